"""The FP64 oracle against its stored results (tests/golden/make_golden.py)."""
import json
import os

import numpy as np

from oracle.mf64 import retrieve
from synth.scenes import make_scene, tiny_spec

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_oracle.json")


def test_oracle_matches_stored_values():
    ref = json.load(open(GOLDEN))
    sc = make_scene(tiny_spec())
    cols = sorted(int(c) for c in ref["columns"])
    a, st = retrieve(sc.radiance, sc.s, 30, ref["lambda"], 1e-9, columns=cols)
    a0, _ = retrieve(sc.radiance, sc.s, 0, ref["lambda"], 1e-9, columns=cols)
    for i, c in enumerate(cols):
        r = ref["columns"][str(c)]
        assert st[i] == r["status"]
        assert int((a[i] > 0).sum()) == r["nonzero"]
        np.testing.assert_allclose(a[i].sum(), r["sum"], rtol=1e-9)
        for j, v in r["samples"].items():
            np.testing.assert_allclose(a[i][int(j)], v, rtol=1e-9, atol=1e-9)
        for j, v in r["k0_samples"].items():
            np.testing.assert_allclose(a0[i][int(j)], v, rtol=1e-9, atol=1e-9)
