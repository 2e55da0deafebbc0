"""Write the stored expected values under tests/golden/.

Every value here comes from the FP64 oracle or from the scene generator; none
comes from the GPU path.  Run:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle.mf64 import retrieve  # noqa: E402
from synth.scenes import make_scene, tiny_spec  # noqa: E402


def main():
    sc = make_scene(tiny_spec())
    lam = json.load(open(os.path.join(HERE, "..", "..", "configs", "tiny.json")))["lambda"]
    out = {
        "about": "64x512x74 synthetic scene, seed 1000: generator digest and FP64 oracle "
                 "results (Fig. 1, 30 iterations, eps 1e-9) for the listed columns",
        "radiance_sha256": hashlib.sha256(sc.radiance.tobytes()).hexdigest(),
        "s_sha256": hashlib.sha256(sc.s.tobytes()).hexdigest(),
        "lambda": lam,
        "columns": {},
    }
    cols = [0, 17, 40, 63]
    a, st = retrieve(sc.radiance, sc.s, 30, lam, 1e-9, columns=cols)
    a0, _ = retrieve(sc.radiance, sc.s, 0, lam, 1e-9, columns=cols)
    for i, c in enumerate(cols):
        nz = np.flatnonzero(a[i] > 0)
        out["columns"][str(c)] = {
            "status": int(st[i]),
            "nonzero": int(len(nz)),
            "sum": float(a[i].sum()),
            "samples": {str(j): float(a[i][j]) for j in list(nz[:4]) + [0, 255, 511]},
            "k0_samples": {str(j): float(a0[i][j]) for j in (0, 100, 511)},
        }
    with open(os.path.join(HERE, "tiny_oracle.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print("wrote tiny_oracle.json")


if __name__ == "__main__":
    main()
