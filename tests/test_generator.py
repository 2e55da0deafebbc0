"""Synthetic scene generator: fixtures of the recipe and reproducibility."""
import hashlib
import json
import os

import numpy as np

from synth.scenes import (batch_specs, make_column, make_globals, make_scene,
                          tiny_spec, SceneSpec)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_oracle.json")


def test_target_dip_and_sign():
    g = make_globals(tiny_spec())
    # 3 % transmittance dip at 1000 ppm*m at the deepest band (Beer-Lambert)
    assert abs(np.exp(1000.0 * float(g.s.min())) - 0.97) < 1e-6
    assert np.all(g.s <= 0)
    assert g.s.dtype == np.float32 and g.s.shape == (74,)
    np.testing.assert_allclose(g.wavelengths[[0, -1]], [2122.0, 2487.0])
    assert g.endmembers.min() >= 1.0 - 1e-12 and g.endmembers.max() <= 10.0 + 1e-12


def test_plumes_are_exactly_zero_outside_3_sigma():
    spec = tiny_spec()
    sc = make_scene(spec)
    g = make_globals(spec)
    assert sc.alpha_true.max() <= spec.peak_range[1] * 3 + 1e-9
    zero = sc.alpha_true == 0
    assert zero.sum() > 0
    cc, ll = np.meshgrid(np.arange(spec.n_columns) + 0.5, np.arange(spec.n_lines) + 0.5,
                         indexing="ij")
    inside_any = np.zeros_like(zero)
    for pc, pl, ps, pk in g.plumes:
        inside_any |= (cc - pc) ** 2 + (ll - pl) ** 2 <= (3 * ps) ** 2
    np.testing.assert_array_equal(zero, ~inside_any)


def test_reproducible_and_column_local():
    spec = tiny_spec()
    a = make_scene(spec)
    g = make_globals(spec)
    L5, al5, _ = make_column(spec, g, 5)
    np.testing.assert_array_equal(a.radiance[5], L5)
    np.testing.assert_array_equal(a.alpha_true[5], al5)
    ref = json.load(open(GOLDEN))
    assert hashlib.sha256(a.radiance.tobytes()).hexdigest() == ref["radiance_sha256"]
    assert hashlib.sha256(a.s.tobytes()).hexdigest() == ref["s_sha256"]


def test_masks_runs_and_nan():
    spec = SceneSpec(4, 3000, 74, 2, seed=7, mask_max_frac=0.2)
    sc = make_scene(spec)
    assert sc.valid is not None and sc.valid.dtype == np.uint8
    frac = 1 - sc.valid.mean(axis=1)
    assert np.all(frac <= 0.2 + 64 / 3000)
    assert np.all(np.isnan(sc.radiance[sc.valid == 0]))
    assert np.all(np.isfinite(sc.radiance[sc.valid == 1]))


def test_batch_lengths():
    specs = batch_specs()
    assert len(specs) == 32
    lens = np.array([s.n_lines for s in specs])
    assert lens.min() >= 1000 and lens.max() <= 12000
    assert all(s.n_columns == 598 and s.mask_max_frac == 0.2 for s in specs)
    # one target spectrum for the whole batch; backgrounds and plumes differ
    g0, g7 = make_globals(specs[0]), make_globals(specs[7])
    assert np.array_equal(g0.s, g7.s)
    assert not np.array_equal(g0.endmembers, g7.endmembers)
    assert not np.array_equal(g0.plumes, g7.plumes)
