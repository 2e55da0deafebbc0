"""The reference gradient (torch FP64 autograd over Fig. 1) against the numpy
oracle: same forward, and gradients equal to central finite differences of the
numpy oracle, which share nothing with autograd."""
import numpy as np
import pytest
import torch

from oracle.grad64 import fd_radiance, fd_target, loss_and_grads, loss_numpy, retrieve_column_torch
from oracle.mf64 import retrieve_column
from synth.scenes import SceneSpec, make_scene


def _scene(mask=0.0, seed=77):
    return make_scene(SceneSpec(3, 160, 12, 2, (800.0, 5000.0), (3.0, 8.0), seed=seed,
                                mask_max_frac=mask))


@pytest.mark.parametrize("K,lam,albedo", [(0, 1.0, True), (1, 0.0, True), (6, 2.0, True), (6, 2.0, False)])
def test_torch_forward_equals_oracle(K, lam, albedo):
    sc = _scene()
    for c in range(3):
        a_np, _ = retrieve_column(sc.radiance[c], sc.s, K, lam, albedo=albedo)
        a_t = retrieve_column_torch(torch.tensor(sc.radiance[c], dtype=torch.float64),
                                    torch.tensor(sc.s, dtype=torch.float64), K, lam, albedo=albedo)
        np.testing.assert_allclose(a_t.numpy(), a_np, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("K,lam,mask", [(0, 1.0, 0.0), (4, 2.0, 0.0), (4, 2.0, 0.15)])
def test_autograd_matches_finite_differences(K, lam, mask):
    sc = _scene(mask)
    L = sc.radiance.astype(np.float64)
    L[np.isnan(L)] = 0.0                       # masked values never enter the sums
    J, gL, gs = loss_and_grads(L, sc.s, sc.alpha_true, K, lam, valid=sc.valid)
    assert abs(J - loss_numpy(L, sc.s, sc.alpha_true, K, lam, valid=sc.valid)) <= 1e-9 * J
    rng = np.random.default_rng(3)
    checked = 0
    while checked < 6:
        c, i, b = int(rng.integers(3)), int(rng.integers(160)), int(rng.integers(12))
        if sc.valid is not None and sc.valid[c, i] == 0:
            assert gL[c, i, b] == 0.0
            continue
        fd = fd_radiance(L, sc.s, sc.alpha_true, (c, i, b), 1e-4, K, lam, valid=sc.valid)
        fd2 = fd_radiance(L, sc.s, sc.alpha_true, (c, i, b), 2e-4, K, lam, valid=sc.valid)
        if abs(fd - fd2) > 1e-3 * (abs(fd) + 1.0):   # a sparsity flip inside the stencil
            continue
        np.testing.assert_allclose(gL[c, i, b], fd, rtol=2e-4, atol=1e-6 * (1 + abs(fd)))
        checked += 1
    for b in np.argsort(np.abs(sc.s))[-2:]:      # the two most absorbing bands
        fd = fd_target(L, sc.s, sc.alpha_true, int(b), 1e-5, K, lam, valid=sc.valid)
        np.testing.assert_allclose(gs[b], fd, rtol=2e-4)
