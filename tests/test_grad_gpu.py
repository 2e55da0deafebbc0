"""The hand-written adjoint (mf_backward through torch.autograd) against the
torch-FP64 reference gradient and central finite differences of the FP64
numpy oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2003_02978_amd as mf  # noqa: E402
from oracle.grad64 import fd_radiance, fd_target, loss_and_grads  # noqa: E402
from synth.scenes import SceneSpec, make_scene, make_globals  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _gpu_grads(sc, K, lam, albedo=True):
    L = torch.from_numpy(sc.radiance).to(DEV).requires_grad_(True)
    s = torch.from_numpy(sc.s).to(DEV).requires_grad_(True)
    valid = None if sc.valid is None else torch.from_numpy(sc.valid).to(DEV)
    at = torch.from_numpy(sc.alpha_true).to(DEV)
    alpha = mf.retrieve_differentiable(L, s, K, lam, 1e-9, albedo, valid)
    m = torch.ones_like(alpha) if valid is None else valid.to(alpha.dtype)
    J = (((alpha.double() - at) ** 2) * m).sum()
    J.backward()
    torch.cuda.synchronize()
    return float(J), L.grad.cpu().numpy().astype(np.float64), s.grad.cpu().numpy().astype(np.float64)


def _rel_err(g, ref):
    return float(np.abs(g - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.mark.parametrize("K,lam,albedo,mask", [(0, 1.0, True, 0.0), (1, 0.0, True, 0.0),
                                               (5, 2.0, True, 0.0), (5, 2.0, False, 0.0),
                                               (5, 2.0, True, 0.15)])
def test_adjoint_matches_reference_gradient(K, lam, albedo, mask):
    sc = make_scene(SceneSpec(4, 300, 74, 2, (800.0, 5000.0), (3.0, 12.0), seed=31, mask_max_frac=mask))
    J, gL, gs = _gpu_grads(sc, K, lam, albedo)
    L = sc.radiance.astype(np.float64)
    L[np.isnan(L)] = 0.0
    Jr, gLr, gsr = loss_and_grads(L, sc.s, sc.alpha_true, K, lam, albedo=albedo, valid=sc.valid)
    print(f"K={K} lam={lam} albedo={albedo} mask={mask}: J {J:.6e} ref {Jr:.6e}, "
          f"grad L rel err {_rel_err(gL, gLr):.2e}, grad s rel err {_rel_err(gs, gsr):.2e}", flush=True)
    assert abs(J - Jr) <= 1e-6 * Jr
    if sc.valid is not None:
        assert np.all(gL[sc.valid == 0] == 0)
    assert _rel_err(gL, gLr) < 1e-4
    assert _rel_err(gs, gsr) < 1e-4


def test_adjoint_odd_lines_ragged_items():
    """Odd line counts (every other column off 16-byte alignment) with 128-line
    work items and ragged chunks, through the plan's backward directly."""
    sc = make_scene(SceneSpec(5, 333, 74, 2, (800.0, 5000.0), (3.0, 12.0), seed=37, mask_max_frac=0.1))
    S, N, B = sc.radiance.shape
    K, lam = 6, 2.0
    plan = mf.Plan([(0, S, N)], B, K, lam, 1e-9, True, "lowrank", chunk_lines=128,
                   save_for_backward=True)
    ws = plan.alloc_workspace(DEV)
    L = torch.from_numpy(sc.radiance).to(DEV)
    s = torch.from_numpy(sc.s).to(DEV)
    valid = torch.from_numpy(sc.valid).to(DEV)
    alpha = torch.empty((S, N), dtype=torch.float32, device=DEV)
    plan.retrieve(L, s, alpha, valid, None, ws)
    at = torch.from_numpy(sc.alpha_true).to(DEV)
    g = (2.0 * (alpha.double() - at) * valid.double()).float()
    gL, gs = plan.backward(L, s, g, valid, ws)
    torch.cuda.synchronize()
    Lr = sc.radiance.astype(np.float64)
    Lr[np.isnan(Lr)] = 0.0
    Jr, gLr, gsr = loss_and_grads(Lr, sc.s, sc.alpha_true, K, lam, valid=sc.valid)
    gL = gL.cpu().numpy().astype(np.float64)
    gs = gs.cpu().numpy()
    print(f"odd lines: grad L rel err {_rel_err(gL, gLr):.2e}, grad s rel err {_rel_err(gs, gsr):.2e}",
          flush=True)
    assert np.all(gL[sc.valid == 0] == 0)
    assert _rel_err(gL, gLr) < 1e-4
    assert _rel_err(gs, gsr) < 1e-4
    plan.close()


def test_adjoint_detector_grouping():
    """Partitions of 3 adjacent columns (remainder 2): the adjoint against the
    reference gradient of each partition run as one column."""
    sc = make_scene(SceneSpec(5, 200, 74, 2, (800.0, 5000.0), (3.0, 12.0), seed=41))
    S, N, B = sc.radiance.shape
    K, lam, g = 5, 2.0, 3
    L = torch.from_numpy(sc.radiance).to(DEV).requires_grad_(True)
    s = torch.from_numpy(sc.s).to(DEV).requires_grad_(True)
    at = torch.from_numpy(sc.alpha_true).to(DEV)
    alpha = mf.retrieve_differentiable(L, s, K, lam, 1e-9, True, None, group=g)
    J = ((alpha.double() - at) ** 2).sum()
    J.backward()
    torch.cuda.synchronize()
    gL = L.grad.cpu().numpy().astype(np.float64)
    gs = s.grad.cpu().numpy().astype(np.float64)
    Jr, gLr, gsr = 0.0, np.zeros_like(gL), np.zeros(B)
    for c0 in range(0, S, g):
        c1 = min(S, c0 + g)
        Lp = sc.radiance[c0:c1].astype(np.float64).reshape(1, (c1 - c0) * N, B)
        Ap = sc.alpha_true[c0:c1].reshape(1, -1)
        j, gl, gsp = loss_and_grads(Lp, sc.s, Ap, K, lam)
        Jr += j
        gLr[c0:c1] = gl.reshape(c1 - c0, N, B)
        gsr += gsp
    print(f"grouping: J {float(J):.6e} ref {Jr:.6e}, grad L rel err {_rel_err(gL, gLr):.2e}, "
          f"grad s rel err {_rel_err(gs, gsr):.2e}", flush=True)
    assert abs(float(J) - Jr) <= 1e-6 * Jr
    assert _rel_err(gL, gLr) < 1e-4
    assert _rel_err(gs, gsr) < 1e-4


def test_adjoint_subscene_16x256_30_iterations():
    """The differentiation workload's reference check: a 16 x 256 sub-scene of
    the 598 x 4000 scene, 30 iterations, against torch FP64 autograd."""
    spec = SceneSpec(598, 4000, 74, 40, (200.0, 8000.0), (3.0, 30.0), seed=1004)
    g = make_globals(spec)
    # the sub-scene: columns 0-15, lines 0-255 of the scene (regenerated per column)
    from synth.scenes import make_column
    Ls, As = [], []
    for c in range(16):
        Lc, ac, _ = make_column(spec, g, c)
        Ls.append(Lc[:256])
        As.append(ac[:256])
    sub = make_scene(SceneSpec(16, 256, 74, 0, seed=5))
    sub.radiance = np.stack(Ls)
    sub.alpha_true = np.stack(As)
    sub.s = g.s
    lam = 4.0
    J, gL, gs = _gpu_grads(sub, 30, lam)
    Jr, gLr, gsr = loss_and_grads(sub.radiance, sub.s, sub.alpha_true, 30, lam)
    print(f"sub-scene: J {J:.6e} ref {Jr:.6e}, grad L rel err {_rel_err(gL, gLr):.2e}, "
          f"grad s rel err {_rel_err(gs, gsr):.2e}", flush=True)
    assert abs(J - Jr) <= 1e-6 * Jr
    assert _rel_err(gL, gLr) < 1e-4
    assert _rel_err(gs, gsr) < 1e-4


def test_adjoint_finite_differences():
    """Central differences (FP64 numpy oracle) on random radiance coordinates
    and on the most absorbing bands of s."""
    sc = make_scene(SceneSpec(3, 1500, 74, 3, (800.0, 6000.0), (3.0, 20.0), seed=41))
    K, lam = 30, 3.0
    J, gL, gs = _gpu_grads(sc, K, lam)
    L = sc.radiance.astype(np.float64)
    rng = np.random.default_rng(5)
    checked, tries = 0, 0
    while checked < 12 and tries < 60:
        tries += 1
        c, i, b = int(rng.integers(3)), int(rng.integers(1500)), int(rng.integers(74))
        fd1 = fd_radiance(L, sc.s, sc.alpha_true, (c, i, b), 1e-3, K, lam)
        fd2 = fd_radiance(L, sc.s, sc.alpha_true, (c, i, b), 5e-4, K, lam)
        if abs(fd1 - fd2) > 1e-3 * (abs(fd1) + 1e-3):     # a sparsity flip in the stencil
            continue
        assert abs(gL[c, i, b] - fd1) <= 2e-3 * abs(fd1) + 1e-6 * np.abs(gL).max(), (c, i, b, gL[c, i, b], fd1)
        checked += 1
    assert checked >= 8
    for b in np.argsort(np.abs(sc.s))[-3:]:
        fd = fd_target(L, sc.s, sc.alpha_true, int(b), 1e-4, K, lam)
        assert abs(gs[b] - fd) <= 2e-3 * abs(fd), (int(b), gs[b], fd)
