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


def _diff_workload():
    """The differentiation workload: 598 x 4000 x 74, 30 iterations, its lambda."""
    from synth.scenes import diff_spec
    from tests.parity_util import config_lambda
    return diff_spec(), config_lambda("diff")


def _subscene(spec, g, c0, l0):
    """Columns c0..c0+15, lines l0..l0+255 of the scene (regenerated per column),
    as a scene of its own (each 256-line column is one partition)."""
    from synth.scenes import make_column
    Ls, As = [], []
    for c in range(c0, c0 + 16):
        Lc, ac, _ = make_column(spec, g, c)
        Ls.append(Lc[l0:l0 + 256])
        As.append(ac[l0:l0 + 256])
    sub = make_scene(SceneSpec(16, 256, 74, 0, seed=5))
    sub.radiance = np.stack(Ls)
    sub.alpha_true = np.stack(As)
    sub.s = g.s
    return sub


def _elementwise(g, ref, rtol=1e-4, floor_frac=1e-6):
    """Per-element check |g - ref| <= rtol |ref| + floor, floor = floor_frac
    max|ref|: returns (violations, largest relative error above the floor)."""
    floor = floor_frac * max(float(np.abs(ref).max()), 1e-300)
    err = np.abs(g - ref)
    viol = int((err > rtol * np.abs(ref) + floor).sum())
    above = np.abs(ref) > floor
    rel = float((err[above] / np.abs(ref[above])).max()) if above.any() else 0.0
    return viol, rel


@pytest.mark.parametrize("window", ["first_columns", "through_plume"])
def test_adjoint_subscene_16x256_30_iterations(window):
    """The differentiation workload's reference check at its own lambda: a
    16 x 256 sub-scene of the 598 x 4000 scene, 30 iterations, against torch
    FP64 autograd, element by element.  Columns 0-15 x lines 0-255 hold no
    plume: every alpha is locked at 0 and both gradients are exactly zero.
    The second window, columns 160-175 x lines 2384-2639, is centred on plume
    4 of the scene (sigma 5.8 px, peak 5244 ppm*m): of the 40 plume-centred
    16 x 256 windows it is the one whose own retrieval at this lambda keeps
    the most nonzero alpha (113, found with the oracle; a wide plume fills a
    256-line column, enters its mean and covariance, and leaves alpha at 0)."""
    spec, lam = _diff_workload()
    g = make_globals(spec)
    c0, l0 = (0, 0) if window == "first_columns" else (160, 2384)
    sub = _subscene(spec, g, c0, l0)
    J, gL, gs = _gpu_grads(sub, 30, lam)
    Jr, gLr, gsr = loss_and_grads(sub.radiance, sub.s, sub.alpha_true, 30, lam)
    vL, rL = _elementwise(gL, gLr)
    vs, rs = _elementwise(gs, gsr)
    print(f"sub-scene {window} (columns {c0}-{c0 + 15}, lines {l0}-{l0 + 255}, lambda {lam:.4g}): "
          f"J {J:.6e} ref {Jr:.6e}; grad L: {vL} violations, max rel err above floor {rL:.2e}; "
          f"grad s: {vs} violations, max rel err {rs:.2e}; max|grad L| {np.abs(gLr).max():.3e}",
          flush=True)
    assert abs(J - Jr) <= 1e-6 * max(Jr, 1e-300)
    if window == "first_columns":
        assert np.all(gLr == 0) and np.all(gsr == 0)
        assert np.all(gL == 0) and np.all(gs == 0)
    else:
        assert np.abs(gLr).max() > 0 and np.abs(gsr).max() > 0
        assert vL == 0 and vs == 0


def test_adjoint_finite_differences_differentiation_scene():
    """Central finite differences (FP64 numpy oracle, h = 1e-3) on 16 random
    coordinates of the 598 x 4000 differentiation scene at its lambda.

    12 radiance coordinates (6 pixels with alpha > 0, 6 pixels of columns
    with a nonzero alpha; only the touched column is re-run), against the
    gradient of the whole loss.  A stencil whose +h or -h run changes the
    sparsity pattern is rejected and resampled, and so is one whose
    difference quotient moves by more than 1e-3 relative between h and h/2
    (a kink inside the stencil).

    4 target bands with |s_b| >= 5 % of max|s| (step 1e-3 |s_b|), on the loss
    of 64 random columns with a nonzero alpha (the columns whose alpha is all
    zero stay locked at zero).  Pixels near the reweighting map's bifurcation
    make J smooth but so curved in s that the difference quotient of a whole
    column moves by percents between h and h/4, so each band keeps the columns
    whose own quotient agrees to 1e-3 between h and h/2, and the adjoint is
    run with the loss restricted to those columns."""
    from oracle.mf64 import retrieve as oracle_retrieve, retrieve_column
    spec, lam = _diff_workload()
    sc = make_scene(spec)
    S, N, B = sc.radiance.shape
    K = 30
    J, gL, gs = _gpu_grads(sc, K, lam)
    L = sc.radiance.astype(np.float64)
    at = sc.alpha_true
    base, _ = oracle_retrieve(sc.radiance, sc.s, K, lam, workers=16)
    pattern = base > 0
    act = np.flatnonzero(pattern.any(axis=1))

    def col_run(c, Lc, s):
        a, _ = retrieve_column(Lc, s, K, lam)
        return a, float(((a - at[c]) ** 2).sum())

    rng = np.random.default_rng(2020)
    on = np.argwhere(pattern)
    checked, tries, worst = 0, 0, 0.0
    while checked < 12 and tries < 80:
        tries += 1
        if checked < 6:
            c, i = on[rng.integers(len(on))]
        else:
            c, i = int(rng.choice(act)), int(rng.integers(N))
        b = int(rng.integers(B))
        q = []
        ok = True
        for h in (1e-3, 5e-4):
            Lp, Lm = L[c].copy(), L[c].copy()
            Lp[i, b] += h
            Lm[i, b] -= h
            ap, Jp = col_run(c, Lp, sc.s)
            am, Jm = col_run(c, Lm, sc.s)
            if np.any((ap > 0) != pattern[c]) or np.any((am > 0) != pattern[c]):
                ok = False
                break
            q.append((Jp - Jm) / (2 * h))
        if not ok or abs(q[0] - q[1]) > 1e-3 * abs(q[0]) + 1e-9:
            continue
        fd = q[0]
        err = abs(gL[c, i, b] - fd)
        assert err <= 2e-3 * abs(fd) + 1e-6 * np.abs(gL).max(), (c, i, b, gL[c, i, b], fd)
        worst = max(worst, err / max(abs(fd), 1e-300))
        checked += 1
    assert checked == 12, (checked, tries)

    # target bands on the loss of a column subset, through the plan's backward
    cols = np.sort(rng.choice(act, 64, replace=False))
    dev_L = torch.from_numpy(sc.radiance).to(DEV)
    dev_s = torch.from_numpy(sc.s).to(DEV)
    dev_at = torch.from_numpy(at).to(DEV)
    plan = mf.Plan([(0, S, N)], B, K, lam, 1e-9, True, "lowrank", save_for_backward=True)
    ws = plan.alloc_workspace(DEV)
    alpha = torch.empty((S, N), dtype=torch.float32, device=DEV)
    bands = np.flatnonzero(np.abs(sc.s) >= 0.05 * np.abs(sc.s).max())
    sb_checked, kept = 0, []
    for b in rng.permutation(bands):
        if sb_checked == 4:
            break
        q = []
        ok = True
        for rel in (1e-3, 5e-4):
            h = rel * abs(float(sc.s[b]))
            per = []
            for sgn in (1.0, -1.0):
                sp = sc.s.astype(np.float64).copy()
                sp[b] += sgn * h
                a, _ = oracle_retrieve(sc.radiance, sp, K, lam, columns=list(cols), workers=16)
                ok = ok and not np.any((a > 0) != pattern[cols])
                per.append(((a - at[cols]) ** 2).sum(axis=1))
            q.append((per[0] - per[1]) / (2 * h))
        if not ok:
            continue
        smooth = np.abs(q[0] - q[1]) <= 1e-3 * np.abs(q[0]) + 1e-9
        if smooth.sum() < 16:
            continue
        fd = float(q[0][smooth].sum())
        mask = torch.zeros((S, 1), dtype=torch.float64, device=DEV)
        mask[torch.from_numpy(cols[smooth]).to(DEV)] = 1.0
        plan.retrieve(dev_L, dev_s, alpha, None, None, ws)
        g = (2.0 * (alpha.double() - dev_at) * mask).float()
        _, gsb = plan.backward(dev_L, dev_s, g, None, ws)
        torch.cuda.synchronize()
        gb = float(gsb.cpu().numpy()[b])
        assert abs(gb - fd) <= 2e-3 * abs(fd), (int(b), gb, fd, int(smooth.sum()))
        kept.append(int(smooth.sum()))
        sb_checked += 1
    plan.close()
    print(f"differentiation scene: 12 radiance coordinates in {tries} draws, worst rel err {worst:.2e}; "
          f"{sb_checked} target bands on {kept} of 64 columns", flush=True)
    assert sb_checked == 4


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


@pytest.mark.parametrize("K,n_streams", [(31, 1), (61, 1), (94, 2), (95, 1)])
def test_adjoint_more_than_thirty_iterations(K, n_streams):
    """K > 30: the gradient assembly runs in several blocks of 64 coefficient
    slots (K = 31: a second block with two slots; 61: two full blocks; 94:
    three full blocks; 95: a fourth with two) summed in FP64; odd line
    counts, 128-line work items, masks."""
    sc = make_scene(SceneSpec(4, 301, 74, 2, (800.0, 5000.0), (3.0, 12.0), seed=53, mask_max_frac=0.1))
    S, N, B = sc.radiance.shape
    lam = 2.0
    plan = mf.Plan([(0, S, N)], B, K, lam, 1e-9, True, "lowrank", chunk_lines=128,
                   save_for_backward=True)
    plan.set_streams(n_streams)
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
    print(f"K={K} streams={n_streams}: grad L rel err {_rel_err(gL, gLr):.2e}, "
          f"grad s rel err {_rel_err(gs, gsr):.2e}", flush=True)
    assert np.all(gL[sc.valid == 0] == 0)
    assert _rel_err(gL, gLr) < 1e-4
    assert _rel_err(gs, gsr) < 1e-4
    plan.close()


def test_adjoint_forty_iterations_grouped_autograd():
    """K = 40 (two assembly blocks) through torch.autograd, with partitions of
    3 columns (remainder 2), albedo off and two partition groups: against
    the reference gradient of each partition run as one column."""
    sc = make_scene(SceneSpec(5, 200, 74, 2, (800.0, 5000.0), (3.0, 12.0), seed=59))
    S, N, B = sc.radiance.shape
    K, lam, g = 40, 2.0, 3
    L = torch.from_numpy(sc.radiance).to(DEV).requires_grad_(True)
    s = torch.from_numpy(sc.s).to(DEV).requires_grad_(True)
    at = torch.from_numpy(sc.alpha_true).to(DEV)
    alpha = mf.retrieve_differentiable(L, s, K, lam, 1e-9, False, None, group=g, streams=2)
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
        j, gl, gsp = loss_and_grads(Lp, sc.s, Ap, K, lam, albedo=False)
        Jr += j
        gLr[c0:c1] = gl.reshape(c1 - c0, N, B)
        gsr += gsp
    print(f"K=40 grouped autograd: J {float(J):.6e} ref {Jr:.6e}, grad L rel err {_rel_err(gL, gLr):.2e}, "
          f"grad s rel err {_rel_err(gs, gsr):.2e}", flush=True)
    assert abs(float(J) - Jr) <= 1e-6 * Jr
    assert _rel_err(gL, gLr) < 1e-4
    assert _rel_err(gs, gsr) < 1e-4


@pytest.mark.parametrize("n_streams", [2, 5])
def test_adjoint_streams_bit_identical(n_streams):
    """Both sweeps with concurrent partition groups (up to one per partition)
    give the one-stream gradients bit for bit: odd line counts, ragged
    128-line work items, masks."""
    sc = make_scene(SceneSpec(5, 333, 74, 2, (800.0, 5000.0), (3.0, 12.0), seed=41, mask_max_frac=0.1))
    S, N, B = sc.radiance.shape
    L = torch.from_numpy(sc.radiance).to(DEV)
    s = torch.from_numpy(sc.s).to(DEV)
    valid = torch.from_numpy(sc.valid).to(DEV)
    at = torch.from_numpy(sc.alpha_true).to(DEV)
    outs = []
    for ns in (1, n_streams):
        plan = mf.Plan([(0, S, N)], B, 8, 2.0, 1e-9, True, "lowrank", chunk_lines=128,
                       save_for_backward=True)
        plan.set_streams(ns)
        ws = plan.alloc_workspace(DEV)
        alpha = torch.empty((S, N), dtype=torch.float32, device=DEV)
        plan.retrieve(L, s, alpha, valid, None, ws)
        g = (2.0 * (alpha.double() - at) * valid.double()).float()
        gL, gs = plan.backward(L, s, g, valid, ws)
        torch.cuda.synchronize()
        outs.append((alpha.cpu().numpy(), gL.cpu().numpy(), gs.cpu().numpy()))
        plan.close()
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(b, a)
    assert np.abs(outs[0][1]).max() > 0
