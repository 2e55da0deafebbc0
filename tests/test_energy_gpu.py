"""The per-iteration energy E^0..E^K (Eq. 8 with the 1/2 of the alpha update)
the low-rank form records on the GPU, against the FP64 oracle's energy list of
each partition, formed there from explicit residuals and Cholesky solves."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2003_02978_amd as mf  # noqa: E402
from oracle.mf64 import retrieve_column  # noqa: E402
from synth.scenes import SceneSpec, make_scene  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _gpu_energy(sc, K, lam, albedo=True, group=1, chunk=0):
    S, N, B = sc.radiance.shape
    plan = mf.Plan([(0, S, N)], B, K, lam, 1e-9, albedo, "lowrank", chunk_lines=chunk, group=group,
                   track_energy=True)
    ws = plan.alloc_workspace(DEV)
    L = torch.from_numpy(sc.radiance).to(DEV)
    s = torch.from_numpy(sc.s).to(DEV)
    valid = None if sc.valid is None else torch.from_numpy(sc.valid).to(DEV)
    alpha = torch.empty((S, N), dtype=torch.float32, device=DEV)
    status = torch.empty(plan.n_columns, dtype=torch.int32, device=DEV)
    plan.retrieve(L, s, alpha, valid, status, ws)
    E = plan.energy(ws)
    torch.cuda.synchronize()
    out = E.cpu().numpy(), status.cpu().numpy()
    plan.close()
    return out


def _oracle_energy(sc, K, lam, albedo=True, group=1):
    S, N, B = sc.radiance.shape
    rows, status = [], []
    for c0 in range(0, S, group):
        c1 = min(S, c0 + group)
        Lp = sc.radiance[c0:c1].reshape(-1, B)
        vp = None if sc.valid is None else sc.valid[c0:c1].reshape(-1)
        e = []
        _, st = retrieve_column(Lp, sc.s, K, lam, 1e-9, albedo, vp, energy=e)
        rows.append(e + [np.nan] * (K + 1 - len(e)))
        status.append(st)
    return np.array(rows).T, np.array(status)


def _check(E, Er, label):
    ok = np.isfinite(Er)
    assert np.array_equal(np.isfinite(E), ok), label
    err = np.abs(E[ok] - Er[ok]) / np.abs(Er[ok])
    print(f"{label}: {int(ok.sum())} energies, max rel err {err.max():.2e}", flush=True)
    assert err.max() < 1e-7, label


@pytest.mark.parametrize("K,lam,albedo,mask,chunk", [(5, 2.0, True, 0.1, 256), (0, 1.0, True, 0.0, 0),
                                                     (3, 0.0, False, 0.0, 128), (30, 4.0, True, 0.05, 0)])
def test_energy_matches_oracle(K, lam, albedo, mask, chunk):
    # 333 lines: odd (unaligned columns) and, with 128/256-pixel items, ragged
    sc = make_scene(SceneSpec(4, 333 if K < 30 else 1200, 74, 2, (800.0, 5000.0), (3.0, 12.0), seed=53,
                              mask_max_frac=mask))
    E, st = _gpu_energy(sc, K, lam, albedo, chunk=chunk)
    Er, rst = _oracle_energy(sc, K, lam, albedo)
    np.testing.assert_array_equal(st, rst)
    _check(E, Er, f"K={K} lam={lam} albedo={albedo} mask={mask} chunk={chunk}")


def test_energy_detector_grouping():
    sc = make_scene(SceneSpec(5, 200, 74, 2, (800.0, 5000.0), (3.0, 12.0), seed=59))
    E, st = _gpu_energy(sc, 6, 2.0, group=3)
    Er, rst = _oracle_energy(sc, 6, 2.0, group=3)
    assert E.shape == (7, 2)
    np.testing.assert_array_equal(st, rst)
    _check(E, Er, "group=3")


def test_energy_of_a_failed_partition_is_nan():
    sc = make_scene(SceneSpec(3, 300, 74, 2, (800.0, 5000.0), (3.0, 12.0), seed=61))
    sc.valid = np.ones((3, 300), np.uint8)
    sc.valid[1, 60:] = 0                      # 60 valid pixels <= B bands
    E, st = _gpu_energy(sc, 4, 1.0)
    Er, rst = _oracle_energy(sc, 4, 1.0)
    assert st[1] == mf.MF_COL_FEW_PIXELS and st[0] == st[2] == mf.MF_COL_OK
    assert np.all(np.isnan(E[:, 1]))
    _check(E, Er, "failed partition")


def test_energy_needs_a_tracking_plan():
    plan = mf.Plan([(0, 2, 200)], 74, 2)
    ws = plan.alloc_workspace(DEV)
    with pytest.raises(Exception, match="track_energy"):
        plan.energy(ws)
    plan.close()


def test_energy_long_run_one_partition():
    """100 iterations with every detector of a small flightline pooled into one
    partition (63 work items of 128 pixels), checked at every iteration."""
    sc = make_scene(SceneSpec(8, 1000, 74, 3, (800.0, 5000.0), (3.0, 12.0), seed=67))
    E, st = _gpu_energy(sc, 100, 1.0, group=8, chunk=128)
    Er, rst = _oracle_energy(sc, 100, 1.0, group=8)
    assert E.shape == (101, 1)
    np.testing.assert_array_equal(st, rst)
    _check(E, Er, "100 iterations, one partition")
