"""Batched form on the GPU: ragged flightlines with masks in one plan, graph
replay, and the chunk autotuner."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2003_02978_amd as mf  # noqa: E402
from oracle.mf64 import retrieve as oracle_retrieve  # noqa: E402
from synth.scenes import SceneSpec, make_scene  # noqa: E402
from tests.parity_util import assert_fp32_parity  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _batch():
    """Three ragged, masked flightlines laid out with a NaN-filled gap."""
    specs = [SceneSpec(5, 900, 74, 2, (500.0, 5000.0), (3.0, 30.0), seed=21, flightline=0,
                       mask_max_frac=0.2),
             SceneSpec(3, 2500, 74, 3, (500.0, 5000.0), (3.0, 30.0), seed=21, flightline=1,
                       mask_max_frac=0.2),
             SceneSpec(7, 1333, 74, 2, (500.0, 5000.0), (3.0, 30.0), seed=21, flightline=2,
                       mask_max_frac=0.2)]
    scenes = [make_scene(sp) for sp in specs]
    fls, off = [], 0
    for i, sc in enumerate(scenes):
        S, N, _ = sc.radiance.shape
        fls.append((off, S, N))
        off += S * N + (777 if i == 0 else 0)          # a gap after the first flightline
    L = np.full((off, 74), np.nan, np.float32)
    V = np.zeros(off, np.uint8)
    for (o, S, N), sc in zip(fls, scenes):
        L[o:o + S * N] = sc.radiance.reshape(S * N, 74)
        V[o:o + S * N] = sc.valid.reshape(S * N)
    return scenes, fls, L, V


@pytest.mark.parametrize("cov", ["lowrank", "fp64"])
def test_ragged_masked_batch_matches_oracle(cov):
    scenes, fls, L, V = _batch()
    s = scenes[0].s
    plan = mf.Plan(fls, 74, 20, 3.0, 1e-9, True, cov, chunk_lines=512)
    Lt = torch.from_numpy(L).to(DEV)
    Vt = torch.from_numpy(V).to(DEV)
    st = torch.from_numpy(s).to(DEV)
    alpha = torch.full((L.shape[0],), -7.0, dtype=torch.float32, device=DEV)
    status = torch.empty(plan.n_columns, dtype=torch.int32, device=DEV)
    plan.retrieve(Lt, st, alpha, Vt, status)
    torch.cuda.synchronize()
    a = alpha.cpu().numpy()
    assert np.all(a[fls[0][1] * fls[0][2]:fls[1][0]] == -7.0)   # the gap is never written
    assert np.all(status.cpu().numpy() == 0)
    for (o, S, N), sc in zip(fls, scenes):
        ref, rst = oracle_retrieve(sc.radiance, s, 20, 3.0, valid=sc.valid)
        got = a[o:o + S * N].reshape(S, N)
        assert np.all(got[sc.valid == 0] == 0)
        assert_fp32_parity(got, ref, label=f"batch flightline at {o} cov={cov}")


def test_graph_replays_match_eager():
    scenes, fls, L, V = _batch()
    plan = mf.Plan(fls, 74, 12, 2.0, 1e-9, True, "lowrank", chunk_lines=256)
    Lt = torch.from_numpy(L).to(DEV)
    Vt = torch.from_numpy(V).to(DEV)
    st = torch.from_numpy(scenes[0].s).to(DEV)
    ws = plan.alloc_workspace()
    eager = torch.empty(L.shape[0], dtype=torch.float32, device=DEV)
    plan.retrieve(Lt, st, eager, Vt, None, ws)
    torch.cuda.synchronize()
    inplan = np.zeros(L.shape[0], bool)          # pixels of the plan (not the gap)
    for o, S, N in fls:
        inplan[o:o + S * N] = True
    ref = eager.cpu().numpy()[inplan]
    stream = torch.cuda.Stream()
    plan.set_graph(True)
    out = torch.empty_like(eager)
    for rep in range(4):
        out.fill_(123.0)
        junk = torch.randn(1 << 20, device=DEV).sum()      # eager work between replays
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            plan.retrieve(Lt, st, out, Vt, None, ws, stream=stream)
        stream.synchronize()
        got = out.cpu().numpy()[inplan]
        np.testing.assert_array_equal(got, ref, err_msg=f"replay {rep}")
        del junk
    plan.set_graph(False)


def test_autotuner_picks_a_candidate(tmp_path):
    scenes, fls, L, V = _batch()
    Lt = torch.from_numpy(L).to(DEV)
    Vt = torch.from_numpy(V).to(DEV)
    st = torch.from_numpy(scenes[0].s).to(DEV)
    cache = str(tmp_path / "tune.json")
    best, times = mf.autotune_chunk(fls, Lt, st, Vt, candidates=(256, 512, 1024), reps=2,
                                    cache_path=cache, n_iter=5, lam=2.0)
    assert best in (256, 512, 1024) and set(times) == {256, 512, 1024}
    best2, _ = mf.autotune_chunk(fls, Lt, st, Vt, candidates=(256, 512, 1024), reps=2,
                                 cache_path=cache, n_iter=5, lam=2.0)
    assert best2 == best
