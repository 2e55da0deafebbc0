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


@pytest.mark.parametrize("tile", ["32x4", "32x2", "64x2", "64x1"])
@pytest.mark.parametrize("wgs", [0, 1, 3])
def test_launch_shapes_give_the_same_alpha(tile, wgs):
    """Every streaming tile shape, with one workgroup per work item or a
    persistent grid taking work items from the queue (1 and 3 workgroups per
    compute unit: far fewer workgroups than items), gives the default launch's
    alpha and statuses bit for bit on the ragged masked batch (chunks of 128
    lines: many items per column, ragged tails), and matches the oracle."""
    scenes, fls, L, V = _batch()
    s = scenes[0].s
    Lt = torch.from_numpy(L).to(DEV)
    Vt = torch.from_numpy(V).to(DEV)
    st = torch.from_numpy(s).to(DEV)
    outs = []
    for shape in (("32x4", 0), (tile, wgs)):
        plan = mf.Plan(fls, 74, 15, 3.0, 1e-9, True, "lowrank", chunk_lines=128)
        plan.set_launch(*shape)
        alpha = torch.full((L.shape[0],), -7.0, dtype=torch.float32, device=DEV)
        status = torch.empty(plan.n_columns, dtype=torch.int32, device=DEV)
        ws = plan.alloc_workspace()
        plan.retrieve(Lt, st, alpha, Vt, status, ws)
        plan.retrieve(Lt, st, alpha, Vt, status, ws)        # the queue counters restart
        torch.cuda.synchronize()
        outs.append((alpha.cpu().numpy(), status.cpu().numpy()))
        plan.close()
    np.testing.assert_array_equal(outs[1][1], outs[0][1])
    np.testing.assert_array_equal(outs[1][0], outs[0][0])
    o, S, N = fls[1]
    ref, _ = oracle_retrieve(scenes[1].radiance, s, 15, 3.0, valid=scenes[1].valid)
    assert_fp32_parity(outs[1][0][o:o + S * N].reshape(S, N), ref, label=f"tile {tile} wgs {wgs}")


def test_persistent_graph_replays_match_eager():
    """The persistent launch captured in a graph: the queue counters are
    cleared by the retrieval's own first kernel, so every replay (with eager
    work in between) equals the eager result."""
    scenes, fls, L, V = _batch()
    plan = mf.Plan(fls, 74, 12, 2.0, 1e-9, True, "lowrank", chunk_lines=256)
    plan.set_launch("32x2", 2)
    Lt = torch.from_numpy(L).to(DEV)
    Vt = torch.from_numpy(V).to(DEV)
    st = torch.from_numpy(scenes[0].s).to(DEV)
    ws = plan.alloc_workspace()
    eager = torch.empty(L.shape[0], dtype=torch.float32, device=DEV)
    plan.retrieve(Lt, st, eager, Vt, None, ws)
    torch.cuda.synchronize()
    inplan = np.zeros(L.shape[0], bool)
    for o, S, N in fls:
        inplan[o:o + S * N] = True
    ref = eager.cpu().numpy()[inplan]
    stream = torch.cuda.Stream()
    plan.set_graph(True)
    out = torch.empty_like(eager)
    for rep in range(4):
        out.fill_(123.0)
        junk = torch.randn(1 << 20, device=DEV).sum()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            plan.retrieve(Lt, st, out, Vt, None, ws, stream=stream)
        stream.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy()[inplan], ref, err_msg=f"replay {rep}")
        del junk
    plan.set_graph(False)
    plan.close()


def test_launch_autotuner(tmp_path):
    """The autotuner searches work-item length, tile shape, persistent grid
    and concurrent partition groups, returns candidates it timed, caches
    them, and its choice retrieves the same alpha as the default launch."""
    scenes, fls, L, V = _batch()
    Lt = torch.from_numpy(L).to(DEV)
    Vt = torch.from_numpy(V).to(DEV)
    st = torch.from_numpy(scenes[0].s).to(DEV)
    cache = str(tmp_path / "tune.json")
    kw = dict(n_iter=5, lam=2.0)
    best, times = mf.autotune(fls, Lt, st, Vt, chunks=(256, 512), tiles=("32x4", "32x2", "64x2"),
                              wgs=(0, 2), streams=(1, 2), reps=1, cache_path=cache, **kw)
    assert best["chunk_lines"] in (256, 512) and best["stream_tile"] in ("32x4", "32x2", "64x2")
    assert best["wgs_per_cu"] in (0, 2) and best["streams"] in (1, 2) and len(times) >= 5
    best2, _ = mf.autotune(fls, Lt, st, Vt, chunks=(256, 512), tiles=("32x4", "32x2", "64x2"),
                           wgs=(0, 2), streams=(1, 2), reps=1, cache_path=cache, **kw)
    assert best2 == best
    outs = []
    for cfg in ({"chunk_lines": 512, "stream_tile": "32x4", "wgs_per_cu": 0, "streams": 1}, best):
        plan = mf.Plan(fls, 74, 5, 2.0, 1e-9, True, "lowrank", chunk_lines=cfg["chunk_lines"])
        plan.set_launch(cfg["stream_tile"], cfg["wgs_per_cu"])
        plan.set_streams(cfg["streams"])
        a = torch.empty(L.shape[0], dtype=torch.float32, device=DEV)
        plan.retrieve(Lt, st, a, Vt)
        torch.cuda.synchronize()
        outs.append(a.cpu().numpy())
        plan.close()
    inplan = np.zeros(L.shape[0], bool)
    for o, S, N in fls:
        inplan[o:o + S * N] = True
    # a different work-item length changes the order of the partial sums, so
    # the comparison is the FP32 bar against the default launch
    d = np.abs(outs[0][inplan] - outs[1][inplan])
    assert np.all(d <= 1e-4 * np.abs(outs[0][inplan]) + 0.1)


@pytest.mark.parametrize("cov,n_streams,wgs", [("lowrank", 2, 0), ("lowrank", 3, 0), ("lowrank", 8, 0),
                                               ("lowrank", 3, 2), ("fp64", 2, 0), ("bf16x3", 3, 0)])
def test_streams_give_the_same_alpha(cov, n_streams, wgs):
    """Partition groups on concurrent streams (mf_plan_set_streams) give the
    one-stream alpha and statuses bit for bit on the ragged masked batch,
    from 2 groups up to the most the library takes (8), with one workgroup per work
    item or a persistent grid (each group on its own queue counters), for
    the low-rank and Gram forms; the call stays ordered on the caller's
    stream (read right after it without a device-wide synchronisation)."""
    scenes, fls, L, V = _batch()
    Lt = torch.from_numpy(L).to(DEV)
    Vt = torch.from_numpy(V).to(DEV)
    st = torch.from_numpy(scenes[0].s).to(DEV)
    caller = torch.cuda.Stream()
    outs = []
    for ns in (1, n_streams):
        plan = mf.Plan(fls, 74, 12, 3.0, 1e-9, True, cov, chunk_lines=256)
        plan.set_launch("32x4", wgs)
        plan.set_streams(ns)
        assert plan.streams == ns
        alpha = torch.full((L.shape[0],), -7.0, dtype=torch.float32, device=DEV)
        status = torch.full((plan.n_columns,), -1, dtype=torch.int32, device=DEV)
        ws = plan.alloc_workspace()
        torch.cuda.synchronize()
        with torch.cuda.stream(caller):
            for _ in range(2):                                  # the queue counters restart
                plan.retrieve(Lt, st, alpha, Vt, status, ws, stream=caller)
            a_host = alpha.to("cpu", non_blocking=False)         # ordered after the call on `caller`
            s_host = status.to("cpu", non_blocking=False)
        caller.synchronize()
        outs.append((a_host.numpy(), s_host.numpy()))
        plan.close()
    np.testing.assert_array_equal(outs[1][1], outs[0][1])
    np.testing.assert_array_equal(outs[1][0], outs[0][0])
    assert np.all(outs[0][0][fls[0][1] * fls[0][2]:fls[1][0]] == -7.0)   # the gap is never written


def test_streams_graph_replays_match_eager():
    """A graph captured with three concurrent partition groups (the capture
    follows the fork to the plan's streams and the join back): every replay,
    with eager work in between, equals the one-stream eager result."""
    scenes, fls, L, V = _batch()
    Lt = torch.from_numpy(L).to(DEV)
    Vt = torch.from_numpy(V).to(DEV)
    st = torch.from_numpy(scenes[0].s).to(DEV)
    plan = mf.Plan(fls, 74, 12, 2.0, 1e-9, True, "lowrank", chunk_lines=256)
    ws = plan.alloc_workspace()
    eager = torch.empty(L.shape[0], dtype=torch.float32, device=DEV)
    plan.retrieve(Lt, st, eager, Vt, None, ws)
    torch.cuda.synchronize()
    inplan = np.zeros(L.shape[0], bool)
    for o, S, N in fls:
        inplan[o:o + S * N] = True
    ref = eager.cpu().numpy()[inplan]
    plan.set_streams(3)
    stream = torch.cuda.Stream()
    plan.set_graph(True)
    out = torch.empty_like(eager)
    for rep in range(4):
        out.fill_(123.0)
        junk = torch.randn(1 << 20, device=DEV).sum()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            plan.retrieve(Lt, st, out, Vt, None, ws, stream=stream)
        stream.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy()[inplan], ref, err_msg=f"replay {rep}")
        del junk
    plan.set_graph(False)
    plan.close()


def test_streams_energy_matches_one_stream():
    """The energy monitor's E^k per partition is the same with concurrent
    partition groups (its last kernel runs after the join)."""
    scenes, fls, L, V = _batch()
    Lt = torch.from_numpy(L).to(DEV)
    Vt = torch.from_numpy(V).to(DEV)
    st = torch.from_numpy(scenes[0].s).to(DEV)
    Es = []
    for ns in (1, 4):
        plan = mf.Plan(fls, 74, 8, 2.0, 1e-9, True, "lowrank", track_energy=True)
        plan.set_streams(ns)
        ws = plan.alloc_workspace()
        alpha = torch.empty(L.shape[0], dtype=torch.float32, device=DEV)
        plan.retrieve(Lt, st, alpha, Vt, None, ws)
        Es.append(plan.energy(ws).cpu().numpy())
        torch.cuda.synchronize()
        plan.close()
    np.testing.assert_array_equal(Es[1], Es[0])
    assert np.all(np.isfinite(Es[0]))


def test_set_streams_rejects_bad_counts():
    scenes, fls, L, V = _batch()
    plan = mf.Plan(fls, 74, 5, 2.0, 1e-9, True, "lowrank")
    lib = mf.load_library()
    for n in (0, -1, mf.MAX_STREAMS + 1):
        assert lib.mf_plan_set_streams(plan._h, n) == mf.MF_E_ARG
    one = mf.Plan([fls[1]], 74, 5, 2.0, 1e-9, True, "lowrank")   # 3 partitions
    assert lib.mf_plan_set_streams(one._h, 4) == mf.MF_E_ARG
    assert lib.mf_plan_set_streams(one._h, 3) == 0 and one.streams == 3
    assert plan.streams == 1
    plan.close()
    one.close()


@pytest.mark.parametrize("tile,wgs,n_streams,reverse", [("32x4", 0, 1, False), ("64x2", 0, 1, False),
                                                        ("64x1", 0, 1, True), ("32x2", 3, 2, False),
                                                        ("32x4", 2, 3, True)])
def test_sparse_alpha_matches_every_entry(tile, wgs, n_streams, reverse):
    """A low-rank retrieval passes alpha between its streaming passes sparsely
    (nonzero entries plus a mask per 32-pixel piece) through two ping-pong
    buffers; one with checkpoints (save_for_backward) keeps every
    iteration's alpha, each with its own mask array.  Both give the same
    alpha bit for bit: ragged masked flightlines with a gap, odd line
    counts, every tile shape's piece layout, and flightlines listed out of
    pixel order (reverse)."""
    scenes, fls, L, V = _batch()
    if reverse:
        fls = fls[::-1]
    Lt = torch.from_numpy(L).to(DEV)
    Vt = torch.from_numpy(V).to(DEV)
    s = torch.from_numpy(scenes[0].s).to(DEV)
    outs = []
    for save in (False, True):
        plan = mf.Plan(fls, 74, 12, 2.0, 1e-9, True, "lowrank", chunk_lines=128, save_for_backward=save)
        plan.set_launch(tile, wgs)
        plan.set_streams(n_streams)
        ws = plan.alloc_workspace(DEV)
        alpha = torch.full((L.shape[0],), -1.0, dtype=torch.float32, device=DEV)
        st = torch.empty((plan.n_columns,), dtype=torch.int32, device=DEV)
        plan.retrieve(Lt, s, alpha, Vt, st, ws)
        torch.cuda.synchronize()
        outs.append((alpha.cpu().numpy(), st.cpu().numpy()))
        plan.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    assert (outs[0][0] > 0).sum() > 100


def test_sparse_alpha_workspace_reused_across_tile_shapes():
    """The masks of the sparse alpha live in the workspace and every pass
    rewrites every word of its pieces, so a workspace reused by retrievals
    with other tile shapes (pieces written by 64-pixel chunks, then by
    32-pixel ones, then by a persistent launch) gives each the alpha of a
    fresh workspace, bit for bit."""
    scenes, fls, L, V = _batch()
    Lt = torch.from_numpy(L).to(DEV)
    Vt = torch.from_numpy(V).to(DEV)
    s = torch.from_numpy(scenes[0].s).to(DEV)
    plan = mf.Plan(fls, 74, 12, 2.0, 1e-9, True, "lowrank", chunk_lines=128)
    shared = plan.alloc_workspace(DEV)
    shared.fill_(0xFF)                       # garbage in every mask word at the start
    for tile, wgs in (("64x2", 0), ("32x4", 0), ("32x2", 2), ("64x1", 0)):
        plan.set_launch(tile, wgs)
        fresh = plan.alloc_workspace(DEV)
        a1 = torch.full((L.shape[0],), -1.0, dtype=torch.float32, device=DEV)
        a2 = torch.full((L.shape[0],), -1.0, dtype=torch.float32, device=DEV)
        plan.retrieve(Lt, s, a1, Vt, None, shared)
        plan.retrieve(Lt, s, a2, Vt, None, fresh)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(a1.cpu().numpy(), a2.cpu().numpy())
    plan.close()
