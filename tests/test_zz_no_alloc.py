"""mf_retrieve_noalloc: the retrieval on the library's fixed device scratch
(no workspace argument, nothing allocated), called through the C ABI and
compared bit for bit with mf_retrieve on a caller workspace, for two calls in
a row where the second plan is smaller and of another covariance form."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2003_02978_amd as mf  # noqa: E402
from synth.scenes import SceneSpec, make_scene, tiny_spec  # noqa: E402
from tests.parity_util import config_lambda  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _inputs(sc):
    S, N, B = sc.radiance.shape
    L = torch.from_numpy(sc.radiance).to(DEV)
    s = torch.from_numpy(sc.s).to(DEV)
    V = None if sc.valid is None else torch.from_numpy(sc.valid).to(DEV)
    return L, s, V


def test_noalloc_matches_retrieve_on_two_calls():
    a_sc = make_scene(tiny_spec())                        # 64 x 512 x 74
    b_sc = make_scene(SceneSpec(8, 300, 74, 2, (500.0, 5000.0), (3.0, 30.0), seed=31,
                                mask_max_frac=0.2))       # 8 x 300, masked
    lam = config_lambda("tiny")
    runs = []
    for sc, cov, K in ((a_sc, "lowrank", 30), (b_sc, "bf16", 12)):
        S, N, B = sc.radiance.shape
        plan = mf.Plan([(0, S, N)], B, K, lam, 1e-9, True, cov)
        assert plan.workspace_bytes <= mf.NOALLOC_SCRATCH_BYTES
        L, s, V = _inputs(sc)
        ref = torch.empty((S, N), dtype=torch.float32, device=DEV)
        ref_st = torch.empty((plan.n_columns,), dtype=torch.int32, device=DEV)
        plan.retrieve(L, s, ref, V, ref_st, plan.alloc_workspace(DEV))
        torch.cuda.synchronize()
        runs.append((plan, L, s, V, ref, ref_st))
    outs = []
    for plan, L, s, V, ref, ref_st in runs:             # two no-alloc calls in a row
        a = torch.full_like(ref, float("nan"))
        st = torch.full_like(ref_st, -1)
        plan.retrieve_noalloc(L, s, a, V, st)
        outs.append((a, st))
    torch.cuda.synchronize()
    for (plan, L, s, V, ref, ref_st), (a, st) in zip(runs, outs):
        np.testing.assert_array_equal(st.cpu().numpy(), ref_st.cpu().numpy())
        np.testing.assert_array_equal(a.cpu().numpy(), ref.cpu().numpy())
        assert int((ref.cpu().numpy() > 0).sum()) > 0
        plan.close()


def test_noalloc_rejects_what_does_not_fit():
    lib = mf.load_library()
    big = mf.Plan([(0, 598, 8000)], 74, 30, 1.0, 1e-9, True, "lowrank")
    assert big.workspace_bytes > mf.NOALLOC_SCRATCH_BYTES
    one = ctypes.c_void_p(256)       # never dereferenced: the size check comes first
    rc = lib.mf_retrieve_noalloc(big._h, one, None, one, one, None, None)
    assert rc == mf.MF_E_UNSUPPORTED and b"workspace" in lib.mf_last_error()
    big.close()
    sfb = mf.Plan([(0, 4, 300)], 74, 5, 1.0, 1e-9, True, "lowrank", save_for_backward=True)
    rc = lib.mf_retrieve_noalloc(sfb._h, one, None, one, one, None, None)
    assert rc == mf.MF_E_UNSUPPORTED
    sfb.close()


def test_noalloc_with_streams_matches_retrieve():
    """With concurrent partition groups (streams and events the plan created
    beforehand), the no-alloc call still equals mf_retrieve bit for bit, on
    two calls in a row, the second with a smaller plan."""
    a_sc = make_scene(tiny_spec())
    b_sc = make_scene(SceneSpec(8, 300, 74, 2, (500.0, 5000.0), (3.0, 30.0), seed=33,
                                mask_max_frac=0.2))
    lam = config_lambda("tiny")
    runs = []
    for sc, ns in ((a_sc, 3), (b_sc, 2)):
        S, N, B = sc.radiance.shape
        plan = mf.Plan([(0, S, N)], B, 12, lam, 1e-9, True, "lowrank")
        plan.set_streams(ns)
        L, s, V = _inputs(sc)
        ref = torch.empty((S, N), dtype=torch.float32, device=DEV)
        plan.retrieve(L, s, ref, V, None, plan.alloc_workspace(DEV))
        torch.cuda.synchronize()
        runs.append((plan, L, s, V, ref))
    for plan, L, s, V, ref in runs:
        a = torch.full_like(ref, float("nan"))
        plan.retrieve_noalloc(L, s, a, V)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(a.cpu().numpy(), ref.cpu().numpy())
        plan.close()
