"""Band counts other than the 74 of the 2122-2487 nm window: every register
layout the kernels instantiate (1 to 5 blocks of 16 bands, the narrow and the
wide layout, B = 2 to the maximum 78), odd B in the paired band loop, with
ragged work items; forward against the FP64 oracle, the adjoint against the
reference gradient, and the energy monitor."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2003_02978_amd as mf  # noqa: E402
from oracle.grad64 import loss_and_grads  # noqa: E402
from oracle.mf64 import retrieve as oracle_retrieve, retrieve_column  # noqa: E402
from synth.scenes import SceneSpec, make_scene  # noqa: E402
from tests.parity_util import assert_fp32_parity  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# narrow layouts with 1..4 blocks (B + 2 <= 16, 32, 48, 64), the last narrow
# B, the first wide one and the maximum
BANDS = [2, 9, 14, 15, 30, 31, 46, 47, 62, 63, 64, 77, 78]


def _scene(B, seed=71):
    return make_scene(SceneSpec(3, 700, B, 2, (500.0, 5000.0), (3.0, 30.0), seed=seed))


@pytest.mark.parametrize("cov", ["lowrank", "fp64"])
@pytest.mark.parametrize("B", BANDS)
def test_band_counts_match_oracle(B, cov):
    sc = _scene(B)
    L = torch.from_numpy(sc.radiance).to(DEV)
    s = torch.from_numpy(sc.s).to(DEV)
    a, st = mf.retrieve(L, s, n_iter=10, lam=2.0, cov=cov, chunk_lines=256)   # items 256, 256, 188
    torch.cuda.synchronize()
    ref, rst = oracle_retrieve(sc.radiance, sc.s, 10, 2.0)
    np.testing.assert_array_equal(st.cpu().numpy(), rst)
    assert_fp32_parity(a.cpu().numpy(), ref, label=f"B={B} cov={cov}")


@pytest.mark.parametrize("cov", ["fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("B", BANDS)
def test_band_counts_rounded_gram_forms(B, cov):
    """The rounded Gram forms at every register layout: refined against the
    exact C^k, they meet the same FP32 bar."""
    sc = _scene(B)
    L = torch.from_numpy(sc.radiance).to(DEV)
    s = torch.from_numpy(sc.s).to(DEV)
    a, st = mf.retrieve(L, s, n_iter=10, lam=2.0, cov=cov, chunk_lines=256)
    torch.cuda.synchronize()
    ref, rst = oracle_retrieve(sc.radiance, sc.s, 10, 2.0)
    np.testing.assert_array_equal(st.cpu().numpy(), rst)
    assert_fp32_parity(a.cpu().numpy(), ref, label=f"B={B} cov={cov}")


@pytest.mark.parametrize("B", [9, 31, 64, 78])
def test_band_counts_adjoint(B):
    sc = _scene(B, seed=73)
    K, lam = 5, 2.0
    L = torch.from_numpy(sc.radiance).to(DEV).requires_grad_(True)
    s = torch.from_numpy(sc.s).to(DEV).requires_grad_(True)
    at = torch.from_numpy(sc.alpha_true).to(DEV)
    alpha = mf.retrieve_differentiable(L, s, K, lam, 1e-9, True, None, chunk_lines=256)
    J = ((alpha.double() - at) ** 2).sum()
    J.backward()
    torch.cuda.synchronize()
    gL = L.grad.cpu().numpy().astype(np.float64)
    gs = s.grad.cpu().numpy().astype(np.float64)
    Jr, gLr, gsr = loss_and_grads(sc.radiance.astype(np.float64), sc.s, sc.alpha_true, K, lam)
    eL = np.abs(gL - gLr).max() / np.abs(gLr).max()
    es = np.abs(gs - gsr).max() / np.abs(gsr).max()
    print(f"B={B}: J {float(J):.6e} ref {Jr:.6e}, grad L rel err {eL:.2e}, grad s rel err {es:.2e}",
          flush=True)
    assert abs(float(J) - Jr) <= 1e-6 * Jr
    assert eL < 1e-4 and es < 1e-4


@pytest.mark.parametrize("B", [2, 31, 78])
def test_band_counts_energy(B):
    sc = _scene(B, seed=79)
    S, N, _ = sc.radiance.shape
    K = 6
    plan = mf.Plan([(0, S, N)], B, K, 2.0, 1e-9, True, "lowrank", chunk_lines=256, track_energy=True)
    ws = plan.alloc_workspace(DEV)
    alpha = torch.empty((S, N), dtype=torch.float32, device=DEV)
    plan.retrieve(torch.from_numpy(sc.radiance).to(DEV), torch.from_numpy(sc.s).to(DEV), alpha, None, None, ws)
    E = plan.energy(ws).cpu().numpy()
    plan.close()
    for c in range(S):
        e = []
        retrieve_column(sc.radiance[c], sc.s, K, 2.0, 1e-9, True, None, energy=e)
        err = np.abs(E[:, c] - np.array(e)) / np.abs(np.array(e))
        print(f"B={B} column {c}: energy max rel err {err.max():.2e}", flush=True)
        assert err.max() < 1e-7
