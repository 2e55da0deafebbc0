"""GPU ingest: the BIL repack kernel (through the C ABI) against the numpy
reference, bit-exact, on ragged sizes with censored values; and BIL ->
repack -> retrieval equals the retrieval of the same cube in its native
layout."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2003_02978_amd as mf  # noqa: E402
from oracle.ingest import repack_bil as ref_repack  # noqa: E402
from synth.scenes import SceneSpec, make_scene  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("N,B,S", [(7, 74, 130), (1, 74, 1), (64, 78, 64), (33, 5, 257)])
def test_repack_matches_reference(N, B, S):
    rng = np.random.default_rng(N * 1000 + S)
    bil = rng.standard_normal((N, B, S)).astype(np.float32)
    bil[rng.random((N, B, S)) < 0.002] = np.nan
    bil[rng.random((N, B, S)) < 0.002] = -9999.0
    rad, val = mf.repack_bil(torch.from_numpy(bil).to(DEV), nodata=-9999.0)
    torch.cuda.synchronize()
    r_ref, v_ref = ref_repack(bil, nodata=-9999.0)
    np.testing.assert_array_equal(rad.cpu().numpy().view(np.uint32), r_ref.view(np.uint32))
    np.testing.assert_array_equal(val.cpu().numpy(), v_ref)


def test_repack_into_flat_buffer_at_offset():
    """Two flightlines repacked into one flat radiance buffer, the layout a
    multi-flightline plan reads; bytes between and after them untouched."""
    rng = np.random.default_rng(3)
    B = 74
    b1 = rng.standard_normal((9, B, 70)).astype(np.float32)
    b2 = rng.standard_normal((5, B, 3)).astype(np.float32)
    off2 = 9 * 70 + 11
    total = off2 + 5 * 3 + 4
    flat = torch.full((total * B,), -1.0, dtype=torch.float32, device=DEV)
    vflat = torch.full((total,), 7, dtype=torch.uint8, device=DEV)
    mf.repack_bil(torch.from_numpy(b1).to(DEV), flat, vflat, first_px=0)
    mf.repack_bil(torch.from_numpy(b2).to(DEV), flat, vflat, first_px=off2)
    torch.cuda.synchronize()
    f = flat.cpu().numpy().reshape(total, B)
    v = vflat.cpu().numpy()
    np.testing.assert_array_equal(f[:9 * 70], ref_repack(b1)[0].reshape(-1, B))
    np.testing.assert_array_equal(f[off2:off2 + 15], ref_repack(b2)[0].reshape(-1, B))
    assert np.all(f[9 * 70:off2] == -1.0) and np.all(f[off2 + 15:] == -1.0)
    assert np.all(v[:9 * 70] == 1) and np.all(v[9 * 70:off2] == 7) and np.all(v[off2 + 15:] == 7)


def test_bil_ingest_then_retrieve_equals_native_layout():
    sc = make_scene(SceneSpec(6, 500, 74, 2, (500.0, 5000.0), (3.0, 20.0), seed=23, mask_max_frac=0.1))
    S, N, B = sc.radiance.shape
    bil = np.ascontiguousarray(np.transpose(sc.radiance, (1, 2, 0)))      # [N, B, S]
    s = torch.from_numpy(sc.s).to(DEV)
    rad, val = mf.repack_bil(torch.from_numpy(bil).to(DEV))
    a1, st1 = mf.retrieve(rad, s, n_iter=10, lam=2.0, valid=val)
    a0, st0 = mf.retrieve(torch.from_numpy(sc.radiance).to(DEV), s, n_iter=10, lam=2.0,
                          valid=torch.from_numpy(sc.valid).to(DEV))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(val.cpu().numpy(), sc.valid)
    np.testing.assert_array_equal(st1.cpu().numpy(), st0.cpu().numpy())
    np.testing.assert_array_equal(a1.cpu().numpy(), a0.cpu().numpy())
