"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded scenes.  Sizes span several work items per column and ragged
tails; the full-size flightline is checked on every pixel (default form) and
on sampled columns (every form)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2003_02978_amd as mf  # noqa: E402
from oracle.mf64 import retrieve as oracle_retrieve  # noqa: E402
from synth.scenes import SceneSpec, make_scene, tiny_spec, flightline_spec, make_globals, make_column  # noqa: E402
from tests.parity_util import assert_fp32_parity, compare, config_lambda  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _gpu(sc, **kw):
    L = torch.from_numpy(sc.radiance).to(DEV)
    s = torch.from_numpy(sc.s).to(DEV)
    valid = None if sc.valid is None else torch.from_numpy(sc.valid).to(DEV)
    a, st = mf.retrieve(L, s, valid=valid, **kw)
    torch.cuda.synchronize()
    return a.cpu().numpy(), st.cpu().numpy()


@pytest.fixture(scope="module")
def tiny():
    return make_scene(tiny_spec())


EXACT = ["lowrank", "fp64"]    # forms whose covariance is accumulated exactly
# every form: the rounded Gram forms (FP32 and BF16 MFMA) refine against the
# exact C^k and are held to the same FP32 bar
FORMS = EXACT + ["fp32", "bf16", "bf16x3"]


@pytest.mark.parametrize("cov", FORMS)
@pytest.mark.parametrize("chunk", [0, 128])
def test_tiny_scene(tiny, chunk, cov):
    lam = config_lambda("tiny")
    a, st = _gpu(tiny, n_iter=30, lam=lam, chunk_lines=chunk, cov=cov)
    ref, rst = oracle_retrieve(tiny.radiance, tiny.s, 30, lam, workers=8)
    np.testing.assert_array_equal(st, rst)
    assert np.all(a >= 0)
    assert_fp32_parity(a, ref, label=f"tiny chunk={chunk} cov={cov}")


@pytest.mark.parametrize("cov", EXACT)
@pytest.mark.parametrize("refine", [0, 2])
def test_refinement_step_counts(tiny, refine, cov):
    """No refinement step and two steps of C^-1 t (the exact forms' default is
    one): the solves stay within the FP32 tolerance of the exact oracle."""
    lam = config_lambda("tiny")
    a, st = _gpu(tiny, n_iter=30, lam=lam, cov=cov, refine_steps=refine)
    ref, rst = oracle_retrieve(tiny.radiance, tiny.s, 30, lam, workers=8)
    np.testing.assert_array_equal(st, rst)
    assert_fp32_parity(a, ref, label=f"tiny refine={refine} cov={cov}")


@pytest.mark.parametrize("cov", FORMS)
@pytest.mark.parametrize("albedo", [True, False])
def test_zero_iterations_is_the_unclamped_filter(tiny, albedo, cov):
    a, st = _gpu(tiny, n_iter=0, lam=1.0, albedo=albedo, cov=cov)
    ref, _ = oracle_retrieve(tiny.radiance, tiny.s, 0, 1.0, albedo=albedo, workers=8)
    assert (a < 0).any()
    assert_fp32_parity(a, ref, iterative=False, label=f"K=0 albedo={albedo}")


@pytest.mark.parametrize("cov", FORMS)
@pytest.mark.parametrize("lam,albedo,K", [(0.0, True, 5), (0.0, False, 5), (1.0, False, 12)])
def test_variants(tiny, lam, albedo, K, cov):
    sub = make_scene(tiny_spec())
    sub.radiance = sub.radiance[:16].copy()
    a, _ = _gpu(sub, n_iter=K, lam=lam, albedo=albedo, cov=cov)
    ref, _ = oracle_retrieve(sub.radiance, sub.s, K, lam, albedo=albedo, workers=8)
    assert_fp32_parity(a, ref, label=f"lam={lam} albedo={albedo} K={K}")


@pytest.mark.parametrize("cov", FORMS)
def test_ragged_lengths_and_many_items(cov):
    spec = SceneSpec(6, 1000, 74, 2, (500.0, 5000.0), (3.0, 30.0), seed=5)
    sc = make_scene(spec)
    for chunk in (128, 256, 0):
        a, st = _gpu(sc, n_iter=15, lam=3.0, chunk_lines=chunk, cov=cov)
        ref, rst = oracle_retrieve(sc.radiance, sc.s, 15, 3.0)
        np.testing.assert_array_equal(st, rst)
        assert_fp32_parity(a, ref, label=f"ragged chunk={chunk}")


@pytest.mark.parametrize("cov", FORMS)
def test_masks_skip_invalid_pixels(cov):
    spec = SceneSpec(8, 1500, 74, 3, (500.0, 5000.0), (3.0, 30.0), seed=9, mask_max_frac=0.2)
    sc = make_scene(spec)
    a, st = _gpu(sc, n_iter=20, lam=3.0, chunk_lines=512, cov=cov)
    ref, rst = oracle_retrieve(sc.radiance, sc.s, 20, 3.0, valid=sc.valid)
    np.testing.assert_array_equal(st, rst)
    assert np.all(a[sc.valid == 0] == 0)
    assert np.all(np.isfinite(a))
    assert_fp32_parity(a, ref, label="masked")


@pytest.mark.parametrize("cov", FORMS)
def test_degenerate_columns_get_status_and_zero(cov):
    spec = SceneSpec(4, 600, 74, 1, (500.0, 5000.0), (3.0, 30.0), seed=11, mask_max_frac=0.0)
    sc = make_scene(spec)
    valid = np.ones((4, 600), np.uint8)
    valid[0, 50:] = 0               # 50 valid pixels <= 74 bands
    sc.radiance[0, 50:] = np.nan
    sc.radiance[1, 123, 7] = np.nan  # a valid pixel with NaN
    valid[3, :] = 0                  # no valid pixel at all
    sc.valid = valid
    a, st = _gpu(sc, n_iter=5, lam=2.0, cov=cov)
    ref, rst = oracle_retrieve(sc.radiance, sc.s, 5, 2.0, valid=valid)
    assert list(st) == [mf.MF_COL_FEW_PIXELS, mf.MF_COL_NONFINITE, mf.MF_COL_OK,
                        mf.MF_COL_FEW_PIXELS]
    np.testing.assert_array_equal(st, rst)
    assert np.all(a[[0, 1, 3]] == 0)
    assert_fp32_parity(a[2:3], ref[2:3], label=f"degenerate, healthy column, cov={cov}")


@pytest.mark.parametrize("cov", ["fp32", "bf16", "bf16x3"])
def test_rounded_forms_refinement_converges(tiny, cov):
    """The rounded Gram forms refine against the exact C^k: the error against
    the oracle after one step is larger than after the form's default steps,
    which meet the FP32 bar (the step counts are the ones whose contraction,
    about 1e-3 per step for the FP32 Gram, 2e-2 for BF16 and 1e-2 for split
    BF16, reaches FP64 rounding)."""
    lam = config_lambda("tiny")
    ref, _ = oracle_retrieve(tiny.radiance, tiny.s, 30, lam, workers=8)
    a1, _ = _gpu(tiny, n_iter=30, lam=lam, cov=cov, refine_steps=1)
    ad, _ = _gpu(tiny, n_iter=30, lam=lam, cov=cov)
    r1, rd = compare(a1, ref), compare(ad, ref)
    print(f"{cov}: one refinement step {r1}; default steps {rd}", flush=True)
    assert rd["max_abs_err"] <= r1["max_abs_err"]
    assert_fp32_parity(ad, ref, label=f"tiny cov={cov} default refinement")


@pytest.mark.parametrize("cov", FORMS)
def test_deterministic_and_column_independent(tiny, cov):
    lam = config_lambda("tiny")
    a1, _ = _gpu(tiny, n_iter=30, lam=lam, cov=cov)
    a2, _ = _gpu(tiny, n_iter=30, lam=lam, cov=cov)
    np.testing.assert_array_equal(a1, a2)
    sub = make_scene(tiny_spec())
    sub.radiance = sub.radiance[17:18].copy()
    a3, _ = _gpu(sub, n_iter=30, lam=lam, cov=cov)
    np.testing.assert_array_equal(a3[0], a1[17])


@pytest.fixture(scope="module")
def flightline():
    return make_scene(flightline_spec())


@pytest.fixture(scope="module")
def flightline_sample(flightline):
    """Columns through plumes and random columns of the flightline, with the
    oracle's alpha for them (30 iterations)."""
    g = make_globals(flightline_spec())
    rng = np.random.default_rng(0)
    cols = sorted(set([int(g.plumes[i, 0]) for i in range(3)] +
                      [int(c) for c in rng.choice(598, 3, replace=False)]))
    ref, _ = oracle_retrieve(flightline.radiance, flightline.s, 30, config_lambda("flightline"),
                             columns=cols, workers=6)
    return cols, ref


def test_full_flightline_every_pixel(flightline):
    """The default form on the whole 598 x 8000 x 74 flightline, 30
    iterations, in the benchmark's launch configuration: every one of the
    4.78 M pixels against the oracle run on every column."""
    lam = config_lambda("flightline")
    a, st = _gpu(flightline, n_iter=30, lam=lam)
    ref, rst = oracle_retrieve(flightline.radiance, flightline.s, 30, lam, workers=16)
    np.testing.assert_array_equal(st, rst)
    rep = assert_fp32_parity(a, ref, label="flightline, every pixel, default form")
    assert rep["flips_over_nonzero"] == 0.0


@pytest.mark.parametrize("cov", FORMS)
def test_full_flightline_sampled_columns(flightline, flightline_sample, cov):
    """598 x 8000 x 74, 30 iterations, the benchmark's launch configuration;
    columns through plumes and random columns are recomputed by the oracle."""
    a, st = _gpu(flightline, n_iter=30, lam=config_lambda("flightline"), cov=cov)
    assert np.all(st == 0)
    cols, ref = flightline_sample
    assert_fp32_parity(a[cols], ref, label=f"flightline cov={cov} cols {cols}")


@pytest.mark.parametrize("cov", FORMS)
@pytest.mark.parametrize("offset", [0, 1, 2])
def test_odd_lines_and_unaligned_radiance(cov, offset):
    """Odd line counts put every other column on an 8-byte (not 16-byte)
    boundary, and an offset view of a larger buffer moves the whole cube off
    16-byte alignment; work items of 128 lines leave ragged chunks."""
    spec = SceneSpec(6, 1001, 74, 2, (500.0, 5000.0), (3.0, 30.0), seed=13)
    sc = make_scene(spec)
    S, N, B = sc.radiance.shape
    big = torch.zeros(S * N * B + 4, dtype=torch.float32, device=DEV)
    L = big[offset:offset + S * N * B]
    L.copy_(torch.from_numpy(sc.radiance.reshape(-1)).to(DEV))
    s = torch.from_numpy(sc.s).to(DEV)
    ref, rst = oracle_retrieve(sc.radiance, sc.s, 15, 3.0)
    for chunk in (128, 0):
        a, st = mf.retrieve(L.view(S, N, B), s, n_iter=15, lam=3.0, cov=cov, chunk_lines=chunk)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(st.cpu().numpy(), rst)
        assert_fp32_parity(a.cpu().numpy(), ref, label=f"odd lines offset={offset} chunk={chunk}")


@pytest.mark.parametrize("cov", FORMS)
def test_detector_grouping(cov):
    """Partitions of g = 5 adjacent columns (the last takes the remaining 3)
    share one mean and covariance (Sec. II-E); masked pixels included."""
    from oracle.mf64 import retrieve_grouped
    spec = SceneSpec(13, 400, 74, 3, (500.0, 5000.0), (3.0, 20.0), seed=17, mask_max_frac=0.15)
    sc = make_scene(spec)
    S, N, B = sc.radiance.shape
    L = torch.from_numpy(sc.radiance).to(DEV)
    s = torch.from_numpy(sc.s).to(DEV)
    V = torch.from_numpy(sc.valid).to(DEV)
    ref, rst = retrieve_grouped(sc.radiance, sc.s, 12, 2.0, valid=sc.valid, group=5)
    assert len(rst) == 3
    for chunk in (128, 0):
        a, st = mf.retrieve(L, s, n_iter=12, lam=2.0, cov=cov, valid=V, chunk_lines=chunk, group=5)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(st.cpu().numpy(), rst)
        assert_fp32_parity(a.cpu().numpy(), ref, label=f"group 5 cov={cov} chunk={chunk}")
    # two flightlines in one plan: 7 columns -> groups of 3, 3, 1; 4 columns -> 3, 1
    spec2 = SceneSpec(4, 300, 74, 1, (500.0, 5000.0), (3.0, 20.0), seed=19)
    sc2 = make_scene(spec2)
    off = 7 * N + 50
    total = off + 4 * 300
    Lb = torch.zeros((total, B), dtype=torch.float32, device=DEV)
    Lb[:7 * N] = L[:7].reshape(-1, B)
    Lb[off:] = torch.from_numpy(sc2.radiance.reshape(-1, B)).to(DEV)
    Vb = torch.ones(total, dtype=torch.uint8, device=DEV)
    Vb[:7 * N] = V[:7].reshape(-1)
    plan = mf.Plan([(0, 7, N), (off, 4, 300)], B, 12, 2.0, 1e-9, True, cov, group=3)
    assert plan.n_columns == 5
    ws = plan.alloc_workspace(DEV)
    ab = torch.empty(total, dtype=torch.float32, device=DEV)
    stb = torch.empty(plan.n_columns, dtype=torch.int32, device=DEV)
    plan.retrieve(Lb, s, ab, Vb, stb, ws)
    torch.cuda.synchronize()
    r1, s1 = retrieve_grouped(sc.radiance[:7], sc.s, 12, 2.0, valid=sc.valid[:7], group=3)
    r2, s2 = retrieve_grouped(sc2.radiance, sc.s, 12, 2.0, group=3)
    np.testing.assert_array_equal(stb.cpu().numpy(), np.concatenate([s1, s2]))
    abh = ab.cpu().numpy()
    assert_fp32_parity(abh[:7 * N].reshape(7, N), r1, label="batch group 3, flightline 0")
    assert_fp32_parity(abh[off:].reshape(4, 300), r2, label="batch group 3, flightline 1")
    plan.close()
