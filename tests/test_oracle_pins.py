"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper it follows.  Equation numbers are the
paper's: (3) classic matched filter, (5) weights, (6) soft-threshold update,
(7) albedo factor, (8) albedo-scaled objective, (9) target, (10)-(11) mean and
covariance with the enhancement removed; Fig. 1 is the algorithm figure.
"""
import numpy as np
import pytest
import scipy.optimize

from oracle.mf64 import (STATUS_FEW_PIXELS, STATUS_NONFINITE, STATUS_OK,
                         alpha_step, energy_k, retrieve, retrieve_column, retrieve_grouped)


BRUTE_RTOL = 1e-6   # resolution of the brute-force searches (see below)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _background_column(rng, N, B, albedo_spread=0.0, noise=0.02):
    """Smooth positive spectra: 3 random smooth endmembers, random mixtures."""
    x = np.linspace(0, 1, B)
    E = np.stack([2 + np.sin(2 * np.pi * (x * f + ph)) for f, ph in
                  zip(rng.uniform(0.3, 1.5, 3), rng.uniform(0, 1, 3))])
    ab = rng.dirichlet(np.ones(3), N)
    a = 1.0 + albedo_spread * rng.uniform(-1, 1, N)
    return a[:, None] * (ab @ E) + noise * rng.standard_normal((N, B))


def _s(rng, B):
    return -1e-4 * rng.uniform(0.0, 1.0, B)


# ---------------------------------------------------------------------------
# Eq. (3): with no iterations and no albedo factor, the filter is the least-
# squares matched filter.  Its scores satisfy exact normal-equation identities:
#   sum_i alpha_i = 0   and   sum_i alpha_i L_i = (sum_i alpha_i^2) (mu (.) s)
# with mu the column mean.  Both follow from alpha_i = (L_i-mu)^T C^-1 t / q
# and C = (1/N) sum (L_i-mu)(L_i-mu)^T; a wrong sign, target, transpose or a
# dropped inverse breaks them.

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_classic_mf_normal_equations(seed):
    rng = _rng(seed)
    L = _background_column(rng, 400, 12)
    s = _s(rng, 12)
    a, st = retrieve_column(L, s, 0, lam=0.0, albedo=False)
    assert st == STATUS_OK
    mu = L.mean(0)
    assert abs(a.sum()) <= 1e-9 * np.abs(a).sum()
    lhs = (a[:, None] * L).sum(0)
    rhs = (a ** 2).sum() * (mu * s)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-9 * np.abs(rhs).max())


@pytest.mark.parametrize("seed", [4, 5])
def test_classic_mf_is_pixelwise_least_squares(seed):
    """Eq. (2)-(3): each alpha_i minimises d^T C^-1 d over alpha (brute force)."""
    rng = _rng(seed)
    L = _background_column(rng, 300, 6)
    s = _s(rng, 6)
    a, _ = retrieve_column(L, s, 0, lam=0.0, albedo=False)
    mu = L.mean(0)
    C = np.cov(L.T, bias=True)          # library sample covariance, 1/N
    Ci = np.linalg.inv(C)
    t = mu * s
    Cil = Ci.astype(np.longdouble)
    for i in rng.choice(300, 8, replace=False):
        Li, mul, tl = (x.astype(np.longdouble) for x in (L[i], mu, t))
        f = lambda al: (Li - mul - al * tl) @ Cil @ (Li - mul - al * tl)
        x = _golden(f, -1e4, 1e4)
        assert abs(x - a[i]) <= BRUTE_RTOL * max(1.0, abs(a[i]))


@pytest.mark.parametrize("seed", [6, 7])
def test_albedo_mf_normal_equations(seed):
    """Fig. 1 initialisation with the albedo factor of Eq. (7): r_i alpha_i is the
    classic score, so sum_i r_i alpha_i = 0 and
    sum_i r_i alpha_i L_i = (sum_i r_i^2 alpha_i^2) (mu (.) s); mean r = 1."""
    rng = _rng(seed)
    L = _background_column(rng, 500, 10, albedo_spread=0.5)
    s = _s(rng, 10)
    a, st = retrieve_column(L, s, 0, lam=1.0, albedo=True)
    assert st == STATUS_OK
    mu = L.mean(0)
    r = L @ mu / (mu @ mu)
    assert abs(r.mean() - 1.0) < 1e-12
    ra = r * a
    assert abs(ra.sum()) <= 1e-9 * np.abs(ra).sum()
    lhs = (ra[:, None] * L).sum(0)
    rhs = (ra ** 2).sum() * (mu * s)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-9 * np.abs(rhs).max())
    # the K = 0 result keeps its sign (non-iterative filters give negatives)
    assert (a < 0).any()


# ---------------------------------------------------------------------------
# Positivity (Eq. 6, Fig. 1; "no negative values" for the iterative filters)

@pytest.mark.parametrize("lam", [0.0, 1.0, 10.0])
def test_iterative_output_nonnegative_with_exact_zeros(lam):
    rng = _rng(11)
    L = _background_column(rng, 600, 16, albedo_spread=0.4)
    s = _s(rng, 16)
    a, st = retrieve_column(L, s, 5, lam=lam)
    assert st == STATUS_OK
    assert np.all(a >= 0.0)
    assert np.all(np.signbit(a[a == 0]) == False)  # +0.0, never -0.0
    assert (a == 0).sum() > 0


# ---------------------------------------------------------------------------
# Brute force of each iteration: given the state the oracle used at iteration k
# (mu^k, C^k, t^k, w^k, r), alpha^k must minimise over alpha >= 0 the sum of
#   E_i(alpha) = 1/2 d_i^T C^-1 d_i + r_i w_i alpha,
#   d_i = L_i - r_i alpha t^k - mu^k                         (Eqs. 6 and 8).
# Solved independently by a grid + golden-section search per pixel and by
# L-BFGS-B jointly.  A search on function values resolves the minimiser of a
# quadratic of curvature a and minimum E0 only to about sqrt(eps E0 / a), which
# is ~1e-7 relative on these columns; hence BRUTE_RTOL.  Plausible mistakes
# (a dropped factor, a wrong sign or index) move alpha by 1e-3 or more.

def _golden(f, lo, hi, iters=400):
    """Golden-section search in extended precision (np.longdouble)."""
    lo, hi = np.longdouble(lo), np.longdouble(hi)
    g = (np.sqrt(np.longdouble(5)) - 1) / 2
    x1, x2 = hi - g * (hi - lo), lo + g * (hi - lo)
    f1, f2 = f(x1), f(x2)
    for _ in range(iters):
        if f1 < f2:
            hi, x2, f2 = x2, x1, f1
            x1 = hi - g * (hi - lo)
            f1 = f(x1)
        else:
            lo, x1, f1 = x1, x2, f2
            x2 = lo + g * (hi - lo)
            f2 = f(x2)
        if hi - lo <= 1e-14 * max(1.0, abs(float(lo))):
            break
    return float((lo + hi) / 2)


def _brute_alpha(L, mu, C, t, r, w):
    Ci = np.linalg.inv(C).astype(np.longdouble)
    Ll, mul, tl = (x.astype(np.longdouble) for x in (L, mu, t))
    out = np.empty(L.shape[0])
    for i in range(L.shape[0]):
        def E(al, i=i):
            d = Ll[i] - r[i] * al * tl - mul
            return 0.5 * d @ Ci @ d + r[i] * w[i] * al
        # dense grid over [0, 1e6] locates the basin; golden section refines it
        grid = np.concatenate([[0.0], np.geomspace(1e-3, 1e6, 400)])
        vals = np.array([E(np.longdouble(gv)) for gv in grid])
        j = int(np.argmin(vals))
        lo, hi = grid[max(j - 1, 0)], grid[min(j + 1, len(grid) - 1)]
        x = _golden(E, lo, hi)
        out[i] = x if E(np.longdouble(x)) < E(np.longdouble(0.0)) else 0.0
    return out


def test_alpha_step_bruteforce_3px_4bands():
    rng = _rng(21)
    B = 4
    A = rng.standard_normal((B, B))
    C = A @ A.T + 0.5 * np.eye(B)        # supplied SPD covariance
    mu = rng.uniform(1, 2, B)
    t = -mu * rng.uniform(0.01, 0.05, B)
    L = mu + rng.standard_normal((3, B)) * 0.3 - np.array([[5.0], [0.5], [-2.0]]) * t
    r = np.array([0.8, 1.0, 1.3])
    w = np.array([0.01, 0.5, 0.001])
    a = alpha_step(L, mu, C, t, r, w)
    b = _brute_alpha(L, mu, C, t, r, w)
    np.testing.assert_allclose(a, b, rtol=BRUTE_RTOL, atol=BRUTE_RTOL)
    # joint L-BFGS-B on the separable sum agrees as well
    Ci = np.linalg.inv(C)

    def Esum(x):
        d = L - (r * x)[:, None] * t[None, :] - mu
        e = 0.5 * np.einsum("ib,bc,ic->i", d, Ci, d) + r * w * x
        g = -(r[:, None] * (d @ Ci) * 1.0) @ t + r * w
        return e.sum(), g
    res = scipy.optimize.minimize(Esum, np.ones(3), jac=True, method="L-BFGS-B",
                                  bounds=[(0, None)] * 3,
                                  options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 1000})
    np.testing.assert_allclose(a, res.x, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("albedo", [True, False])
def test_full_run_bruteforce_16px_4bands(albedo):
    rng = _rng(31)
    N, B = 16, 4
    L = _background_column(rng, N, B, albedo_spread=0.3, noise=0.05)
    s = _s(rng, B) * 50
    L[3] *= np.exp(2000 * s)            # one enhanced pixel
    L[9] *= np.exp(800 * s)
    trace = []
    a, st = retrieve_column(L, s, 6, lam=0.05, albedo=albedo, trace=trace)
    assert st == STATUS_OK and len(trace) == 7
    mu0 = L.mean(0)
    r = L @ mu0 / (mu0 @ mu0) if albedo else np.ones(N)
    for it in trace[1:]:
        b = _brute_alpha(L, it.mu, it.C, it.t, r, it.w)
        np.testing.assert_allclose(it.alpha, b, rtol=BRUTE_RTOL, atol=BRUTE_RTOL)
    np.testing.assert_array_equal(a, trace[-1].alpha)


# ---------------------------------------------------------------------------
# Mean and covariance with the current enhancement removed (Eqs. 10-11).
# mu^k solves the normal equations of least squares over the de-enhanced data,
# and C^k whitens the residuals d_i exactly: (1/N) sum_i C^-1 d_i d_i^T = I,
# so the mean Mahalanobis norm of the residuals equals the band count.

def test_mean_and_covariance_updates():
    rng = _rng(41)
    N, B = 200, 8
    L = _background_column(rng, N, B, albedo_spread=0.3)
    s = _s(rng, B) * 10
    L[:20] *= np.exp(rng.uniform(500, 3000, 20)[:, None] * s)
    trace = []
    retrieve_column(L, s, 4, lam=0.5, trace=trace)
    mu0 = L.mean(0)
    r = L @ mu0 / (mu0 @ mu0)
    # C^0 is the library sample covariance (1/N normalisation)
    np.testing.assert_allclose(trace[0].C, np.cov(L.T, bias=True), rtol=1e-12)
    for prev, it in zip(trace[:-1], trace[1:]):
        c = r * it.alpha_prev
        # normal equations of min_mu sum |L_i - c_i t^{k-1} - mu|^2
        resid = L - c[:, None] * prev.t[None, :] - it.mu
        np.testing.assert_allclose(resid.sum(0), 0.0, atol=1e-10 * np.abs(L).sum(0).max())
        # whitening identity with the residual of Fig. 1 (target t^k)
        d = L - c[:, None] * it.t[None, :] - it.mu
        W = np.linalg.solve(it.C, d.T @ d) / N
        np.testing.assert_allclose(W, np.eye(B), atol=1e-9)
        # target spectrum Eq. (9)
        np.testing.assert_allclose(it.t, it.mu * s, rtol=0, atol=0)


# ---------------------------------------------------------------------------
# Invariances of Fig. 1 (exact up to rounding; epsilon only perturbs them at
# the 1e-9 level)

def test_invariance_uniform_scaling_and_permutation():
    rng = _rng(51)
    L = _background_column(rng, 300, 10, albedo_spread=0.5)
    s = _s(rng, 10) * 5
    L[:15] *= np.exp(rng.uniform(300, 3000, 15)[:, None] * s)
    a, _ = retrieve_column(L, s, 8, lam=1.0)
    a2, _ = retrieve_column(3.7 * L, s, 8, lam=1.0)
    np.testing.assert_allclose(a2, a, rtol=1e-8, atol=1e-8)
    perm = rng.permutation(300)
    a3, _ = retrieve_column(L[perm], s, 8, lam=1.0)
    np.testing.assert_allclose(a3, a[perm], rtol=1e-8, atol=1e-8)


def test_invariance_per_band_scaling_without_albedo():
    rng = _rng(52)
    L = _background_column(rng, 300, 10)
    s = _s(rng, 10) * 5
    L[:15] *= np.exp(rng.uniform(300, 3000, 15)[:, None] * s)
    a, _ = retrieve_column(L, s, 8, lam=1.0, albedo=False)
    g = rng.uniform(0.5, 2.0, 10)
    a2, _ = retrieve_column(L * g, s, 8, lam=1.0, albedo=False)
    np.testing.assert_allclose(a2, a, rtol=1e-7, atol=1e-7)


def test_target_scaling_without_sparsity():
    """alpha(L, c s) = alpha(L, s) / c when w = 0 (t, v scale by c, q by c^2)."""
    rng = _rng(53)
    L = _background_column(rng, 300, 10, albedo_spread=0.4)
    s = _s(rng, 10) * 5
    L[:15] *= np.exp(rng.uniform(300, 3000, 15)[:, None] * s)
    a, _ = retrieve_column(L, s, 6, lam=0.0)
    a2, _ = retrieve_column(L, 2.5 * s, 6, lam=0.0)
    np.testing.assert_allclose(a2, a / 2.5, rtol=1e-8, atol=1e-8)


def test_columns_are_independent():
    rng = _rng(54)
    L = np.stack([_background_column(rng, 200, 8, 0.3) for _ in range(3)])
    s = _s(rng, 8) * 5
    a, st = retrieve(L, s, 5, lam=1.0)
    for c in range(3):
        ac, _ = retrieve_column(L[c], s, 5, lam=1.0)
        np.testing.assert_array_equal(a[c], ac)


# ---------------------------------------------------------------------------
# Detector grouping (Sec. II-E): g adjacent columns share one mean and one
# covariance.  Pins that do not restate the grouping itself:
#  * g = 1 is the per-column retrieval;
#  * a partition made of g identical copies of one column has the same 1/N
#    means and covariances as the column alone (R2), so every copy gets the
#    single-column alpha - by induction over the iterations;
#  * pixels are exchangeable: permuting the columns inside a partition
#    permutes the outputs;
#  * the remainder partition of S = 7, g = 3 is the last column alone.

def _group_scene(rng, S=7, N=150, B=8):
    L = np.stack([_background_column(rng, N, B, 0.3) for _ in range(S)])
    s = _s(rng, B) * 5
    for c in range(S):                       # a few plume pixels per column
        L[c, :6] *= np.exp(800.0 * s)[None, :]
    return L, s


def test_grouping_of_one_is_the_per_column_retrieval():
    rng = _rng(61)
    L, s = _group_scene(rng)
    a1, st1 = retrieve(L, s, 6, lam=0.5)
    ag, stg = retrieve_grouped(L, s, 6, lam=0.5, group=1)
    np.testing.assert_array_equal(ag, a1)
    np.testing.assert_array_equal(stg, st1)


def test_grouping_identical_copies_keep_the_column_result():
    rng = _rng(62)
    L, s = _group_scene(rng, S=1, N=200)
    a1, _ = retrieve_column(L[0], s, 8, lam=0.5)
    Lg = np.repeat(L, 4, axis=0)             # 4 copies in one partition
    ag, st = retrieve_grouped(Lg, s, 8, lam=0.5, group=4)
    assert list(st) == [STATUS_OK]
    for c in range(4):
        np.testing.assert_allclose(ag[c], a1, rtol=1e-9, atol=1e-9)


def test_grouping_permutation_and_remainder():
    rng = _rng(63)
    L, s = _group_scene(rng)
    a, st = retrieve_grouped(L, s, 6, lam=0.5, group=3)
    assert len(st) == 3                      # partitions {0,1,2}, {3,4,5}, {6}
    perm = [2, 0, 1, 5, 3, 4, 6]             # permute inside each partition
    ap, _ = retrieve_grouped(L[perm], s, 6, lam=0.5, group=3)
    np.testing.assert_allclose(ap, a[perm], rtol=1e-10, atol=1e-10)
    a6, _ = retrieve_column(L[6], s, 6, lam=0.5)
    np.testing.assert_array_equal(a[6], a6)
    # a partition differs from its columns run alone (shared statistics)
    a0, _ = retrieve_column(L[0], s, 6, lam=0.5)
    assert np.abs(a[0] - a0).max() > 1e-6


# ---------------------------------------------------------------------------
# Energy monitor (Eq. 8 with the 1/2 of R5; R14).
#  * K = 0, no albedo: the sample covariance gives sum_i (L_i-mu)^T C^-1
#    (L_i-mu) = N B exactly, and alpha_i = p_i / q, so E^0 = N B/2 - q/2 sum
#    alpha_i^2 (a dropped 1/2 or a wrong residual breaks it).
#  * the update minimises E at fixed mu^k, C^k, w^k: moving any alpha^k_i
#    (within alpha >= 0) cannot lower it.
#  * the column part used on the GPU: with C^k = C^0 + U S U^T (rank 3),
#    sum_i (L_i - mu^k)^T C^k^-1 (L_i - mu^k) = N (B - tr(S M)) + N abar^2
#    e^T M e, M = U^T C^k^-1 U = W - W (I + S W)^-1 S W, W = U^T C^0^-1 U,
#    e = (1, 1, 0); checked against the direct sum.

def test_energy_closed_form_k0():
    rng = _rng(71)
    L = _background_column(rng, 300, 8, 0.0)
    s = _s(rng, 8) * 5
    E = []
    a, st = retrieve_column(L, s, 0, lam=1.0, albedo=False, energy=E)
    mu = L.mean(axis=0)
    C = (L - mu).T @ (L - mu) / len(L)
    t = mu * s
    q = t @ np.linalg.solve(C, t)
    assert len(E) == 1
    np.testing.assert_allclose(E[0], 0.5 * len(L) * 8 - 0.5 * q * np.sum(a ** 2), rtol=1e-10)


def test_energy_update_is_a_minimiser():
    rng = _rng(72)
    L = _background_column(rng, 250, 8, 0.3)
    s = _s(rng, 8) * 5
    L[:10] *= np.exp(700.0 * s)[None, :]
    trace = []
    retrieve_column(L, s, 4, lam=0.3, trace=trace)
    mu0 = L.mean(axis=0)
    r = L @ mu0 / (mu0 @ mu0)
    for it in trace[1:]:
        base = energy_k(L, it.mu, it.C, it.t, r, it.w, it.alpha)
        act = np.flatnonzero(it.alpha > 0)[:5]
        zero = np.flatnonzero(it.alpha == 0)[:5]
        assert len(act) > 0
        for i in act:
            for dlt in (1e-3, -1e-3):
                a2 = it.alpha.copy()
                a2[i] = max(0.0, a2[i] + dlt * max(1.0, a2[i]))
                assert energy_k(L, it.mu, it.C, it.t, r, it.w, a2) >= base - 1e-9 * abs(base)
        for i in zero:
            a2 = it.alpha.copy()
            a2[i] = 1e-2
            assert energy_k(L, it.mu, it.C, it.t, r, it.w, a2) >= base


def test_energy_column_term_by_rank3_identity():
    rng = _rng(73)
    N, B = 400, 8
    L = _background_column(rng, N, B, 0.3)
    s = _s(rng, B) * 5
    L[:15] *= np.exp(900.0 * s)[None, :]
    trace = []
    retrieve_column(L, s, 3, lam=0.2, trace=trace)
    Lbar = L.mean(axis=0)
    C0 = (L - Lbar).T @ (L - Lbar) / N
    r = L @ Lbar / (Lbar @ Lbar)
    for k in range(1, len(trace)):
        it, prev = trace[k], trace[k - 1]
        c = r * it.alpha_prev
        abar, S2 = c.mean(), np.sum(c * c)
        m = ((L - Lbar) * c[:, None]).sum(axis=0)
        U = np.stack([prev.t - it.t, it.t, m], axis=1)
        S = np.array([[abar ** 2, 0, 0], [0, S2 / N - abar ** 2, -1 / N], [0, -1 / N, 0]])
        np.testing.assert_allclose(C0 + U @ S @ U.T, it.C, rtol=1e-9, atol=1e-12)
        W = U.T @ np.linalg.solve(C0, U)
        M = W - W @ np.linalg.solve(np.eye(3) + S @ W, S @ W)
        e = np.array([1.0, 1.0, 0.0])
        fast = N * (B - np.trace(S @ M)) + N * abar ** 2 * (e @ M @ e)
        D = L - it.mu
        direct = np.sum(D * np.linalg.solve(it.C, D.T).T)
        np.testing.assert_allclose(fast, direct, rtol=1e-9)


# ---------------------------------------------------------------------------
# Closed form at convergence with a known background (linear model of Eq. 1):
# L_i = mu_bg + alpha_i t + n_i with n ~ N(0, Sigma).  With lambda large
# enough to zero every background pixel, mu^k and C^k become background
# statistics and each plume pixel converges to the fixed point of
#   alpha = z - lambda / (r q alpha),  z = alpha_true + e,  e ~ N(0, 1/q),
# i.e. alpha = (z + sqrt(z^2 - 4 lambda / q)) / 2 for r = 1.

def test_recovery_fixed_point_linear_model():
    rng = _rng(61)
    N, B = 40000, 8
    x = np.linspace(0, 1, B)
    mu_bg = 3 + np.sin(3 * x)
    s = -1e-4 * (0.2 + np.exp(-((x - 0.5) / 0.15) ** 2))
    t = mu_bg * s
    A = rng.standard_normal((B, B)) * 0.01
    Sigma = A @ A.T + 1e-4 * np.eye(B)
    q_true = t @ np.linalg.solve(Sigma, t)
    sd = 1.0 / np.sqrt(q_true)
    n = rng.multivariate_normal(np.zeros(B), Sigma, N)
    alpha_true = np.zeros(N)
    idx = rng.choice(N, 400, replace=False)
    alpha_true[idx] = rng.uniform(20, 60, 400) * sd
    L = mu_bg + alpha_true[:, None] * t + n
    lam = 25.0                       # zeros pixels with z < 10 sd
    a, st = retrieve_column(L, s, 30, lam=lam, albedo=False)
    assert st == STATUS_OK
    bg = alpha_true == 0
    assert (a[bg] > 0).mean() < 1e-3
    at = alpha_true[idx]
    pred = 0.5 * (at + np.sqrt(at ** 2 - 4 * lam / q_true))
    err = a[idx] - pred
    assert abs(err.mean()) < 4 * sd / np.sqrt(400)
    assert 0.85 < err.std() / sd < 1.15
    # the shrink itself is resolved: without it the mean error would be
    # lambda/(q alpha) ~ 0.5 sd, far outside the band above
    assert abs((a[idx] - at).mean() + (lam / q_true / at).mean()) < 4 * sd / np.sqrt(400)


def test_recovery_with_albedo_variation():
    """Same with a per-pixel albedo a_i scaling background and signal.  The
    filter of Eq. (8) scales the target by r_i (Eq. 7, from the observed L_i,
    which includes the absorption), so a plume pixel's score is
    z_i = (a_i / r_i) alpha_true_i + noise, shrunk as above with r_i q."""
    rng = _rng(62)
    N, B = 40000, 8
    x = np.linspace(0, 1, B)
    mu_bg = 3 + np.sin(3 * x)
    s = -1e-4 * (0.2 + np.exp(-((x - 0.5) / 0.15) ** 2))
    t = mu_bg * s
    Sigma = 1e-4 * np.eye(B)
    alb = rng.uniform(0.6, 1.4, N)
    alb /= alb.mean()
    C_true = alb.var() * np.outer(mu_bg, mu_bg) + Sigma
    q = t @ np.linalg.solve(C_true, t)
    sd = 1.0 / np.sqrt(q)
    alpha_true = np.zeros(N)
    idx = rng.choice(N, 400, replace=False)
    alpha_true[idx] = rng.uniform(30, 60, 400) * sd
    L = alb[:, None] * (mu_bg + alpha_true[:, None] * t) + \
        rng.multivariate_normal(np.zeros(B), Sigma, N)
    lam = 25.0
    a, st = retrieve_column(L, s, 30, lam=lam, albedo=True)
    assert st == STATUS_OK
    assert (a[alpha_true == 0] > 0).mean() < 1e-3
    mu = L.mean(0)
    r = (L @ mu / (mu @ mu))[idx]
    z = alb[idx] / r * alpha_true[idx]
    pred = 0.5 * (z + np.sqrt(z ** 2 - 4 * lam / (r * q)))
    err = a[idx] - pred
    se = sd * np.sqrt((1 / r ** 2).mean())
    assert abs(err.mean()) < 5 * se / np.sqrt(400)
    assert 0.8 < err.std() / se < 1.2
    # dropping the albedo factor of the observed radiance would bias by
    # mean((a/r - 1) alpha_true), far outside the band above
    assert abs(((alb[idx] / r - 1) * alpha_true[idx]).mean()) > 10 * se / np.sqrt(400)


# ---------------------------------------------------------------------------
# Zero-locking (Eq. 5 with small epsilon): once alpha_i = 0 the weight is
# lambda/epsilon, so a pixel stays 0 whenever lambda/(epsilon r q) > p_i.

def test_zero_locking():
    rng = _rng(71)
    L = _background_column(rng, 800, 12, albedo_spread=0.5)
    s = _s(rng, 12) * 5
    L[:30] *= np.exp(rng.uniform(300, 3000, 30)[:, None] * s)
    trace = []
    retrieve_column(L, s, 10, lam=1.0, eps=1e-9, trace=trace)
    viol = 0
    for prev, it in zip(trace[1:-1], trace[2:]):
        viol += int(((prev.alpha == 0) & (it.alpha > 0)).sum())
    assert viol == 0


def test_lambda_monotone_sparsity():
    from synth.scenes import make_scene, tiny_spec
    sc = make_scene(tiny_spec())
    L = sc.radiance[:8]
    counts = []
    for lam in [0.0, 0.5, 1.0, 2.0, 4.0]:
        a, _ = retrieve(L, sc.s, 30, lam=lam)
        counts.append(int((a > 0).sum()))
    assert all(c1 >= c2 for c1, c2 in zip(counts, counts[1:])), counts


# ---------------------------------------------------------------------------
# Degenerate columns (status codes) and masks

def test_status_few_pixels_and_nonfinite():
    rng = _rng(81)
    L = _background_column(rng, 10, 12)
    a, st = retrieve_column(L, _s(rng, 12), 3)
    assert st == STATUS_FEW_PIXELS and np.all(a == 0)
    L = _background_column(rng, 100, 12)
    L[5, 3] = np.nan
    a, st = retrieve_column(L, _s(rng, 12), 3)
    assert st == STATUS_NONFINITE and np.all(a == 0)
    valid = np.ones(100, np.uint8)
    valid[5] = 0
    a, st = retrieve_column(L, _s(rng, 12), 3, valid=valid)
    assert st == STATUS_OK and a[5] == 0


def test_mask_equals_removal():
    rng = _rng(82)
    L = _background_column(rng, 300, 10, 0.3)
    s = _s(rng, 10) * 5
    valid = (rng.uniform(size=300) > 0.2).astype(np.uint8)
    Lm = L.copy()
    Lm[valid == 0] = np.nan
    a, st = retrieve_column(Lm, s, 6, lam=1.0, valid=valid)
    b, _ = retrieve_column(L[valid == 1], s, 6, lam=1.0)
    np.testing.assert_array_equal(a[valid == 1], b)
    assert np.all(a[valid == 0] == 0)
