"""Host emulation of the rounded Gram forms' solve (no GPU): the covariance of
iteration k accumulated from FP32-, BF16- or split-BF16-rounded residuals in
FP32 per block (as the FP32 and BF16 MFMA passes do; split BF16 takes
hi hi' + hi lo' + lo hi' with hi = bf16(y), lo = bf16(y - hi)), factored in
FP64, used only to precondition iterative refinement whose residual takes the
exact C^k.  The error of v = C^-1 t contracts by about 1e-3 (FP32), 2e-2
(BF16) and 1e-2 (split BF16) per step and falls below 1e-10 (FP32) and 1e-9
(BF16, split BF16) relative in the library's default step counts (3, 5 and 4;
FP64 rounding is about 1e-12 here),
while a refinement against the rounded matrix itself keeps the Gram's
rounding error.  The exact C^k, t^k and alpha^{k-1} come from the oracle's
trace of one column of the flightline workload."""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle.mf64 import retrieve_column
from synth.scenes import flightline_spec, make_column, make_globals
from tests.parity_util import config_lambda


def _bf16(x):
    x = np.asarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = ((u + ((u >> 16) & 1) + 0x7FFF) >> 16) << 16          # round to nearest even
    return u.astype(np.uint32).view(np.float32)


@pytest.fixture(scope="module")
def column_trace():
    spec = flightline_spec()
    g = make_globals(spec)
    c = int(g.plumes[0, 0])                                    # a column through a plume
    L, _, _ = make_column(spec, g, c)
    trace = []
    retrieve_column(L, g.s, 30, config_lambda("flightline"), 1e-9, True, trace=trace)
    return L.astype(np.float64), trace


@pytest.mark.parametrize("form,block,steps,rho_max,v_tol", [("fp32", 1024, 3, 5e-3, 1e-10),
                                                            ("bf16", 1024, 5, 5e-2, 1e-9),
                                                            ("bf16x3", 1024, 4, 3e-2, 1e-9)])
def test_exact_residual_refinement_converges(column_trace, form, block, steps, rho_max, v_tol):
    L, trace = column_trace
    N, B = L.shape
    mu0 = trace[0].mu
    r = (L @ mu0) / (mu0 @ mu0)
    for k in (1, 15, 30):
        it, prev = trace[k], trace[k - 1]
        c = (r * it.alpha_prev).astype(np.float32)
        y = (L.astype(np.float32) - prev.mu.astype(np.float32)) - c[:, None] * prev.t.astype(np.float32)
        Y = np.concatenate([y, np.ones((N, 1), np.float32), c[:, None]], axis=1)
        if form == "bf16":
            Y = _bf16(Y)
        G = np.zeros((B + 2, B + 2))
        for b0 in range(0, N, block):                        # FP32 sums per block, FP64 across
            Yb = Y[b0:b0 + block].astype(np.float32)
            if form == "bf16x3":
                hi = _bf16(Yb)
                lo = _bf16(Yb - hi)
                G += (hi.T @ hi + hi.T @ lo + lo.T @ hi).astype(np.float64)
            else:
                G += (Yb.T @ Yb).astype(np.float64)
        # the shifted-Gram assembly of C about mu^k (the solve's formula)
        D = prev.mu.astype(np.float32).astype(np.float64) - it.mu
        E = prev.t.astype(np.float32).astype(np.float64) - it.t
        g1, g2, n, S1, S2 = G[B, :B], G[B + 1, :B], G[B, B], G[B + 1, B], G[B + 1, B + 1]
        NC = (G[:B, :B] + np.outer(g1, D) + np.outer(D, g1) + np.outer(g2, E) + np.outer(E, g2)
              + n * np.outer(D, D) + S1 * (np.outer(D, E) + np.outer(E, D)) + S2 * np.outer(E, E))
        Cf = NC / n
        C, t = it.C, it.t
        v_exact = np.linalg.solve(C, t)
        fac = sl.cho_factor(Cf, lower=True)
        err = lambda v: np.linalg.norm(v - v_exact) / np.linalg.norm(v_exact)
        v = sl.cho_solve(fac, t)
        e0 = err(v)
        v_self = v.copy()
        for _ in range(steps):
            v = v + sl.cho_solve(fac, t - C @ v)               # residual with the exact C^k
            v_self = v_self + sl.cho_solve(fac, t - Cf @ v_self)   # ... with the rounded matrix
        rho = np.abs(np.linalg.eigvals(np.eye(B) - sl.cho_solve(fac, C))).max()
        assert rho < rho_max, (k, rho)
        assert err(v) < v_tol, (k, e0, err(v))
        assert err(v_self) > 0.5 * e0                          # the rounding error stays
