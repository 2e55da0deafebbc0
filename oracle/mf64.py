"""FP64 CPU oracle for the albedo-corrected reweighted-l1 matched filter.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The library never calls it: there is
no CPU fallback.  It shares no code with the GPU path.

It follows the paper's algorithm figure ("AlbedoReWeightL1Filter", Fig. 1)
step by step, in float64, on one detector partition (one cross-track column,
Sec. II-E) at a time.  The covariance is recomputed from its definition every
iteration (Eq. 11) - no shifted moments, no low-rank updates, no fusion.

Readings of the paper that this oracle takes (each is listed with its reason
in the design notes of the repository):
  R1  C^0 is the outer-product sample covariance (the figure prints an inner
      product; Eq. 11 and the iteration body use the outer product).
  R2  all means and covariances are normalised by 1/N.
  R3  r_i is computed once, from mu^0 and the observed L_i, and kept fixed.
  R4  alpha^0 is clamped at 0 before it is used in w^1, mu^1, C^1 (positivity
      inside each iteration, Sec. III-D); with zero iterations the unclamped
      alpha^0 is returned (the non-iterative filters have negative values).
  R5  the per-pixel update is the one printed in Fig. 1 / Eq. 6, i.e. the exact
      minimiser over alpha >= 0 of 1/2 d^T C^-1 d + r w alpha.
  R6  epsilon is a parameter (default 1e-9 ppm*m).
  R7  w = lambda / (alpha + epsilon); lambda = 1 is the paper, lambda = 0
      switches the sparsity prior off ("Iter. Pos." variants of Table I).
  R8  mu^k removes r alpha^{k-1} (mu^{k-1} * s), d_i uses mu^k * s (as printed
      both in Fig. 1 and in Eqs. 10-11).
  R12 invalid (masked) pixels are excluded from every sum; N = number of valid
      pixels; their output is 0.
  R13 a column with N <= B valid pixels, a non-finite valid pixel, or a
      covariance that is not positive definite gets a non-zero status and
      alpha = 0.  A pixel with r_i <= 0 keeps alpha = 0 (it stays in the
      background statistics).
  R14 the energy monitored per iteration (Eq. 8, Sec. III-B) is the objective
      the update of R5 minimises: E^k = sum_i 1/2 d_i^T C^k^-1 d_i
      + r_i w^k_i alpha^k_i with d_i = L_i - r_i alpha^k_i t^k - mu^k, alpha^k
      as carried into the next iteration (alpha^0 clamped unless K = 0) and
      w^0 = 0.
"""
from __future__ import annotations

import os
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.linalg

STATUS_OK = 0
STATUS_FEW_PIXELS = 1
STATUS_NOT_SPD = 2
STATUS_NONFINITE = 3


@dataclass
class IterState:
    """Per-iteration state of one column, recorded when a trace list is given."""
    k: int
    mu: np.ndarray        # mu^k
    C: np.ndarray         # C^k
    t: np.ndarray         # t^k = mu^k * s
    w: Optional[np.ndarray]   # w^k (None for k = 0)
    alpha_prev: Optional[np.ndarray]  # alpha^{k-1} as used (clamped)
    alpha: np.ndarray     # alpha^k (unclamped for k = 0)


def _solve_spd(C: np.ndarray, t: np.ndarray) -> np.ndarray:
    """C^-1 t through a Cholesky factorisation (LAPACK potrf/potrs)."""
    cf = scipy.linalg.cho_factor(C, lower=True, check_finite=True)
    return scipy.linalg.cho_solve(cf, t, check_finite=False)


def energy_k(X, mu, C, t, r, w, alpha) -> float:
    """E^k of R14 (Eq. 8 with the 1/2 of R5), from its definition: the
    residuals d_i formed explicitly and solved against C^k."""
    d = X - (r * alpha)[:, None] * t[None, :] - mu
    cf = scipy.linalg.cho_factor(C, lower=True, check_finite=True)
    quad = np.einsum("ij,ji->i", d, scipy.linalg.cho_solve(cf, d.T, check_finite=False))
    pen = 0.0 if w is None else float(np.sum(r * w * alpha))
    return float(0.5 * quad.sum() + pen)


def alpha_step(L, mu, C, t, r, w):
    """One albedo-scaled soft-threshold step (Fig. 1, inner loop; Eq. 6, 8).

    alpha_i = max(((L_i - mu)^T C^-1 t - w_i) / (r_i t^T C^-1 t), 0)
    """
    v = _solve_spd(C, t)
    q = t @ v
    return np.maximum(((L - mu) @ v - w) / (r * q), 0.0)


def retrieve_column(L, s, n_iter: int, lam: float = 1.0, eps: float = 1e-9,
                    albedo: bool = True, valid=None, trace: Optional[List] = None,
                    energy: Optional[List] = None):
    """Run Fig. 1 on one column.

    L      [N, B] radiance (any float dtype; used in float64)
    s      [B] unit absorption spectrum, (ppm*m)^-1
    n_iter number of reweighting iterations K (>= 0)
    lam    weight scale (w = lam / (alpha + eps))
    valid  [N] bool/uint8 or None
    energy if a list, E^0..E^K (R14) are appended to it
    Returns (alpha [N] float64, status int).
    """
    L = np.asarray(L, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    Nall, B = L.shape
    out = np.zeros(Nall)
    idx = np.arange(Nall) if valid is None else np.flatnonzero(np.asarray(valid) != 0)
    X = L[idx]                      # the partition D = {L_i}
    N = X.shape[0]
    if N <= B:
        return out, STATUS_FEW_PIXELS
    if not np.all(np.isfinite(X)):
        return out, STATUS_NONFINITE

    # Initialize mu^0 = (1/N) sum L_i
    mu = X.sum(axis=0) / N
    # Initialize C^0 = (1/N) sum (L_i - mu^0)(L_i - mu^0)^T    (R1, R2)
    D0 = X - mu
    C = (D0.T @ D0) / N
    t = mu * s                      # target t(mu^0) = mu^0 (.) s  (Eq. 9)
    # r_i = L_i^T mu / mu^T mu  (Eq. 7), fixed from here on (R3)
    if albedo:
        r = (X @ mu) / (mu @ mu)
    else:
        r = np.ones(N)
    dark = r <= 0.0                 # R13: such pixels keep alpha = 0
    r_safe = np.where(dark, 1.0, r)
    # alpha^0_i = (L_i - mu^0)^T C^0^-1 t / (r_i t^T C^0^-1 t)
    try:
        v = _solve_spd(C, t)
    except np.linalg.LinAlgError:
        return out, STATUS_NOT_SPD
    q = t @ v
    if not (q > 0.0):
        return out, STATUS_NOT_SPD
    alpha = (D0 @ v) / (r_safe * q)
    alpha = np.where(dark, 0.0, alpha)
    if trace is not None:
        trace.append(IterState(0, mu.copy(), C.copy(), t.copy(), None, None, alpha.copy()))
    if n_iter == 0:
        if energy is not None:
            energy.append(energy_k(X, mu, C, t, r, None, alpha))
        out[idx] = alpha
        return out, STATUS_OK
    alpha = np.maximum(alpha, 0.0)  # R4
    if energy is not None:
        energy.append(energy_k(X, mu, C, t, r, None, alpha))

    for k in range(1, n_iter + 1):
        # w^k = lam / (alpha^{k-1} + eps)      (Eq. 5, R7)
        w = lam / (alpha + eps)
        # mu^k = (1/N) sum (L_i - r_i alpha_i^{k-1} mu^{k-1} (.) s)   (R8)
        mu_new = (X - (r * alpha)[:, None] * (mu * s)[None, :]).sum(axis=0) / N
        t = mu_new * s
        # d_Ci = L_i - r_i alpha_i^{k-1} mu^k (.) s - mu^k
        d = X - (r * alpha)[:, None] * t[None, :] - mu_new
        # C^k = (1/N) sum d_Ci d_Ci^T
        C = (d.T @ d) / N
        try:
            v = _solve_spd(C, t)
        except np.linalg.LinAlgError:
            out[:] = 0.0
            return out, STATUS_NOT_SPD
        q = t @ v
        if not (q > 0.0):
            out[:] = 0.0
            return out, STATUS_NOT_SPD
        # alpha_i^k = max(((L_i - mu^k)^T C^k^-1 t - w_i) / (r_i t^T C^k^-1 t), 0)
        alpha_new = np.maximum(((X - mu_new) @ v - w) / (r_safe * q), 0.0)
        alpha_new = np.where(dark, 0.0, alpha_new)
        if trace is not None:
            trace.append(IterState(k, mu_new.copy(), C.copy(), t.copy(), w.copy(),
                                   alpha.copy(), alpha_new.copy()))
        if energy is not None:
            energy.append(energy_k(X, mu_new, C, t, r, w, alpha_new))
        alpha = alpha_new
        mu = mu_new
    out[idx] = alpha
    return out, STATUS_OK


# ---------------------------------------------------------------------------
# Whole scenes: columns are independent problems (Sec. II-E), so they are
# spread over a process pool with one BLAS thread per process.

_POOL_ARGS = None


def _pool_init(args):
    global _POOL_ARGS
    _POOL_ARGS = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover - threadpoolctl is optional
        pass


def _pool_column(c):
    L, s, n_iter, lam, eps, albedo, valid = _POOL_ARGS
    return retrieve_column(L[c], s, n_iter, lam, eps, albedo,
                           None if valid is None else valid[c])


def retrieve(L, s, n_iter: int, lam: float = 1.0, eps: float = 1e-9,
             albedo: bool = True, valid=None, workers: int = 1,
             columns=None):
    """Run every column (or the listed ones) of a [S, N, B] cube.

    Returns (alpha [S', N] float64, status [S'] int32) for the selected columns.
    """
    S = L.shape[0]
    cols = list(range(S)) if columns is None else list(columns)
    args = (L, s, n_iter, lam, eps, albedo, valid)
    if workers <= 1 or len(cols) <= 1:
        _pool_init(args)
        res = [_pool_column(c) for c in cols]
    else:
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        with ctx.Pool(workers, initializer=_pool_init, initargs=(args,)) as pool:
            res = pool.map(_pool_column, cols, chunksize=max(1, len(cols) // (4 * workers)))
    alpha = np.stack([a for a, _ in res]) if res else np.zeros((0, L.shape[1]))
    status = np.array([st for _, st in res], dtype=np.int32)
    return alpha, status


def retrieve_grouped(L, s, n_iter: int, lam: float = 1.0, eps: float = 1e-9,
                     albedo: bool = True, valid=None, group: int = 1):
    """Detector grouping (Sec. II-E): `group` adjacent columns of a [S, N, B]
    cube form one partition (the last partition takes the remainder) whose
    pixels share one mean and one covariance.  Each partition is run through
    Fig. 1 as a single column of (columns x N) pixels.

    Returns (alpha [S, N] float64, status [ceil(S / group)] int32).
    """
    L = np.asarray(L)
    S, N, B = L.shape
    alpha = np.zeros((S, N))
    status = []
    for c0 in range(0, S, group):
        c1 = min(S, c0 + group)
        Lp = L[c0:c1].reshape((c1 - c0) * N, B)
        vp = None if valid is None else np.asarray(valid)[c0:c1].reshape(-1)
        a, st = retrieve_column(Lp, s, n_iter, lam, eps, albedo, vp)
        alpha[c0:c1] = a.reshape(c1 - c0, N)
        status.append(st)
    return alpha, np.array(status, dtype=np.int32)


def host_cores() -> int:
    return len(os.sched_getaffinity(0))
