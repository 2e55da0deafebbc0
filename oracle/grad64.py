"""Reference gradient of the retrieval (FP64, CPU) - TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the library never does.  It re-states the algorithm figure of the
paper (Fig. 1; Eqs. 3, 5-11) with torch FP64 tensor operations so that
torch.autograd differentiates it, and provides central finite differences of
the numpy oracle (oracle/mf64.py), which are independent of autograd.

Loss: J = sum_i (alpha_i^K - alpha_true_i)^2 over the valid pixels.
The derivative of max(z, 0) is taken as 1 for z > 0 and 0 otherwise.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle.mf64 import retrieve_column


def retrieve_column_torch(L, s, n_iter, lam, eps=1e-9, albedo=True, valid=None):
    """Fig. 1 on one column with torch FP64 ops; returns alpha on the valid pixels."""
    X = L if valid is None else L[torch.as_tensor(np.asarray(valid) != 0)]
    N = X.shape[0]
    mu = X.sum(0) / N
    D0 = X - mu
    C = D0.T @ D0 / N
    t = mu * s
    r = (X @ mu) / (mu @ mu) if albedo else torch.ones(N, dtype=X.dtype)
    v = torch.linalg.solve(C, t)
    q = t @ v
    a = (D0 @ v) / (r * q)
    if n_iter == 0:
        return a
    a = torch.where(a > 0, a, torch.zeros_like(a))
    for _ in range(n_iter):
        w = lam / (a + eps)
        c = r * a
        mu_new = (X - c[:, None] * (mu * s)[None, :]).sum(0) / N
        t = mu_new * s
        d = X - c[:, None] * t[None, :] - mu_new
        C = d.T @ d / N
        v = torch.linalg.solve(C, t)
        q = t @ v
        z = ((X - mu_new) @ v - w) / (r * q)
        a = torch.where(z > 0, z, torch.zeros_like(z))
        mu = mu_new
    return a


def loss_and_grads(L, s, alpha_true, n_iter, lam, eps=1e-9, albedo=True, valid=None):
    """J and (dJ/dL [S,N,B], dJ/ds [B]) by autograd over every column."""
    Lt = torch.tensor(np.asarray(L, dtype=np.float64), requires_grad=True)
    st = torch.tensor(np.asarray(s, dtype=np.float64), requires_grad=True)
    J = torch.zeros((), dtype=torch.float64)
    for c in range(Lt.shape[0]):
        vc = None if valid is None else valid[c]
        a = retrieve_column_torch(Lt[c], st, n_iter, lam, eps, albedo, vc)
        at = np.asarray(alpha_true[c], dtype=np.float64)
        if vc is not None:
            at = at[np.asarray(vc) != 0]
        J = J + ((a - torch.from_numpy(at)) ** 2).sum()
    J.backward()
    return float(J.detach()), Lt.grad.numpy(), st.grad.numpy()


def loss_numpy(L, s, alpha_true, n_iter, lam, eps=1e-9, albedo=True, valid=None, columns=None):
    """J from the numpy oracle (FP64)."""
    L = np.asarray(L, dtype=np.float64)
    cols = range(L.shape[0]) if columns is None else columns
    J = 0.0
    for c in cols:
        vc = None if valid is None else valid[c]
        a, _ = retrieve_column(L[c], s, n_iter, lam, eps, albedo, vc)
        m = np.ones(L.shape[1], bool) if vc is None else (np.asarray(vc) != 0)
        J += float(((a - alpha_true[c])[m] ** 2).sum())
    return J


def fd_radiance(L, s, alpha_true, coord, h, n_iter, lam, eps=1e-9, albedo=True, valid=None):
    """Central difference of J in L[coord] (only the touched column is re-run)."""
    c, i, b = coord
    Lp = np.array(L[c:c + 1], dtype=np.float64)
    Lm = Lp.copy()
    Lp[0, i, b] += h
    Lm[0, i, b] -= h
    vc = None if valid is None else valid[c:c + 1]
    at = alpha_true[c:c + 1]
    return (loss_numpy(Lp, s, at, n_iter, lam, eps, albedo, vc) -
            loss_numpy(Lm, s, at, n_iter, lam, eps, albedo, vc)) / (2 * h)


def fd_target(L, s, alpha_true, b, h_rel, n_iter, lam, eps=1e-9, albedo=True, valid=None,
              columns=None):
    """Central difference of J in s[b] with the step h_rel * max|s| (bands far
    from absorption lines have |s_b| many orders below the maximum)."""
    s = np.asarray(s, dtype=np.float64)
    h = h_rel * float(np.abs(s).max())
    sp, sm = s.copy(), s.copy()
    sp[b] += h
    sm[b] -= h
    return (loss_numpy(L, sp, alpha_true, n_iter, lam, eps, albedo, valid, columns) -
            loss_numpy(L, sm, alpha_true, n_iter, lam, eps, albedo, valid, columns)) / (2 * h)
