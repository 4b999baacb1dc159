"""Boundary-condition-enforced immersed boundary step (oracle; test infrastructure).

Follows Section 2.3 of the paper:

* the regularised delta of Eq. 18 (a four-point kernel, support |r| < 2);
* the discrete delta of Eq. 17, D_ij = prod_d h^-1 delta((x_j,d - X_i,d)/h); the
  interpolation weight used here is w_ij = h^3 D_ij, so that the interpolated
  velocity of Eq. 6 at point i is sum_j w_ij u_j (the h^3 factor of Eqs. 20 and 23);
* the force system of Eqs. 20-24, A_F F = B_F with
  A_F = (dt/rho) h^3 [D dS] [D^T] and B_F = U_B - h^3 D^T u~.  With Lambda = c F,
  c = (dt/rho) dS / h^3 and the correction restricted to free velocity nodes, this
  is G Lambda = U_B - I u~ with G = I_F I_F^T;
* spreading (Eq. 19) and the velocity update u = u~ + dt f / rho (Eq. 14), i.e.
  u_F = u~_F + I_F^T Lambda.

Readings: I reads every node (nodes outside the vessel hold zero velocity);
only free nodes F are corrected; the 4x4x4 support starts at
floor((X - x0)/h) - 1 per axis; support nodes outside the box are dropped.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import krylov


def delta4(r):
    """Four-point kernel of Eq. 18 (credited in the paper to Lai and Peskin)."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(r)
    a = r <= 1.0
    b = (r > 1.0) & (r <= 2.0)
    out[a] = (3.0 - 2.0 * r[a] + np.sqrt(1.0 + 4.0 * r[a] - 4.0 * r[a] ** 2)) / 8.0
    out[b] = (5.0 - 2.0 * r[b] - np.sqrt(-7.0 + 12.0 * r[b] - 4.0 * r[b] ** 2)) / 8.0
    return out


def interpolation_matrix(X: np.ndarray, nx: int, ny: int, nz: int, h: float,
                         origin: np.ndarray) -> sp.csr_matrix:
    """I (M x N) with I_ij = w_ij = prod_d delta((x_j,d - X_i,d)/h) over the 4x4x4
    support of each point (Eq. 17 times h^3)."""
    M = X.shape[0]
    N = (nx + 1) * (ny + 1) * (nz + 1)
    dims = np.array([nx, ny, nz])
    offs = np.array([[a, b, c] for c in range(4) for b in range(4) for a in range(4)])
    base = np.floor((X - origin[None, :]) / h).astype(np.int64) - 1         # (M, 3)
    idx = base[:, None, :] + offs[None, :, :]                              # (M, 64, 3)
    inside = ((idx >= 0) & (idx <= dims)).all(axis=2)                      # (M, 64)
    xn = origin + idx * h                                                  # node coords
    w = np.prod(delta4((xn - X[:, None, :]) / h), axis=2)                  # (M, 64)
    n = idx[..., 0] + (nx + 1) * (idx[..., 1] + (ny + 1) * idx[..., 2])
    rows = np.repeat(np.arange(M), 64).reshape(M, 64)
    return sp.coo_matrix((w[inside], (rows[inside], n[inside])), shape=(M, N)).tocsr()


class SingularIB(RuntimeError):
    """A Lagrangian point has no (numerically) free support node."""


def bce_correction(I: sp.csr_matrix, in_F: np.ndarray, U_B: np.ndarray, u_tilde: np.ndarray,
                   direct_max: int = 2000):
    """Solve G Lambda = U_B - I u~ (G = I_F I_F^T) for the three components and return
    (u_ib, Lambda, info).  u_ib = u~ + I_F^T Lambda on free nodes, u~ elsewhere.

    The paper solves its force system with a direct solver; for M <= direct_max a dense
    Cholesky factorisation is used here, otherwise CG iterated to stagnation."""
    IF = I @ sp.diags(in_F.astype(np.float64))
    row_norm2 = np.asarray(IF.multiply(IF).sum(axis=1)).ravel()
    if I.shape[0] and row_norm2.min() < 1e-12:
        raise SingularIB("Lagrangian point without free support")
    G = (IF @ IF.T).tocsr()
    b = U_B.T - np.stack([I @ u_tilde[d] for d in range(3)], axis=0)      # (3, M)
    lam = np.zeros_like(b)
    info = {}
    if I.shape[0] == 0:
        return u_tilde.copy(), lam, info
    if G.shape[0] <= direct_max:
        L = krylov.cholesky(G.toarray())
        for d in range(3):
            lam[d] = krylov.cholesky_solve(L, b[d])
        info["method"] = "cholesky"
    else:
        its = []
        for d in range(3):
            lam[d], it, res = krylov.cg(G, b[d], diag=G.diagonal())
            its.append((it, res))
        info["method"] = "cg"
        info["iters"] = its
    u_ib = u_tilde.copy()
    for d in range(3):
        u_ib[d] += IF.T @ lam[d]
    return u_ib, lam, info
