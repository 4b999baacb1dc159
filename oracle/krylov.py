"""Linear solvers for the oracle (test infrastructure).

The paper does not name its solver backend (FEniCS defaults) and solves the IB
force system "with a direct solver" (Section 2.3).  The discrete solution of every
sub-problem is unique, so the oracle iterates textbook Jacobi-preconditioned
CG / BiCGStab until stagnation: the relative residual reaches `rtol` or has not
improved for `patience` iterations.  The result is the best iterate seen.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

RTOL = 1e-14
PATIENCE = 400


def cg(A, b: np.ndarray, x0: np.ndarray | None = None, diag: np.ndarray | None = None,
       rtol: float = RTOL, patience: int = PATIENCE, max_iter: int | None = None):
    """Preconditioned conjugate gradients on SPD (or consistent singular SPD) A."""
    n = b.size
    max_iter = max_iter or 20 * n + 100
    x = np.zeros(n) if x0 is None else x0.copy()
    dinv = np.ones(n) if diag is None else 1.0 / diag
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0
    r = b - A @ x
    z = dinv * r
    p = z.copy()
    rz = r @ z
    best_x, best_res, since = x.copy(), np.linalg.norm(r) / bnorm, 0
    it = 0
    while it < max_iter and best_res > rtol and since < patience:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        res = np.linalg.norm(r) / bnorm
        if res < best_res:
            best_x, best_res, since = x.copy(), res, 0
        else:
            since += 1
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return best_x, it, best_res


def bicgstab(A, b: np.ndarray, x0: np.ndarray | None = None, diag: np.ndarray | None = None,
             rtol: float = RTOL, patience: int = PATIENCE, max_iter: int | None = None):
    """Right-preconditioned BiCGStab (van der Vorst) for nonsymmetric A."""
    n = b.size
    max_iter = max_iter or 20 * n + 100
    x = np.zeros(n) if x0 is None else x0.copy()
    dinv = np.ones(n) if diag is None else 1.0 / diag
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0
    r = b - A @ x
    r_hat = r.copy()
    rho_old = alpha = omega = 1.0
    v = np.zeros(n)
    p = np.zeros(n)
    best_x, best_res, since = x.copy(), np.linalg.norm(r) / bnorm, 0
    it = 0
    while it < max_iter and best_res > rtol and since < patience:
        rho = r_hat @ r
        if rho == 0.0:
            break
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        phat = dinv * p
        v = A @ phat
        alpha = rho / (r_hat @ v)
        s = r - alpha * v
        shat = dinv * s
        t = A @ shat
        tt = t @ t
        omega = (t @ s) / tt if tt > 0.0 else 0.0
        x += alpha * phat + omega * shat
        r = s - omega * t
        rho_old = rho
        it += 1
        res = np.linalg.norm(r) / bnorm
        if res < best_res:
            best_x, best_res, since = x.copy(), res, 0
        else:
            since += 1
        if omega == 0.0:
            break
    # Report the true residual of the returned iterate.
    true_res = np.linalg.norm(b - A @ best_x) / bnorm
    return best_x, it, true_res


def cholesky(A: np.ndarray) -> np.ndarray:
    """Dense lower Cholesky factor (the direct solver for the IB force system)."""
    return np.linalg.cholesky(A)


def cholesky_solve(L: np.ndarray, b: np.ndarray) -> np.ndarray:
    y = sla.solve_triangular(L, b, lower=True)
    return sla.solve_triangular(L.T, y, lower=False)
