"""Steady-state test and exact solution of the Poiseuille experiment (oracle;
test infrastructure only).

Section 3.1 runs the pressure-driven tube until the normalised root-mean-square
difference between two successive velocity fields is below 1e-8 for every
component, and compares the steady field with the Poiseuille profile
u_z(r) = U_max (1 - r^2/R^2), U_max = -(R^2 / (4 mu)) dp/dz, with the maximum error
L_inf and the root-mean-square error L_2 = (1/N) sqrt(sum of squared errors).

Readings: the N nodes of both norms are the nodes of P (the velocity lives there;
it is identically zero elsewhere), max and min are taken over the same nodes, and
a component whose old field is constant has NRMSE 0 when it did not change and
+inf when it did.
"""
from __future__ import annotations

import numpy as np


def nrmse(u_new: np.ndarray, u_old: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """(3,) step-to-step NRMSE of the three components over the node ids `nodes`."""
    out = np.empty(3)
    n = nodes.size
    for d in range(3):
        a = u_old[d][nodes]
        b = u_new[d][nodes]
        ssq = 0.0
        for v in (b - a):
            ssq += float(v) * float(v)
        rng = float(a.max() - a.min()) if n else 0.0
        rms = np.sqrt(ssq / (n * n)) if n else 0.0
        out[d] = rms / rng if rng > 0.0 else (0.0 if ssq == 0.0 else np.inf)
    return out


def poiseuille_u_max(p_drop: float, length: float, radius: float, mu: float) -> float:
    """U_max = R^2 (p_in - p_out) / (4 mu L): the centre-line speed of the
    pressure-driven tube flow."""
    return radius * radius * p_drop / (4.0 * mu * length)


def poiseuille_velocity(xyz: np.ndarray, p_drop: float, length: float, radius: float,
                        mu: float) -> np.ndarray:
    """(3, n) exact velocity at the points xyz (n, 3) of a tube along z centred on
    x = y = 0: (0, 0, U_max (1 - r^2/R^2)) inside, 0 outside."""
    r2 = xyz[:, 0] ** 2 + xyz[:, 1] ** 2
    uz = poiseuille_u_max(p_drop, length, radius, mu) * (1.0 - r2 / (radius * radius))
    out = np.zeros((3, xyz.shape[0]))
    out[2] = np.where(r2 < radius * radius, uz, 0.0)
    return out


def error_norms(u: np.ndarray, u_exact: np.ndarray) -> tuple[float, float]:
    """(L_inf, L_2) of the velocity error over the given nodes (u, u_exact: (3, n)):
    the largest component-wise error and (1/N) sqrt of the sum of squares of all
    component errors."""
    e = u - u_exact
    n = u.shape[1]
    return float(np.abs(e).max()), float(np.sqrt((e * e).sum()) / n)
