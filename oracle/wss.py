"""Wall shear stress at the Lagrangian points (oracle; test infrastructure).

The paper defines the wall shear stress as the tangential part of the traction
2 mu eps n (Section 2.6) and computes it on a body-fitted mesh of its vessels.
Here it is evaluated at the immersed wall points from the grid velocity, in four
plain steps:

1. nodal velocity gradient by the lumped L2 projection of the Q1 gradient:
   g_de(j) = (G_e u_d)_j / m_j with the weak gradient G_e of the momentum
   equation's forms and the lumped mass m_j = sum_k M_jk (nodes of P);
2. strain rate eps = (g + g^T) / 2 at every node;
3. eps at point X_i interpolated with the kernel of Eq. 18: eps(X_i) =
   sum_j w_ij eps_j (the weights of the interpolation I, every grid node);
4. traction t = 2 mu eps n for the wall normal n of the point, and the wall
   shear stress is its tangential part tau = t - (t . n) n.

Parity unpinned beyond the exact cases: linear velocity fields (exact nodal
gradients where every cell around a node is kept, exact interpolation of a
constant tensor) and rigid rotations (zero strain).
"""
from __future__ import annotations

import numpy as np


def nodal_strain(problem, u: np.ndarray) -> np.ndarray:
    """(3, 3, N) strain rate at every node of P (zero elsewhere)."""
    ops, s = problem.ops, problem.sets
    m = np.asarray(ops.M.sum(axis=1)).ravel()
    g = np.zeros((3, 3, m.size))
    P = s.in_P
    for d in range(3):
        for e in range(3):
            ge = ops.G[e] @ u[d]
            g[d, e][P] = ge[P] / m[P]
    return 0.5 * (g + g.transpose(1, 0, 2))


def wall_shear(problem, u: np.ndarray, normals: np.ndarray) -> np.ndarray:
    """(M, 3) wall shear stress vectors at the Lagrangian points of `problem` for the
    velocity u (3, N) and unit wall normals (M, 3)."""
    eps = nodal_strain(problem, u)
    I = problem.I
    eX = np.stack([np.stack([I @ eps[d, e] for e in range(3)], axis=1) for d in range(3)], axis=1)  # (M,3,3)
    n = np.asarray(normals, np.float64)
    t = 2.0 * problem.mu * np.einsum("ide,ie->id", eX, n)
    return t - np.sum(t * n, axis=1)[:, None] * n
