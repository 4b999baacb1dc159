"""Q1 finite-element forms on the masked grid (oracle; test infrastructure).

The paper discretises the IPCS sub-problems (Section 2.2, Eqs. 7-12) with
equal-order finite elements.  Here the element is the trilinear cube of
side h.  Every form is integrated with the 2x2x2 Gauss rule, which is exact
for all integrands below (polynomial degree at most 3 per axis), and
assembled over the kept cells only:

    M_ij     = int N_i N_j                       (mass)
    K_ij     = int grad N_i . grad N_j           (stiffness, viscous term mu (grad u, grad v))
    G_d,ij   = int N_i d_d N_j                   (weak gradient; divergence B = [G_1 G_2 G_3])
    C(a)_ij  = int N_i (a_h . grad N_j)          (advection with a_h = sum_k a_k N_k)
    X_de,ij  = int d_e N_i d_d N_j               (the part of the strain-rate form
               2 mu (eps(u), eps(v)) beyond mu (grad u, grad v): the viscous form of
               the momentum equation, Section 2.1, written with eps(u) = (grad u +
               grad u^T)/2, couples component d of the test function with
               component e of the trial function through mu X_de)

Local corner a of a cell has offsets (a & 1, (a >> 1) & 1, (a >> 2) & 1).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

_GP = np.array([-1.0 / math.sqrt(3.0), 1.0 / math.sqrt(3.0)])


def _reference_shape():
    """Values and xi-derivatives of the 8 trilinear shape functions at the 8 Gauss
    points of [-1,1]^3.  Returns N (8g, 8a) and dN (8g, 8a, 3)."""
    pts = np.array([[_GP[gx], _GP[gy], _GP[gz]] for gz in range(2) for gy in range(2)
                    for gx in range(2)])
    sgn = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1]
                    for a in range(8)], dtype=np.float64)
    Nv = np.ones((8, 8))
    dN = np.zeros((8, 8, 3))
    for g in range(8):
        for a in range(8):
            f = [(1.0 + sgn[a, d] * pts[g, d]) / 2.0 for d in range(3)]
            Nv[g, a] = f[0] * f[1] * f[2]
            for d in range(3):
                prod = sgn[a, d] / 2.0
                for e in range(3):
                    if e != d:
                        prod *= f[e]
                dN[g, a, d] = prod
    return Nv, dN


def element_matrices(h: float):
    """Element mass, stiffness, weak gradients and the advection tensor of a cube of
    side h.  Gauss weights are 1, the Jacobian is (h/2) per axis.

    Returns Me (8,8), Ke (8,8), Ge (3,8,8) and Ce (8,8,3,8) with
    C^e(a)_{ib} = sum_{c,d} a_{c,d} Ce[i, c, d, b]."""
    Me, Ke, Ge, Ce, _ = element_matrices_all(h)
    return Me, Ke, Ge, Ce


def element_matrices_all(h: float):
    """element_matrices plus Xe (3,3,8,8): Xe[d, e, i, j] = int d_e N_i d_d N_j."""
    Nv, dNxi = _reference_shape()
    dV = (h / 2.0) ** 3
    dN = dNxi * (2.0 / h)                       # physical derivatives
    Me = np.einsum("ga,gb->ab", Nv, Nv) * dV
    Ke = np.einsum("gad,gbd->ab", dN, dN) * dV
    Ge = np.einsum("ga,gbd->dab", Nv, dN) * dV
    Ce = np.einsum("gi,gc,gbd->icdb", Nv, Nv, dN) * dV
    Xe = np.einsum("gie,gjd->deij", dN, dN) * dV
    return Me, Ke, Ge, Ce, Xe


def _assemble(corners: np.ndarray, local: np.ndarray, N: int) -> sp.csr_matrix:
    """Sum element matrices local[e] (or one shared matrix) into an N x N CSR."""
    ne = corners.shape[0]
    rows = np.repeat(corners, 8, axis=1).ravel()          # corners[e, a] repeated over b
    cols = np.tile(corners, (1, 8)).ravel()               # corners[e, b]
    if local.ndim == 2:
        vals = np.broadcast_to(local.ravel(), (ne, 64)).ravel()
    else:
        vals = local.reshape(ne, 64).ravel()
    return sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()


class Operators:
    """Assembled global (N x N) matrices over the kept cells; rows and columns of
    nodes outside P are empty."""

    def __init__(self, sets, h: float):
        self.N = sets.in_P.size
        self.corners = sets.corners
        self.Me, self.Ke, self.Ge, self.Ce, self.Xe = element_matrices_all(h)
        self.M = _assemble(self.corners, self.Me, self.N)
        self.K = _assemble(self.corners, self.Ke, self.N)
        self.G = [_assemble(self.corners, self.Ge[d], self.N) for d in range(3)]
        self._X = None

    def strain_cross(self):
        """X[d][e] = int d_e N_i d_d N_j assembled (3 x 3 list of N x N), so that the
        strain-rate viscous form is mu (K delta_de + X[d][e]) between test component d
        and trial component e."""
        if self._X is None:
            self._X = [[_assemble(self.corners, self.Xe[d, e], self.N) for e in range(3)] for d in range(3)]
        return self._X

    def advection(self, a: np.ndarray) -> sp.csr_matrix:
        """C(a) for the nodal velocity field a (3, N) (all nodes, Dirichlet values
        included)."""
        aloc = np.stack([a[d][self.corners] for d in range(3)], axis=2)   # (ne, 8c, 3d)
        local = np.einsum("ecd,icdb->eib", aloc, self.Ce)
        return _assemble(self.corners, local, self.N)

    def divergence(self, u: np.ndarray) -> np.ndarray:
        """(B u)_i = sum_d (G_d u_d)_i."""
        return self.G[0] @ u[0] + self.G[1] @ u[1] + self.G[2] @ u[2]
