"""Pressure-driven Poiseuille flow of Section 3.1 on the Q1 grids of Table 1.

Tube of radius R = 5 mm and length L = 10 R along z in the box
[-6, 6] mm x [-6, 6] mm x [0, 50] mm, rho = 1050, mu = 0.00345, dt = 2.5e-3,
pressure p_in on the inlet disk (z = 0) and 0 on the outlet disk (z = L), no-slip
on the other box faces; grid spacing h = 1e-3 / 2^level (13 x 13 x 51, 25 x 25 x 101
and 49 x 49 x 201 nodes: the Eulerian node counts of Table 1).

Inputs only: node mask, boundary tags, Lagrangian wall points, initial fields.
"""
from __future__ import annotations

import math

import numpy as np

from .cases import TAG_OUTLET, TAG_WALL, Case, _ring_points

R = 0.005
L = 0.05
HALF_WIDTH = 0.006
RHO = 1050.0
MU = 0.00345
DT = 2.5e-3


def poiseuille_e1(level: int = 0, p_in: float = 1.0, spacing: float = 1.5, nsteps: int = 3) -> Case:
    """The tube on grid `level` (0, 1, 2 = h 1, 0.5, 0.25 mm).

    * mask: nodes with x^2 + y^2 < R^2;
    * boundary tags: every box-face node is wall, except the masked nodes of the two
      end faces, which are pressure boundaries (natural velocity, fixed pressure);
    * Lagrangian points: rings at z = (k + 1/2) L / rings with `per_ring` points at
      equal angles, point spacing close to `spacing` * h both ways, dS = 2 pi R L / M;
    * initial state: at rest, pressure p_in on the inlet disk and 0 elsewhere.
    """
    f = 2 ** int(level)
    h = 1e-3 / f
    nxy, nz = 12 * f, 50 * f
    per_ring = int(round(2.0 * math.pi * R / (spacing * h)))
    rings = int(round(L / (spacing * h)))
    c = Case(
        name=f"poiseuille_e1_h{h:g}_p{p_in:g}", nx=nxy, ny=nxy, nz=nz, h=h,
        origin=np.array([-HALF_WIDTH, -HALF_WIDTH, 0.0]),
        node_mask=np.zeros(0, np.uint8), bc_tag=None, X=np.zeros((0, 3)), dS=0.0, U_B=None,
        rho=RHO, mu=MU, dt=DT, nsteps=nsteps, inlet_K=0, inlet_omega=0.0,
        inlet_ids=np.zeros(0, np.int64), inlet_shape=np.zeros((1, 0, 3)),
        u0=np.zeros((3, 0)), p0=np.zeros(0))
    N = c.N
    k = np.arange(N)
    i = k % (nxy + 1)
    j = (k // (nxy + 1)) % (nxy + 1)
    kz = k // ((nxy + 1) * (nxy + 1))
    x = c.origin[0] + i * h
    y = c.origin[1] + j * h
    mask = (x * x + y * y < R * R).astype(np.uint8)
    c.node_mask = mask
    tag = np.zeros(N, np.uint8)
    face = (i == 0) | (i == nxy) | (j == 0) | (j == nxy) | (kz == 0) | (kz == nz)
    tag[face] = TAG_WALL
    inlet = (kz == 0) & (mask == 1)
    outlet = (kz == nz) & (mask == 1)
    tag[inlet | outlet] = TAG_OUTLET
    c.bc_tag = tag
    z_levels = (np.arange(rings, dtype=np.float64) + 0.5) * (L / rings)
    c.X = _ring_points(R, z_levels, per_ring)
    c.dS = 2.0 * math.pi * R * L / c.M
    c.u0 = np.zeros((3, N))
    c.p0 = np.where(inlet, p_in, 0.0)
    return c

