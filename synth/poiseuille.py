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

from .cases import TAG_INLET, TAG_OUTLET, TAG_WALL, Case, _ring_points

R = 0.005
L = 0.05
HALF_WIDTH = 0.006
RHO = 1050.0
MU = 0.00345
DT = 2.5e-3


def poiseuille_e1(level: int = 0, p_in: float = 1.0, spacing: float = 1.5, nsteps: int = 3,
                  domain: str = "reduced", refine_band: float | None = None) -> Case:
    """The tube on grid `level` (0, 1, 2 = h 1, 0.5, 0.25 mm).

    With refine_band (metres), the base cells whose centre lies within refine_band of
    the wall radius R are split 2:1: every node array lives on the fine lattice of
    spacing h/2, and the Lagrangian points follow the fine spacing (the IB kernel uses
    the lattice spacing).

    * mask: nodes with x^2 + y^2 < R^2 (domain = "reduced"), or every node of the box
      (domain = "box": the whole box is fluid and the immersed wall separates the
      inside of the tube from the fluid around it, as in the paper's BoxMesh);
    * boundary tags: every box-face node is wall, except the masked nodes of the two
      end faces, which are pressure boundaries (natural velocity, fixed pressure);
    * Lagrangian points: rings at z = (k + 1/2) L / rings with `per_ring` points at
      equal angles, point spacing close to `spacing` * h both ways, dS = 2 pi R L / M;
    * initial state: at rest, pressure p_in on the inlet disk and 0 elsewhere.
    """
    f = 2 ** int(level)
    h = 1e-3 / f
    nxy, nz = 12 * f, 50 * f
    refine = None
    if refine_band is not None:
        ci = (np.arange(nxy) + 0.5) * h - HALF_WIDTH
        _, cy, cx = np.meshgrid(np.arange(nz), ci, ci, indexing="ij")
        refine = (np.abs(np.sqrt(cx * cx + cy * cy) - R) <= refine_band).astype(np.uint8).ravel()
    g = 2 if refine is not None else 1      # lattice steps per base cell
    hl = h / g                              # lattice spacing (the IB kernel's h)
    per_ring = int(round(2.0 * math.pi * R / (spacing * hl)))
    rings = int(round(L / (spacing * hl)))
    c = Case(
        name=f"poiseuille_e1_h{h:g}_p{p_in:g}", nx=nxy, ny=nxy, nz=nz, h=h,
        origin=np.array([-HALF_WIDTH, -HALF_WIDTH, 0.0]),
        node_mask=np.zeros(0, np.uint8), bc_tag=None, X=np.zeros((0, 3)), dS=0.0, U_B=None,
        rho=RHO, mu=MU, dt=DT, nsteps=nsteps, inlet_K=0, inlet_omega=0.0,
        inlet_ids=np.zeros(0, np.int64), inlet_shape=np.zeros((1, 0, 3)),
        u0=np.zeros((3, 0)), p0=np.zeros(0), refine_cell=refine)
    if refine is not None:
        c.name += f"_band{refine_band:g}"
    nxy, nz = g * nxy, g * nz               # lattice cells
    N = c.N
    k = np.arange(N)
    i = k % (nxy + 1)
    j = (k // (nxy + 1)) % (nxy + 1)
    kz = k // ((nxy + 1) * (nxy + 1))
    x = c.origin[0] + i * hl
    y = c.origin[1] + j * hl
    disk = (x * x + y * y < R * R)
    if domain == "reduced":
        mask = disk.astype(np.uint8)
    elif domain == "box":
        mask = np.ones(N, np.uint8)
        c.name += "_box"
    else:
        raise ValueError(domain)
    c.node_mask = mask
    tag = np.zeros(N, np.uint8)
    face = (i == 0) | (i == nxy) | (j == 0) | (j == nxy) | (kz == 0) | (kz == nz)
    tag[face] = TAG_WALL
    inlet = (kz == 0) & disk
    outlet = (kz == nz) & disk
    tag[inlet | outlet] = TAG_OUTLET
    c.bc_tag = tag
    z_levels = (np.arange(rings, dtype=np.float64) + 0.5) * (L / rings)
    c.X = _ring_points(R, z_levels, per_ring)
    c.dS = 2.0 * math.pi * R * L / c.M
    c.u0 = np.zeros((3, N))
    c.p0 = np.where(inlet, p_in, 0.0)
    return c



def tube_in_box(cells_d: int, length: float = 2.0, margin_cells: int = 4, nsteps: int = 8,
                mu: float = 0.01, rho: float = 1.0, dt: float = 0.01) -> tuple[Case, np.ndarray]:
    """A tube of radius 1/2 along z immersed in a box that is fluid everywhere (the
    paper's Poiseuille test meshes the whole box and lets the immersed wall separate
    the tube from the fluid around it, Section 3.1), `cells_d` cells per diameter and
    `margin_cells` cells between the tube and the side walls.  Parabolic inlet
    u_z = 1 - r^2/R^2 on the z = 0 disk, pressure outlet on the z = L disk, walls on
    the rest of the box; rings of wall points about 2h apart.  Initial state: the
    Poiseuille profile inside the tube (at rest outside) and the matching linear
    pressure 4 mu (L - z)/R^2 everywhere.  Returns the case and the in-tube node mask."""
    R = 0.5
    h = 2 * R / cells_d
    nxy = cells_d + 2 * margin_cells
    nz = int(round(length / h))
    width = nxy * h
    c = Case(name=f"tube_in_box_{cells_d}", nx=nxy, ny=nxy, nz=nz, h=h,
             origin=np.array([-width / 2, -width / 2, 0.0]),
             node_mask=np.zeros(0, np.uint8), bc_tag=None, X=np.zeros((0, 3)), dS=0.0, U_B=None,
             rho=rho, mu=mu, dt=dt, nsteps=nsteps, inlet_K=0, inlet_omega=0.0,
             inlet_ids=np.zeros(0, np.int64), inlet_shape=np.zeros((1, 0, 3)),
             u0=np.zeros((3, 0)), p0=np.zeros(0))
    xyz = c.node_coords()
    r2 = xyz[:, 0] ** 2 + xyz[:, 1] ** 2
    disk = r2 < R * R
    c.node_mask = np.ones(c.N, np.uint8)
    n = np.arange(c.N)
    i = n % (nxy + 1)
    j = (n // (nxy + 1)) % (nxy + 1)
    k = n // ((nxy + 1) * (nxy + 1))
    tag = np.zeros(c.N, np.uint8)
    tag[(i == 0) | (i == nxy) | (j == 0) | (j == nxy) | (k == 0) | (k == nz)] = TAG_WALL
    tag[(k == 0) & disk] = TAG_INLET
    tag[(k == nz) & disk] = TAG_OUTLET
    c.bc_tag = tag
    rings = int(length * cells_d / 2)
    per = int(round(2 * math.pi * R / (2.0 / cells_d)))
    c.X = _ring_points(R, (np.arange(rings, dtype=np.float64) + 0.5) * (length / rings), per)
    c.dS = 2 * math.pi * R * length / c.M
    ids = np.nonzero((k == 0) & disk)[0].astype(np.int64)
    shape = np.zeros((1, ids.size, 3))
    shape[0, :, 2] = 1.0 - r2[ids] / (R * R)
    c.inlet_ids, c.inlet_shape = ids, shape
    c.u0 = np.zeros((3, c.N))
    c.u0[2] = np.where(disk, 1.0 - r2 / (R * R), 0.0)
    c.p0 = 4.0 * mu / (R * R) * (length - xyz[:, 2])
    return c, disk
