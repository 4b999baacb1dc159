"""Derived sets on the masked Cartesian grid (oracle; test infrastructure).

The paper reduces the box mesh to the vessel by removing unused elements
(domain reduction and cropping, Section 4 and Section 4.3) and applies
velocity Dirichlet data at inlets and no-slip on the remaining box walls,
with a zero pressure at outlets (Section 3.1, Fig. 1a).  On the Q1 grid
this becomes (reading stated in the design notes):

* kept cells E: cells with at least one corner inside the vessel (m = 1);
* pressure/velocity nodes P: the corners of kept cells;
* box-face tags: z = 0 inlet, z = max outlet, the four other faces wall,
  wall wins on edges and corners (unless a tag array is supplied);
* velocity Dirichlet D_u: nodes of P with m = 0, wall-tagged and
  inlet-tagged nodes of P; free velocity nodes F = P minus D_u;
* pressure Dirichlet: outlet-tagged nodes of P (Phi = 0 there);
* canonical order: ascending node id n = i + (nx+1)(j + (ny+1)k).
"""
from __future__ import annotations

import dataclasses

import numpy as np

TAG_NONE, TAG_WALL, TAG_INLET, TAG_OUTLET = 0, 1, 2, 3


def node_index_arrays(nx: int, ny: int, nz: int):
    """Integer (i, j, k) of every node id, x fastest."""
    n = np.arange((nx + 1) * (ny + 1) * (nz + 1), dtype=np.int64)
    i = n % (nx + 1)
    j = (n // (nx + 1)) % (ny + 1)
    k = n // ((nx + 1) * (ny + 1))
    return i, j, k


def default_tags(nx: int, ny: int, nz: int) -> np.ndarray:
    """Face tags: inlet at k = 0, outlet at k = nz, wall on the x and y faces
    (applied last, so wall wins on shared edges and corners)."""
    i, j, k = node_index_arrays(nx, ny, nz)
    tag = np.zeros(i.size, np.uint8)
    tag[k == 0] = TAG_INLET
    tag[k == nz] = TAG_OUTLET
    wall = (i == 0) | (i == nx) | (j == 0) | (j == ny)
    tag[wall] = TAG_WALL
    return tag


def cell_corner_ids(nx: int, ny: int, nz: int) -> np.ndarray:
    """(ncells, 8) node ids of each cell's corners; local corner a = ax + 2 ay + 4 az.
    Cells are numbered c = ci + nx (cj + ny ck)."""
    c = np.arange(nx * ny * nz, dtype=np.int64)
    ci = c % nx
    cj = (c // nx) % ny
    ck = c // (nx * ny)
    out = np.empty((c.size, 8), np.int64)
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        out[:, a] = (ci + ax) + (nx + 1) * ((cj + ay) + (ny + 1) * (ck + az))
    return out


@dataclasses.dataclass
class Sets:
    nx: int
    ny: int
    nz: int
    kept_cells: np.ndarray   # (ncells,) bool
    corners: np.ndarray      # (n_kept, 8) node ids of the kept cells
    in_P: np.ndarray         # (N,) bool
    in_F: np.ndarray         # (N,) bool, free velocity nodes
    in_Du: np.ndarray        # (N,) bool, velocity Dirichlet nodes
    p_dir: np.ndarray        # (N,) bool, pressure Dirichlet (outlet) nodes
    tag: np.ndarray          # (N,) uint8
    P: np.ndarray            # ascending node ids of P
    F: np.ndarray            # ascending node ids of F
    D: np.ndarray            # ascending node ids of D_u
    Pp: np.ndarray           # ascending node ids of P minus outlet (pressure unknowns)


def derive_sets(nx: int, ny: int, nz: int, mask: np.ndarray, tag: np.ndarray | None) -> Sets:
    mask = np.asarray(mask, np.uint8)
    N = (nx + 1) * (ny + 1) * (nz + 1)
    if mask.shape != (N,):
        raise ValueError("mask shape")
    if tag is None:
        tag = default_tags(nx, ny, nz)
    corners_all = cell_corner_ids(nx, ny, nz)
    kept = (mask[corners_all] == 1).any(axis=1)
    corners = corners_all[kept]
    in_P = np.zeros(N, bool)
    in_P[corners.ravel()] = True
    in_Du = in_P & ((mask == 0) | (tag == TAG_WALL) | (tag == TAG_INLET))
    in_F = in_P & ~in_Du
    p_dir = in_P & (tag == TAG_OUTLET)
    return Sets(nx=nx, ny=ny, nz=nz, kept_cells=kept, corners=corners, in_P=in_P, in_F=in_F,
                in_Du=in_Du, p_dir=p_dir, tag=np.asarray(tag, np.uint8),
                P=np.nonzero(in_P)[0], F=np.nonzero(in_F)[0], D=np.nonzero(in_Du)[0],
                Pp=np.nonzero(in_P & ~p_dir)[0])


def dirichlet_values(sets: Sets, mask: np.ndarray, inlet_ids: np.ndarray,
                     inlet_shape: np.ndarray, K: int, omega: float, t: float) -> np.ndarray:
    """(3, N) prescribed velocity g(t): zero on every D_u node except the inlet
    table nodes, where u_in(t) = W_0 + sum_k [Re W_k cos(k w t) - Im W_k sin(k w t)],
    i.e. the real part of sum_k W_k exp(i k w t) (inlet profiles, Sections 3.2 and 4)."""
    N = sets.in_P.size
    g = np.zeros((3, N))
    if inlet_ids.size == 0:
        return g
    val = inlet_shape[0].copy()                      # (n, 3)
    for k in range(1, K + 1):
        val += inlet_shape[2 * k - 1] * np.cos(k * omega * t)
        val -= inlet_shape[2 * k] * np.sin(k * omega * t)
    keep = sets.in_P[inlet_ids]                      # all of them on a uniform grid
    g[:, inlet_ids[keep]] = val[keep].T
    return g


def check_inlet_table(sets: Sets, mask: np.ndarray, inlet_ids: np.ndarray,
                      skip_non_mesh: bool = False) -> None:
    """Every listed node must be an in-vessel inlet node of P.  On a refined lattice
    (skip_non_mesh) listed points that are not nodes of P (interior points of unrefined
    cells, hanging nodes) carry no unknown and are skipped."""
    sel = sets.in_P[inlet_ids] if skip_non_mesh else np.ones(inlet_ids.size, bool)
    ids = inlet_ids[sel]
    ok = (sets.in_P[ids] & (sets.tag[ids] == TAG_INLET) & (mask[ids] == 1))
    if not ok.all():
        raise ValueError("inlet table lists a node that is not an in-vessel inlet node of P")
    if np.unique(inlet_ids).size != inlet_ids.size:
        raise ValueError("duplicate inlet node")
