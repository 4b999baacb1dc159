"""Seeded synthetic inputs for the IPCS + BCE-IB time step.

This module produces plain arrays only: a Cartesian grid description, a
node mask that reduces the box to the vessel, Lagrangian wall points with
their uniform surface element, an inlet velocity table and initial fields.
It contains none of the method's arithmetic (no finite-element forms, no
delta kernel, no solver) so that the oracle and the GPU library can both
consume the very same bytes without sharing any computation.

Geometries stand in for the paper's vessels (straight-tube Poiseuille
benchmark of Section 3.1; the patient geometries of Section 4 are not
available, so synthetic tubes are used).  Node ids follow
n = i + (nx+1) * (j + (ny+1) * k), x fastest.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TAG_NONE, TAG_WALL, TAG_INLET, TAG_OUTLET = 0, 1, 2, 3


@dataclasses.dataclass
class Case:
    """One flow problem: everything the library and the oracle take as input."""

    name: str
    nx: int
    ny: int
    nz: int
    h: float
    origin: np.ndarray          # (3,) float64, coordinates of node (0,0,0)
    node_mask: np.ndarray       # (N,) uint8, 1 = node inside the vessel
    bc_tag: np.ndarray | None   # (N,) uint8 or None for the face defaults
    X: np.ndarray               # (M,3) float64 Lagrangian wall points
    dS: float                   # uniform surface element of each point
    U_B: np.ndarray | None      # (M,3) float64 wall velocity, None = at rest
    rho: float
    mu: float
    dt: float
    nsteps: int
    inlet_K: int                # number of harmonics beyond the mean
    inlet_omega: float          # angular frequency of the first harmonic
    inlet_ids: np.ndarray       # (n,) int64 node ids carrying a prescribed inlet velocity
    inlet_shape: np.ndarray     # (2K+1, n, 3) float64: W_0, then Re W_k, Im W_k per harmonic
    u0: np.ndarray              # (3, N) float64 initial velocity on every node
    p0: np.ndarray              # (N,) float64 initial pressure on every node
    refine_cell: np.ndarray | None = None   # (nx*ny*nz,) uint8: base cells split 2:1

    @property
    def N(self) -> int:
        """Nodes of the grid the arrays live on (the fine lattice when refined)."""
        f = 2 if self.refine_cell is not None else 1
        return (f * self.nx + 1) * (f * self.ny + 1) * (f * self.nz + 1)

    @property
    def M(self) -> int:
        return int(self.X.shape[0])

    def node_coords(self) -> np.ndarray:
        """(N,3) physical coordinates of the array nodes, x fastest."""
        f = 2 if self.refine_cell is not None else 1
        i = np.arange(f * self.nx + 1, dtype=np.float64)
        j = np.arange(f * self.ny + 1, dtype=np.float64)
        k = np.arange(f * self.nz + 1, dtype=np.float64)
        K, J, I = np.meshgrid(k, j, i, indexing="ij")
        xyz = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1) * (self.h / f)
        return xyz + self.origin[None, :]


def _ring_points(radius: float, z_levels: np.ndarray, per_ring: int) -> np.ndarray:
    theta = 2.0 * math.pi * np.arange(per_ring, dtype=np.float64) / per_ring
    zz, tt = np.meshgrid(z_levels, theta, indexing="ij")
    return np.stack([radius * np.cos(tt).ravel(), radius * np.sin(tt).ravel(), zz.ravel()], axis=1)


def cylinder_case(
    name: str,
    cells_xy: int,
    cells_z: int,
    width: float,
    length: float,
    radius: float,
    rings: int,
    per_ring: int,
    rho: float,
    mu: float,
    dt: float,
    nsteps: int,
    u_max: float = 1.0,
    pulsatile_amp: float = 0.0,
    period: float = 1.0,
    ic: str = "rest",
) -> Case:
    """Straight tube of the given radius along z inside the box
    [-width/2, width/2]^2 x [0, length], resolved by a uniform grid.

    * mask: strict test x^2 + y^2 < R^2 (nodes exactly on the wall are outside);
    * Lagrangian points: `rings` rings at z = (k + 1/2) * length / rings, each with
      `per_ring` points at equal angles; uniform dS = 2 pi R L / M (the mean facet area
      of the ring triangulation);
    * inlet (z = 0): parabolic profile u_z = u_max (1 - r^2/R^2) times
      (1 + pulsatile_amp sin(2 pi t / period));
    * initial condition: at rest, or the exact Poiseuille profile with the matching
      linear pressure when ic == "poiseuille".
    """
    h = width / cells_xy
    if abs(h * cells_z - length) > 1e-12 * length:
        raise ValueError("box length must be a whole number of cells")
    nx = ny = cells_xy
    nz = cells_z
    origin = np.array([-width / 2, -width / 2, 0.0])
    case = Case(
        name=name, nx=nx, ny=ny, nz=nz, h=h, origin=origin,
        node_mask=np.zeros(0, np.uint8), bc_tag=None,
        X=np.zeros((0, 3)), dS=0.0, U_B=None,
        rho=rho, mu=mu, dt=dt, nsteps=nsteps,
        inlet_K=0, inlet_omega=0.0, inlet_ids=np.zeros(0, np.int64),
        inlet_shape=np.zeros((1, 0, 3)), u0=np.zeros((3, 0)), p0=np.zeros(0),
    )
    xyz = case.node_coords()
    r2 = xyz[:, 0] ** 2 + xyz[:, 1] ** 2
    mask = (r2 < radius * radius).astype(np.uint8)
    case.node_mask = mask

    z_levels = (np.arange(rings, dtype=np.float64) + 0.5) * (length / rings)
    case.X = _ring_points(radius, z_levels, per_ring)
    case.dS = 2.0 * math.pi * radius * length / case.M

    # Inlet table: every in-vessel node of the z = 0 face.
    on_inlet = (np.abs(xyz[:, 2] - 0.0) == 0.0) & (mask == 1)
    ids = np.nonzero(on_inlet)[0].astype(np.int64)
    prof = u_max * (1.0 - r2[ids] / (radius * radius))
    if pulsatile_amp != 0.0:
        K = 1
        shape = np.zeros((3, ids.size, 3))
        shape[0, :, 2] = prof
        # Re[(W_re + i W_im) e^{i w t}] = W_re cos(wt) - W_im sin(wt) = amp sin(wt) prof
        shape[2, :, 2] = -pulsatile_amp * prof
        case.inlet_omega = 2.0 * math.pi / period
    else:
        K = 0
        shape = np.zeros((1, ids.size, 3))
        shape[0, :, 2] = prof
        case.inlet_omega = 0.0
    case.inlet_K = K
    case.inlet_ids = ids
    case.inlet_shape = shape

    N = case.N
    case.u0 = np.zeros((3, N))
    case.p0 = np.zeros(N)
    if ic == "poiseuille":
        case.u0[2] = np.where(mask == 1, u_max * (1.0 - r2 / (radius * radius)), 0.0)
        grad = 4.0 * mu * u_max / (radius * radius)
        case.p0 = grad * (length - xyz[:, 2])
    elif ic != "rest":
        raise ValueError(ic)
    return case


def poiseuille_c1(ic: str = "rest") -> Case:
    """Poiseuille flow, cylinder R = 0.5, L = 4 in a 16x16x64 grid (box 1x1x4),
    rho = 1, mu = 0.01, parabolic inlet u_max = 1, dt = 0.01, 20 steps,
    32 rings x 25 points (200 points per unit length)."""
    return cylinder_case("poiseuille_16x16x64", 16, 64, 1.0, 4.0, 0.5, 32, 25,
                         rho=1.0, mu=0.01, dt=0.01, nsteps=20, ic=ic)


def pulsatile_c2(ic: str = "rest") -> Case:
    """Pulsatile flow, cylinder R = 0.5, L = 8 on a 64x64x512 grid, inlet
    u_max(t) = 1 + 0.5 sin(2 pi t), dt = 0.005, 200 steps; 256 rings of 100 points
    (point spacing close to 2h both ways, sqrt(dS)/h = 2, inside the paper's
    0.1..2.5 range; spacing h makes the Gram matrix of the four-point kernel
    numerically singular)."""
    return cylinder_case("pulsatile_64x64x512", 64, 512, 1.0, 8.0, 0.5, 256, 100,
                         rho=1.0, mu=0.01, dt=0.005, nsteps=200,
                         pulsatile_amp=0.5, period=1.0, ic=ic)


def small_cylinder(cells_xy: int = 8, cells_z: int = 16, length: float = 2.0,
                   rings: int = 8, per_ring: int = 12, pulsatile: bool = False,
                   ic: str = "rest", nsteps: int = 3, dt: float = 0.02) -> Case:
    """Reduced cylinder for fast tests (same geometry family as the two above)."""
    return cylinder_case(f"cyl_{cells_xy}x{cells_xy}x{cells_z}", cells_xy, cells_z, 1.0,
                         length, 0.5, rings, per_ring, rho=1.0, mu=0.01, dt=dt,
                         nsteps=nsteps, pulsatile_amp=0.5 if pulsatile else 0.0, ic=ic)


def closed_box(cells: int = 4, seed: int = 0) -> Case:
    """All nodes active, every box node tagged wall except nothing: a closed box with
    no outlet (exercises the pressure null space).  Random initial velocity inside."""
    rng = np.random.default_rng(seed)
    h = 1.0 / cells
    c = cylinder_case("closed_box", cells, cells, 1.0, 1.0, 10.0, 1, 4,
                      rho=1.0, mu=0.01, dt=0.05, nsteps=1)
    c.node_mask[:] = 1
    N = c.N
    xyz = c.node_coords()
    tag = np.zeros(N, np.uint8)
    eps = 1e-12
    on_face = ((np.abs(xyz[:, 0] + 0.5) < eps) | (np.abs(xyz[:, 0] - 0.5) < eps) |
               (np.abs(xyz[:, 1] + 0.5) < eps) | (np.abs(xyz[:, 1] - 0.5) < eps) |
               (np.abs(xyz[:, 2]) < eps) | (np.abs(xyz[:, 2] - 1.0) < eps))
    tag[on_face] = TAG_WALL
    c.bc_tag = tag
    c.X = np.array([[0.1, -0.05, 0.5], [-0.2, 0.1, 0.45]])
    c.dS = h * h
    c.inlet_K = 0
    c.inlet_omega = 0.0
    c.inlet_ids = np.zeros(0, np.int64)
    c.inlet_shape = np.zeros((1, 0, 3))
    u0 = rng.standard_normal((3, N))
    u0[:, on_face] = 0.0
    c.u0 = u0
    c.p0 = np.zeros(N)
    return c


def random_blob_case(cells: tuple[int, int, int] = (6, 5, 7), seed: int = 1,
                     n_points: int = 6) -> Case:
    """Irregular small problem: random node mask (about half the nodes), random
    Lagrangian points well inside the box, random wall velocity and a two-harmonic
    inlet on every z = 0 face node with m = 1 that is not on a side face.  Used for
    parity of the whole step on an irregular domain."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = cells
    h = 0.25
    origin = np.array([-0.3, 0.2, -0.1])
    c = Case(name=f"blob_{nx}x{ny}x{nz}_s{seed}", nx=nx, ny=ny, nz=nz, h=h, origin=origin,
             node_mask=np.zeros(0, np.uint8), bc_tag=None, X=np.zeros((0, 3)), dS=0.0,
             U_B=None, rho=1.3, mu=0.02, dt=0.03, nsteps=3, inlet_K=2, inlet_omega=2.0,
             inlet_ids=np.zeros(0, np.int64), inlet_shape=np.zeros((5, 0, 3)),
             u0=np.zeros((3, 0)), p0=np.zeros(0))
    N = c.N
    mask = (rng.random(N) < 0.55).astype(np.uint8)
    c.node_mask = mask
    ii = np.arange(N) % (nx + 1)
    jj = (np.arange(N) // (nx + 1)) % (ny + 1)
    kk = np.arange(N) // ((nx + 1) * (ny + 1))
    inlet = (kk == 0) & (ii > 0) & (ii < nx) & (jj > 0) & (jj < ny) & (mask == 1)
    ids = np.nonzero(inlet)[0].astype(np.int64)
    c.inlet_ids = ids
    c.inlet_shape = rng.standard_normal((5, ids.size, 3)) * 0.3
    lo = origin + 2.0 * h
    hi = origin + h * np.array([nx, ny, nz]) - 2.0 * h
    c.X = lo + (hi - lo) * rng.random((n_points, 3))
    c.dS = 0.8 * h * h
    c.U_B = 0.1 * rng.standard_normal((n_points, 3))
    u0 = rng.standard_normal((3, N)) * 0.2
    u0[:, mask == 0] = 0.0
    c.u0 = u0
    c.p0 = rng.standard_normal(N) * 0.1
    return c


def channel_case(cells_y: int = 8, cells_xz: tuple[int, int] = (2, 4), length: float = 0.5,
                 mu: float = 0.05, rho: float = 1.0, dt: float = 0.02, grad: float = 1.0,
                 ic: str = "rest", nsteps: int = 5) -> Case:
    """Plane channel between grid-aligned walls y = +-1/2 (wall-tagged), every node
    active, no Lagrangian points, natural conditions on the x faces and at z = 0,
    zero pressure at z = length, driven by the linear pressure p = grad (length - z).
    With ic == "steady" the velocity starts at the plane Poiseuille profile
    u_z = grad (1/4 - y^2) / (2 mu)."""
    h = 1.0 / cells_y
    nx, nz = cells_xz
    ny = cells_y
    if abs(nz * h - length) > 1e-12:
        raise ValueError("length must be cells_xz[1] * h")
    c = Case(name=f"channel_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, h=h,
             origin=np.array([0.0, -0.5, 0.0]), node_mask=np.zeros(0, np.uint8), bc_tag=None,
             X=np.zeros((0, 3)), dS=h * h, U_B=None, rho=rho, mu=mu, dt=dt, nsteps=nsteps,
             inlet_K=0, inlet_omega=0.0, inlet_ids=np.zeros(0, np.int64),
             inlet_shape=np.zeros((1, 0, 3)), u0=np.zeros((3, 0)), p0=np.zeros(0))
    N = c.N
    c.node_mask = np.ones(N, np.uint8)
    xyz = c.node_coords()
    j = np.rint((xyz[:, 1] + 0.5) / h).astype(np.int64)
    k = np.rint(xyz[:, 2] / h).astype(np.int64)
    tag = np.zeros(N, np.uint8)
    tag[k == nz] = TAG_OUTLET
    tag[(j == 0) | (j == ny)] = TAG_WALL
    c.bc_tag = tag
    c.u0 = np.zeros((3, N))
    if ic == "steady":
        c.u0[2] = grad * (0.25 - xyz[:, 1] ** 2) / (2.0 * mu)
    elif ic != "rest":
        raise ValueError(ic)
    c.p0 = grad * (length - xyz[:, 2])
    return c


def shear_advection_case(cells_x: int = 10, U: float = 0.8, force: float = 0.6,
                         mu: float = 0.03, rho: float = 1.1, dt: float = 0.05) -> Case:
    """Uniform stream U along x carrying a transverse profile w(x) in u_z: every node
    active on [0,1] x [0,h] x [0,h], both x faces carry the prescribed velocity
    (U, 0, 0) (inlet-tagged, listed in the inlet table), the y and z faces are
    natural, no outlet, no Lagrangian points, pressure p = -force z driving u_z,
    initial u = (U, 0, sin(pi x))."""
    h = 1.0 / cells_x
    nx, ny, nz = cells_x, 1, 1
    c = Case(name=f"shear_{nx}", nx=nx, ny=ny, nz=nz, h=h, origin=np.zeros(3),
             node_mask=np.zeros(0, np.uint8), bc_tag=None, X=np.zeros((0, 3)), dS=h * h,
             U_B=None, rho=rho, mu=mu, dt=dt, nsteps=3, inlet_K=0, inlet_omega=0.0,
             inlet_ids=np.zeros(0, np.int64), inlet_shape=np.zeros((1, 0, 3)),
             u0=np.zeros((3, 0)), p0=np.zeros(0))
    N = c.N
    c.node_mask = np.ones(N, np.uint8)
    xyz = c.node_coords()
    i = np.rint(xyz[:, 0] / h).astype(np.int64)
    tag = np.zeros(N, np.uint8)
    xface = (i == 0) | (i == nx)
    tag[xface] = TAG_INLET
    c.bc_tag = tag
    ids = np.nonzero(xface)[0].astype(np.int64)
    c.inlet_ids = ids
    shape = np.zeros((1, ids.size, 3))
    shape[0, :, 0] = U
    c.inlet_shape = shape
    c.u0 = np.zeros((3, N))
    c.u0[0] = U
    c.u0[2] = np.sin(math.pi * xyz[:, 0])
    c.u0[2][xface] = 0.0
    c.p0 = -force * xyz[:, 2]
    return c


def refined_cylinder(cells_xy: int = 8, cells_z: int = 8, length: float = 1.0, radius: float = 0.5,
                     band: float = 0.2, width: float = 1.25, rho: float = 1.0, mu: float = 0.01,
                     dt: float = 0.02, nsteps: int = 3, mask_all: bool = False) -> Case:
    """Cylinder along z on a base grid whose cells within `band` of the wall are split
    2:1 (cell centre distance to the wall).  Arrays live on the fine lattice (spacing
    h/2): mask x^2 + y^2 < R^2, Lagrangian rings at spacing close to 2 h_f (= h) placed
    at least 2 h_f inside the box, parabolic inlet on the lattice z = 0 face."""
    h = width / cells_xy
    if abs(h * cells_z - length) > 1e-12 * length:
        raise ValueError("length must be a whole number of cells")
    nx = ny = cells_xy
    nz = cells_z
    origin = np.array([-width / 2, -width / 2, 0.0])
    ci = (np.arange(nx) + 0.5) * h + origin[0]
    cz_, cy_, cx_ = np.meshgrid(np.arange(nz), ci, ci, indexing="ij")
    rc = np.sqrt(cx_ ** 2 + cy_ ** 2)
    refine = (np.abs(rc - radius) <= band).astype(np.uint8).ravel()
    c = Case(name=f"refined_cyl_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, h=h, origin=origin,
             node_mask=np.zeros(0, np.uint8), bc_tag=None, X=np.zeros((0, 3)), dS=h * h, U_B=None,
             rho=rho, mu=mu, dt=dt, nsteps=nsteps, inlet_K=0, inlet_omega=0.0,
             inlet_ids=np.zeros(0, np.int64), inlet_shape=np.zeros((1, 0, 3)),
             u0=np.zeros((3, 0)), p0=np.zeros(0), refine_cell=refine)
    xyz = c.node_coords()
    r2 = xyz[:, 0] ** 2 + xyz[:, 1] ** 2
    c.node_mask = np.ones(c.N, np.uint8) if mask_all else (r2 < radius * radius).astype(np.uint8)
    hf = h / 2
    spacing = 2 * hf
    nr = max(1, int(round((length - 4 * hf) / spacing)))
    zl = 2 * hf + (np.arange(nr) + 0.5) * ((length - 4 * hf) / nr)
    c.X = _ring_points(radius, zl, max(6, int(round(2 * math.pi * radius / spacing))))
    c.dS = spacing * spacing
    lo, hi = origin[0], origin[0] + width
    side = (xyz[:, 0] == lo) | (xyz[:, 0] == hi) | (xyz[:, 1] == lo) | (xyz[:, 1] == hi)
    on_inlet = (xyz[:, 2] == 0.0) & (c.node_mask == 1) & ~side
    ids = np.nonzero(on_inlet)[0].astype(np.int64)
    shape = np.zeros((1, ids.size, 3))
    shape[0, :, 2] = np.maximum(0.0, 1.0 - r2[ids] / (radius * radius))
    c.inlet_ids, c.inlet_shape = ids, shape
    c.u0 = np.zeros((3, c.N))
    c.p0 = np.zeros(c.N)
    return c
