"""Seeded request stream for the serving benchmark (inputs only).

Each request is a complete flow problem: a synthetic vessel (straight cylinder,
aneurysm = tube plus a spherical bulge, or a Y-branch = parent tube splitting
into two daughters of radius 2^{-1/3} r), a grid from 32^3 to 128x128x256, a
parabolic inlet of peak velocity 1 on the parent tube at z = 0, zero pressure at
z = max, 50 steps with dt = h/4.  Geometry is described by signed distances of
primitives (capsules and spheres); the node mask is "inside the union" and the
Lagrangian points sample the union surface at spacing close to 2h.  These stand
in for the paper's patient vessels (Section 4), whose meshes are not available.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .cases import Case

GRIDS = [(32, 32, 32), (48, 48, 64), (64, 64, 128), (96, 96, 192), (128, 128, 256)]
KINDS = ["cylinder", "aneurysm", "branch"]
WIDTH = {"cylinder": 2.5, "aneurysm": 5.5, "branch": 6.0}   # box width in units of r


@dataclasses.dataclass
class Request:
    index: int
    arrival: float      # seconds after the start of the stream
    kind: str
    radius: float
    case: Case


def _capsule_sdf(p, a, b, r):
    ab = b - a
    t = np.clip(((p - a) @ ab) / (ab @ ab), 0.0, 1.0)
    q = a + t[:, None] * ab
    return np.linalg.norm(p - q, axis=1) - r


def _sphere_sdf(p, c, r):
    return np.linalg.norm(p - c, axis=1) - r


def _tube_surface(a, b, r, spacing):
    """Rings on the side of the segment a-b (radius r), spacing close to `spacing`."""
    ab = b - a
    L = np.linalg.norm(ab)
    axis = ab / L
    helper = np.array([1.0, 0.0, 0.0]) if abs(axis[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(axis, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(axis, e1)
    nr = max(1, int(round(L / spacing)))
    nt = max(6, int(round(2 * math.pi * r / spacing)))
    s = (np.arange(nr) + 0.5) / nr * L
    th = 2 * math.pi * np.arange(nt) / nt
    S, T = np.meshgrid(s, th, indexing="ij")
    pts = (a[None, :] + S.ravel()[:, None] * axis[None, :]
           + r * (np.cos(T).ravel()[:, None] * e1[None, :] + np.sin(T).ravel()[:, None] * e2[None, :]))
    return pts


def _sphere_surface(c, r, spacing):
    """Fibonacci points on a sphere with spacing close to `spacing`."""
    n = max(12, int(round(4 * math.pi * r * r / (spacing * spacing))))
    k = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * k / n)
    th = math.pi * (1 + 5 ** 0.5) * k
    return c[None, :] + r * np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)


def vessel_case(kind: str, r: float, grid: tuple[int, int, int], nsteps: int = 50,
                seed: int = 0, name: str | None = None) -> Case:
    nx, ny, nz = grid
    W = WIDTH[kind] * r
    h = W / nx
    L = nz * h
    origin = np.array([-W / 2, -W / 2, 0.0])
    spacing = 2.0 * h
    # primitives: list of (sdf, surface points)
    prims = []
    far = 2.0 * h   # extend the tubes past the box so that the faces cut them cleanly
    if kind == "cylinder":
        a, b = np.array([0, 0, -far]), np.array([0, 0, L + far])
        prims.append((lambda p, a=a, b=b: _capsule_sdf(p, a, b, r), _tube_surface(a, b, r, spacing)))
    elif kind == "aneurysm":
        a, b = np.array([0, 0, -far]), np.array([0, 0, L + far])
        c = np.array([0.5 * r, 0.0, 0.5 * L])
        prims.append((lambda p, a=a, b=b: _capsule_sdf(p, a, b, r), _tube_surface(a, b, r, spacing)))
        prims.append((lambda p, c=c: _sphere_sdf(p, c, 2.0 * r), _sphere_surface(c, 2.0 * r, spacing)))
    elif kind == "branch":
        rng = np.random.default_rng(seed)
        theta = math.radians(rng.uniform(10.0, 20.0))
        zs = 0.6 * L
        rd = r * 2.0 ** (-1.0 / 3.0)
        a, s = np.array([0, 0, -far]), np.array([0, 0, zs])
        prims.append((lambda p, a=a, s=s: _capsule_sdf(p, a, s, r), _tube_surface(a, s, r, spacing)))
        for sign in (-1.0, 1.0):
            top = np.array([sign * math.tan(theta) * (L + far - zs), 0.0, L + far])
            prims.append((lambda p, s=s, top=top: _capsule_sdf(p, s, top, rd), _tube_surface(s, top, rd, spacing)))
    else:
        raise ValueError(kind)

    c = Case(name=name or f"{kind}_r{r:.2f}_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, h=h, origin=origin,
             node_mask=np.zeros(0, np.uint8), bc_tag=None, X=np.zeros((0, 3)), dS=spacing * spacing,
             U_B=None, rho=1.0, mu=0.01 * r, dt=0.25 * h, nsteps=nsteps, inlet_K=0,
             inlet_omega=0.0, inlet_ids=np.zeros(0, np.int64), inlet_shape=np.zeros((1, 0, 3)),
             u0=np.zeros((3, 0)), p0=np.zeros(0))
    xyz = c.node_coords()
    sdf = np.min(np.stack([f(xyz) for f, _ in prims]), axis=0)
    mask = (sdf < 0.0).astype(np.uint8)
    c.node_mask = mask
    # union surface: points of each primitive that lie outside every other primitive,
    # inside the box with a margin of h (so that their support reaches free nodes)
    pts = []
    for i, (_, surf) in enumerate(prims):
        keep = np.ones(len(surf), bool)
        for j, (f, _) in enumerate(prims):
            if j != i:
                keep &= f(surf) > 0.25 * h
        lo, hi = origin + h, origin + np.array([nx, ny, nz]) * h - h
        keep &= np.all((surf >= lo) & (surf <= hi), axis=1)
        pts.append(surf[keep])
    c.X = np.concatenate(pts, axis=0)
    # inlet: parabolic profile on the parent tube at z = 0
    on_inlet = (xyz[:, 2] == 0.0) & (mask == 1)
    ids = np.nonzero(on_inlet)[0].astype(np.int64)
    rr = xyz[ids, 0] ** 2 + xyz[ids, 1] ** 2
    shape = np.zeros((1, ids.size, 3))
    shape[0, :, 2] = np.maximum(0.0, 1.0 - rr / (r * r))
    c.inlet_ids = ids
    c.inlet_shape = shape
    c.u0 = np.zeros((3, c.N))
    c.p0 = np.zeros(c.N)
    return c


def request_stream(n: int = 64, rate: float = 4.0, nsteps: int = 50, seed: int = 20070208 + 5,
                   grids=GRIDS, build: bool = True) -> list[Request]:
    """n requests with exponential inter-arrival times of mean 1/rate seconds."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        kind = KINDS[int(rng.integers(len(KINDS)))]
        r = float(rng.uniform(0.4, 2.5))
        grid = grids[int(rng.integers(len(grids)))]
        sub = int(rng.integers(1 << 30))
        case = vessel_case(kind, r, grid, nsteps=nsteps, seed=sub) if build else None
        out.append(Request(i, t, kind, r, case))
        t += float(rng.exponential(1.0 / rate))
    return out
