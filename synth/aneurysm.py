"""Seeded synthetic aneurysm on a 2:1 locally refined grid (inputs only).

A tube of radius r follows the sinusoidal centreline c(s) = (A sin(2 pi s / T),
0, s) through a box of length L; a sphere of radius Rb bulges out of it at a
seeded height on a seeded side (+y or -y).  Base cells whose centre lies within
`band` of the vessel wall (|signed distance| <= band) are split 2:1; every node
array lives on the fine lattice (spacing h/2).  The Lagrangian points sample
the union surface (rings on the tube, a Fibonacci set on the sphere) at spacing
close to the base spacing h = 2 h_f, thinned to a Poisson-disk set (no two points
closer than 0.7 h); the inlet is a parabolic profile on the
lattice z = 0 face.  This stands in for the paper's aneurysmal vessels
(Section 4), whose meshes are not available.  Signed distances only decide the
mask and the refinement flags, which are inputs: the rule does not have to be
exact, only deterministic.
"""
from __future__ import annotations

import math

import numpy as np

from .cases import Case


def _tube_distance(x, y, z, amp, k, iters=6):
    """Distance to the centreline (amp sin(k s), 0, s) by Newton steps on s from s = z."""
    s = z.copy()
    for _ in range(iters):
        cx = amp * np.sin(k * s)
        dcx = amp * k * np.cos(k * s)
        ddcx = -amp * k * k * np.sin(k * s)
        g = -(x - cx) * dcx - (z - s)              # half derivative of |p - c(s)|^2
        gp = dcx * dcx - (x - cx) * ddcx + 1.0
        s = s - g / gp
    return np.sqrt((x - amp * np.sin(k * s)) ** 2 + y * y + (z - s) ** 2)


def _poisson_disk(X, rmin):
    """Greedy Poisson-disk thinning in input order: a point is kept unless a kept point
    lies closer than rmin (removes the near-duplicates where the two surfaces meet)."""
    from scipy.spatial import cKDTree

    pairs = cKDTree(X).query_pairs(rmin, output_type="ndarray")
    if pairs.size == 0:
        return X
    nbrs = [[] for _ in range(len(X))]
    for a, b in pairs:
        nbrs[max(a, b)].append(min(a, b))
    keep = np.ones(len(X), bool)
    for i in range(len(X)):
        if any(keep[j] for j in nbrs[i]):
            keep[i] = False
    return X[keep]


def aneurysm_case(base=(128, 128, 320), length: float = 20.0, width: float = 8.0, radius: float = 1.0,
                  amp: float = 1.0, period: float = 10.0, bulge: float = 2.5, band: float = 0.5,
                  nsteps: int = 20, seed: int = 20070208 + 2, rho: float = 1.0, mu: float = 0.01,
                  dt: float | None = None, name: str | None = None) -> Case:
    nx, ny, nz = base
    h = length / nz
    if abs(h * nx - width) > 1e-9 * width or abs(h * ny - width) > 1e-9 * width:
        raise ValueError("cells must be cubes: width / nx = length / nz")
    origin = np.array([-width / 2, -width / 2, 0.0])
    rng = np.random.default_rng(seed)
    zb = float(rng.uniform(0.35, 0.65)) * length
    side = 1.0 if rng.integers(2) else -1.0
    k = 2.0 * math.pi / period
    off = 1.2 * radius
    cb = np.array([amp * math.sin(k * zb), side * off, zb])

    def sdf(x, y, z):
        tube = _tube_distance(x, y, z, amp, k) - radius
        sph = np.sqrt((x - cb[0]) ** 2 + (y - cb[1]) ** 2 + (z - cb[2]) ** 2) - bulge
        return np.minimum(tube, sph)

    # refinement flags from base-cell centres
    ci = origin[0] + (np.arange(nx) + 0.5) * h
    cj = origin[1] + (np.arange(ny) + 0.5) * h
    refine = np.zeros((nz, ny, nx), np.uint8)
    Y, X = np.meshgrid(cj, ci, indexing="ij")
    for kk in range(nz):
        Z = np.full_like(X, (kk + 0.5) * h)
        refine[kk] = (np.abs(sdf(X, Y, Z)) <= band).astype(np.uint8)

    c = Case(name=name or f"aneurysm_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, h=h, origin=origin,
             node_mask=np.zeros(0, np.uint8), bc_tag=None, X=np.zeros((0, 3)), dS=h * h, U_B=None,
             rho=rho, mu=mu, dt=dt if dt is not None else 0.25 * h, nsteps=nsteps, inlet_K=0,
             inlet_omega=0.0, inlet_ids=np.zeros(0, np.int64), inlet_shape=np.zeros((1, 0, 3)),
             u0=np.zeros((3, 0)), p0=np.zeros(0), refine_cell=refine.ravel())
    # mask on the fine lattice, one z-plane at a time
    hf = h / 2
    lx, ly, lz = 2 * nx, 2 * ny, 2 * nz
    xi = origin[0] + np.arange(lx + 1) * hf
    yj = origin[1] + np.arange(ly + 1) * hf
    YL, XL = np.meshgrid(yj, xi, indexing="ij")
    mask = np.empty((lz + 1, ly + 1, lx + 1), np.uint8)
    for kk in range(lz + 1):
        mask[kk] = (sdf(XL, YL, np.full_like(XL, kk * hf)) < 0.0).astype(np.uint8)
    c.node_mask = mask.ravel()

    # Lagrangian points: tube rings (outside the sphere) and sphere points (outside the tube)
    spacing = 2.0 * hf
    nring = max(6, int(round(2 * math.pi * radius / spacing)))
    ss = np.arange(0.0, length, spacing / math.sqrt(1.0 + (amp * k) ** 2) * 0.999)
    pts = []
    th = 2 * math.pi * np.arange(nring) / nring
    for s in ss:
        cpt = np.array([amp * math.sin(k * s), 0.0, s])
        t = np.array([amp * k * math.cos(k * s), 0.0, 1.0])
        t /= np.linalg.norm(t)
        e1 = np.cross(t, [0.0, 1.0, 0.0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(t, e1)
        pts.append(cpt[None, :] + radius * (np.cos(th)[:, None] * e1[None, :] + np.sin(th)[:, None] * e2[None, :]))
    tube_pts = np.concatenate(pts, 0)
    nsp = max(12, int(round(4 * math.pi * bulge * bulge / (spacing * spacing))))
    q = np.arange(nsp) + 0.5
    phi = np.arccos(1 - 2 * q / nsp)
    tt = math.pi * (1 + 5 ** 0.5) * q
    sph_pts = cb[None, :] + bulge * np.stack([np.cos(tt) * np.sin(phi), np.sin(tt) * np.sin(phi), np.cos(phi)], 1)
    d_sph = np.linalg.norm(tube_pts - cb[None, :], axis=1) - bulge
    d_tube = _tube_distance(sph_pts[:, 0], sph_pts[:, 1], sph_pts[:, 2], amp, k) - radius
    X = np.concatenate([tube_pts[d_sph > 0.25 * hf], sph_pts[d_tube > 0.25 * hf]], 0)
    X = _poisson_disk(X, 0.7 * spacing)
    lo = origin + 3 * hf
    hi = origin + np.array([nx, ny, nz]) * h - 3 * hf
    X = X[np.all((X >= lo) & (X <= hi), axis=1)]
    # keep the points whose kernel support (4 lattice nodes per axis from
    # floor((X - origin) / h_f) - 1) only touches refined base cells: the flags
    # come from cell centres, so the few points near a crease of the band are
    # dropped rather than widening it
    i0 = np.floor((X - origin[None, :]) / hf).astype(np.int64) - 1
    lo_c = (i0 - 1) // 2
    hi_c = (i0 + 3) // 2
    dims = np.array([nx, ny, nz])
    ok = np.ones(len(X), bool)
    for a in range(3):
        for b in range(3):
            for d in range(3):
                cc = np.minimum(lo_c + np.array([a, b, d])[None, :], hi_c)
                cc = np.clip(cc, 0, dims[None, :] - 1)
                ok &= refine[cc[:, 2], cc[:, 1], cc[:, 0]] == 1
    c.X = X[ok]
    c.dS = spacing * spacing
    # inlet: parabolic profile around the centreline on the lattice z = 0 face
    ids = np.nonzero(mask[0].ravel() == 1)[0].astype(np.int64)
    px, py = XL.ravel()[ids], YL.ravel()[ids]
    shape = np.zeros((1, ids.size, 3))
    shape[0, :, 2] = np.maximum(0.0, 1.0 - (px * px + py * py) / (radius * radius))
    c.inlet_ids, c.inlet_shape = ids, shape
    c.u0 = np.zeros((3, c.N))
    c.p0 = np.zeros(c.N)
    return c
