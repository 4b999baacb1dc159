"""Seeded synthetic aorta-like vessel on a uniform grid (inputs only).

An arch tube of radius R follows the cubic Bezier curve with control points
(4,5,0), (4,5,28), (12,5,28), (12,5,0) inside the box [0,16] x [0,10] x [0,24];
it enters and leaves through two disks on the z = 0 face (per-node inlet and
outlet tags on the same face).  Three straight branch tubes start on the arch
centreline at curve parameters near 0.38, 0.5 and 0.62, lean away from the
vertical by a seeded polar angle (0 to 25 degrees) and azimuth, have seeded
radii in [0.4, 0.6] and leave through outlet disks on the z = 24 face; draws
whose branches come closer than their radii plus a margin are rejected.  The
inlet carries a Womersley-type pulsatile profile of period 1 with two harmonics
(mean parabola plus the oscillatory Bessel shapes).  The Lagrangian points
sample the union surface (rings on every tube, spacing 1.5 h) thinned to a
Poisson-disk set.  This stands in for the paper's aortas (Section 4), whose
meshes and inflow waveforms are not available.  Signed distances only decide the
mask, the tags and the points, which are inputs: the rule does not have to be
exact, only deterministic.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special

from .aneurysm import _poisson_disk
from .cases import TAG_INLET, TAG_OUTLET, TAG_WALL, Case

BOX = (16.0, 10.0, 24.0)
CTRL = np.array([[4.0, 5.0, 0.0], [4.0, 5.0, 28.0], [12.0, 5.0, 28.0], [12.0, 5.0, 0.0]])


def bezier(t):
    t = np.asarray(t, np.float64)[..., None]
    return ((1 - t) ** 3 * CTRL[0] + 3 * (1 - t) ** 2 * t * CTRL[1] + 3 * (1 - t) * t * t * CTRL[2]
            + t ** 3 * CTRL[3])


def bezier_tangent(t):
    t = np.asarray(t, np.float64)[..., None]
    return 3 * ((1 - t) ** 2 * (CTRL[1] - CTRL[0]) + 2 * (1 - t) * t * (CTRL[2] - CTRL[1])
                + t * t * (CTRL[3] - CTRL[2]))


def _segment_distance(P, a, b):
    """Distance of the points P (..., 3) to the segment [a, b]."""
    ab = b - a
    w = P - a
    s = np.clip((w @ ab) / float(ab @ ab), 0.0, 1.0)
    return np.linalg.norm(w - s[..., None] * ab, axis=-1)


def _stamp(dist, h, a, b, radius):
    """dist = min(dist, |p - [a, b]| - radius) over the lattice nodes near the segment."""
    lz, ly, lx = (d - 1 for d in dist.shape)
    reach = radius + 2.0 * h
    lo = np.floor((np.minimum(a, b) - reach) / h).astype(int)
    hi = np.ceil((np.maximum(a, b) + reach) / h).astype(int)
    lo = np.maximum(lo, 0)
    hi = np.minimum(hi, [lx, ly, lz])
    if np.any(hi < lo):
        return
    i = np.arange(lo[0], hi[0] + 1) * h
    j = np.arange(lo[1], hi[1] + 1) * h
    k = np.arange(lo[2], hi[2] + 1) * h
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    P = np.stack([I, J, K], axis=-1)
    d = (_segment_distance(P, a, b) - radius).astype(np.float32)
    view = dist[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
    np.minimum(view, d, out=view)


def _rings(center, tangent, radius, spacing, ref):
    """Points at spacing ~spacing on the circle of `radius` around `center` normal to
    `tangent`; `ref` fixes the angular origin."""
    t = tangent / np.linalg.norm(tangent)
    e1 = np.cross(ref, t)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(t, e1)
    n = max(6, int(round(2 * math.pi * radius / spacing)))
    th = 2 * math.pi * np.arange(n) / n
    return center[None, :] + radius * (np.cos(th)[:, None] * e1[None, :] + np.sin(th)[:, None] * e2[None, :])


def womersley_shapes(r, R, omega, rho, mu, coefs):
    """Profile shapes C_k W_k(r) for k = 0..K: W_0 = 1 - r^2/R^2 and, for k >= 1,
    W_k = 1 - J0(i^{3/2} a_k r / R) / J0(i^{3/2} a_k) with a_k = R sqrt(k omega rho / mu)."""
    out = [coefs[0] * np.maximum(0.0, 1.0 - (r / R) ** 2)]
    z = (1j) ** 1.5
    for k in range(1, len(coefs)):
        a = R * math.sqrt(k * omega * rho / mu)
        w = 1.0 - scipy.special.jv(0, z * a * r / R) / scipy.special.jv(0, z * a)
        out.append(coefs[k] * w)
    return out


def _draw_branches(rng, h):
    """Three branch axes (root, unit direction, radius, exit point on z = 24)."""
    t_nom = (0.38, 0.5, 0.62)
    for _ in range(1000):
        br = []
        for tn in t_nom:
            t = tn + rng.uniform(-0.03, 0.03)
            theta = math.radians(rng.uniform(0.0, 25.0))
            phi = rng.uniform(0.0, 2 * math.pi)
            r = rng.uniform(0.4, 0.6)
            root = bezier(t)
            d = np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])
            top = root + d * (BOX[2] - root[2]) / d[2]
            br.append((root, d, r, top))
        ok = all(r + 0.5 <= top[0] <= BOX[0] - r - 0.5 and r + 0.5 <= top[1] <= BOX[1] - r - 0.5
                 for _, _, r, top in br)
        # no two branches closer than their radii plus a margin above the arch wall
        for a in range(3):
            for b in range(a + 1, 3):
                ra, da, rad_a, ta = br[a]
                rb, db, rad_b, tb = br[b]
                s = np.linspace(0.0, 1.0, 64)
                pa = ra + (ta - ra) * s[:, None]
                pb = rb + (tb - rb) * s[:, None]
                above = (pa[:, 2] > ra[2] + 1.5) & (pb[:, 2] > rb[2] + 1.5)
                if np.any(above):
                    dd = np.linalg.norm(pa[above][:, None, :] - pb[above][None, :, :], axis=-1).min()
                    ok &= dd > rad_a + rad_b + 4 * h
        if ok:
            return br
    raise RuntimeError("could not place the branches")


def aorta_case(scale: int = 1, nsteps: int = 20, seed: int = 20070208 + 3, radius: float = 1.2,
               rho: float = 1.0, mu: float = 0.01, dt: float = 0.002, period: float = 1.0,
               coefs=(1.0, 0.5, 0.25j), spacing: float = 1.5, name: str | None = None) -> Case:
    """Aorta-like arch with three branches on the 256x160x384 grid (h = 1/16) divided by
    `scale` per axis (scale 4: 64x40x96, h = 1/4).  Lagrangian points lie `spacing` h
    apart: at 1 h the points on the thin branches (radius 0.4, a few cells across)
    outnumber the free nodes their kernels reach and G = I_F I_F^T is numerically
    singular, so the default is 1.5 h."""
    nx, ny, nz = 256 // scale, 160 // scale, 384 // scale
    h = BOX[0] / nx
    rng = np.random.default_rng(seed)
    branches = _draw_branches(rng, h)

    # signed distance to the union of the tubes, stamped segment by segment
    dist = np.full((nz + 1, ny + 1, nx + 1), np.inf, np.float32)
    ts = np.linspace(0.0, 1.0, 257)
    B = bezier(ts)
    # extend both legs below z = 0 so that the tube crosses the face squarely
    legs = [(B[0] - np.array([0, 0, 2.0]), B[0]), (B[-1], B[-1] - np.array([0, 0, 2.0]))]
    for a, b in list(zip(B[:-1], B[1:])) + legs:
        _stamp(dist, h, a, b, radius)
    for root, d, r, top in branches:
        _stamp(dist, h, root, top + 2.0 * d, r)
    mask = (dist < 0.0).astype(np.uint8)

    c = Case(name=name or f"aorta_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, h=h, origin=np.zeros(3),
             node_mask=mask.ravel(), bc_tag=None, X=np.zeros((0, 3)), dS=h * h, U_B=None, rho=rho,
             mu=mu, dt=dt, nsteps=nsteps, inlet_K=len(coefs) - 1, inlet_omega=2 * math.pi / period,
             inlet_ids=np.zeros(0, np.int64), inlet_shape=np.zeros((len(coefs) * 2 - 1, 0, 3)),
             u0=np.zeros((3, 0)), p0=np.zeros(0))

    # boundary tags: walls everywhere on the box, then the inlet and outlet disks
    ii = np.arange(nx + 1)
    jj = np.arange(ny + 1)
    tag = np.zeros((nz + 1, ny + 1, nx + 1), np.uint8)
    tag[0] = tag[-1] = TAG_WALL
    tag[:, 0, :] = tag[:, -1, :] = TAG_WALL
    tag[:, :, 0] = tag[:, :, -1] = TAG_WALL
    JJ, II = np.meshgrid(jj * h, ii * h, indexing="ij")
    side = (JJ == 0) | (JJ == BOX[1]) | (II == 0) | (II == BOX[0])
    rin = np.hypot(II - CTRL[0, 0], JJ - CTRL[0, 1])
    rout = np.hypot(II - CTRL[3, 0], JJ - CTRL[3, 1])
    tag[0][(rin < radius + 2 * h) & ~side] = TAG_INLET
    tag[0][(rout < radius + 2 * h) & ~side] = TAG_OUTLET
    for _, _, r, top in branches:
        rt = np.hypot(II - top[0], JJ - top[1])
        tag[-1][(rt < r + 2 * h) & ~side] = TAG_OUTLET
    c.bc_tag = tag.ravel()

    # inlet: Womersley-type shapes on the in-vessel nodes of the inlet disk
    face = mask[0].ravel() == 1
    inl = face & (tag[0].ravel() == TAG_INLET)
    ids = np.nonzero(inl)[0].astype(np.int64)
    r = rin.ravel()[ids]
    shapes = womersley_shapes(r, radius, c.inlet_omega, rho, mu, coefs)
    table = np.zeros((2 * len(coefs) - 1, ids.size, 3))
    table[0, :, 2] = np.real(shapes[0])
    for k in range(1, len(coefs)):
        table[2 * k - 1, :, 2] = np.real(shapes[k])
        table[2 * k, :, 2] = np.imag(shapes[k])
    c.inlet_ids, c.inlet_shape = ids, table

    # Lagrangian points: arch rings outside the branches, branch rings outside the arch
    # and the other branches, thinned to a Poisson-disk set
    seg = np.linalg.norm(np.diff(B, axis=0), axis=1)
    s_cum = np.concatenate([[0.0], np.cumsum(seg)])
    y_ref = np.array([0.0, 1.0, 0.0])
    pts = []
    ds = spacing * h
    for s in np.arange(0.5 * ds, s_cum[-1], ds):
        t = np.interp(s, s_cum, ts)
        pts.append(("arch", _rings(bezier(t), bezier_tangent(t), radius, ds, y_ref)))
    for b, (root, d, r, top) in enumerate(branches):
        ref = y_ref if abs(d[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
        length = float(np.linalg.norm(top - root))
        for s in np.arange(0.5 * ds, length, ds):
            pts.append((b, _rings(root + s * d, d, r, ds, ref)))

    def d_arch(P):
        return np.min(np.stack([_segment_distance(P, a, bb) for a, bb in zip(B[:-1], B[1:])]), axis=0) - radius

    def d_branch(P, b):
        root, d, r, top = branches[b]
        return _segment_distance(P, root, top + 2.0 * d) - r

    keep = []
    for owner, P in pts:
        ok = np.ones(len(P), bool)
        if owner != "arch":
            ok &= d_arch(P) > 0.25 * h
        for b in range(3):
            if b != owner:
                ok &= d_branch(P, b) > 0.25 * h
        keep.append(P[ok])
    X = _poisson_disk(np.concatenate(keep, 0), 0.7 * ds)
    lo = 3 * h
    hi = np.array(BOX) - 3 * h
    c.X = X[np.all((X >= lo) & (X <= hi), axis=1)]
    c.dS = ds * ds
    c.u0 = np.zeros((3, c.N))
    c.p0 = np.zeros(c.N)
    return c
