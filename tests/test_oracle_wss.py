"""Pins of the wall shear stress at the Lagrangian points (oracle).

Exact cases: for a linear velocity field u = A x the lumped projection of the Q1
gradient returns A at every node whose eight cells are kept, and the kernel of
Eq. 18 interpolates a constant tensor exactly (partition of unity), so at points
whose support only holds such nodes the stress is tau = t - (t.n) n with
t = mu (A + A^T) n; a rigid rotation has no strain and no wall shear."""
import numpy as np
import pytest

import synth
from oracle import ipcs, wss


def _box_with_ring_points():
    # a tube of radius 0.5 in a 2 x 2 x 1 box (h = 1/8) with every cell kept, so that
    # the supports of the wall points only hold nodes with all eight cells kept
    c = synth.cylinder_case("wss_box", 16, 8, 2.0, 1.0, 0.5, 4, 24, rho=1.0, mu=0.02, dt=0.01, nsteps=1)
    c.node_mask[:] = 1
    return c


@pytest.fixture(scope="module")
def cyl():
    c = _box_with_ring_points()
    pr = ipcs.Problem.from_case(c)
    return c, pr


def _normals(c):
    n = c.X.copy()
    n[:, 2] = 0.0
    return n / np.linalg.norm(n, axis=1)[:, None]


def _interior_points(c, pr):
    """Points whose 4x4x4 support only holds nodes with all eight cells kept."""
    full = np.zeros(c.N, bool)
    nx, ny = c.nx, c.ny
    ii = np.arange(c.N) % (nx + 1)
    jj = (np.arange(c.N) // (nx + 1)) % (ny + 1)
    kk = np.arange(c.N) // ((nx + 1) * (ny + 1))
    full = (ii > 0) & (ii < nx) & (jj > 0) & (jj < ny) & (kk > 0) & (kk < c.nz)
    I = pr.I.tocsr()
    ok = np.array([full[I.indices[I.indptr[i]:I.indptr[i + 1]]].all() for i in range(c.M)])
    return ok


def test_linear_field_exact(cyl):
    c, pr = cyl
    rng = np.random.default_rng(4)
    A = rng.standard_normal((3, 3))
    xyz = c.node_coords()
    u = (A @ xyz.T) * pr.sets.in_P[None, :]
    n = _normals(c)
    tau = wss.wall_shear(pr, u, n)
    ok = _interior_points(c, pr)
    assert ok.sum() >= 48           # the two middle rings
    t = pr.mu * np.einsum("de,ie->id", A + A.T, n)
    ref = t - np.sum(t * n, axis=1)[:, None] * n
    assert np.abs(tau[ok] - ref[ok]).max() < 1e-12 * np.abs(ref).max()
    # tangential: no normal component anywhere
    assert np.abs(np.sum(tau * n, axis=1)).max() < 1e-14 * np.abs(tau).max()


def test_rigid_rotation_has_no_wall_shear(cyl):
    c, pr = cyl
    xyz = c.node_coords()
    P = pr.sets.in_P
    u = np.stack([-xyz[:, 1] * P, xyz[:, 0] * P, 0.3 * P])
    tau = wss.wall_shear(pr, u, _normals(c))
    ok = _interior_points(c, pr)
    assert np.abs(tau[ok]).max() < 1e-13


def test_plane_shear_magnitude():
    # u = (s z, 0, 0) in the interior: tau on a wall with normal e_z is mu s e_x
    c = _box_with_ring_points()
    pr = ipcs.Problem.from_case(c)
    xyz = c.node_coords()
    s_ = 0.7
    u = np.stack([s_ * xyz[:, 2], 0 * xyz[:, 2], 0 * xyz[:, 2]]) * pr.sets.in_P[None, :]
    n = np.tile([0.0, 0.0, 1.0], (c.M, 1))
    tau = wss.wall_shear(pr, u, n)
    ok = _interior_points(c, pr)
    assert np.allclose(tau[ok], np.tile([pr.mu * s_, 0.0, 0.0], (ok.sum(), 1)), rtol=0, atol=1e-14)


def test_linear_field_exact_on_refined_lattice():
    # every cell kept: the constrained space holds trilinear fields, the lumped
    # projection of their gradient is exact at every node and the points' supports
    # lie in the fine band away from the box faces
    c = synth.refined_cylinder(8, 8, length=1.25, band=0.3, mask_all=True)
    pr = ipcs.Problem.from_case(c)
    rng = np.random.default_rng(8)
    A = rng.standard_normal((3, 3))
    u = (A @ c.node_coords().T) * pr.sets.in_P[None, :]
    n = _normals(c)
    tau = wss.wall_shear(pr, u, n)
    t = pr.mu * np.einsum("de,ie->id", A + A.T, n)
    ref = t - np.sum(t * n, axis=1)[:, None] * n
    assert np.abs(tau - ref).max() < 1e-12 * np.abs(ref).max()
