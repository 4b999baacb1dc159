"""Pins for the 2:1 refined (composite) discretisation of the oracle: full refinement
reproduces the uniform grid at h/2, trilinear fields pass the patch test across the
hanging-node interface, and the mass, gradient and null-space identities hold."""
import numpy as np
import pytest

import synth
from oracle import fem, grid, ipcs, refine


def _mesh(case):
    return refine.CompositeMesh(case.nx, case.ny, case.nz, case.h, case.node_mask, case.bc_tag,
                                case.refine_cell)


def test_full_refinement_equals_uniform_half_spacing():
    c = synth.refined_cylinder(4, 4, length=1.25, band=10.0)        # every cell refined
    assert c.refine_cell.all()
    m = _mesh(c)
    assert m.hanging.size == 0 and m.coarse.size == 0
    ops = refine.CompositeOperators(m)
    s_u = grid.derive_sets(2 * c.nx, 2 * c.ny, 2 * c.nz, c.node_mask, None)
    ref = fem.Operators(s_u, c.h / 2)
    for A, B in ((ops.M, ref.M), (ops.K, ref.K), (ops.G[0], ref.G[0]), (ops.G[2], ref.G[2])):
        assert abs(A - B).max() < 1e-15
    a = np.random.default_rng(0).standard_normal((3, m.N)) * s_u.in_P
    assert abs(ops.advection(a) - ref.advection(a)).max() < 1e-13
    s_c = m.derive_sets(None)
    assert (s_c.P == s_u.P).all() and (s_c.F == s_u.F).all() and (s_c.Pp == s_u.Pp).all()


def test_hanging_nodes_of_one_interface():
    """Two base cells side by side, the first refined: the shared face carries one
    face-centre node (4 parents) and four edge midpoints (2 parents each)."""
    nx, ny, nz, h = 2, 1, 1, 1.0
    N = 5 * 3 * 3
    c = synth.Case(name="pair", nx=nx, ny=ny, nz=nz, h=h, origin=np.zeros(3),
                   node_mask=np.ones(N, np.uint8), bc_tag=None, X=np.zeros((0, 3)), dS=1.0,
                   U_B=None, rho=1, mu=1, dt=1, nsteps=1, inlet_K=0, inlet_omega=0,
                   inlet_ids=np.zeros(0, np.int64), inlet_shape=np.zeros((1, 0, 3)),
                   u0=np.zeros((3, N)), p0=np.zeros(N), refine_cell=np.array([1, 0], np.uint8))
    m = _mesh(c)
    counts = sorted(len(v) for v in m.parents.values())
    assert counts == [2, 2, 2, 2, 4]
    for n, par in m.parents.items():
        i = n % 5
        assert i == 2                      # all on the shared face x = 1 (lattice i = 2)
        assert all(q % 5 == 2 for q in par)


def _band_all_active():
    return synth.refined_cylinder(6, 6, length=1.25, band=0.25, mask_all=True)


def test_patch_test_trilinear_fields_across_interface():
    c = _band_all_active()
    m = _mesh(c)
    assert m.hanging.size > 0 and m.coarse.size > 0
    ops = refine.CompositeOperators(m)
    s = m.derive_sets(None)
    xyz = c.node_coords()
    x, y, z = xyz.T
    f = 0.4 + x - 2 * y + 0.7 * z + x * y - 3 * y * z + 2 * x * z + 4 * x * y * z
    fd = np.where(s.in_P, f, 0.0)
    lx, ly, lz = m.lx, m.ly, m.lz
    i = np.arange(m.N) % (lx + 1)
    j = (np.arange(m.N) // (lx + 1)) % (ly + 1)
    k = np.arange(m.N) // ((lx + 1) * (ly + 1))
    interior = s.in_P & (i > 0) & (i < lx) & (j > 0) & (j < ly) & (k > 0) & (k < lz)
    assert np.abs((ops.K @ fd)[interior]).max() < 1e-12
    # the constrained space holds the field exactly: C (dof values) = field at hanging nodes
    assert np.abs((m.C @ fd)[m.hanging] - f[m.hanging]).max() < 1e-13


def test_composite_identities():
    c = _band_all_active()
    m = _mesh(c)
    ops = refine.CompositeOperators(m)
    s = m.derive_sets(None)
    one = s.in_P.astype(float)
    vol = m.fine.shape[0] * m.hf ** 3 + m.coarse.shape[0] * m.h ** 3
    assert one @ (ops.M @ one) == pytest.approx(vol, rel=1e-13)
    assert abs(vol - (c.nx * c.h) * (c.ny * c.h) * (c.nz * c.h)) < 1e-12
    assert abs(ops.K - ops.K.T).max() < 1e-15
    assert np.abs(ops.K @ one).max() < 1e-13
    xyz = c.node_coords()
    slope = np.array([0.3, -1.2, 0.8])
    lin = np.where(s.in_P, xyz @ slope, 0.0)
    M1 = ops.M @ one
    for d in range(3):
        assert np.abs(ops.G[d] @ lin - slope[d] * M1).max() < 1e-13
    a = np.tile(np.array([0.5, -0.25, 1.0])[:, None], (1, m.N)) * one
    C = ops.advection(a)
    assert np.abs(C @ one).max() < 1e-13
    assert np.abs(C @ lin - (a[:, 0] @ slope) * M1).max() < 1e-13


def test_refined_step_matches_dense_direct_solve():
    from test_oracle_flow import _dense_step
    c = synth.refined_cylinder(8, 8, length=1.25, band=0.3)
    pr = ipcs.Problem.from_case(c)
    assert pr.mesh.hanging.size > 0 and c.M > 0
    u, p = pr.initial_state(c.u0, c.p0)
    t = 0.0
    for _ in range(2):
        un, pn, t1, info = pr.step(u, p, t)
        ud, pd, us, uib, phi = _dense_step(pr, u, p, t)
        scale = np.abs(ud).max()
        assert np.abs(info.u_star - us).max() < 1e-11 * scale
        assert np.abs(info.u_ib - uib).max() < 1e-11 * scale
        assert np.abs(un - ud).max() < 1e-11 * scale
        assert np.abs(pn - pd).max() < 1e-10 * np.abs(pd).max()
        assert np.abs(pr.I @ info.u_ib[2]).max() < 1e-12
        u, p, t = un, pn, t1
    assert np.abs(u[:, pr.mesh.hanging]).max() == 0.0


def test_support_outside_band_rejected():
    c = synth.refined_cylinder(8, 8, length=1.25, band=0.3)
    c.X = np.array([[0.0, 0.0, 0.6]])                 # on the axis, in the coarse core
    with pytest.raises(ValueError, match="refined band"):
        ipcs.Problem.from_case(c)
