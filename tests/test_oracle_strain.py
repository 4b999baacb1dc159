"""Pins of the strain-rate viscous form 2 mu (eps(u), eps(v)) in the oracle.

The momentum equation of Section 2.1 carries the viscous stress through the
strain rate eps(u) = (grad u + grad u^T)/2.  Its weak form couples the velocity
components: block (d, e) between test component d and trial component e is
mu (K delta_de + X_de) with X_de,ij = int d_e N_i d_d N_j.  The pins below do not
retype that formula: they check it against the tensor-product derivation of the
element entries, the rigid-motion null space of the strain, closed-form strain
energies of linear fields, and a dense direct solve of a whole step."""
import numpy as np
import pytest

import synth
from oracle import fem, ipcs



def test_element_cross_blocks_match_tensor_products():
    h = 0.37
    _, Ke, _, _, Xe = fem.element_matrices_all(h)
    # 1-D pieces on [0, h]: int phi_i' phi_j = s_i / 2, int phi_i phi_j' = s_j / 2,
    # int phi_i phi_j = h (1/3 or 1/6), int phi_i' phi_j' = s_i s_j / h, s_0 = -1, s_1 = +1
    s = [-1.0, 1.0]
    m = lambda i, j: h / 3 if i == j else h / 6
    for d in range(3):
        for e in range(3):
            for a in range(8):
                la = [(a >> k) & 1 for k in range(3)]
                for b in range(8):
                    lb = [(b >> k) & 1 for k in range(3)]
                    v = 1.0
                    for f in range(3):
                        if f == d and f == e:
                            v *= s[la[f]] * s[lb[f]] / h
                        elif f == e:
                            v *= s[la[f]] / 2
                        elif f == d:
                            v *= s[lb[f]] / 2
                        else:
                            v *= m(la[f], lb[f])
                    assert Xe[d, e, a, b] == pytest.approx(v, rel=1e-13, abs=1e-15)
    assert np.allclose(Xe[0, 0] + Xe[1, 1] + Xe[2, 2], Ke, rtol=0, atol=1e-15)
    for d in range(3):
        for e in range(3):
            assert np.allclose(Xe[d, e], Xe[e, d].T, rtol=0, atol=1e-16)


@pytest.fixture(scope="module")
def blob():
    c = synth.random_blob_case(cells=(5, 4, 6), seed=7)
    pr = ipcs.Problem.from_case(c, viscous=1)
    return c, pr


def _strain_op(pr):
    ops = pr.ops
    X = ops.strain_cross()
    import scipy.sparse as sp
    return sp.bmat([[ops.K + X[d][e] if d == e else X[d][e] for e in range(3)] for d in range(3)]).tocsr()


def test_strain_form_symmetric_with_rigid_null_space(blob):
    c, pr = blob
    Keps = _strain_op(pr)
    assert abs(Keps - Keps.T).max() < 1e-14
    xyz = c.node_coords()
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    P = pr.sets.in_P
    one, zero = np.where(P, 1.0, 0.0), np.zeros(c.N)
    motions = [(one, zero, zero), (zero, one, zero), (zero, zero, one),     # translations
               (-y * P, x * P, zero), (zero, -z * P, y * P), (z * P, zero, -x * P)]  # rotations
    for u in motions:
        r = Keps @ np.concatenate(u)
        assert np.abs(r).max() < 1e-12 * max(1.0, np.abs(np.concatenate(u)).max())
    # the component-wise Laplacian form does not annihilate rotations
    rot = np.concatenate(motions[3])
    lap = np.concatenate([pr.ops.K @ motions[3][d] for d in range(3)])
    assert np.abs(lap).max() > 1e-3 * np.abs(rot).max()


def test_strain_energy_of_linear_fields(blob):
    c, pr = blob
    Keps = _strain_op(pr)
    xyz = c.node_coords()
    P = pr.sets.in_P
    vol = pr.sets.kept_cells.sum() * c.h ** 3
    x, y = xyz[:, 0] * P, xyz[:, 1] * P
    zero = np.zeros(c.N)
    # u = (y, x, 0): eps_12 = eps_21 = 1, 2 eps:eps = 4; grad u:grad u = 2
    u = np.concatenate([y, x, zero])
    assert u @ (Keps @ u) == pytest.approx(4.0 * vol, rel=1e-12)
    assert sum(w @ (pr.ops.K @ w) for w in (y, x)) == pytest.approx(2.0 * vol, rel=1e-12)
    # u = (x, 0, 0): eps_11 = 1, 2 eps:eps = 2
    u = np.concatenate([x, zero, zero])
    assert u @ (Keps @ u) == pytest.approx(2.0 * vol, rel=1e-12)


@pytest.mark.parametrize("advection", [0, 1])
def test_strain_step_matches_dense_direct_solve(blob, advection):
    c, _ = blob
    pr = ipcs.Problem.from_case(c, viscous=1, advection=advection)
    s, ops = pr.sets, pr.ops
    rho, mu, dt = pr.rho, pr.mu, pr.dt
    u, p = pr.initial_state(c.u0, c.p0)
    t = 0.05
    un, pn, t1, info = pr.step(u, p, t)
    # dense coupled S1
    F = s.F
    g = pr.g(t + dt)
    C = ops.advection(u).toarray()
    A = (rho / dt) * ops.M.toarray() + mu * ops.K.toarray() + (rho * C if advection == 0 else 0.0)
    X = [[ops.strain_cross()[d][e].toarray() for e in range(3)] for d in range(3)]
    full = [[(A if d == e else 0.0) + mu * X[d][e] for e in range(3)] for d in range(3)]
    rhs = []
    for d in range(3):
        r = (rho / dt) * (ops.M @ u[d]) - ops.G[d] @ p - sum(full[d][e] @ g[e] for e in range(3))
        if advection == 1:
            r = r - rho * (C @ u[d])
        rhs.append(r[F])
    big = np.block([[full[d][e][np.ix_(F, F)] for e in range(3)] for d in range(3)])
    x = np.linalg.solve(big, np.concatenate(rhs))
    us = np.array(g, copy=True)
    for d in range(3):
        us[d][F] = x[d * F.size:(d + 1) * F.size]
    assert np.abs(info.u_star - us).max() < 1e-11 * np.abs(us).max()
    # the coupling matters: the component-wise solve differs
    pr0 = ipcs.Problem.from_case(c, viscous=0, advection=advection)
    _, _, _, info0 = pr0.step(u, p, t)
    assert np.abs(info0.u_star - us).max() > 1e-6 * np.abs(us).max()


def test_refined_strain_form_rigid_null_space_and_dense_step():
    # composite mesh with every cell kept: rigid motions are in the constrained space
    c = synth.refined_cylinder(6, 4, length=1.25 * 4 / 6, band=0.25, mask_all=True)
    c.X = np.zeros((0, 3))      # the operator alone: no wall points needed
    c.U_B = None
    pr = ipcs.Problem.from_case(c, viscous=1)
    Keps = _strain_op(pr)
    assert abs(Keps - Keps.T).max() < 1e-14
    xyz = c.node_coords()
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    P = pr.sets.in_P
    zero = np.zeros(c.N)
    for u in ((-y * P, x * P, zero), (zero, -z * P, y * P), (P * 1.0, zero, zero)):
        r = Keps @ np.concatenate(u)
        assert np.abs(r).max() < 1e-12
    # a refined step equals the dense direct solve of the coupled composite system
    cs = synth.refined_cylinder(8, 8, length=1.25, band=0.3)
    pr = ipcs.Problem.from_case(cs, viscous=1)
    ops, s = pr.ops, pr.sets
    rng = np.random.default_rng(9)
    u = np.where(s.in_P[None, :], rng.standard_normal((3, cs.N)) * 0.1, 0.0)
    p = np.zeros(cs.N)
    un, pn, t1, info = pr.step(u, p, 0.05)
    F = s.F
    g = pr.g(0.05 + pr.dt)
    A = ((pr.rho / pr.dt) * ops.M + pr.rho * ops.advection(u) + pr.mu * ops.K).toarray()
    X = [[ops.strain_cross()[d][e].toarray() for e in range(3)] for d in range(3)]
    full = [[(A if d == e else 0.0) + pr.mu * X[d][e] for e in range(3)] for d in range(3)]
    rhs = [((pr.rho / pr.dt) * (ops.M @ u[d]) - ops.G[d] @ p - sum(full[d][e] @ g[e] for e in range(3)))[F]
           for d in range(3)]
    big = np.block([[full[d][e][np.ix_(F, F)] for e in range(3)] for d in range(3)])
    xs = np.linalg.solve(big, np.concatenate(rhs))
    for d in range(3):
        assert np.abs(info.u_star[d][F] - xs[d * F.size:(d + 1) * F.size]).max() < 1e-10 * np.abs(xs).max()


def test_refined_strain_explicit_step_matches_dense_direct_solve():
    # explicit advection: the convection at u^n moves to the right-hand side and the
    # coupled composite system (rho/dt) M + mu K + mu X is solved by CG
    cs = synth.refined_cylinder(8, 8, length=1.25, band=0.3)
    pr = ipcs.Problem.from_case(cs, viscous=1, advection=1)
    ops, s = pr.ops, pr.sets
    rng = np.random.default_rng(11)
    u = np.where(s.in_P[None, :], rng.standard_normal((3, cs.N)) * 0.1, 0.0)
    p = np.where(s.in_P, rng.standard_normal(cs.N) * 0.01, 0.0)
    _, _, _, info = pr.step(u, p, 0.05)
    F = s.F
    g = pr.g(0.05 + pr.dt)
    A = ((pr.rho / pr.dt) * ops.M + pr.mu * ops.K).toarray()
    C = ops.advection(u)
    X = [[ops.strain_cross()[d][e].toarray() for e in range(3)] for d in range(3)]
    full = [[(A if d == e else 0.0) + pr.mu * X[d][e] for e in range(3)] for d in range(3)]
    rhs = [((pr.rho / pr.dt) * (ops.M @ u[d]) - pr.rho * (C @ u[d]) - ops.G[d] @ p
            - sum(full[d][e] @ g[e] for e in range(3)))[F] for d in range(3)]
    big = np.block([[full[d][e][np.ix_(F, F)] for e in range(3)] for d in range(3)])
    assert np.abs(big - big.T).max() < 1e-12 * np.abs(big).max()
    xs = np.linalg.solve(big, np.concatenate(rhs))
    for d in range(3):
        assert np.abs(info.u_star[d][F] - xs[d * F.size:(d + 1) * F.size]).max() < 1e-10 * np.abs(xs).max()
