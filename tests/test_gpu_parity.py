"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

FP64 mode: relative L2 <= 1e-10 for every field of every step (the bound the
design targets), operator applies within the FP64 rounding bound of the row
sums, FP32 applies within the FP32 rounding bound."""
import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from gpu_util import check_steps, make_solver, rel_l2, run_pair, say
from oracle import fem, ib, ipcs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _check_steps(out, tol, label):
    check_steps(out, tol, label)


@pytest.mark.parametrize("seed", [1, 3])
def test_step_parity_fp64_irregular(seed):
    case = synth.random_blob_case(seed=seed)
    say("case", case.name, "N", case.N, "M", case.M)
    _, out = run_pair(case, 3, t0=0.1)
    _check_steps(out, TOL64, case.name)


def test_step_parity_fp64_poiseuille_16x16x64():
    case = synth.poiseuille_c1()
    say("case", case.name, "N", case.N, "M", case.M)
    _, out = run_pair(case, case.nsteps)
    _check_steps(out, TOL64, case.name)


def test_step_parity_fp64_closed_box_null_space():
    case = synth.closed_box(6)
    say("case", case.name)
    _, out = run_pair(case, 2)
    _check_steps(out, TOL64, case.name)
    phi = out[-1]["g_phi"]
    assert abs(phi.mean()) < 1e-12 * np.abs(phi).max()


@pytest.mark.parametrize("make", [lambda: synth.channel_case(ic="rest"),
                                  lambda: synth.shear_advection_case(),
                                  lambda: synth.small_cylinder(8, 16, pulsatile=True, nsteps=3)])
def test_step_parity_fp64_special_cases(make):
    case = make()
    say("case", case.name)
    _, out = run_pair(case, 3)
    _check_steps(out, TOL64, case.name)


# ---------------------------------------------------------------------------
# operator applies
# ---------------------------------------------------------------------------

def _ops_case():
    return synth.random_blob_case(cells=(9, 7, 8), seed=5, n_points=10)


def _bound(A, x):
    return np.abs(A) @ np.abs(x)


@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 2e-6)])
def test_symmetric_applies(precision, tol):
    case = _ops_case()
    pr = ipcs.Problem.from_case(case)
    s = make_solver(case)
    P = pr.sets.P
    rng = np.random.default_rng(11)
    x = rng.standard_normal(P.size)
    xf = np.zeros(case.N)
    xf[P] = x
    for op, A in ((ibfe.OP_MASS, pr.ops.M), (ibfe.OP_STIFF, pr.ops.K)):
        say("apply", op, "precision", precision)
        y = s.apply(op, x, precision)
        yo = (A @ xf)[P]
        bound = _bound(A, xf)[P]
        assert np.all(np.abs(y - yo) <= tol * bound + 1e-300), op
    s.close()


def test_gradient_divergence_interp_spread_fp64():
    case = _ops_case()
    pr = ipcs.Problem.from_case(case)
    s = make_solver(case)
    P = pr.sets.P
    rng = np.random.default_rng(12)
    x = rng.standard_normal(P.size)
    xf = np.zeros(case.N)
    xf[P] = x
    g = s.apply(ibfe.OP_GRAD, x).reshape(3, -1)
    for d in range(3):
        G = pr.ops.G[d]
        assert np.all(np.abs(g[d] - (G @ xf)[P]) <= 1e-13 * _bound(G, xf)[P])
    u = rng.standard_normal((3, P.size))
    uf = np.zeros((3, case.N))
    uf[:, P] = u
    dv = s.apply(ibfe.OP_DIV, u.ravel())
    bound = sum(_bound(pr.ops.G[d], uf[d]) for d in range(3))[P]
    assert np.all(np.abs(dv - pr.ops.divergence(uf)[P]) <= 1e-13 * bound)
    Iu = s.apply(ibfe.OP_INTERP, u.ravel()).reshape(-1, 3)
    for d in range(3):
        ref = pr.I @ uf[d]
        assert np.all(np.abs(Iu[:, d] - ref) <= 1e-13 * _bound(pr.I, uf[d]) + 1e-300)
    lam = rng.standard_normal((case.M, 3))
    sp = s.apply(ibfe.OP_SPREAD, lam.ravel()).reshape(3, -1)
    IF = pr.I.multiply(pr.sets.in_F[None, :].astype(float)).tocsr()
    for d in range(3):
        ref = (IF.T @ lam[:, d])[P]
        assert np.all(np.abs(sp[d] - ref) <= 1e-13 * (np.abs(IF.T) @ np.abs(lam[:, d]))[P] + 1e-300)
    s.close()


@pytest.mark.parametrize("advdiff", [0, 1])
@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 2e-6)])
def test_advection_diffusion_apply(precision, tol, advdiff):
    # advdiff 0: rows formed on the fly (matrix-free); 1: assembled stencil
    case = _ops_case()
    pr = ipcs.Problem.from_case(case)
    s = make_solver(case, advdiff=advdiff)
    P = pr.sets.P
    rng = np.random.default_rng(13)
    u = rng.standard_normal((3, P.size))
    s.set_state(u.ravel(), np.zeros(P.size), 0.0)
    uf = np.zeros((3, case.N))
    uf[:, P] = u
    A = ((pr.rho / pr.dt) * pr.ops.M + pr.rho * pr.ops.advection(uf) + pr.mu * pr.ops.K).tocsr()
    x = rng.standard_normal((3, P.size))
    xf = np.zeros((3, case.N))
    xf[:, P] = x
    y = s.apply(ibfe.OP_ADVDIFF, x.ravel(), precision).reshape(3, -1)
    for d in range(3):
        assert np.all(np.abs(y[d] - (A @ xf[d])[P]) <= tol * _bound(A, xf[d])[P] + 1e-300), d
    s.close()


# ---------------------------------------------------------------------------
# full-size pulsatile cylinder (64x64x512): sampled rows and step properties
# ---------------------------------------------------------------------------

def _row_apply(sets, Me, xf, nodes, nx, ny):
    """y_i = sum over kept cells around node i of the element row: the definition of
    the assembled operator, evaluated one output at a time."""
    out = []
    for i in nodes:
        ii = i % (nx + 1)
        jj = (i // (nx + 1)) % (ny + 1)
        kk = i // ((nx + 1) * (ny + 1))
        acc = 0.0
        for s in range(8):
            ci, cj, ck = ii - 1 + (s & 1), jj - 1 + ((s >> 1) & 1), kk - 1 + ((s >> 2) & 1)
            if min(ci, cj, ck) < 0 or ci >= nx or cj >= ny or ck >= sets.nz:
                continue
            c = ci + nx * (cj + ny * ck)
            if not sets.kept_cells[c]:
                continue
            a = (ii - ci) + 2 * (jj - cj) + 4 * (kk - ck)
            for b in range(8):
                nb = (ci + (b & 1)) + (nx + 1) * ((cj + ((b >> 1) & 1)) + (ny + 1) * (ck + ((b >> 2) & 1)))
                acc += Me[a, b] * xf[nb]
        out.append(acc)
    return np.array(out)


@pytest.fixture(scope="module")
def c2():
    return synth.pulsatile_c2()


def test_full_size_stiffness_rows_sampled(c2):
    from oracle import grid
    say("case", c2.name, "N", c2.N, "M", c2.M)
    sets = grid.derive_sets(c2.nx, c2.ny, c2.nz, c2.node_mask, None)
    s = make_solver(c2)
    P = sets.P
    rng = np.random.default_rng(21)
    x = rng.standard_normal(P.size)
    xf = np.zeros(c2.N)
    xf[P] = x
    Me, Ke, _, _ = fem.element_matrices(c2.h)
    for op, E in ((ibfe.OP_STIFF, Ke), (ibfe.OP_MASS, Me)):
        for prec, tol in ((0, 1e-12), (1, 1e-5)):
            y = s.apply(op, x, prec)
            pick = rng.choice(P.size, 400, replace=False)
            ref = _row_apply(sets, E, xf, P[pick], c2.nx, c2.ny)
            bound = _row_apply(sets, np.abs(E), np.abs(xf), P[pick], c2.nx, c2.ny)
            say("full-size apply", op, prec, "max rel", float(np.max(np.abs(y[pick] - ref) / bound)))
            assert np.all(np.abs(y[pick] - ref) <= tol * bound)
    s.close()


def test_full_size_steps_fp64_properties(c2):
    say("case", c2.name, "FP64, 2 steps from rest")
    s = make_solver(c2)
    n = s.n_u
    s.set_state(np.zeros(3 * n), np.zeros(n), 0.0)
    ids = s.node_ids()
    I = ib.interpolation_matrix(c2.X, c2.nx, c2.ny, c2.nz, c2.h, c2.origin)
    for k in range(2):
        s.step(1)
        st = s.stats()
        say("step", k, st)
        uib = s.field(ibfe.FIELD_UIB)
        uf = np.zeros((3, c2.N))
        uf[:, ids] = uib
        for d in range(3):
            assert np.abs(I @ uf[d]).max() < 1e-9
        u, p, t = s.get_state()
        assert np.isfinite(u).all() and np.isfinite(p).all()
        d_ib = np.linalg.norm(s.apply(ibfe.OP_DIV, uib.ravel()))
        d_new = np.linalg.norm(s.apply(ibfe.OP_DIV, u.ravel()))
        say("divergence", d_ib, d_new)
        assert d_new < 0.5 * d_ib
        assert st["s3_res"] <= 1e-13 and st["s1_res"] <= 1e-13 and st["s4_res"] <= 1e-13
    s.close()


def _advdiff_rows(sets, xf, uf, rows, nx, ny, h, rho, mu, dt):
    """Rows of A = (rho/dt) M + rho C(u) + mu K applied to the three components of xf,
    from the oracle's element matrices (cells kept, corner velocities of each cell),
    and the matching rounding bound (the same sum over absolute values)."""
    Me, Ke, _, Ce = fem.element_matrices(h)
    out = np.zeros((3, len(rows)))
    bnd = np.zeros((3, len(rows)))
    for q, i in enumerate(rows):
        ii = i % (nx + 1)
        jj = (i // (nx + 1)) % (ny + 1)
        kk = i // ((nx + 1) * (ny + 1))
        for s_ in range(8):
            ci, cj, ck = ii - 1 + (s_ & 1), jj - 1 + ((s_ >> 1) & 1), kk - 1 + ((s_ >> 2) & 1)
            if min(ci, cj, ck) < 0 or ci >= nx or cj >= ny or ck >= sets.nz:
                continue
            if not sets.kept_cells[ci + nx * (cj + ny * ck)]:
                continue
            a = (ii - ci) + 2 * (jj - cj) + 4 * (kk - ck)
            nb = np.array([(ci + (b & 1)) + (nx + 1) * ((cj + ((b >> 1) & 1)) + (ny + 1) * (ck + ((b >> 2) & 1)))
                           for b in range(8)])
            aloc = uf[:, nb].T                                    # (8 corners, 3 directions)
            row = (rho / dt) * Me[a] + rho * np.einsum("cd,cdb->b", aloc, Ce[a]) + mu * Ke[a]
            for d in range(3):
                out[d, q] += row @ xf[d][nb]
                bnd[d, q] += np.abs(row) @ np.abs(xf[d][nb])
    return out, bnd


def test_full_size_advection_diffusion_rows_sampled(c2):
    """The tentative-velocity operator at the benchmark size, sampled rows against the
    oracle's element forms (FP64 and FP32 applies)."""
    from oracle import grid
    sets = grid.derive_sets(c2.nx, c2.ny, c2.nz, c2.node_mask, None)
    P = sets.P
    rng = np.random.default_rng(22)
    u = rng.standard_normal((3, P.size)) * 0.5
    x = rng.standard_normal((3, P.size))
    uf = np.zeros((3, c2.N))
    uf[:, P] = u
    xf = np.zeros((3, c2.N))
    xf[:, P] = x
    pick = rng.choice(P.size, 300, replace=False)
    ref, bound = _advdiff_rows(sets, xf, uf, P[pick], c2.nx, c2.ny, c2.h, c2.rho, c2.mu, c2.dt)
    for advdiff in (0, 1):  # matrix-free rows, then the assembled stencil
        s = make_solver(c2, advdiff=advdiff)
        s.set_state(u.ravel(), np.zeros(P.size), 0.0)
        for prec, tol in ((0, 1e-12), (1, 1e-5)):
            y = s.apply(ibfe.OP_ADVDIFF, x.ravel(), prec).reshape(3, -1)
            err = np.abs(y[:, pick] - ref) / bound
            say("full-size advection-diffusion apply, advdiff", advdiff, "precision", prec,
                "max rel", float(err.max()))
            assert np.all(err <= tol)
        s.close()


def _c2_steps(c2, sets, precision, tol):
    """Two steps from rest on the full benchmark cylinder.  After each, every row of
    the three sub-step equations is checked with the library's operator applies
    (each checked row by row against the oracle above): the tentative velocity
    A(u^n) u* = (rho/dt) M u^n - G p^n on the free rows (A at the old velocity, applied
    by a second context holding u^n), the IB constraint I u_ib = 0 at every point, the
    pressure increment K Phi = -(rho/dt) B u_ib on the pressure unknowns and the
    correction (rho/dt) M (u_ib - u^{n+1}) = G Phi on the free rows."""
    s = make_solver(c2, precision=precision, precond=2)
    aux = make_solver(c2)
    n = s.n_u
    s.set_state(np.zeros(3 * n), np.zeros(n), 0.0)
    ids = s.node_ids()
    onF = sets.in_F[ids]
    onPp = (sets.in_P & ~sets.p_dir)[ids]
    I = ib.interpolation_matrix(c2.X, c2.nx, c2.ny, c2.nz, c2.h, c2.origin)
    rho, dt = c2.rho, c2.dt
    for k in range(2):
        u_n, p_n, t_n = s.get_state()
        s.step(1)
        st = s.stats()
        say("precision", precision, "step", k, {x: st[x] for x in ("s1_iters", "ib_iters", "s3_iters",
                                                                    "s4_iters", "s1_res", "s3_res", "s4_res")})
        ustar = s.field(ibfe.FIELD_USTAR)
        uib = s.field(ibfe.FIELD_UIB)
        phi = s.field(ibfe.FIELD_PHI)
        u, p, t = s.get_state()
        assert np.isfinite(u).all() and np.isfinite(p).all()
        assert np.allclose(p, p_n + phi, rtol=0, atol=1e-12 * np.abs(p).max())
        # tentative velocity
        aux.set_state(u_n.ravel(), p_n, t_n)
        # A_FF u*_F and the Dirichlet lifting A_FD g as separate applies: from rest the
        # right-hand side vanishes and the two cancel, so the residual is measured
        # against the largest of the three terms (a component at rest gives 0 = 0)
        us = ustar.reshape(3, -1)
        a_free = aux.apply(ibfe.OP_ADVDIFF, (us * onF).ravel(), 0).reshape(3, -1)
        a_lift = aux.apply(ibfe.OP_ADVDIFF, (us * ~onF).ravel(), 0).reshape(3, -1)
        gp = aux.apply(ibfe.OP_GRAD, p_n, 0).reshape(3, -1)
        e1 = 0.0
        for d in range(3):
            rhs1 = (rho / dt) * aux.apply(ibfe.OP_MASS, u_n[d], 0) - gp[d]
            scale = max(np.abs(rhs1[onF]).max(), np.abs(a_free[d][onF]).max(), np.abs(a_lift[d][onF]).max())
            r1 = np.abs((a_free[d] + a_lift[d] - rhs1)[onF]).max()
            e1 = max(e1, r1 / scale if scale > 0 else r1)
        # IB constraint (force solve to 1e-13 in FP64, 1e-10 in mixed precision)
        uf = np.zeros((3, c2.N))
        uf[:, ids] = uib.reshape(3, -1)
        for d in range(3):
            assert np.abs(I @ uf[d]).max() < (1e-9 if precision == 0 else 1e-7)
        # pressure increment
        rhs3 = -(rho / dt) * s.apply(ibfe.OP_DIV, uib.ravel(), 0)
        e3 = np.abs((s.apply(ibfe.OP_STIFF, phi, 0) - rhs3)[onPp]).max() / np.abs(rhs3[onPp]).max()
        # correction
        du = (uib - u).reshape(3, -1)
        gphi = s.apply(ibfe.OP_GRAD, phi, 0).reshape(3, -1)
        e4 = max(np.abs(((rho / dt) * s.apply(ibfe.OP_MASS, du[d], 0) - gphi[d])[onF]).max()
                 / np.abs(gphi[d][onF]).max() for d in range(3))
        say("equation residuals (max row / max term): tentative", e1, "pressure", e3,
            "correction", e4)
        assert e1 <= tol and e3 <= tol and e4 <= tol
    u, p, t = s.get_state()
    s.close()
    aux.close()
    return u, p


def test_full_size_c2_steps_fp64_and_mixed(c2):
    """The benchmark cylinder at full size in both precisions: the sub-step equations
    on every row, and mixed precision against FP64 after two steps (relative L2 and
    entry by entry against the field maximum) at the 1e-6 of the accuracy target."""
    from oracle import grid
    from gpu_util import rel_max
    sets = grid.derive_sets(c2.nx, c2.ny, c2.nz, c2.node_mask, None)
    say("case", c2.name, "N", c2.N, "M", c2.M)
    u64, p64 = _c2_steps(c2, sets, 0, 1e-10)
    u32, p32 = _c2_steps(c2, sets, 1, 1e-6)
    eu, ep = rel_l2(u32, u64), rel_l2(p32, p64)
    mu_, mp = rel_max(u32, u64), rel_max(p32, p64)
    say("mixed vs FP64 after 2 steps: rel L2 u", eu, "p", ep, "| max u", mu_, "p", mp)
    assert eu <= 1e-6 and ep <= 1e-6 and mu_ <= 1e-6 and mp <= 1e-6


# ---------------------------------------------------------------------------
# mixed precision: FP32 inner solves inside FP64 refinement, 1e-6 relative L2
# ---------------------------------------------------------------------------

TOL_MIXED = 1e-6


@pytest.mark.parametrize("make", [lambda: synth.random_blob_case(seed=1),
                                  lambda: synth.small_cylinder(8, 16, pulsatile=True, nsteps=3),
                                  lambda: synth.closed_box(6)])
def test_step_parity_mixed_small(make):
    case = make()
    say("case", case.name, "mixed precision")
    _, out = run_pair(case, 3, precision=1)
    _check_steps(out, TOL_MIXED, case.name + "/mixed")


def test_step_parity_mixed_poiseuille_16x16x64():
    case = synth.poiseuille_c1()
    say("case", case.name, "mixed precision, 20 steps")
    _, out = run_pair(case, case.nsteps, precision=1)
    _check_steps(out, TOL_MIXED, case.name + "/mixed")
    st = out[-1]["stats"]
    assert st["s3_outer"] >= 1 and st["s3_res"] <= 1e-8


# ---------------------------------------------------------------------------
# multigrid-preconditioned pressure solve (precond = 2): same discrete solution
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [(0, TOL64), (1, TOL_MIXED)])
@pytest.mark.parametrize("make", [lambda: synth.random_blob_case(seed=3),
                                  lambda: synth.closed_box(8),
                                  lambda: synth.small_cylinder(8, 16, pulsatile=True, nsteps=3)])
def test_step_parity_multigrid_small(make, precision, tol):
    case = make()
    say("case", case.name, "multigrid, precision", precision)
    _, out = run_pair(case, 3, precision=precision, precond=2)
    _check_steps(out, tol, case.name + "/mg")
    # the same steps with the assembled advection-diffusion stencil
    _, out = run_pair(case, 3, precision=precision, precond=2, advdiff=1)
    _check_steps(out, tol, case.name + "/mg/stencil")


@pytest.mark.parametrize("precision,tol", [(0, TOL64), (1, TOL_MIXED)])
def test_step_parity_multigrid_poiseuille_16x16x64(precision, tol):
    case = synth.poiseuille_c1()
    say("case", case.name, "multigrid, precision", precision)
    _, out = run_pair(case, case.nsteps, precision=precision, precond=2)
    _check_steps(out, tol, case.name + "/mg")
    assert out[-1]["stats"]["s3_iters"] < 60


# ---------------------------------------------------------------------------
# Chebyshev-Jacobi polynomial preconditioner for the pressure increment
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [(0, TOL64), (1, TOL_MIXED)])
@pytest.mark.parametrize("make", [lambda: synth.poiseuille_c1(),
                                  lambda: synth.closed_box(6),
                                  lambda: synth.refined_cylinder(8, 8, length=1.25, band=0.3)])
def test_step_parity_chebyshev_preconditioner(make, precision, tol):
    case = make()
    say("case", case.name, "Chebyshev preconditioner, precision", precision)
    _, out = run_pair(case, 3, precision=precision, precond=1)
    _check_steps(out, tol, case.name + "/cheb")
    _, out_j = run_pair(case, 1, precision=precision, precond=0)
    say("s3 iterations: Chebyshev", out[0]["stats"]["s3_iters"], "Jacobi", out_j[0]["stats"]["s3_iters"])
    assert out[0]["stats"]["s3_iters"] < out_j[0]["stats"]["s3_iters"]


# ---------------------------------------------------------------------------
# explicit advection (the convection of Eq. 13 at the old velocity)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [(0, TOL64), (1, TOL_MIXED)])
@pytest.mark.parametrize("make", [lambda: synth.shear_advection_case(),
                                  lambda: synth.random_blob_case(seed=3),
                                  lambda: synth.small_cylinder(8, 16, pulsatile=True, nsteps=3),
                                  lambda: synth.refined_cylinder(8, 8, length=1.25, band=0.3)])
def test_step_parity_explicit_advection(make, precision, tol):
    case = make()
    say("case", case.name, "explicit advection, precision", precision)
    _, out = run_pair(case, 3, t0=0.05, precision=precision, precond=2, advection=1)
    _check_steps(out, tol, case.name + "/explicit")


# ---------------------------------------------------------------------------
# strain-rate viscous form 2 mu (eps(u), eps(v)) (components coupled in S1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("advdiff", [0, 1])
@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 2e-6)])
def test_advection_diffusion_apply_strain(precision, tol, advdiff):
    case = _ops_case()
    pr = ipcs.Problem.from_case(case, viscous=1)
    s = make_solver(case, viscous=1, advdiff=advdiff)
    P = pr.sets.P
    rng = np.random.default_rng(17)
    u = rng.standard_normal((3, P.size))
    s.set_state(u.ravel(), np.zeros(P.size), 0.0)
    uf = np.zeros((3, case.N))
    uf[:, P] = u
    A = ((pr.rho / pr.dt) * pr.ops.M + pr.rho * pr.ops.advection(uf) + pr.mu * pr.ops.K).tocsr()
    X = pr.ops.strain_cross()
    x = rng.standard_normal((3, P.size))
    xf = np.zeros((3, case.N))
    xf[:, P] = x
    y = s.apply(ibfe.OP_ADVDIFF, x.ravel(), precision).reshape(3, -1)
    for d in range(3):
        ref = A @ xf[d] + pr.mu * sum(X[d][c] @ xf[c] for c in range(3))
        bound = _bound(A, xf[d]) + pr.mu * sum(_bound(X[d][c], xf[c]) for c in range(3))
        assert np.all(np.abs(y[d] - ref[P]) <= tol * bound[P] + 1e-300), d
    s.close()


@pytest.mark.parametrize("advection", [0, 1])
@pytest.mark.parametrize("precision,tol", [(0, TOL64), (1, TOL_MIXED)])
@pytest.mark.parametrize("make", [lambda: synth.random_blob_case(seed=3),
                                  lambda: synth.small_cylinder(8, 16, pulsatile=True, nsteps=3),
                                  lambda: synth.poiseuille_c1()])
def test_step_parity_strain_rate_form(make, precision, tol, advection):
    case = make()
    say("case", case.name, "strain-rate viscous form, precision", precision, "advection", advection)
    _, out = run_pair(case, 3, t0=0.05, precision=precision, precond=2, viscous=1, advection=advection)
    _check_steps(out, tol, case.name + "/strain")


# ---------------------------------------------------------------------------
# wall shear stress at the Lagrangian points
# ---------------------------------------------------------------------------

def _cyl_normals(case):
    n = case.X.copy()
    n[:, 2] = 0.0
    return n / np.linalg.norm(n, axis=1)[:, None]


@pytest.mark.parametrize("make", [lambda: synth.small_cylinder(8, 16, pulsatile=True, nsteps=3),
                                  lambda: synth.poiseuille_c1(ic="poiseuille")])
def test_wall_shear_parity(make):
    from oracle import wss
    case = make()
    pr, out = run_pair(case, 2, t0=0.05)
    s = make_solver(case)
    P = pr.sets.P
    # the state after the oracle's second step, on both sides
    uf = np.zeros((3, case.N))
    uf[:, P] = out[-1]["o_u"]
    s.set_state(out[-1]["o_u"].ravel(), out[-1]["o_p"], out[-1]["o_t"])
    n = _cyl_normals(case)
    g = s.wall_shear(n)
    o = wss.wall_shear(pr, uf, n)
    err = np.abs(g - o).max() / np.abs(o).max()
    say(case.name, "wall shear max", np.abs(o).max(), "rel err", err)
    assert err < 1e-12
    s.close()
