"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

FP64 mode: relative L2 <= 1e-10 for every field of every step (the bound the
design targets), operator applies within the FP64 rounding bound of the row
sums, FP32 applies within the FP32 rounding bound."""
import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from gpu_util import make_solver, rel_l2, run_pair, say
from oracle import fem, ib, ipcs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _check_steps(out, tol, label):
    """Relative L2 per field; the pressure increment is measured against the pressure
    scale (it vanishes identically in some exact solutions)."""
    for k, r in enumerate(out):
        errs = {f: rel_l2(r["g_" + f], r["o_" + f]) for f in ("ustar", "uib", "u", "p")}
        floor = max(np.linalg.norm(r["o_phi"]), np.linalg.norm(r["o_p"]))
        errs["phi"] = float(np.linalg.norm(r["g_phi"] - r["o_phi"]) / floor)
        say(f"{label} step {k}: " + " ".join(f"{f}={e:.2e}" for f, e in errs.items()),
            "gpu iters", {x: r["stats"][x] for x in ("s1_iters", "ib_iters", "s3_iters", "s4_iters")})
        assert r["g_t"] == pytest.approx(r["o_t"], abs=1e-15)
        for f, e in errs.items():
            assert e <= tol, (label, k, f, e)


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


@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 2e-6)])
def test_advection_diffusion_apply(precision, tol):
    case = _ops_case()
    pr = ipcs.Problem.from_case(case)
    s = make_solver(case)
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

@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 2e-6)])
def test_advection_diffusion_apply_strain(precision, tol):
    case = _ops_case()
    pr = ipcs.Problem.from_case(case, viscous=1)
    s = make_solver(case, viscous=1)
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
