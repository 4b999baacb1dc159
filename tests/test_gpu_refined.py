"""GPU parity on 2:1 refined lattices (hanging-node constraints): composite
operator applies within rounding bounds, whole steps against the FP64 oracle
in FP64 (1e-10) and mixed precision (1e-6), and the null-space treatment of a
refined vessel without outlet."""
import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from gpu_util import check_steps, make_solver, rel_l2, run_pair, say
from oracle import fem, grid, ipcs, refine

pytestmark = pytest.mark.gpu


def _cyl():
    return synth.refined_cylinder(8, 8, length=1.25, band=0.3)


def _aneurysm():
    return synth.aneurysm_case((16, 16, 40), band=1.2, nsteps=2)


def _abs_bound(mesh, lf, lc, x):
    """|C|^T |A| |C| |x| with |A| assembled from absolute element entries: the scale of
    the rounding error of any summation order of the constrained row."""
    N = mesh.N
    A = refine._assemble(mesh.fine, np.abs(lf), N) + refine._assemble(mesh.coarse, np.abs(lc), N)
    C = abs(mesh.C)
    return C.T @ (A @ (C @ np.abs(x)))


@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 2e-6)])
def test_refined_symmetric_applies(precision, tol):
    case = _cyl()
    pr = ipcs.Problem.from_case(case)
    s = make_solver(case)
    P = pr.sets.P
    x = np.random.default_rng(21).standard_normal(P.size)
    xf = np.zeros(case.N)
    xf[P] = x
    Mf, Kf, _, _ = fem.element_matrices(case.h / 2)
    Mc, Kc, _, _ = fem.element_matrices(case.h)
    for op, A, lf, lc in ((ibfe.OP_MASS, pr.ops.M, Mf, Mc), (ibfe.OP_STIFF, pr.ops.K, Kf, Kc)):
        say("refined apply", op, "precision", precision)
        y = s.apply(op, x, precision)
        yo = (A @ xf)[P]
        bound = _abs_bound(pr.mesh, lf, lc, xf)[P]
        err = np.abs(y - yo)
        assert np.all(err <= tol * bound + 1e-300), (op, float((err / np.maximum(bound, 1e-300)).max()))
    s.close()


def test_refined_gradient_divergence_fp64():
    case = _cyl()
    pr = ipcs.Problem.from_case(case)
    s = make_solver(case)
    P = pr.sets.P
    rng = np.random.default_rng(22)
    x = rng.standard_normal(P.size)
    xf = np.zeros(case.N)
    xf[P] = x
    _, _, Gf, _ = fem.element_matrices(case.h / 2)
    _, _, Gc, _ = fem.element_matrices(case.h)
    g = s.apply(ibfe.OP_GRAD, x).reshape(3, -1)
    for d in range(3):
        bound = _abs_bound(pr.mesh, Gf[d], Gc[d], xf)[P]
        assert np.all(np.abs(g[d] - (pr.ops.G[d] @ xf)[P]) <= 1e-13 * bound + 1e-300), d
    u = rng.standard_normal((3, P.size))
    uf = np.zeros((3, case.N))
    uf[:, P] = u
    dv = s.apply(ibfe.OP_DIV, u.ravel())
    bound = sum(_abs_bound(pr.mesh, Gf[d], Gc[d], uf[d]) for d in range(3))[P]
    assert np.all(np.abs(dv - pr.ops.divergence(uf)[P]) <= 1e-13 * bound + 1e-300)
    s.close()


@pytest.mark.parametrize("advdiff", [0, 1])
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-6)])
def test_refined_advection_diffusion_apply(precision, tol, advdiff):
    # advdiff 0: rows formed on the fly (matrix-free); 1: assembled 54-plane stencil
    case = _cyl()
    pr = ipcs.Problem.from_case(case)
    s = make_solver(case, advdiff=advdiff)
    P = pr.sets.P
    rng = np.random.default_rng(23)
    a = rng.standard_normal((3, P.size))
    s.set_state(a, np.zeros(P.size), 0.0)
    af = np.zeros((3, case.N))
    af[:, P] = a
    A = (case.rho / case.dt) * pr.ops.M + case.rho * pr.ops.advection(af) + case.mu * pr.ops.K
    x = rng.standard_normal((3, P.size))
    xf = np.zeros((3, case.N))
    xf[:, P] = x
    y = s.apply(ibfe.OP_ADVDIFF, x.ravel(), precision).reshape(3, -1)
    for d in range(3):
        e = rel_l2(y[d], (A @ xf[d])[P])
        say("advdiff", precision, d, e)
        assert e <= tol
    s.close()


@pytest.mark.parametrize("advdiff", [0, 1])
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-6)])
def test_refined_advection_diffusion_apply_strain(precision, tol, advdiff):
    # the composite operator plus the strain-rate cross blocks mu X_dc of the fine
    # and of the unrefined cells (components coupled)
    case = _cyl()
    pr = ipcs.Problem.from_case(case, viscous=1)
    s = make_solver(case, viscous=1, advdiff=advdiff)
    P = pr.sets.P
    rng = np.random.default_rng(29)
    a = rng.standard_normal((3, P.size))
    s.set_state(a, np.zeros(P.size), 0.0)
    af = np.zeros((3, case.N))
    af[:, P] = a
    A = (case.rho / case.dt) * pr.ops.M + case.rho * pr.ops.advection(af) + case.mu * pr.ops.K
    X = pr.ops.strain_cross()
    x = rng.standard_normal((3, P.size))
    xf = np.zeros((3, case.N))
    xf[:, P] = x
    y = s.apply(ibfe.OP_ADVDIFF, x.ravel(), precision).reshape(3, -1)
    for d in range(3):
        ref = A @ xf[d] + case.mu * sum(X[d][c] @ xf[c] for c in range(3))
        e = rel_l2(y[d], ref[P])
        say("advdiff strain", precision, d, e)
        assert e <= tol
    s.close()


def _check(out, tol, label):
    check_steps(out, tol, label)


@pytest.mark.parametrize("make", [_cyl, _aneurysm])
def test_refined_step_parity_fp64(make):
    case = make()
    say("refined case", case.name, "N", case.N, "M", case.M)
    _, out = run_pair(case, 3)
    _check(out, 1e-10, case.name)


@pytest.mark.parametrize("make", [_cyl, _aneurysm])
def test_refined_step_parity_mixed(make):
    case = make()
    say("refined case mixed", case.name)
    _, out = run_pair(case, 3, precision=1)
    _check(out, 1e-6, case.name + " mixed")


def test_refined_without_outlet_null_space():
    """No outlet: the pressure increment is normalised to zero nodal mean."""
    case = _cyl()
    tag = grid.default_tags(2 * case.nx, 2 * case.ny, 2 * case.nz)
    tag[tag == grid.TAG_OUTLET] = grid.TAG_WALL
    case.bc_tag = tag
    rng = np.random.default_rng(24)
    case.u0 = 0.1 * rng.standard_normal((3, case.N))
    say("refined closed", case.name)
    pr, out = run_pair(case, 2)
    assert len(pr.floating) == 1
    _check(out, 1e-10, "refined closed")
    phi = out[-1]["g_phi"]
    assert abs(phi.mean()) < 1e-12 * np.abs(phi).max()


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
@pytest.mark.parametrize("make", [_cyl, _aneurysm])
def test_refined_step_parity_multigrid(make, precision, tol):
    """Pressure increment with the composite-level V-cycle (base grid below it)."""
    case = make()
    say("refined multigrid", case.name, precision)
    _, out = run_pair(case, 3, precision=precision, precond=2)
    _check(out, tol, f"{case.name} mg p{precision}")
    _, out = run_pair(case, 2, precision=precision, precond=2, advdiff=1)
    _check(out, tol, f"{case.name} mg p{precision} stencil")
    _, out_j = run_pair(case, 1, precision=precision, precond=0)
    mg_it, j_it = out[0]["stats"]["s3_iters"], out_j[0]["stats"]["s3_iters"]
    say("s3 iterations: multigrid", mg_it, "Jacobi", j_it)
    assert mg_it < j_it


def test_refined_wall_shear_parity():
    from oracle import wss
    case = _cyl()
    pr = ipcs.Problem.from_case(case)
    s = make_solver(case)
    P = pr.sets.P
    rng = np.random.default_rng(41)
    u = rng.standard_normal((3, P.size))
    s.set_state(u.ravel(), np.zeros(P.size), 0.0)
    uf = np.zeros((3, case.N))
    uf[:, P] = u
    n = case.X.copy()
    n[:, 2] = 0.0
    n /= np.linalg.norm(n, axis=1)[:, None]
    g = s.wall_shear(n)
    o = wss.wall_shear(pr, uf, n)
    err = np.abs(g - o).max() / np.abs(o).max()
    say("refined wall shear rel err", err)
    assert err < 1e-12
    s.close()


@pytest.mark.parametrize("advection", [0, 1])
@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
def test_refined_step_parity_strain_rate_form(precision, tol, advection):
    case = _cyl()
    say("case", case.name, "refined, strain-rate viscous form, precision", precision, "advection", advection)
    _, out = run_pair(case, 3, t0=0.05, precision=precision, precond=2, viscous=1, advection=advection)
    _check(out, tol, case.name + "/strain")
