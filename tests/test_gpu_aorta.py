"""GPU checks of the aorta-like arch with three branches: inlet and outlet disks on
the same face, branch outlets on the opposite face, a two-harmonic Womersley-type
inlet and a 5 % active fill of the box.

* quarter resolution (64x40x96): whole-step parity with the oracle, FP64 to 1e-10
  and mixed precision to 1e-6, with the Jacobi and the multigrid pressure solve;
* full size (256x160x384, 15.9 M grid nodes, 0.97 M nodes of P): the derived sets
  bit for bit, sampled operator rows against their definition, and two steps whose
  IB constraint and sub-step equations are checked, with the mixed precision result
  within 1e-6 of the FP64 one."""
import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from gpu_util import make_solver, rel_l2, run_pair, say
from oracle import fem, grid, ib
from test_gpu_parity import _check_steps, _row_apply

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,precond,tol", [(0, 0, 1e-10), (0, 2, 1e-10), (1, 2, 1e-6)])
def test_quarter_aorta_step_parity(precision, precond, tol):
    case = synth.aorta_case(scale=4, spacing=1.5, nsteps=3)
    say("case", case.name, "M", case.M, "precision", precision, "precond", precond)
    _, out = run_pair(case, 3, precision=precision, precond=precond)
    _check_steps(out, tol, f"{case.name}/p{precision}/pc{precond}")


@pytest.fixture(scope="module")
def c4():
    c = synth.aorta_case(scale=1, nsteps=2)
    say("case", c.name, "N", c.N, "M", c.M, "active", int(c.node_mask.sum()))
    return c


@pytest.fixture(scope="module")
def c4_sets(c4):
    return grid.derive_sets(c4.nx, c4.ny, c4.nz, c4.node_mask, c4.bc_tag)


def test_full_size_aorta_sets_and_rows(c4, c4_sets):
    sets = c4_sets
    s = make_solver(c4, precision=1, precond=2)
    assert np.array_equal(s.node_ids(), sets.P)
    P = sets.P
    rng = np.random.default_rng(23)
    x = rng.standard_normal(P.size)
    xf = np.zeros(c4.N)
    xf[P] = x
    Me, Ke, _, _ = fem.element_matrices(c4.h)
    for op, E in ((ibfe.OP_STIFF, Ke), (ibfe.OP_MASS, Me)):
        for prec, tol in ((0, 1e-12), (1, 1e-5)):
            y = s.apply(op, x, prec)
            pick = rng.choice(P.size, 400, replace=False)
            ref = _row_apply(sets, E, xf, P[pick], c4.nx, c4.ny)
            bound = _row_apply(sets, np.abs(E), np.abs(xf), P[pick], c4.nx, c4.ny)
            say("full-size apply", op, prec, "max rel", float(np.max(np.abs(y[pick] - ref) / bound)))
            assert np.all(np.abs(y[pick] - ref) <= tol * bound)
    s.close()


def _run(c4, sets, precision, tol):
    """Two steps from rest; after each, the IB constraint on every point and the
    equations of the pressure increment and of the mass correction on every row,
    evaluated with the library's operator applies (checked row by row above)."""
    s = make_solver(c4, precision=precision, precond=2)
    n = s.n_u
    s.set_state(np.zeros(3 * n), np.zeros(n), 0.0)
    ids = s.node_ids()
    onF = sets.in_F[ids]
    onPp = (sets.in_P & ~sets.p_dir)[ids]
    I = ib.interpolation_matrix(c4.X, c4.nx, c4.ny, c4.nz, c4.h, c4.origin)
    rho, dt = c4.rho, c4.dt
    _, p_prev, _ = s.get_state()
    for k in range(2):
        s.step(1)
        st = s.stats()
        say("precision", precision, "step", k, {x: st[x] for x in ("s1_iters", "ib_iters", "s3_iters", "s4_iters",
                                                                    "s1_res", "s3_res", "s4_res")})
        uib = s.field(ibfe.FIELD_UIB)
        phi = s.field(ibfe.FIELD_PHI)
        u, p, t = s.get_state()
        assert np.isfinite(u).all() and np.isfinite(p).all()
        assert np.allclose(p, p_prev + phi, rtol=0, atol=1e-12 * np.abs(p).max())
        p_prev = p
        uf = np.zeros((3, c4.N))
        uf[:, ids] = uib.reshape(3, -1)
        # the force solve stops at 1e-13 (FP64) or 1e-10 (mixed) relative residual
        for d in range(3):
            assert np.abs(I @ uf[d]).max() < (1e-9 if precision == 0 else 1e-7)
        # pressure increment: K phi = -(rho/dt) B u_ib on the pressure unknowns
        rhs3 = -(rho / dt) * s.apply(ibfe.OP_DIV, uib.ravel(), 0)
        r3 = s.apply(ibfe.OP_STIFF, phi, 0) - rhs3
        e3 = np.abs(r3[onPp]).max() / np.abs(rhs3[onPp]).max()
        # correction: (rho/dt) M (u_ib - u) = G phi on the free rows
        du = (uib - u).reshape(3, -1)
        gphi = s.apply(ibfe.OP_GRAD, phi, 0).reshape(3, -1)
        e4 = max(np.abs(((rho / dt) * s.apply(ibfe.OP_MASS, du[d], 0) - gphi[d])[onF]).max()
                 / np.abs(gphi[d][onF]).max() for d in range(3))
        say("equation residuals: pressure", e3, "correction", e4)
        assert e3 <= tol and e4 <= tol
    u, p, t = s.get_state()
    s.close()
    return u, p


def test_full_size_aorta_steps_fp64_and_mixed(c4, c4_sets):
    u64, p64 = _run(c4, c4_sets, 0, 1e-10)
    u32, p32 = _run(c4, c4_sets, 1, 1e-6)
    eu, ep = rel_l2(u32, u64), rel_l2(p32, p64)
    say("mixed vs FP64 after 2 steps: u", eu, "p", ep)
    assert eu <= 1e-6 and ep <= 1e-6
