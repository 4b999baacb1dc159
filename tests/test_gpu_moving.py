"""Moving Lagrangian points on the GPU: the device rebuild of the IB operators
(stencils, spreading lists, G = I_F I_F^T and its block inverses) against the
oracle, which rebuilds I from its definition at every step.  A radially pulsating
vessel wall (prescribed positions and velocities) is stepped on both sides; the
rebuild at the initial positions reproduces the static plan; the same motion gives
bit-identical states on two contexts; error paths keep the context safe."""
import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from gpu_util import compact_state, make_solver, run_pair, say
from oracle import ipcs
from test_gpu_parity import TOL64, TOL_MIXED, _check_steps

pytestmark = pytest.mark.gpu


def _run_moving(case, wall, nsteps, t0, **kw):
    """Both sides move the points to X(t^{n+1}) with U_B(t^{n+1}) before each step."""
    pr = ipcs.Problem.from_case(case, advection=kw.get("advection", 0))
    u, p = pr.initial_state(case.u0, case.p0)
    s = make_solver(case, **kw)
    s.set_state(*compact_state(pr, u, p), t0)
    P = pr.sets.P
    t = t0
    out = []
    for _ in range(nsteps):
        X, U = wall.at(t + case.dt)
        pr.set_points(X, U)
        s.set_points(X, U)
        u, p, t, info = pr.step(u, p, t)
        s.step(1)
        gu, gp, gt = s.get_state()
        out.append(dict(o_u=u[:, P], o_p=p[P], g_u=gu, g_p=gp, o_t=t, g_t=gt,
                        o_ustar=info.u_star[:, P], g_ustar=s.field(ibfe.FIELD_USTAR),
                        o_uib=info.u_ib[:, P], g_uib=s.field(ibfe.FIELD_UIB),
                        o_phi=info.phi[P], g_phi=s.field(ibfe.FIELD_PHI),
                        stats=s.stats(), o_iters=info.iters))
        # the constraint holds at the new positions: I u_ib = U_B
        Iu = np.stack([pr.I @ info.u_ib[d] for d in range(3)], axis=1)
        assert np.abs(Iu - U).max() <= 1e-8 * max(1.0, np.abs(U).max())
    s.close()
    return out


@pytest.mark.parametrize("precision,tol", [(0, TOL64), (1, TOL_MIXED)])
def test_moving_wall_step_parity(precision, tol):
    case, wall = synth.pulsating_cylinder(nsteps=4)
    say("case", case.name, "M", case.M, "precision", precision)
    out = _run_moving(case, wall, 4, 0.0, precision=precision, precond=2)
    _check_steps(out, tol, case.name)


def test_moving_wall_explicit_advection_parity():
    case, wall = synth.pulsating_cylinder(cells_xy=8, cells_z=16, nsteps=3)
    out = _run_moving(case, wall, 3, 0.05, precision=0, precond=2, advection=1)
    _check_steps(out, TOL64, case.name + "/explicit")


def test_rebuild_at_initial_positions_matches_static_plan():
    case = synth.small_cylinder(8, 16, pulsatile=True, nsteps=3)
    _, ref = run_pair(case, 3, t0=0.05, precision=0, precond=2)
    pr = ipcs.Problem.from_case(case)
    u, p = pr.initial_state(case.u0, case.p0)
    s = make_solver(case, precision=0, precond=2)
    s.set_state(*compact_state(pr, u, p), 0.05)
    s.set_points(case.X, case.U_B)
    for k in range(3):
        s.step(1)
        gu, gp, _ = s.get_state()
        e = np.linalg.norm(gu - ref[k]["g_u"]) / np.linalg.norm(ref[k]["g_u"])
        say("step", k, "rebuilt vs static plan", e, s.stats()["ib_iters"], ref[k]["stats"]["ib_iters"])
        assert e <= 1e-12
        assert np.linalg.norm(gp - ref[k]["g_p"]) <= 1e-12 * max(1.0, np.linalg.norm(ref[k]["g_p"]))
    s.close()


def test_moving_points_are_deterministic():
    case, wall = synth.pulsating_cylinder(nsteps=3)
    states = []
    for _ in range(2):
        s = make_solver(case, precision=1, precond=2)
        pr = ipcs.Problem.from_case(case)
        s.set_state(*compact_state(pr, *pr.initial_state(case.u0, case.p0)), 0.0)
        t = 0.0
        for _ in range(3):
            s.set_points(*wall.at(t + case.dt))
            s.step(1)
            t += case.dt
        states.append(s.get_state())
        s.close()
    assert np.array_equal(states[0][0], states[1][0]) and np.array_equal(states[0][1], states[1][1])


def test_set_points_errors_keep_the_context_safe():
    case, wall = synth.pulsating_cylinder(nsteps=1)
    s = make_solver(case, precision=0, precond=2)
    far = case.X.copy()
    far[5] = [100.0, 100.0, 100.0]      # support outside the grid: no free node
    with pytest.raises(ibfe.IbfeError, match="ESINGULAR"):
        s.set_points(far)
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        s.step(1)
    bad = case.X.copy()
    bad[0, 0] = np.nan
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        s.set_points(bad)
    s.set_points(*wall.at(case.dt))
    s.step(1)
    s.close()


@pytest.mark.parametrize("precision,tol", [(0, TOL64), (1, TOL_MIXED)])
def test_moving_wall_refined_lattice_parity(precision, tol):
    """Moving points on the 2:1 refined lattice: the kernel on the fine lattice, the
    supports re-checked against the band at every rebuild, against the oracle."""
    case, wall = synth.pulsating_refined_cylinder(nsteps=3)
    say("case", case.name, "M", case.M, "precision", precision)
    out = _run_moving(case, wall, 3, 0.0, precision=precision, precond=2)
    _check_steps(out, tol, case.name)


def test_refined_points_leaving_the_band_are_refused():
    case, wall = synth.pulsating_refined_cylinder(nsteps=1)
    X, U = wall.at(case.dt)
    inward = X * np.array([0.6, 0.6, 1.0])   # supports reach the unrefined core
    pr = ipcs.Problem.from_case(case)
    with pytest.raises(ValueError):
        pr.set_points(inward, U)
    s = make_solver(case, precision=0, precond=2)
    with pytest.raises(ibfe.IbfeError, match="refined band"):
        s.set_points(inward, U)
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        s.step(1)
    s.set_points(X, U)
    s.step(1)
    s.close()


def test_set_points_from_device_tensors():
    """Device pointers (CUDA tensors) give the same rebuild as host arrays."""
    import torch

    case, wall = synth.pulsating_cylinder(nsteps=2)
    pr = ipcs.Problem.from_case(case)
    states = []
    for on_device in (False, True):
        s = make_solver(case, precision=0, precond=2)
        s.set_state(*compact_state(pr, *pr.initial_state(case.u0, case.p0)), 0.0)
        t = 0.0
        for _ in range(2):
            X, U = wall.at(t + case.dt)
            if on_device:
                s.set_points(torch.tensor(X, device="cuda"), torch.tensor(U, device="cuda"))
            else:
                s.set_points(X, U)
            s.step(1)
            t += case.dt
        states.append(s.get_state())
        s.close()
    assert np.array_equal(states[0][0], states[1][0]) and np.array_equal(states[0][1], states[1][1])


def test_translating_ring_band_changes_the_force_pattern():
    """A band of wall rings moved along the axis by 0.8 h per step (with the wall held
    at rest: U_B is an input of its own, and a wall speed of 0.8 h / dt would dominate
    the flow): the supports, the spreading lists and the sparsity of G change from
    step to step; every step against the oracle (FP64), and the empty point set is
    accepted."""
    case = synth.small_cylinder(8, 16, nsteps=3)
    th = 2 * np.pi * np.arange(12) / 12
    zl = np.array([0.6, 0.75, 0.9, 1.05])
    zz, tt = np.meshgrid(zl, th, indexing="ij")
    X0 = np.stack([0.5 * np.cos(tt).ravel(), 0.5 * np.sin(tt).ravel(), zz.ravel()], axis=1)
    v = 0.8 * case.h / case.dt
    U = np.zeros_like(X0)
    case.X, case.U_B = X0, U
    case.dS = 0.1 * case.h

    class Translate:
        def at(self, t):
            return X0 + np.array([0.0, 0.0, v * t]), U

    out = _run_moving(case, Translate(), 3, 0.0, precision=0, precond=2)
    _check_steps(out, TOL64, "translating band")
    # no points at all: a no-op
    c0 = synth.small_cylinder(8, 16, nsteps=1)
    c0.X = np.zeros((0, 3))
    c0.U_B = None
    s = make_solver(c0, precision=0)
    s.set_points(np.zeros((0, 3)))
    s.step(1)
    s.close()


def test_too_dense_points_are_rejected():
    """All 96 points inside half a cell: a row of G would gather 64 x 96 support
    products, more than the 1024 a row holds; the rebuild reports IBFE_EINVAL (the kernel checks the count
    before it stages anything) and the context refuses to step until valid points
    are set."""
    case, wall = synth.pulsating_cylinder(nsteps=1)
    s = make_solver(case, precision=0, precond=2)
    rng = np.random.default_rng(5)
    dense = case.X.copy()
    dense[:] = np.array([0.3, 0.0, 1.0]) + 0.5 * case.h * rng.random((case.M, 3))
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        s.set_points(dense)
    with pytest.raises(ibfe.IbfeError, match="EINVAL"):
        s.step(1)
    s.set_points(*wall.at(case.dt))
    s.step(1)
    s.close()
