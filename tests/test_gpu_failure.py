"""Failure paths and checkpoints through the C ABI: a failed step keeps the last
completed state, a restart from a checkpoint continues bit for bit, and a BiCGStab
breakdown (forced from the host) is recovered by a restart without changing the
result beyond the solver tolerance.  All conditions are normal error returns: no
kernel faults or waits here."""
import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from gpu_util import check_steps, compact_state, make_solver, say
from oracle import ipcs

pytestmark = pytest.mark.gpu


def _state_after(case, nsteps, **kw):
    s = make_solver(case, **kw)
    pr = ipcs.Problem.from_case(case)
    s.set_state(*compact_state(pr, *pr.initial_state(case.u0, case.p0)), 0.0)
    s.step(nsteps)
    u, p, t = s.get_state()
    s.close()
    return u, p, t


@pytest.mark.parametrize("precision", [0, 1])
def test_iteration_cap_keeps_the_last_state(precision):
    case = synth.small_cylinder(8, 16, pulsatile=True)
    u, p, t = _state_after(case, 2, precision=precision, precond=2)
    say("iteration cap, precision", precision)
    s = make_solver(case, precision=precision, precond=2, max_iters=1)
    s.set_state(u.ravel(), p, t)
    for _ in range(2):
        with pytest.raises(ibfe.IbfeError) as e:
            s.step(1)
        assert e.value.code == -4, str(e.value)          # IBFE_ENOCONV
        gu, gp, gt = s.get_state()
        assert np.array_equal(gu, u) and np.array_equal(gp, p) and gt == t
        assert s.stats()["steps"] == 0
    s.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_non_finite_state_is_reported_and_kept(precision):
    case = synth.small_cylinder(8, 16, pulsatile=True)
    u, p, t = _state_after(case, 1, precision=precision)
    bad = u.copy()
    bad[2, bad.shape[1] // 2] = np.nan
    say("non-finite input, precision", precision)
    s = make_solver(case, precision=precision)
    s.set_state(bad.ravel(), p, t)
    with pytest.raises(ibfe.IbfeError) as e:
        s.step(1)
    assert e.value.code == -5, str(e.value)              # IBFE_ENONFINITE
    gu, gp, gt = s.get_state()
    assert np.array_equal(gu, bad, equal_nan=True) and np.array_equal(gp, p) and gt == t
    # the context recovers: a finite state steps exactly as in a fresh context
    s.set_state(u.ravel(), p, t)
    s.step(1)
    ref = make_solver(case, precision=precision)
    ref.set_state(u.ravel(), p, t)
    ref.step(1)
    a, b = s.get_state(), ref.get_state()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    s.close()
    ref.close()


CASES = {
    "cylinder_mixed_mg": (lambda: synth.small_cylinder(8, 16, pulsatile=True), dict(precision=1, precond=2)),
    "blob_fp64": (lambda: synth.random_blob_case(seed=3), dict(precision=0)),
    "refined_mixed_mg": (lambda: synth.refined_cylinder(8, 8, length=1.25, band=0.3),
                         dict(precision=1, precond=2)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_checkpoint_restart_is_bitwise(name):
    make, kw = CASES[name]
    case = make()
    pr = ipcs.Problem.from_case(case)
    u0, p0 = compact_state(pr, *pr.initial_state(case.u0, case.p0))
    n, k = 6, 3
    say("checkpoint", name, "steps", n, "save after", k)
    full = make_solver(case, **kw)
    full.set_state(u0, p0, 0.05)
    full.step(n)
    uf, pf, tf = full.get_state()
    full.close()

    first = make_solver(case, **kw)
    first.set_state(u0, p0, 0.05)
    first.step(k)
    blob = first.checkpoint()
    uk, pk, tk = first.get_state()
    first.close()

    second = make_solver(case, **kw)
    second.load_checkpoint(blob)
    u2, p2, t2 = second.get_state()
    assert np.array_equal(u2, uk) and np.array_equal(p2, pk) and t2 == tk
    assert second.stats()["steps"] == k
    second.step(n - k)
    u2, p2, t2 = second.get_state()
    say("max |diff| after restart:", float(np.abs(u2 - uf).max()), float(np.abs(p2 - pf).max()))
    assert np.array_equal(u2, uf) and np.array_equal(p2, pf) and t2 == tf
    assert second.stats()["steps"] == n
    second.close()

    # a plain set_state restart starts the solvers cold: equal within the tolerance only
    cold = make_solver(case, **kw)
    cold.set_state(uk.ravel(), pk, tk)
    cold.step(n - k)
    uc, pc, _ = cold.get_state()
    cold.close()
    tol = 1e-6 if kw.get("precision") == 1 else 1e-10
    assert np.linalg.norm(uc - uf) <= tol * np.linalg.norm(uf)


def test_checkpoint_of_another_problem_is_refused():
    a = make_solver(synth.small_cylinder(8, 16))
    b = make_solver(synth.small_cylinder(8, 8, length=1.0))
    blob = a.checkpoint()
    with pytest.raises(ibfe.IbfeError) as e:
        b.load_checkpoint(blob)
    assert e.value.code == -1
    with pytest.raises(ibfe.IbfeError):
        a.load_checkpoint(blob[:100])
    with pytest.raises(ibfe.IbfeError):
        a.load_checkpoint(b"\0" * len(blob))
    a.close()
    b.close()


@pytest.mark.parametrize("precision,tol,at", [(0, 1e-10, 2), (1, 1e-6, 1)])
def test_forced_breakdown_restarts_and_matches_the_oracle(precision, tol, at):
    """A breakdown reported by the tentative-velocity BiCGStab restarts the method
    from its current iterate with a fresh shadow residual; the step still reaches the
    oracle's solution, and the iteration total stays within the cap."""
    case = synth.small_cylinder(8, 16, pulsatile=True, nsteps=3)
    pr = ipcs.Problem.from_case(case)
    u, p = pr.initial_state(case.u0, case.p0)
    maxit = 400
    s = make_solver(case, precision=precision, max_iters=maxit)
    s.set_state(*compact_state(pr, u, p), 0.0)
    P = pr.sets.P
    t = 0.0
    out = []
    restarts = 0
    for k in range(3):
        u, p, t, info = pr.step(u, p, t)
        s.inject_breakdown(at)
        s.step(1)
        st = s.stats()
        restarts += st["s1_restarts"]
        say("precision", precision, "step", k, "s1 iters", st["s1_iters"], "restarts", st["s1_restarts"])
        assert st["s1_iters"] <= maxit * max(1, st["s1_outer"])
        gu, gp, gt = s.get_state()
        out.append(dict(o_u=u[:, P], o_p=p[P], g_u=gu, g_p=gp, o_t=t, g_t=gt,
                        o_ustar=info.u_star[:, P], g_ustar=s.field(ibfe.FIELD_USTAR),
                        o_uib=info.u_ib[:, P], g_uib=s.field(ibfe.FIELD_UIB),
                        o_phi=info.phi[P], g_phi=s.field(ibfe.FIELD_PHI), stats=st))
    assert restarts >= 3                       # one per step at least
    check_steps(out, tol, f"forced breakdown/{precision}")
    # cancelled injection: no restart
    s.inject_breakdown(0)
    s.step(1)
    assert s.stats()["s1_restarts"] == 0
    s.close()
