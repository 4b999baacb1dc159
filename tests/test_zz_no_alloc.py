"""The allocation-free point update through the C ABI: ibfe_set_points_noalloc
(scratch in the library's static per-GPU array) against ibfe_set_points (scratch
allocated on its first call) on twin contexts.  Two calls in a row share the
static array, the second on a context with fewer points; each is compared with the
allocating entry point bit for bit (the rebuild is deterministic): the IB
interpolation and spreading operators it rebuilt, and a full step that uses G and
its block inverses."""
import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from gpu_util import compact_state, make_solver, say
from oracle import ipcs

pytestmark = pytest.mark.gpu


def _twins(case):
    kw = dict(precision=1, precond=2)
    return make_solver(case, **kw), make_solver(case, **kw)


def _same_rebuild(case, wall, t, seed):
    ref, na = _twins(case)
    X, U = wall.at(t)
    ref.set_points(X, U)
    na.set_points_noalloc(X, U)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(3 * ref.n_u)
    f = rng.standard_normal(3 * ref.M)
    for op, v in ((ibfe.OP_INTERP, x), (ibfe.OP_SPREAD, f)):
        a, b = ref.apply(op, v), na.apply(op, v)
        say(case.name, "M", case.M, "op", op, "max |diff|", float(np.abs(a - b).max()))
        assert np.array_equal(a, b)
    pr = ipcs.Problem.from_case(case)
    u0, p0 = compact_state(pr, *pr.initial_state(case.u0, case.p0))
    for s in (ref, na):
        s.set_state(u0, p0, t - case.dt)
        s.step(1)
    (ua, pa, ta), (ub, pb, tb) = ref.get_state(), na.get_state()
    assert np.array_equal(ua, ub) and np.array_equal(pa, pb) and ta == tb
    assert ref.stats()["ib_iters"] == na.stats()["ib_iters"]
    ref.close()
    na.close()


def test_noalloc_point_update_matches_the_allocating_one():
    big, wall_big = synth.pulsating_cylinder(cells_xy=12, cells_z=24, rings=16, per_ring=20)
    small, wall_small = synth.pulsating_cylinder(cells_xy=8, cells_z=16, rings=8, per_ring=12)
    assert small.M < big.M <= ibfe.Solver.set_points_noalloc_max_points()
    say("max points", ibfe.Solver.set_points_noalloc_max_points())
    _same_rebuild(big, wall_big, 0.07, 1)
    _same_rebuild(small, wall_small, 0.13, 2)


def test_noalloc_point_update_refuses_too_many_points():
    case = synth.pulsatile_c2()
    assert case.M > ibfe.Solver.set_points_noalloc_max_points()
    s = make_solver(case, precision=1, precond=2)
    with pytest.raises(ibfe.IbfeError) as e:
        s.set_points_noalloc(case.X)
    assert e.value.code == -1 and "at most" in str(e.value)
    s.close()
