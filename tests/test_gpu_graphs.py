"""GPU: the solves replayed through captured HIP graphs give bitwise the same
states as eager launches, over several steps (many replays of each graph) with
eager work (operator applies, state reads) between them."""
import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from gpu_util import make_solver, say

pytestmark = pytest.mark.gpu


def _run(case, graphs, nsteps, **kw):
    s = make_solver(case, **kw)
    s.set_graphs(graphs)
    n = s.n_u
    s.set_state(np.zeros(3 * n), np.zeros(n), 0.0)
    x = np.random.default_rng(5).standard_normal(n)
    out = []
    for k in range(nsteps):
        s.step(1)
        u, p, _ = s.get_state()
        y = s.apply(ibfe.OP_STIFF, x)          # eager work between the replays
        out.append((u.copy(), p.copy(), y, s.stats()["s3_iters"]))
    s.close()
    return out


@pytest.mark.parametrize("make,kw", [
    (lambda: synth.small_cylinder(12, 24, pulsatile=True), dict(precision=1, precond=2)),
    (lambda: synth.small_cylinder(12, 24, pulsatile=True), dict(precision=0, precond=0)),
    (lambda: synth.refined_cylinder(8, 8, length=1.25, band=0.3), dict(precision=1, precond=2)),
    (lambda: synth.vessel_case("aneurysm", 1.0, (16, 16, 24), seed=7), dict(precision=0, precond=2)),
])
def test_graph_replay_equals_eager(make, kw):
    case = make()
    say("graphs vs eager:", case.name, kw)
    eager = _run(case, False, 6, **kw)
    graph = _run(case, True, 6, **kw)
    for k, (a, b) in enumerate(zip(eager, graph)):
        say("step", k, "s3 iters", a[3], b[3])
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), k
        assert np.array_equal(a[2], b[2])
