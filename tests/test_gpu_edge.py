"""GPU parity on the degenerate cases of the step: no Lagrangian points (the IB
correction is the identity), no free velocity node at all (every sub-step has an
empty or a pure null-space system), and a closed box whose only free nodes are
interior (pressure null space with a tiny free set)."""
import numpy as np
import pytest

import synth
from gpu_util import run_pair, say
from test_gpu_parity import TOL64, TOL_MIXED, _check_steps

pytestmark = pytest.mark.gpu


def _no_points():
    c = synth.small_cylinder(8, 16, pulsatile=True)
    c.X = np.zeros((0, 3))
    c.U_B = None
    return c


def _single_cell():
    # a 1x1x1 box: every node is a corner, hence wall: F is empty, no outlet
    c = synth.random_blob_case(cells=(1, 1, 1), seed=2, n_points=0)
    c.node_mask[:] = 1
    return c


def _closed_box_no_points():
    c = synth.closed_box(3)
    c.X = np.zeros((0, 3))
    c.U_B = None
    return c


@pytest.mark.parametrize("precision,tol", [(0, TOL64), (1, TOL_MIXED)])
@pytest.mark.parametrize("make", [_no_points, _single_cell, _closed_box_no_points])
def test_degenerate_step_parity(make, precision, tol):
    case = make()
    say("case", case.name, "M", case.M, "precision", precision)
    _, out = run_pair(case, 2, t0=0.05, precision=precision, precond=2)
    for r in out:
        assert r["stats"]["ib_iters"] == 0
    if case.M == 0 and make is _single_cell:
        for r in out:
            assert np.all(r["g_u"] == 0.0) and np.all(r["o_u"] == 0.0)
    _check_steps(out, tol, case.name + "/degenerate")
