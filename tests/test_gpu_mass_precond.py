"""GPU tests of the two preconditioners of the consistent-mass correction
(Sections 2.2 and 2.4): the Jacobi-preconditioned Chebyshev iteration and the one
preconditioned by the tensor-product approximate inverse of the Q1 mass reach
the oracle's step (FP64 and mixed precision, uniform and refined lattices), and
the tensor-product one needs far fewer iterations."""
import pytest

import synth
from gpu_util import check_steps, run_pair, say

pytestmark = pytest.mark.gpu

CASES = {
    "cylinder": lambda: synth.small_cylinder(8, 16, pulsatile=True, nsteps=3),
    "blob": lambda: synth.random_blob_case(seed=3),
    "channel": lambda: synth.channel_case(ic="rest"),
    "aneurysm": lambda: synth.aneurysm_case((16, 16, 40), band=1.2, nsteps=2),
}


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
@pytest.mark.parametrize("name", list(CASES))
def test_mass_preconditioners_reach_the_oracle(name, precision, tol):
    case = CASES[name]()
    iters = {}
    for mp in (0, 1):
        say("case", case.name, "precision", precision, "mass_precond", mp)
        _, out = run_pair(case, 2, precision=precision, precond=2, mass_precond=mp)
        check_steps(out, tol, f"{case.name}/mass{mp}")
        iters[mp] = sum(o["stats"]["s4_iters"] for o in out)
        assert all(o["stats"]["s4_res"] <= (1e-13 if precision == 0 else 1e-8) for o in out)
    say("s4 iterations (Jacobi, tensor)", iters[0], iters[1])
    # two passes per tensor step: fewer than half the Jacobi steps
    assert 2 * iters[1] < iters[0]
