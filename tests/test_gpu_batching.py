"""GPU tests of the batched mass-correction kernels: solvers stepping from
different threads with a shared batcher, and a server with batching on, give
results bitwise identical to the same solves run alone, and the batches did
carry several requests."""
import threading

import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

CASES = [lambda: synth.small_cylinder(8, 16, pulsatile=True),
         lambda: synth.small_cylinder(10, 20),
         lambda: synth.vessel_case("branch", 1.0, (24, 24, 32), nsteps=3, seed=4),
         lambda: synth.vessel_case("aneurysm", 1.0, (16, 16, 24), nsteps=3, seed=9)]


def _alone(case, nsteps):
    s = ibfe.Solver(**ibfe.inputs_from_case(case, precision=1, precond=2, mass_precond=0))
    s.set_state(np.zeros(3 * s.n_u), np.zeros(s.n_u), 0.0)
    s.step(nsteps)
    u, p, _ = s.get_state()
    it = s.stats()["s4_iters"]
    s.close()
    return u, p, it


def test_threads_with_shared_batcher_bitwise():
    cases = [mk() for mk in CASES]
    ref = [_alone(c, 4) for c in cases]
    say("alone s4 iterations", [r[2] for r in ref])
    solvers = [ibfe.Solver(**ibfe.inputs_from_case(c, precision=1, precond=2, mass_precond=0)) for c in cases]
    b = ibfe.Batcher(window_us=5000.0)
    for s in solvers:
        s.set_state(np.zeros(3 * s.n_u), np.zeros(s.n_u), 0.0)
        b.attach(s)
    errors = []

    def run(s):
        try:
            s.step(4)
        except Exception as e:  # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=run, args=(s,)) for s in solvers]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    st = b.stats()
    say("batcher", st)
    for s, (ua, pa, _) in zip(solvers, ref):
        u, p, _ = s.get_state()
        assert np.array_equal(u, ua) and np.array_equal(p, pa)
        b.detach(s)
        s.close()
    b.close()
    assert st["widest"] >= 2 and st["members"] > st["batches"]


def test_served_with_batching_bitwise():
    cases = [mk() for mk in CASES]
    ref = [_alone(c, 3) for c in cases]
    srv = ibfe.Server(max_slots=4, batch_window_us=5000.0)
    ids = [srv.submit(3, **ibfe.inputs_from_case(c, precision=1, precond=2, mass_precond=0)) for c in cases]
    out = []
    for rid in ids:
        r = srv.wait(rid, 300.0)
        assert r["status"] == ibfe.REQ_DONE, r
        u, p, _ = srv.fetch(rid, r["n_u"], r["n_p"])
        out.append((u, p))
    st = srv.batch_stats()
    srv.close()
    say("server batches", st)
    for (u, p), (ua, pa, _) in zip(out, ref):
        assert np.array_equal(u, ua) and np.array_equal(p, pa)
    assert st["widest"] >= 2


def test_batcher_refuses_destroy_with_members():
    s = ibfe.Solver(**ibfe.inputs_from_case(synth.small_cylinder(8, 16), precision=1, precond=2, mass_precond=0))
    b = ibfe.Batcher()
    b.attach(s)
    with pytest.raises(ibfe.IbfeError):
        b.close()
    b.detach(s)
    b.close()
    s.close()
