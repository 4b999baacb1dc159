"""GPU tests of the serving loop: a served request equals the direct run, results
are bitwise identical alone and in a concurrent mix, admission respects the
memory budget, and served synthetic vessels match the oracle."""
import numpy as np
import pytest

import paper_2007_02082_amd as ibfe
import synth
from gpu_util import rel_l2, say
from oracle import ipcs

pytestmark = pytest.mark.gpu


def _kw(case, **extra):
    return ibfe.inputs_from_case(case, **extra)


def _run_direct(case, nsteps, **extra):
    s = ibfe.Solver(**_kw(case, **extra))
    n = s.n_u
    s.set_state(np.zeros(3 * n), np.zeros(n), 0.0)
    s.step(nsteps)
    u, p, _ = s.get_state()
    ids = s.node_ids()
    s.close()
    return u, p, ids


def _serve(server, case, nsteps, **extra):
    return server.submit(nsteps, **_kw(case, **extra))


def _collect(server, rid):
    r = server.wait(rid, 300.0)
    assert r["status"] == ibfe.REQ_DONE, r
    u, p, ids = server.fetch(rid, r["n_u"], r["n_p"])
    return r, u, p, ids


def test_served_request_equals_direct_run():
    case = synth.small_cylinder(8, 16, pulsatile=True)
    say("served vs direct:", case.name)
    ud, pd, idd = _run_direct(case, 4, precision=1, precond=2)
    srv = ibfe.Server(max_slots=2)
    rid = _serve(srv, case, 4, precision=1, precond=2)
    r, u, p, ids = _collect(srv, rid)
    srv.close()
    assert (ids == idd).all()
    assert np.array_equal(u, ud) and np.array_equal(p, pd)
    assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


def test_alone_and_in_mix_are_bitwise_identical():
    target = synth.vessel_case("aneurysm", 1.0, (16, 16, 24), nsteps=6, seed=7)
    others = [synth.vessel_case("branch", 0.7, (16, 16, 16), seed=1),
              synth.vessel_case("cylinder", 1.3, (24, 24, 24)),
              synth.small_cylinder(12, 24),
              synth.vessel_case("aneurysm", 0.5, (32, 32, 32), seed=3),
              synth.vessel_case("branch", 2.0, (24, 24, 32), seed=9)]
    say("alone")
    srv = ibfe.Server(max_slots=1)
    _, ua, pa, _ = _collect(srv, _serve(srv, target, 6, precision=1, precond=2))
    srv.close()
    say("in a mix of", len(others) + 1)
    srv = ibfe.Server(max_slots=4)
    ids = [_serve(srv, c, 6, precision=1, precond=2) for c in others[:2]]
    tid = _serve(srv, target, 6, precision=1, precond=2)
    ids += [_serve(srv, c, 6, precision=1, precond=2) for c in others[2:]]
    _, um, pm, _ = _collect(srv, tid)
    for rid in ids:
        _collect(srv, rid)
    peak = srv.peak_concurrency()
    srv.close()
    say("peak concurrency", peak)
    assert peak >= 2
    assert np.array_equal(ua, um) and np.array_equal(pa, pm)


def test_admission_respects_budget():
    cases = [synth.small_cylinder(8, 16), synth.small_cylinder(10, 20), synth.small_cylinder(12, 24)]
    fps = [ibfe.request_footprint(**_kw(c, precision=1, precond=2)) for c in cases]
    budget = int(1.05 * max(fps))          # room for exactly one at a time
    assert budget < min(fps[0] + fps[1], fps[1] + fps[2], fps[0] + fps[2])
    srv = ibfe.Server(budget_bytes=budget, max_slots=4)
    ids = [_serve(srv, c, 3, precision=1, precond=2) for c in cases]
    big = synth.small_cylinder(16, 32)
    rbig = _serve(srv, big, 3, precision=1, precond=2)
    spans = []
    for rid in ids:
        r, _, _, _ = _collect(srv, rid)
        spans.append((r["t_admit"], r["t_done"]))
    rb = srv.wait(rbig, 10.0)
    peak = srv.peak_concurrency()
    srv.close()
    say("spans", spans, "peak", peak, "big", rb["status"], rb["error"])
    assert peak == 1
    spans.sort()
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert b0 >= a1 - 1e-6
    assert rb["status"] == ibfe.REQ_FAILED and rb["error"] == -2


@pytest.mark.parametrize("kind", ["cylinder", "aneurysm", "branch"])
def test_served_vessels_match_oracle(kind):
    case = synth.vessel_case(kind, 1.0, (16, 16, 16), nsteps=3, seed=11)
    say("served", case.name, "vs oracle")
    pr = ipcs.Problem.from_case(case)
    u, p, _, _ = pr.run(case.u0, case.p0, 3)
    srv = ibfe.Server(max_slots=2)
    rid64 = _serve(srv, case, 3, precision=0, precond=2)
    rid32 = _serve(srv, case, 3, precision=1, precond=2)
    _, u64, p64, ids = _collect(srv, rid64)
    _, u32, p32, _ = _collect(srv, rid32)
    srv.close()
    assert (ids == pr.sets.P).all()
    P = pr.sets.P
    e64 = (rel_l2(u64, u[:, P]), rel_l2(p64, p[P]))
    e32 = (rel_l2(u32, u[:, P]), rel_l2(p32, p[P]))
    say("fp64", e64, "mixed", e32)
    assert max(e64) <= 1e-10 and max(e32) <= 1e-6


def test_request_footprint_bounds_real_allocation():
    """The admission footprint is an upper bound of what a request really allocates
    (largest serving grid, 128 x 128 x 256 cells)."""
    import torch
    case = synth.vessel_case("cylinder", 1.0, (128, 128, 256), nsteps=2, seed=5)
    kw = _kw(case, precision=1, precond=2)
    fp = ibfe.request_footprint(**kw)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    s = ibfe.Solver(**kw)
    s.set_state(np.zeros(3 * s.n_u), np.zeros(s.n_u), 0.0)
    s.step(1)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    s.close()
    used = free0 - free1
    say("footprint", fp, "allocated", used)
    assert 0 < used <= fp


def test_request_stream_under_4gb_budget():
    """Serving requests of the seeded stream (grids up to 128 x 128 x 256) under a
    4 GiB device budget and more slots than requests, so that only memory limits
    admission: every request completes, some request waits for another to finish,
    the footprints of the requests running at any admission never exceed the
    budget, and the largest request's result is bitwise the one it has alone."""
    budget = 4 << 30
    reqs = synth.request_stream(n=16, nsteps=2)
    kws = [_kw(r.case, precision=1, precond=2) for r in reqs]
    fps = [ibfe.request_footprint(**kw) for kw in kws]
    say("footprints GiB", [round(f / 2**30, 2) for f in fps])
    assert max(fps) <= budget < sum(fps)
    srv = ibfe.Server(budget_bytes=budget, max_slots=16)
    ids = [srv.submit(2, **kw) for kw in kws]
    res = []
    for rid in ids:
        r, u, p, _ = _collect(srv, rid)
        res.append((r, u, p))
    peak = srv.peak_concurrency()
    srv.close()
    spans = [(r["t_admit"], r["t_done"], r["footprint"]) for r, _, _ in res]
    for a, _, _ in spans:
        held = sum(f for a2, d2, f in spans if a2 <= a < d2)
        assert held <= budget, (a, held)
    first_done = min(d for _, d, _ in spans)
    waited = [k for k, (a, _, _) in enumerate(spans) if a >= first_done]
    say("peak concurrency", peak, "requests admitted after a completion", len(waited))
    assert waited and peak >= 2
    big = int(np.argmax(fps))
    ua, pa, _ = _run_direct(reqs[big].case, 2, precision=1, precond=2)
    assert np.array_equal(res[big][1], ua) and np.array_equal(res[big][2], pa)
