"""Shared helpers for the GPU parity tests (inputs come from synth, expected values
from the oracle; nothing here computes the method)."""
import sys

import numpy as np

import paper_2007_02082_amd as ibfe
from oracle import ipcs


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def make_solver(case, **kw):
    return ibfe.Solver(**ibfe.inputs_from_case(case, **kw))


def compact_state(pr: ipcs.Problem, u_full: np.ndarray, p_full: np.ndarray):
    P = pr.sets.P
    return np.ascontiguousarray(u_full[:, P]), np.ascontiguousarray(p_full[P])


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def run_pair(case, nsteps, t0=0.0, **solver_kw):
    """Run the oracle and the GPU library from the case's initial state; returns a list
    of per-step dicts with both sides' u*, u_ib, Phi, u, p in canonical order."""
    pr = ipcs.Problem.from_case(case, advection=solver_kw.get("advection", 0),
                                viscous=solver_kw.get("viscous", 0))
    u, p = pr.initial_state(case.u0, case.p0)
    s = make_solver(case, **solver_kw)
    assert (s.node_ids() == pr.sets.P).all()
    cu, cp = compact_state(pr, u, p)
    s.set_state(cu, cp, t0)
    t = t0
    P = pr.sets.P
    out = []
    for _ in range(nsteps):
        u, p, t, info = pr.step(u, p, t)
        s.step(1)
        gu, gp, gt = s.get_state()
        out.append(dict(
            o_u=u[:, P], o_p=p[P], g_u=gu, g_p=gp, o_t=t, g_t=gt,
            o_ustar=info.u_star[:, P], g_ustar=s.field(ibfe.FIELD_USTAR),
            o_uib=info.u_ib[:, P], g_uib=s.field(ibfe.FIELD_UIB),
            o_phi=info.phi[P], g_phi=s.field(ibfe.FIELD_PHI),
            stats=s.stats(), o_iters=info.iters))
    s.close()
    return pr, out
