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


def rel_max(a: np.ndarray, b: np.ndarray, scale: float | None = None) -> float:
    """max |a - b| over every entry, relative to max |b| (or to the given scale)."""
    s = float(np.abs(b).max()) if scale is None and b.size else (scale or 0.0)
    d = float(np.abs(a - b).max()) if b.size else 0.0
    return d / (s if s > 0 else 1.0)


def check_steps(out, tol, label):
    """Every field of every step: relative L2 <= tol and, entry by entry,
    max |gpu - oracle| <= tol * max |oracle| (an error confined to the wall or the
    inlet rows shows in the second even when the first averages it away).  The
    pressure increment is measured against the pressure scale (it vanishes
    identically in some exact solutions)."""
    import pytest

    for k, r in enumerate(out):
        errs = {f: rel_l2(r["g_" + f], r["o_" + f]) for f in ("ustar", "uib", "u", "p")}
        floor = max(np.linalg.norm(r["o_phi"]), np.linalg.norm(r["o_p"]))
        errs["phi"] = float(np.linalg.norm(r["g_phi"] - r["o_phi"]) / (floor if floor > 0 else 1.0))
        emax = {f: rel_max(r["g_" + f], r["o_" + f]) for f in ("ustar", "uib", "u", "p")}
        pscale = max(float(np.abs(r["o_phi"]).max()), float(np.abs(r["o_p"]).max()))
        emax["phi"] = rel_max(r["g_phi"], r["o_phi"], pscale)
        say(f"{label} step {k}: L2 " + " ".join(f"{f}={e:.2e}" for f, e in errs.items()),
            "| max " + " ".join(f"{f}={e:.2e}" for f, e in emax.items()),
            "| gpu iters", {x: r["stats"][x] for x in ("s1_iters", "ib_iters", "s3_iters", "s4_iters")})
        assert r["g_t"] == pytest.approx(r["o_t"], abs=1e-15)
        for f in errs:
            assert errs[f] <= tol, (label, k, f, "L2", errs[f])
            assert emax[f] <= tol, (label, k, f, "max", emax[f])


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
