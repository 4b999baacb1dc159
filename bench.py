"""Benchmark: IPCS + BCE-IB time steps per second on one MI355X.

Workload: pulsatile flow in a cylinder of radius 0.5 and length 8 on a 64x64x512
Q1 grid (2.17 M nodes, 1.78 M pressure/velocity nodes after domain reduction),
25,600 Lagrangian wall points, inlet u_max(t) = 1 + 0.5 sin(2 pi t), dt = 0.005,
synthetic inputs.  One step = tentative velocity solve, IB force solve and
spreading, pressure increment solve, velocity/pressure correction, all on the GPU.

Prints one JSON line.  The dominant kernel (the masked Q1 stiffness apply inside
the pressure CG) is timed with HIP events on the library's stream over the timed
region; its algorithmic bytes are (2 s + 0.125) per pressure node (read x, write
y, s bytes per value, plus the domain bits), s = 4 in mixed mode, 8 in FP64 mode.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2007_02082_amd", "csrc")


def counted_traffic(precision: str):
    """HBM bytes per dispatch of the pressure apply from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size), or None when the
    kernel sources changed after the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"pressure_apply_traffic_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for name in ("kernels.hpp", "zblock.hpp"):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return rec["traffic_bytes"] if h.hexdigest()[:16] == rec["source_hash"] else None
METRIC = "IPCS steps/sec + apply HBM GB/s at 1e-6 rel; served solves/sec, p50/p99"


def cpu_baseline(seconds_hint: float = 15.0) -> dict:
    """Oracle (FP64, numpy/scipy, one thread) on a bounded sample: a 64x64x64-cell slab
    of the same cylinder (same h, mask rule, point density and inlet), two steps after
    set-up; seconds per step scaled by the ratio of pressure nodes to the full grid."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import ipcs

    full = synth.pulsatile_c2()
    slab = synth.cylinder_case("pulsatile_slab_64x64x64", 64, 64, 1.0, 1.0, 0.5, 32, 100,
                               rho=1.0, mu=0.01, dt=0.005, nsteps=2, pulsatile_amp=0.5)
    with threadpool_limits(1):
        pr = ipcs.Problem.from_case(slab)
        u, p = pr.initial_state(slab.u0, slab.p0)
        t = 0.0
        t0 = time.perf_counter()
        nsteps = 0
        while nsteps < 2 or (time.perf_counter() - t0) < 0.3 * seconds_hint and nsteps < 4:
            u, p, t, _ = pr.step(u, p, t)
            nsteps += 1
        sec_per_step = (time.perf_counter() - t0) / nsteps
    from oracle import grid
    n_full = grid.derive_sets(full.nx, full.ny, full.nz, full.node_mask, None).P.size
    scale = n_full / pr.sets.P.size
    return {"value": 1.0 / (sec_per_step * scale), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{nsteps} oracle steps of a 64x64x64-cell slab of the same cylinder "
                      f"({pr.sets.P.size} nodes, {sec_per_step:.2f} s/step), scaled by the "
                      f"node ratio {scale:.2f} to the 64x64x512 grid"}


def serve_stream(n: int, slots: int, nsteps: int) -> dict:
    """Serving stream: n seeded requests (cylinder / aneurysm / Y-branch vessels, radius
    0.4-2.5, grids 32^3 .. 128x128x256, 50 steps each, mixed precision, multigrid) submitted
    at their Poisson arrival times (4 per second) to a server with `slots` concurrent
    slots; latency = completion - submission, solves/s = n / (last completion - first
    submission)."""
    import numpy as np

    import paper_2007_02082_amd as ibfe
    import synth

    reqs = synth.request_stream(n=n, nsteps=nsteps)
    kws = [ibfe.inputs_from_case(r.case, precision=1, precond=2) for r in reqs]
    srv = ibfe.Server(max_slots=slots)
    ids = []
    t0 = time.perf_counter()
    for r, kw in zip(reqs, kws):
        delay = r.arrival - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        ids.append(srv.submit(nsteps, **kw))
    res = [srv.wait(i) for i in ids]
    peak = srv.peak_concurrency()
    for i, r in zip(ids, res):
        if r["status"] == ibfe.REQ_DONE:
            srv.fetch(i, r["n_u"], r["n_p"])
    srv.close()
    failed = sum(r["status"] != ibfe.REQ_DONE for r in res)
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    wait = np.array([r["t_admit"] - r["t_submit"] for r in res])
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    busy = sum(r["t_done"] - r["t_admit"] for r in res)
    nodes = [int(kw["node_mask"].size) for kw in kws]

    def nearest_rank(a, q):
        a = np.sort(a)
        return float(a[max(0, int(np.ceil(q * len(a))) - 1)])

    return {"requests": n, "failed": failed, "steps_each": nsteps, "slots": slots,
            "solves_per_s": round(n / span, 3), "p50_latency_s": round(nearest_rank(lat, 0.5), 3),
            "p99_latency_s": round(nearest_rank(lat, 0.99), 3), "mean_latency_s": round(float(lat.mean()), 3),
            "mean_admission_wait_s": round(float(wait.mean()), 3),
            "mean_concurrency": round(busy / span, 2), "peak_concurrency": peak,
            "wall_s": round(span, 2), "grid_nodes_total": int(sum(nodes))}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--precond", choices=["mg", "jacobi"], default="mg",
                    help="pressure preconditioner: geometric multigrid or Jacobi")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check", action="store_true",
                    help="also run the same steps in FP64 mode and report the difference")
    ap.add_argument("--serve", action="store_true",
                    help="also run the serving stream (64 requests, Poisson arrivals at 4/s)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the run, copy a device buffer of this size 5 times (a plain copy "
                         "kernel of known size for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the boxes have one GPU); --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2007_02082_amd as ibfe
    import synth

    torch.cuda.set_device(0)
    case = synth.pulsatile_c2()
    prec = 1 if args.precision == "mixed" else 0
    pc = 2 if args.precond == "mg" else 0
    s = ibfe.Solver(**ibfe.inputs_from_case(case, precision=prec, precond=pc))
    n = s.n_u
    u0 = np.zeros(3 * n)
    p0 = np.zeros(n)
    s.set_state(u0, p0, 0.0)
    s.step(args.warmup)
    torch.cuda.synchronize()
    s.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = s.stats()
    s.set_kernel_timing(False)
    ms_per_step = 1e3 * elapsed / args.steps

    bytes_per_value = 4 if prec == 1 else 8
    n_p = s.n_p
    alg_bytes = (2 * bytes_per_value + 0.125) * n_p
    avg_ms = st["poisson_apply_ms"] / max(1, st["poisson_applies"])
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = counted_traffic(args.precision) if pc == 2 else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(traffic) if traffic else None,
            "kernel": "k_cg_q_zb<%s,1> (masked Q1 stiffness apply + p.q)" % (
                "float" if prec == 1 else "double"), "avg_us": round(avg_ms * 1e3, 3),
            "launches": st["poisson_applies"], "alg_bytes_per_launch": int(alg_bytes)}

    extra = {"iters_last_step": {k: st[k] for k in ("s1_iters", "ib_iters", "s3_iters", "s4_iters",
                                                      "s1_outer", "s3_outer", "s4_outer")}}
    if args.check:
        u_a, p_a, _ = s.get_state()
        ref = ibfe.Solver(**ibfe.inputs_from_case(case, precision=0, precond=pc))
        ref.set_state(u0, p0, 0.0)
        ref.step(args.warmup + args.steps)
        u_b, p_b, _ = ref.get_state()
        extra["rel_l2_vs_fp64"] = {"u": float(np.linalg.norm(u_a - u_b) / np.linalg.norm(u_b)),
                                   "p": float(np.linalg.norm(p_a - p_b) / np.linalg.norm(p_b))}
        ref.close()
    s.close()
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    out = {
        "metric": METRIC, "value": round(args.steps / elapsed, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-inner/f64-outer" if prec == 1 else "f64", "data": "synthetic",
        "config": {"workload": case.name, "grid": [case.nx, case.ny, case.nz], "n_nodes": case.N,
                   "n_active": n_p, "lagrangian_points": case.M, "dt": case.dt,
                   "precision": args.precision, "pressure_preconditioner": args.precond},
        "roofline": roof,
    }
    out.update(extra)
    if args.serve:
        out["serving"] = serve_stream(args.serve_requests, args.serve_slots, 50)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
