"""Benchmark: IPCS + BCE-IB time steps per second on one MI355X.

Default workload: pulsatile flow in a cylinder of radius 0.5 and length 8 on a
64x64x512 Q1 grid (2.17 M nodes, 1.78 M pressure/velocity nodes after domain
reduction), 25,600 Lagrangian wall points, inlet u_max(t) = 1 + 0.5 sin(2 pi t),
dt = 0.005, synthetic inputs.  One step = tentative velocity solve, IB force solve
and spreading, pressure increment solve, velocity/pressure correction, all on the
GPU.  `--workload aneurysm` runs the synthetic aneurysm instead: a tube of radius 1
along a sinusoidal centreline (amplitude 1, period 10, length 20) with a spherical
bulge of radius 2.5, on a 128x128x320 base grid whose cells within 0.5 of the wall
are split 2:1 (a 257x257x641 lattice, 2.8 M unknown nodes), parabolic inlet.
`--workload aorta` runs the aorta-like arch (radius 1.2 along a cubic Bezier, three
branches of radius 0.4-0.6) on a uniform 256x160x384 grid (15.9 M nodes, 5 % of
them active), inlet and outlet disks on the same face, two-harmonic Womersley-type
inlet, dt = 0.002.

Prints one JSON line.  The two matrix-free applies that carry the step are timed
with HIP events on the library's stream over the timed region: the masked Q1
stiffness apply inside the pressure CG, (2 s + b) algorithmic bytes per pressure
node (read p, write q), and the masked Q1 mass Chebyshev step of the velocity
correction, (15 s + b) per free node (three components, read x, b, d, write d,
x); s = 4 in mixed mode, 8 in FP64 mode, b = 1/8 (one bit of domain data) or 1/4
on the refined lattice (fine and coarse element bits).  `roofline` reports the
one with the larger summed time; the other one is listed under `roofline.other`.
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


KERNEL_SOURCES = {"pulsatile": ("kernels.hpp", "zblock.hpp"),
                  "aneurysm": ("kernels.hpp", "zblock.hpp", "composite.hpp"),
                  "aorta": ("kernels.hpp", "zblock.hpp")}


def counted_traffic(workload: str, precision: str, kernel: str):
    """HBM bytes per dispatch of the dominant apply (`pressure` or `mass`) from the
    committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, scaled by a copy of
    known size), or None when the kernel sources changed after the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel}_apply_traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[workload]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return rec["traffic_bytes"] if h.hexdigest()[:16] == rec["source_hash"] else None


METRIC = "IPCS steps/sec + apply HBM GB/s at 1e-6 rel; served solves/sec, p50/p99"


def cpu_baseline_aneurysm(n_full: int) -> dict:
    """Oracle (FP64, one thread) on a bounded sample: the same aneurysm geometry on a
    48x48x120 base grid (same band rule and point spacing in units of h), one step after
    set-up, scaled by the ratio of unknown nodes to the 128x128x320 case (a lower bound
    on the oracle's time at full size: its Jacobi-CG iteration counts grow with the
    resolution)."""
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import ipcs

    sample = synth.aneurysm_case((48, 48, 120), nsteps=1)
    with threadpool_limits(1):
        pr = ipcs.Problem.from_case(sample)
        u, p = pr.initial_state(sample.u0, sample.p0)
        t0 = time.perf_counter()
        pr.step(u, p, 0.0)
        sec = time.perf_counter() - t0
    scale = n_full / pr.sets.P.size
    return {"value": 1.0 / (sec * scale), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 oracle step of the aneurysm on a 48x48x120 base grid ({pr.sets.P.size} "
                      f"nodes, {sec:.2f} s/step), scaled by the node ratio {scale:.2f}"}


def cpu_baseline_aorta(n_full: int) -> dict:
    """Oracle (FP64, one thread) on a bounded sample: the same aorta-like geometry at half
    resolution (128x80x192, same point spacing in units of h), one step after set-up,
    scaled by the ratio of nodes of P to the 256x160x384 case (a lower bound on the
    oracle's time at full size: its Jacobi-CG iteration counts grow with the resolution)."""
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import ipcs

    sample = synth.aorta_case(scale=2, nsteps=1)
    with threadpool_limits(1):
        pr = ipcs.Problem.from_case(sample)
        u, p = pr.initial_state(sample.u0, sample.p0)
        t0 = time.perf_counter()
        pr.step(u, p, 0.0)
        sec = time.perf_counter() - t0
    scale = n_full / pr.sets.P.size
    return {"value": 1.0 / (sec * scale), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 oracle step of the aorta-like arch at half resolution (128x80x192, "
                      f"{pr.sets.P.size} nodes, {sec:.2f} s/step), scaled by the node ratio {scale:.2f}"}


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


def poiseuille_study(levels=(0, 1, 2), pressures=(1.0, 2.0), tol=1e-8, max_steps=8000) -> list:
    """The pressure-driven tube of Section 3.1 on the three grids of Table 1 (h = 1, 0.5,
    0.25 mm), run with the library's steady-state driver until the step-to-step NRMSE of
    every velocity component is below tol.  Reported per run: steps, wall time, the
    centre-line speed against U_max = R^2 p_in / (4 mu L), and the maximum and
    root-mean-square velocity errors against the Poiseuille profile over the nodes
    inside the tube; a run whose step fails is reported with the step it reached."""
    import numpy as np

    import paper_2007_02082_amd as ibfe
    import synth
    from synth import poiseuille as e1

    rows = []
    for level in levels:
        for p_in in pressures:
            case = synth.poiseuille_e1(level, p_in=p_in)
            s = ibfe.Solver(**ibfe.inputs_from_case(case, precision=1, precond=2))
            ids = s.node_ids()
            s.set_state(np.zeros(3 * s.n_u), np.ascontiguousarray(case.p0[ids]), 0.0)
            total, nr, err = 0, None, None
            t0 = time.perf_counter()
            while total < max_steps:
                try:
                    k, nr = s.run_steady(tol, min(500, max_steps - total))
                except ibfe.IbfeError as e:
                    err = str(e)
                    break
                total += k
                print(f"[e1] h={case.h:g} p_in={p_in:g} steps={total} nrmse={np.max(nr):.3e}",
                      file=sys.stderr, flush=True)
                if np.all(nr < tol):
                    break
            wall = time.perf_counter() - t0
            u, p, t = s.get_state()
            s.close()
            xyz = case.node_coords()[ids]
            inside = case.node_mask[ids] == 1
            r2 = xyz[inside, 0] ** 2 + xyz[inside, 1] ** 2
            umax_exact = e1.R ** 2 * p_in / (4.0 * e1.MU * e1.L)
            ex = np.zeros((3, int(inside.sum())))
            ex[2] = umax_exact * (1.0 - r2 / e1.R ** 2)
            e = u[:, inside] - ex
            row = {"h": case.h, "p_in": p_in, "nodes": case.N, "n_u": int(ids.size), "M": case.M,
                   "steps": total, "t": t, "wall_s": round(wall, 3),
                   "steps_per_s": round(total / wall, 1) if wall > 0 else None,
                   "steady": err is None and bool(np.all(nr < tol)),
                   "nrmse": None if nr is None else [float(x) for x in nr],
                   "u_max": float(u[2].max()), "u_max_exact": umax_exact,
                   "Re": e1.RHO * float(u[2].max()) * e1.L / e1.MU,
                   "L_inf": float(np.abs(e).max()), "L_2": float(np.sqrt((e * e).sum()) / e.shape[1]),
                   "transverse_max": float(np.abs(u[:2]).max())}
            if err is not None:
                row["error"] = err
            rows.append(row)
    return rows


def moving_points(s, case, nsteps: int = 20) -> dict:
    """Moving Lagrangian points on the benchmark cylinder: the wall rings pulsate
    radially (R(t) = R0 (1 + 0.02 sin 2 pi t)); every step first moves the points
    (ibfe_set_points rebuilds the stencils, the spreading lists, G and its block
    inverses on the device) and then advances.  Reports the rebuild time and the step
    rate with a rebuild per step next to the rate without motion."""
    import numpy as np
    import torch

    import synth

    rings, per_ring = 256, 100
    z = (np.arange(rings, dtype=np.float64) + 0.5) * (8.0 / rings)
    wall = synth.PulsatingWall(0.5, z, per_ring, 0.02, 1.0)
    _, _, t = s.get_state()
    s.set_points(*wall.at(t + case.dt))     # first call: allocation
    s.step(1)
    t += case.dt
    rebuild = []
    t0 = time.perf_counter()
    for _ in range(nsteps):
        X, U = wall.at(t + case.dt)
        r0 = time.perf_counter()
        s.set_points(X, U)
        torch.cuda.synchronize()
        rebuild.append(time.perf_counter() - r0)
        s.step(1)
        t += case.dt
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    st = s.stats()
    return {"M": case.M, "steps": nsteps, "rebuild_ms_median": round(1e3 * float(np.median(rebuild)), 3),
            "steps_per_s_with_rebuild": round(nsteps / wall_s, 2), "ib_iters_last": st["ib_iters"],
            "amplitude": 0.02, "period": 1.0}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["pulsatile", "aneurysm", "aorta"], default="pulsatile",
                    help="pulsatile cylinder on 64x64x512 (default), the refined aneurysm or the "
                         "aorta-like arch on 256x160x384")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--precond", choices=["mg", "jacobi"], default="mg",
                    help="pressure preconditioner: geometric multigrid or Jacobi")
    ap.add_argument("--viscous", choices=["laplacian", "strain"], default="laplacian",
                    help="viscous form: mu (grad u, grad v) or the strain-rate form 2 mu (eps(u), eps(v))")
    ap.add_argument("--wss", action="store_true",
                    help="also time the wall shear stress at the Lagrangian points (after the timed steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check", action="store_true",
                    help="also run the same steps in FP64 mode and report the difference")
    ap.add_argument("--serve", action="store_true",
                    help="also run the serving stream (64 requests, Poisson arrivals at 4/s)")
    ap.add_argument("--e1", action="store_true",
                    help="also run the pressure-driven Poiseuille study of Section 3.1 to steady "
                         "state on the three grids of Table 1 (after the timed steps)")
    ap.add_argument("--moving", action="store_true",
                    help="also step the benchmark cylinder with its wall points moving radially "
                         "(a device rebuild of the IB operators before every step)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the run, copy a device buffer of this size 5 times (a plain copy "
                         "kernel of known size for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures the path on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design, not an implementation)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2007_02082_amd as ibfe
    import synth

    torch.cuda.set_device(0)
    refined = args.workload == "aneurysm"
    case = {"pulsatile": synth.pulsatile_c2, "aneurysm": synth.aneurysm_case,
            "aorta": synth.aorta_case}[args.workload]()
    prec = 1 if args.precision == "mixed" else 0
    pc = 2 if args.precond == "mg" else 0
    visc = 1 if args.viscous == "strain" else 0
    s = ibfe.Solver(**ibfe.inputs_from_case(case, precision=prec, precond=pc, viscous=visc))
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
    n_free = ibfe.Plan(**ibfe.inputs_from_case(case, precision=prec, precond=0)).sizes()["n_free"]
    bits = 0.25 if refined else 0.125
    tname = "float" if prec == 1 else "double"
    # the two matrix-free applies that carry most of the step, timed with HIP events
    kernels = {
        "pressure": {
            "kernel": (f"k_cg_q_zb<{tname},1> (composite Q1 stiffness apply + p.q: fine-cell walk "
                       "+ precomputed coarse/hanging terms)" if refined
                       else f"k_cg_q_zb<{tname},1> (masked Q1 stiffness apply + p.q)"),
            "ms": st["poisson_apply_ms"], "launches": st["poisson_applies"],
            # read p, write q per pressure node
            "alg_bytes_per_launch": (2 * bytes_per_value + bits) * n_p},
        "mass": {
            "kernel": (f"k_zb_cheb<{tname}, false, 3> (composite Q1 mass Chebyshev step: fine-cell walk "
                       "+ precomputed coarse/hanging terms)"
                       if refined else f"k_zb_cheb<{tname}, false, 3> (masked Q1 mass Chebyshev step)"),
            "ms": st["mass_apply_ms"], "launches": st["mass_applies"],
            # per free node and component: read x, b, d; write d, x
            "alg_bytes_per_launch": (15 * bytes_per_value + bits) * n_free},
    }
    dominant = max(kernels, key=lambda k: kernels[k]["ms"])
    rows = {}
    for name, k in kernels.items():
        avg_ms = k["ms"] / max(1, k["launches"])
        ach = k["alg_bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
        rows[name] = {"kernel": k["kernel"], "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                      "avg_us": round(avg_ms * 1e3, 3), "launches": k["launches"],
                      "total_ms": round(k["ms"], 3), "alg_bytes_per_launch": int(k["alg_bytes_per_launch"])}
    d = rows[dominant]
    traffic = counted_traffic(args.workload, args.precision, dominant) if pc == 2 else None
    roof = {"bound": "hbm", "achieved": d["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": d["frac"], "traffic": round(traffic) if traffic else None,
            "kernel": d["kernel"], "avg_us": d["avg_us"], "launches": d["launches"],
            "alg_bytes_per_launch": d["alg_bytes_per_launch"],
            "other": {k: v for k, v in rows.items() if k != dominant}}

    extra = {"iters_last_step": {k: st[k] for k in ("s1_iters", "ib_iters", "s3_iters", "s4_iters",
                                                      "s1_outer", "s3_outer", "s4_outer")}}
    if args.wss and not refined:
        # unit normals from the vessel axis of the point's tube (timing only: any unit vectors do)
        nrm = case.X - case.X.mean(axis=0)
        nrm[:, 2] = 0.0
        nrm /= np.maximum(np.linalg.norm(nrm, axis=1), 1e-30)[:, None]
        s.wall_shear(nrm)
        torch.cuda.synchronize()
        t0w = time.perf_counter()
        for _ in range(5):
            tau = s.wall_shear(nrm)
        extra["wall_shear_ms"] = round(1e3 * (time.perf_counter() - t0w) / 5, 3)
        extra["wall_shear_max"] = float(np.abs(tau).max())
    if args.check:
        u_a, p_a, _ = s.get_state()
        ref = ibfe.Solver(**ibfe.inputs_from_case(case, precision=0, precond=pc, viscous=visc))
        ref.set_state(u0, p0, 0.0)
        ref.step(args.warmup + args.steps)
        u_b, p_b, _ = ref.get_state()
        extra["rel_l2_vs_fp64"] = {"u": float(np.linalg.norm(u_a - u_b) / np.linalg.norm(u_b)),
                                   "p": float(np.linalg.norm(p_a - p_b) / np.linalg.norm(p_b))}
        ref.close()
    if args.moving:
        if args.workload != "pulsatile":
            print("--moving runs on the pulsatile cylinder only", file=sys.stderr)
            return 2
        extra["moving_points"] = moving_points(s, case)
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
                   "refined_cells": int(case.refine_cell.sum()) if refined else 0,
                   "n_active": n_p, "lagrangian_points": case.M, "dt": case.dt,
                   "precision": args.precision, "pressure_preconditioner": args.precond,
                   "viscous_form": args.viscous},
        "roofline": roof,
    }
    out.update(extra)
    if args.serve:
        out["serving"] = serve_stream(args.serve_requests, args.serve_slots, 50)
    if args.e1:
        out["poiseuille_e1"] = poiseuille_study()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = {"pulsatile": cpu_baseline, "aneurysm": lambda: cpu_baseline_aneurysm(n_p),
                               "aorta": lambda: cpu_baseline_aorta(n_p)}[args.workload]()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
