"""Benchmark: IPCS + BCE-IB time steps per second on one MI355X.

Default workload: the synthetic aneurysm, the largest single-GPU configuration: a tube of
radius 1 along a sinusoidal centreline (amplitude 1, period 10, length 20) with a spherical
bulge of radius 2.5, on a 128x128x320 base grid whose cells within 0.5 of the wall are
split 2:1 (a 257x257x641 lattice of 42.3 M positions, 2.8 M unknown nodes), 46,602
Lagrangian wall points, parabolic inlet, mixed precision (FP32 inner solves in FP64
refinement), multigrid pressure solve.  One step = tentative velocity solve, IB force
solve and spreading, pressure increment solve, velocity/pressure correction, all on the
GPU.  `--workload pulsatile` runs the pulsatile cylinder (64x64x512, 1.78 M nodes) and
`--workload aorta` the aorta-like arch (256x160x384, 5 % active) instead.

Prints one JSON line.  During the timed steps every kernel dispatch records its own
start and end HIP events on the library's stream; the durations are summed per kernel,
and `roofline` reports the kernel with the largest summed time against the HBM peak,
with its algorithmic bytes per dispatch (`kernel_model`).  By default the line also
carries the relative error of the mixed-precision state against an FP64 run of the same
steps, the rates of the other two workloads and the serving stream (64 requests arriving
at 4 per second, served plain and with the mass-correction kernels batched across the
running requests, and the same requests submitted at once with twice the slots).
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
# published vector peaks of MI355X (256 CUs at 2.4 GHz); the library is built
# without packed FP32 instructions, which halves the FP32 figure in practice
FP32_VECTOR_TFLOPS = 157.3
FP64_VECTOR_TFLOPS = 78.6
CSRC = os.path.join(ROOT, "paper_2007_02082_amd", "csrc")


def kernel_sources_hash() -> str:
    """Hash of every device header of the library (the kernels' sources)."""
    import hashlib

    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hpp"):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def counted_traffic(workload: str, precision: str, kernel: str):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size), or None when the
    summary is for another kernel or the kernel sources changed after the counters
    were taken."""
    path = os.path.join(ROOT, "profiles", f"kernel_traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != kernel_sources_hash() or kernel not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel]["traffic_bytes"]


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


def serve_stream(n: int, slots: int, nsteps: int, batch_window_us: float | None = None,
                 rate: float = 4.0) -> dict:
    """Serving stream: n seeded requests (cylinder / aneurysm / Y-branch vessels, radius
    0.4-2.5, grids 32^3 .. 128x128x256, 50 steps each, mixed precision, multigrid) submitted
    at their Poisson arrival times (4 per second) to a server with `slots` concurrent
    slots; latency = completion - submission, solves/s = n / (last completion - first
    submission)."""
    import numpy as np

    import paper_2007_02082_amd as ibfe
    import synth

    reqs = synth.request_stream(n=n, rate=rate, nsteps=nsteps)
    # the batcher joins the Jacobi-preconditioned mass corrections only
    mp = 0 if batch_window_us is not None else 1
    kws = [ibfe.inputs_from_case(r.case, precision=1, precond=2, mass_precond=mp) for r in reqs]
    srv = ibfe.Server(max_slots=slots, batch_window_us=batch_window_us)
    ids = []
    t0 = time.perf_counter()
    for r, kw in zip(reqs, kws):
        delay = r.arrival - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        ids.append(srv.submit(nsteps, **kw))
    res = [srv.wait(i) for i in ids]
    peak = srv.peak_concurrency()
    bstats = srv.batch_stats()
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
            "wall_s": round(span, 2), "grid_nodes_total": int(sum(nodes)),
            "batch_window_us": batch_window_us, "mass_batches": bstats}


def poiseuille_study(levels=(0, 1, 2), pressures=(1.0, 2.0), tol=1e-8, max_steps=8000, domain="box",
                     band_h=None) -> list:
    """The pressure-driven tube of Section 3.1 on the three grids of Table 1 (h = 1, 0.5,
    0.25 mm), run with the library's steady-state driver until the step-to-step NRMSE of
    every velocity component is below tol.  Reported per run: steps, wall time, the
    centre-line speed against U_max = R^2 p_in / (4 mu L), the maximum and
    root-mean-square velocity errors against the Poiseuille profile over the nodes
    inside the tube, and the parabola u_z = U (1 - r^2 / R_eff^2) fitted (least squares)
    to the nodes inside the tube between 0.2 L and 0.8 L (the effective radius at which
    the immersed wall holds the flow); a run whose step fails is reported with the step
    it reached.  band_h: cells within band_h * h of the wall split 2:1."""
    import numpy as np

    import paper_2007_02082_amd as ibfe
    import synth
    from synth import poiseuille as e1

    rows = []
    for level in levels:
        for p_in in pressures:
            h = 1e-3 / 2 ** level
            case = synth.poiseuille_e1(level, p_in=p_in, domain=domain,
                                       refine_band=None if band_h is None else band_h * h)
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
            # nodes inside the tube (the box domain also holds fluid around it)
            inside = xyz[:, 0] ** 2 + xyz[:, 1] ** 2 < e1.R ** 2
            r2 = xyz[inside, 0] ** 2 + xyz[inside, 1] ** 2
            umax_exact = e1.R ** 2 * p_in / (4.0 * e1.MU * e1.L)
            ex = np.zeros((3, int(inside.sum())))
            ex[2] = umax_exact * (1.0 - r2 / e1.R ** 2)
            e = u[:, inside] - ex
            row = {"h": case.h, "p_in": p_in, "domain": domain, "nodes": case.N, "n_u": int(ids.size), "M": case.M,
                   "steps": total, "t": t, "wall_s": round(wall, 3),
                   "steps_per_s": round(total / wall, 1) if wall > 0 else None,
                   "steady": err is None and bool(np.all(nr < tol)),
                   "nrmse": None if nr is None else [float(x) for x in nr],
                   "u_max": float(u[2][inside].max()), "u_max_exact": umax_exact,
                   "Re": e1.RHO * float(u[2][inside].max()) * e1.L / e1.MU,
                   "L_inf": float(np.abs(e).max()), "L_2": float(np.sqrt((e * e).sum()) / e.shape[1]),
                   "transverse_max": float(np.abs(u[:2][:, inside]).max())}
            mid = inside & (xyz[:, 2] > 0.2 * e1.L) & (xyz[:, 2] < 0.8 * e1.L)
            if err is None and mid.sum() > 3:
                rr = xyz[mid, 0] ** 2 + xyz[mid, 1] ** 2
                a, b = np.linalg.lstsq(np.stack([np.ones_like(rr), rr], 1), u[2][mid], rcond=None)[0]
                row["fit_U"] = float(a)
                row["fit_R_eff"] = float(np.sqrt(-a / b)) if b < 0 < a else None
            row["band_h"] = band_h
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


WORKLOADS = {"pulsatile": "pulsatile_c2", "aneurysm": "aneurysm_case", "aorta": "aorta_case"}


def make_case(workload: str):
    import synth
    return getattr(synth, WORKLOADS[workload])()


def sizes_of(case, prec: int) -> dict:
    """Node counts the byte models need: pressure nodes P, free velocity nodes F and the
    active lattice nodes (P plus hanging nodes), from the host-only plan."""
    import paper_2007_02082_amd as ibfe
    pl = ibfe.Plan(**ibfe.inputs_from_case(case, precision=prec, precond=0))
    sz = pl.sizes()
    flags = pl.node_flags()
    n_act = int(((flags & (ibfe.FLAG_P | ibfe.FLAG_HANG)) != 0).sum())
    pl.close()
    return {"n_p": sz["n_p"], "n_free": sz["n_free"], "n_act": n_act, "M": case.M,
            "refined": getattr(case, "refine_cell", None) is not None}


# Floating-point operations of one matrix-free advection-diffusion row where all 8
# cells are kept (the factorised form, an FMA counted as 2): eight 1-D passes of 9
# lines at 5 operations (360), the two sums of the direction blocks (54) and the
# scaled accumulation into the 27 entries (54), then the product with the three
# components of x (81 FMA, 162).
CONV_ROW_FLOPS = 360 + 54 + 54 + 162


def kernel_model(name: str, z: dict):
    """Algorithmic work of one dispatch of a kernel, with a short description and the
    bound: "hbm" (minimum bytes: each operand read or written once, b = 1/8 B of
    domain data per node, 1/4 on a refined lattice) or "alu" (floating-point
    operations of the minimum-work formulation); None for kernels without a model.
    s = 4 for float instantiations, 8 for double."""
    s = 4 if "<float" in name else 8
    b = 0.25 if z["refined"] else 0.125
    n_p, n_f = z["n_p"], z["n_free"]
    if name.startswith("k_zb_cheb<") and name.endswith((", false, 3>", ", false, 3, true>", ", false, 3, false>")):
        return (15 * s + b) * n_f, "Q1 mass Chebyshev step, 3 components: read x, b, d; write d, x per free node", "hbm"
    if name.startswith("k_tm_cheb<") and name.endswith(", false>"):
        return (15 * s + b) * n_f, ("tensor-preconditioned mass Chebyshev update, 3 components: read the scaled "
                                    "residual w, d, x; write d, x per free node"), "hbm"
    if name.startswith("k_tm_resid<"):
        return (9 * s + b) * n_f, "scaled mass residual, 3 components: read x, b; write w per free node", "hbm"
    if name.startswith("k_cg_q_zb<") and name.endswith(", 1>"):
        return (2 * s + b) * n_p, "Q1 stiffness apply + p.q: read p, write q per pressure node", "hbm"
    if name.startswith("k_bi_apply<") and "OpCStencil<" in name:
        return (63 * s) * n_f, ("stored composite advection-diffusion stencil, 3 components: 54 coefficient "
                                "planes, read x and w, write y per free node"), "hbm"
    if name.startswith("k_bi_apply<") and "OpStencil<" in name:
        return (36 * s) * n_f, ("stored advection-diffusion stencil, 3 components: 27 coefficient planes, "
                                "read x and w, write y per free node"), "hbm"
    if name.startswith("k_residual<") and "OpCStencil<double, 3>" in name:
        return (54 * 8 + 6 * 8 + 3 * 4) * n_f, ("FP64 residual of the composite stored stencil: 54 planes, "
                                                 "read x, b, write r (FP32) per free node"), "hbm"
    if name.startswith("k_residual<") and "OpStencil<double, 3>" in name:
        return (27 * 8 + 6 * 8 + 3 * 4) * n_f, ("FP64 residual of the stored stencil: 27 planes, read x, b, "
                                                 "write r (FP32) per free node"), "hbm"
    if name.startswith("k_bi_apply<") and ("OpConv<" in name or "OpCConv<" in name):
        return CONV_ROW_FLOPS * n_f, ("matrix-free advection-diffusion apply, 3 components: each row formed "
                                      "from u^n at its 27 neighbours and applied to x, %d operations per free "
                                      "node in the factorised form (%.2f B of operands)" % (CONV_ROW_FLOPS, 12 * s + b)), "alu"
    if name.startswith("k_residual<") and ("OpConv<double>" in name or "OpCConv<double>" in name):
        return (9 * 8 + 3 * 4 + b) * n_f, ("FP64 matrix-free residual: read x, u^n, b, write r (FP32) per free "
                                           "node (rows formed on the fly)"), "hbm"
    if name == "k_s1_build":
        planes = 54 if z["refined"] else 27
        return (3 * 8 + planes * 12) * n_p, ("advection-diffusion stencil assembly: read u^n, write the "
                                              "FP64 and FP32 coefficient planes per node"), "hbm"
    return None


def achieved_of(name: str, m, seconds: float) -> dict:
    """Achieved rate of one dispatch of `seconds` for the kernel model m against its
    peak: HBM GB/s, or vector TFLOP/s (FP32 or FP64 by the instantiation)."""
    amount, what, bound = m
    if bound == "alu":
        peak = FP32_VECTOR_TFLOPS if "<float" in name else FP64_VECTOR_TFLOPS
        ach = amount / seconds / 1e12
        return {"bound": "alu", "alg_flops_per_launch": int(amount), "achieved": round(ach, 3),
                "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4), "what": what}
    ach = amount / seconds / 1e9
    return {"bound": "hbm", "alg_bytes_per_launch": int(amount), "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "what": what}


def run_workload(workload: str, prec: int, pc: int, visc: int, steps: int, warmup: int, case=None,
                 keep_state: bool = False, profile_steps: int = 3, advdiff: int = 0, mass_precond: int = 1) -> dict:
    """W untimed steps from rest; then `profile_steps` steps in which every kernel
    dispatch records its own start and end HIP events (the whole-step breakdown, which
    names the dominant kernel: the largest summed duration); then the K timed steps,
    bracketed by torch.cuda.synchronize() and the host clock, in which only the dominant
    kernel's dispatches carry events (events on every dispatch cost about 5 us each and
    would slow the timed steps; one kernel's do not measurably)."""
    import numpy as np
    import torch

    import paper_2007_02082_amd as ibfe

    case = case if case is not None else make_case(workload)
    z = sizes_of(case, prec)
    print(f"[bench] {case.name}: {z['n_p']} nodes of P, {z['n_free']} free, M = {case.M}", file=sys.stderr,
          flush=True)
    s = ibfe.Solver(**ibfe.inputs_from_case(case, precision=prec, precond=pc, viscous=visc, advdiff=advdiff,
                                            mass_precond=mass_precond))
    n = s.n_u
    s.set_state(np.zeros(3 * n), np.zeros(n), 0.0)
    s.step(warmup)
    # profile pass: every kernel timed
    s.set_kernel_timing(True)
    s.step(profile_steps)
    table = s.kernel_times()
    s.set_kernel_timing(False)
    dominant = table[0][0]
    # timed steps: the dominant kernel's dispatches timed
    s.set_kernel_timing_filter(dominant)
    s.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = s.stats()
    timed = {name: (ms, cnt) for name, ms, cnt in s.kernel_times()}
    s.set_kernel_timing(False)
    s.set_kernel_timing_filter(None)
    total_ms = sum(ms for _, ms, _ in table)
    rows = []
    for name, ms, cnt in table:
        m = kernel_model(name, z)
        avg_us = 1e3 * ms / max(1, cnt)
        row = {"kernel": name, "total_ms": round(ms, 3), "share": round(ms / total_ms, 4) if total_ms else 0.0,
               "launches": cnt, "avg_us": round(avg_us, 3)}
        if m is not None:
            row.update(achieved_of(name, m, avg_us * 1e-6))
        rows.append(row)
    dom = dict(rows[0])
    ms, cnt = timed.get(dominant, (0.0, 0))
    dom.update({"timed_launches": cnt, "timed_total_ms": round(ms, 3),
                "avg_us": round(1e3 * ms / max(1, cnt), 3)})
    m = kernel_model(dominant, z)
    if m is not None and cnt > 0:
        dom.update(achieved_of(dominant, m, 1e-3 * ms / cnt))
    out = {"case": case, "sizes": z, "steps_per_s": steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
           "elapsed_s": elapsed, "stats": st, "kernels": rows, "dominant": dom,
           "profile_steps": profile_steps, "kernel_ms_per_step": total_ms / profile_steps}
    if keep_state:
        out["state"] = s.get_state()
        out["solver"] = s
    else:
        s.close()
    return out


def roofline_of(res: dict, workload: str, precision: str, pc: int) -> dict:
    """The dominant kernel of the timed steps (largest summed duration over all kernels)
    against the HBM peak."""
    d = res["dominant"]
    traffic = counted_traffic(workload, precision, d["kernel"]) if pc == 2 else None
    roof = {"bound": d.get("bound", "hbm"), "achieved": d.get("achieved"), "peak": d.get("peak", HBM_PEAK_GBS),
            "unit": d.get("unit", "GB/s"), "frac": d.get("frac"), "traffic": round(traffic) if traffic else None,
            "kernel": d["kernel"], "share_of_kernel_time": d["share"], "avg_us": d["avg_us"],
            "launches": d["timed_launches"], "what": d.get("what")}
    for k in ("alg_bytes_per_launch", "alg_flops_per_launch"):
        if k in d:
            roof[k] = d[k]
    return roof


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["pulsatile", "aneurysm", "aorta"], default="aneurysm",
                    help="the refined aneurysm (default: the largest configuration, 2.8 M unknown nodes on "
                         "a 257x257x641 lattice), the pulsatile cylinder on 64x64x512 or the aorta-like arch "
                         "on 256x160x384")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--mass-precond", choices=["tensor", "jacobi"], default="tensor",
                    help="preconditioner of the consistent-mass correction's Chebyshev iteration: the "
                         "tensor-product approximate inverse of the Q1 mass or Jacobi")
    ap.add_argument("--precond", choices=["mg", "jacobi"], default="mg",
                    help="pressure preconditioner: geometric multigrid or Jacobi")
    ap.add_argument("--viscous", choices=["laplacian", "strain"], default="laplacian",
                    help="viscous form: mu (grad u, grad v) or the strain-rate form 2 mu (eps(u), eps(v))")
    ap.add_argument("--advdiff", choices=["matrix-free", "stencil"], default="matrix-free",
                    help="tentative-velocity operator: rows formed on the fly, or the stencil "
                         "assembled once per step")
    ap.add_argument("--wss", action="store_true",
                    help="also time the wall shear stress at the Lagrangian points (after the timed steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the FP64 run of the same steps (the mixed-vs-FP64 error of the line)")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the steps/s of the other two workloads")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--e1", action="store_true",
                    help="also run the pressure-driven Poiseuille study of Section 3.1 to steady "
                         "state on the three grids of Table 1 (after the timed steps)")
    ap.add_argument("--e1-band", type=float, default=None,
                    help="split the cells within this many h of the tube wall 2:1 in the --e1 runs")
    ap.add_argument("--e1-levels", type=int, nargs="+", default=[0, 1, 2],
                    help="grid levels of the --e1 runs (0, 1, 2 = h 1, 0.5, 0.25 mm)")
    ap.add_argument("--e1-domain", choices=["box", "reduced"], default="box",
                    help="the pressure-driven tube in the whole box (the paper's mesh, default) or in the "
                         "domain reduced to the tube")
    ap.add_argument("--moving", action="store_true",
                    help="also step the pulsatile cylinder with its wall points moving radially "
                         "(a device rebuild of the IB operators before every step)")
    ap.add_argument("--kernel-table", type=int, default=8,
                    help="kernels listed from the profile pass (largest summed time first)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-batch-window-us", type=float, default=200.0,
                    help="batching window of the second serving run (mass-correction kernels joined "
                         "across running requests)")
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

    torch.cuda.set_device(0)
    prec = 1 if args.precision == "mixed" else 0
    pc = 2 if args.precond == "mg" else 0
    visc = 1 if args.viscous == "strain" else 0
    ad = 1 if args.advdiff == "stencil" else 0
    refined = args.workload == "aneurysm"
    case = make_case(args.workload)
    mp = 1 if args.mass_precond == "tensor" else 0
    res = run_workload(args.workload, prec, pc, visc, args.steps, args.warmup, case=case, keep_state=True,
                       advdiff=ad, mass_precond=mp)
    s = res.pop("solver")
    st = res["stats"]
    print(f"[bench] {case.name}: {res['steps_per_s']:.2f} steps/s", file=sys.stderr, flush=True)
    roof = roofline_of(res, args.workload, args.precision, pc)

    extra = {"iters_last_step": {k: st[k] for k in ("s1_iters", "ib_iters", "s3_iters", "s4_iters",
                                                      "s1_outer", "s3_outer", "s4_outer", "s1_restarts")},
             "profile_pass": {"steps": res["profile_steps"],
                              "kernel_ms_per_step": round(res["kernel_ms_per_step"], 3),
                              "kernels_top": res["kernels"][:args.kernel_table]}}
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
    if args.moving:
        if args.workload != "pulsatile":
            print("--moving runs on the pulsatile cylinder only", file=sys.stderr)
            return 2
        extra["moving_points"] = moving_points(s, case)
    u_a, p_a, _ = res["state"]
    s.close()
    del res["state"]
    if prec == 1 and not args.no_check:
        # the same warm-up and timed steps in FP64: the accuracy the mixed-precision rate is quoted at
        import paper_2007_02082_amd as ibfe
        ref = ibfe.Solver(**ibfe.inputs_from_case(case, precision=0, precond=pc, viscous=visc, advdiff=ad,
                                                  mass_precond=mp))
        ref.set_state(np.zeros(3 * ref.n_u), np.zeros(ref.n_p), 0.0)
        t0r = time.perf_counter()
        ref.step(args.warmup + res["profile_steps"] + args.steps)
        u_b, p_b, _ = ref.get_state()
        fp64_rate = (args.warmup + res["profile_steps"] + args.steps) / (time.perf_counter() - t0r)
        ref.close()
        extra["rel_vs_fp64"] = {
            "steps": args.warmup + res["profile_steps"] + args.steps,
            "u_rel_l2": float(np.linalg.norm(u_a - u_b) / np.linalg.norm(u_b)),
            "p_rel_l2": float(np.linalg.norm(p_a - p_b) / np.linalg.norm(p_b)),
            "u_rel_max": float(np.abs(u_a - u_b).max() / np.abs(u_b).max()),
            "p_rel_max": float(np.abs(p_a - p_b).max() / np.abs(p_b).max()),
            "fp64_steps_per_s": round(fp64_rate, 2)}
        print(f"[bench] mixed vs FP64: {extra['rel_vs_fp64']}", file=sys.stderr, flush=True)
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    out = {
        "metric": METRIC, "value": round(res["steps_per_s"], 3), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-inner/f64-outer" if prec == 1 else "f64", "data": "synthetic",
        "config": {"workload": case.name, "grid": [case.nx, case.ny, case.nz], "n_nodes": case.N,
                   "refined_cells": int(case.refine_cell.sum()) if refined else 0,
                   "n_active": res["sizes"]["n_p"], "lagrangian_points": case.M, "dt": case.dt,
                   "precision": args.precision, "pressure_preconditioner": args.precond,
                   "viscous_form": args.viscous, "advdiff_operator": args.advdiff,
                   "mass_preconditioner": args.mass_precond},
        "roofline": roof,
    }
    out.update(extra)
    if not args.no_others:
        others = {}
        for w in ("pulsatile", "aneurysm", "aorta"):
            if w == args.workload:
                continue
            r = run_workload(w, prec, pc, visc, args.steps, args.warmup, advdiff=ad, mass_precond=mp)
            rf = roofline_of(r, w, args.precision, pc)
            others[r["case"].name] = {
                "steps_per_s": round(r["steps_per_s"], 3), "ms_per_step": round(r["ms_per_step"], 3),
                "n_active": r["sizes"]["n_p"], "lagrangian_points": r["case"].M,
                "dominant_kernel": rf["kernel"], "dominant_share": rf["share_of_kernel_time"],
                "dominant_avg_us": rf["avg_us"], "dominant_frac": rf["frac"],
                "profile_kernels_top": r["kernels"][:4]}
            print(f"[bench] {r['case'].name}: {r['steps_per_s']:.2f} steps/s", file=sys.stderr, flush=True)
        out["other_workloads"] = others
    if not args.no_serve:
        out["serving"] = serve_stream(args.serve_requests, args.serve_slots, 50)
        print(f"[bench] serving: {out['serving']['solves_per_s']} solves/s", file=sys.stderr, flush=True)
        out["serving_batched"] = serve_stream(args.serve_requests, args.serve_slots, 50,
                                              batch_window_us=args.serve_batch_window_us)
        print(f"[bench] serving, batched mass steps: {out['serving_batched']['solves_per_s']} solves/s",
              file=sys.stderr, flush=True)
        # capacity: the same requests all submitted at once, twice the slots
        out["serving_saturated"] = serve_stream(args.serve_requests, 2 * args.serve_slots, 50, rate=1e9)
        print(f"[bench] serving, all submitted at once: {out['serving_saturated']['solves_per_s']} solves/s",
              file=sys.stderr, flush=True)
    if args.e1:
        out["poiseuille_e1"] = poiseuille_study(domain=args.e1_domain, band_h=args.e1_band,
                                                levels=tuple(args.e1_levels))
    if not args.no_cpu_baseline:
        n_p = res["sizes"]["n_p"]
        out["cpu_baseline"] = {"pulsatile": cpu_baseline, "aneurysm": lambda: cpu_baseline_aneurysm(n_p),
                               "aorta": lambda: cpu_baseline_aorta(n_p)}[args.workload]()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
