#!/usr/bin/env python3
"""Throughput of the second-order Trotter-Suzuki solve on one MI355X.

Workload (one bench "step" = one whole solve of the hot path):
  4096 x 4096 periodic mesh, four seeded Gaussian packets in a harmonic well
  plus 32 seeded Gaussian bumps, dt = 0.05, 1000 second-order steps:
  phase-table setup (FP64) + 1000 fused steps + FP64 norm/energy reduction.
  Run in complex64 (headline line) and complex128 (nested object).
Inputs are generated on the device before the timed region.  Prints ONE JSON
line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "site-steps/s and % HBM roofline (c64/c128); batched p50/p99 solve latency"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


# The sources the benchmarked 2D march kernels and their launches are built from
# (the 3D and time-dependent paths live in files of their own).
KERNEL_SOURCES = ("tsq_march.hpp", "tsq_internal.h", "tsq_kernels.hip", "march_c64_single.hip",
                  "march_c128_single.hip")
# the 3D march includes the 2D march templates
KERNEL3_SOURCES = ("tsq_march.hpp", "tsq_internal.h", "tsq_march3.hpp", "tsq_internal3.h",
                   "tsq_kernels3.hip", "march3_c64.hip", "march3_c128.hip")


def code_text(src: str) -> str:
    """C++ source without its comments, whitespace runs collapsed to one space:
    what the compiler sees, so an edit of a comment keeps the hash."""
    out = []
    i, n = 0, len(src)
    while i < n:
        c = src[i]
        if c == "/" and src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif c == "/" and src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_hash(sources=KERNEL_SOURCES) -> str:
    """sha256[:16] of the code (comments and layout removed) of the sources of the
    benchmarked march kernels (the 2D march by default)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1208_2407_amd", "csrc")
    for name in sources:
        h.update(name.encode())
        with open(os.path.join(csrc, name), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def committed_traffic(dtype: str, schedule, nx: int, ny: int, nz: int = 0) -> float | None:
    """HBM bytes per launch from the committed rocprofv3 counter runs (keyed by
    kernel code hash, mesh "NXxNY" or "NXxNYxNZ", dtype and schedule "S,seg,ppl,store",
    or "1" for the one-step 3D pass), if they were taken on this exact kernel code,
    mesh and schedule; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        return None
    code = kernel_hash(KERNEL3_SOURCES) if nz else kernel_hash()
    mesh = f"{nx}x{ny}x{nz}" if nz else f"{nx}x{ny}"
    e = (db.get(code, {}).get(mesh, {}).get(dtype, {})
         .get(",".join(str(int(v)) for v in schedule)))
    if not e:
        return None
    return float(e["bytes_per_launch"])


def run_dtype(dtype: str, p, psi0, V, args, order: int = 2, bc: str = "periodic"):
    import torch
    import paper_1208_2407_amd as tsq
    from paper_1208_2407_amd import autotune

    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    psi = psi0.to(tdt).contiguous()
    plan = tsq.Plan(p.nx, p.ny, p.dt, dtype, order=order, bc=bc, device=psi.device)
    plan.set_potential(V)
    if args.schedule:
        plan.set_schedule(*[int(v) for v in args.schedule.split(",")])
    elif not args.no_tune:
        sched, _ = autotune.tune(plan, psi, log=log if args.verbose else None)
        log(f"{dtype}: autotuned schedule S={sched[0]} seg={sched[1]} ppl={sched[2]} "
            f"store={sched[3]}")
    sched = plan.schedule()
    passes, copy_back = plan.passes(p.steps)
    ws = plan.workspace()
    n_begin, e_begin = plan.observables(psi, V)

    def solve(events=None):
        plan.set_potential(V)
        if events is not None:
            events[0].record()
        plan.evolve(psi, p.steps)
        if events is not None:
            events[1].record()
        return plan.observables(psi, V)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        norm, energy = solve(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    evolve_ms = sum(a.elapsed_time(b) for a, b in evs)
    wall = t1 - t0
    site_steps = p.nx * p.ny * p.steps * args.steps
    elem = 16 if dtype == "c128" else 8
    alg_bytes = p.nx * p.ny * (2 * elem + 16)   # read psi, write psi, read phase table
    launch_s = evolve_ms * 1e-3 / (args.steps * passes)
    achieved = alg_bytes / launch_s / 1e9
    # counters were taken on second-order passes; fourth-order launches mix pass sizes
    traffic = (committed_traffic(dtype, sched, p.nx, p.ny)
               if order == 2 and bc == "periodic" else None)
    # one pass per step would need the same bytes every step: site-steps/s times those
    # bytes over the peak says how far fusion takes the solve past that roofline (> 1)
    eff_frac = (site_steps / wall) * (2 * elem + 16) / (HBM_PEAK_GBS * 1e9)
    log(f"{dtype}: {wall / args.steps * 1e3:.2f} ms/solve, {site_steps / wall:.4e} site-steps/s, "
        f"pass {launch_s * 1e6:.1f} us, {achieved:.0f} GB/s algorithmic, norm {norm:.15f}")
    del ws
    return {
        "value": site_steps / wall,
        "ms_per_step": wall / args.steps * 1e3,
        "schedule": {"steps_per_pass": sched[0], "segment_rows": sched[1],
                     "pairs_per_lane": sched[2],
                     "phase_store": {1: "registers", 2: "lds"}[sched[3]],
                     "passes_per_solve": passes, "copy_back": copy_back},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_GBps": round(traffic / launch_s / 1e9, 1) if traffic else None,
                     "traffic_frac": (round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
                                      if traffic else None),
                     "eff_frac_one_pass_per_step": round(eff_frac, 3),
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "kernel": "march_kernel", "avg_launch_us": round(launch_s * 1e6, 2)},
        "norm_drift": norm - n_begin,
        "energy": energy,
    }


def run_td(dtype: str, p, psi0, V0, W, f, args, bc: str = "periodic"):
    """One solve under the time-dependent potential V0 + f(t) W: table setup,
    len(f) fused steps (the phase formed in FP64 in the march), FP64 observables
    at the final time."""
    import torch
    import paper_1208_2407_amd as tsq

    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    psi = psi0.to(tdt).contiguous()
    plan = tsq.Plan(p.nx, p.ny, p.dt, dtype, bc=bc, device=psi.device)
    plan.set_potential_td(V0, W)
    if args.schedule:
        plan.set_schedule(*[int(v) for v in args.schedule.split(",")])
    else:
        scratch = psi.clone()
        best = None
        for cand in [(S, 0, 1, st) for S in (1, 2, 3, 4) for st in (1, 2)]:
            plan.set_schedule(*cand)
            plan.evolve_td(scratch, f[:8])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.evolve_td(scratch, f[:120])
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            if args.verbose:
                log(f"td {dtype} S={cand[0]} store={cand[3]}: {ms:.3f} ms / 120 steps")
            if best is None or ms < best[0]:
                best = (ms, cand)
        plan.set_schedule(*best[1])
        del scratch
    sched = plan.schedule()
    passes, copy_back = plan.passes(len(f))
    V_end = V0 + float(f[-1]) * W   # potential at the last step's midpoint, for the energy

    def solve(events=None):
        plan.set_potential_td(V0, W)
        if events is not None:
            events[0].record()
        plan.evolve_td(psi, f)
        if events is not None:
            events[1].record()
        return plan.observables(psi, V_end)

    n_begin, _ = plan.observables(psi, V_end)
    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        norm, energy = solve(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evolve_ms = sum(a.elapsed_time(b) for a, b in evs)
    site_steps = p.nx * p.ny * len(f) * args.steps
    elem = 16 if dtype == "c128" else 8
    alg_bytes = p.nx * p.ny * (2 * elem + 16)   # read psi, write psi, read (theta0, w)
    launch_s = evolve_ms * 1e-3 / (args.steps * passes)
    achieved = alg_bytes / launch_s / 1e9
    log(f"td {dtype}: S={sched[0]} store={sched[3]}: {wall / args.steps * 1e3:.2f} ms/solve, "
        f"{site_steps / wall:.4e} site-steps/s, pass {launch_s * 1e6:.1f} us, norm {norm:.15f}")
    return {
        "value": site_steps / wall, "ms_per_step": wall / args.steps * 1e3,
        "schedule": {"steps_per_pass": sched[0], "pairs_per_lane": sched[2],
                     "phase_store": {1: "registers", 2: "lds"}[sched[3]],
                     "passes_per_solve": passes, "copy_back": copy_back},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes_per_launch": alg_bytes, "kernel": "march_kernel (td)",
                     "avg_launch_us": round(launch_s * 1e6, 2)},
        "norm_drift": norm - n_begin,
    }


def run_3d(dtype: str, p, psi0, V, args):
    """One solve of a 3D mesh (one step per pass): phase table, p.steps steps,
    FP64 observables."""
    import torch
    import paper_1208_2407_amd as tsq

    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    psi = psi0.to(tdt).contiguous()
    plan = tsq.Plan(p.nx, p.ny, p.dt, dtype, nz=p.nz, device=psi.device)
    passes, copy_back = plan.passes(p.steps)
    def solve(events=None):
        plan.set_potential(V)
        if events is not None:
            events[0].record()
        plan.evolve(psi, p.steps)
        if events is not None:
            events[1].record()
        return plan.observables(psi, V)

    plan.set_potential(V)
    n_begin, _ = plan.observables(psi, V)
    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        norm, energy = solve(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evolve_ms = sum(a.elapsed_time(b) for a, b in evs)
    site_steps = p.sites * p.steps * args.steps
    elem = 16 if dtype == "c128" else 8
    alg_bytes = p.sites * (2 * elem + 16)
    launch_s = evolve_ms * 1e-3 / (args.steps * passes)
    achieved = alg_bytes / launch_s / 1e9
    traffic = committed_traffic(dtype, (1,), p.nx, p.ny, p.nz)
    log(f"3d {dtype}: {wall / args.steps * 1e3:.2f} ms/solve, {site_steps / wall:.4e} site-steps/s, "
        f"pass {launch_s * 1e6:.1f} us, {achieved:.0f} GB/s algorithmic, norm {norm:.15f}")
    return {
        "value": site_steps / wall, "ms_per_step": wall / args.steps * 1e3,
        "schedule": {"steps_per_pass": 1, "passes_per_solve": passes, "copy_back": copy_back},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_GBps": round(traffic / launch_s / 1e9, 1) if traffic else None,
                     "traffic_frac": (round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
                                      if traffic else None),
                     "algorithmic_bytes_per_launch": alg_bytes, "kernel": "march3_kernel",
                     "avg_launch_us": round(launch_s * 1e6, 2)},
        "norm_drift": norm - n_begin,
    }


def profile_mode(p, psi0, V, args) -> int:
    """A short, fixed run for hardware-counter collection (no tuning, no timing loop)."""
    import torch
    import paper_1208_2407_amd as tsq

    from paper_1208_2407_amd import autotune

    if not args.schedule:
        print("--profile-passes needs --schedule (or --schedule tuned)", file=sys.stderr)
        return 2
    out = {"kernel_hash": kernel_hash(), "mesh": [p.nx, p.ny], "runs": {}}
    # reference copy of known size (1 GiB read + 1 GiB written)
    src = torch.empty(2**27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    out["copy_bytes"] = src.numel() * 8
    for d in args.dtypes.split(","):
        tdt = torch.complex128 if d == "c128" else torch.complex64
        psi = psi0.to(tdt).contiguous()
        plan = tsq.Plan(p.nx, p.ny, p.dt, d, device=psi.device)
        plan.set_potential(V)
        if args.schedule == "tuned":
            autotune.tune(plan, psi)          # cached choice of an earlier bench run
        else:
            plan.set_schedule(*[int(v) for v in args.schedule.split(",")])
        sched = plan.schedule()
        steps = sched[0] * args.profile_passes
        torch.cuda.synchronize()
        plan.evolve(psi, steps)
        torch.cuda.synchronize()
        elem = 16 if d == "c128" else 8
        out["runs"][d] = {"schedule": list(sched), "steps": steps,
                          "passes": plan.passes(steps)[0],
                          "algorithmic_bytes_per_launch": p.nx * p.ny * (2 * elem + 16)}
    print(json.dumps(out), flush=True)
    return 0


def sweep_mode(p, psi0, V, args) -> int:
    """Every candidate schedule (the tuner's, plus 7 and 8 steps per pass) for
    exactly --profile-passes passes after a warm-up, each timed with HIP events
    on the current stream; one JSON line per dtype and schedule.  Run under
    rocprofv3 --pmc it also gives the HBM counters of every schedule."""
    import torch
    import paper_1208_2407_amd as tsq
    from paper_1208_2407_amd import autotune

    cands = list(autotune.DEFAULT_CANDIDATES) + [(7, 0, 1, 2), (8, 0, 1, 2)]
    stream = torch.cuda.current_stream()
    # reference copy of known size (1 GiB read + 1 GiB written) to scale the counters
    src = torch.empty(2**27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    for d in args.dtypes.split(","):
        tdt = torch.complex128 if d == "c128" else torch.complex64
        elem = 16 if d == "c128" else 8
        alg = p.nx * p.ny * (2 * elem + 16)
        for sched in cands:
            psi = psi0.to(tdt).clone()
            plan = tsq.Plan(p.nx, p.ny, p.dt, d, device=psi.device)
            plan.set_potential(V)
            plan.set_schedule(*sched)
            S = sched[0]
            plan.evolve(psi, 2 * S)
            steps = S * args.profile_passes
            passes = plan.passes(steps)[0]
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            plan.evolve(psi, steps)
            e1.record(stream)
            e1.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3
            pass_s = sec / passes
            print(json.dumps({"sweep": True, "dtype": d, "schedule": list(sched),
                              "kernel_hash": kernel_hash(), "mesh": [p.nx, p.ny],
                              "steps": steps, "passes": passes,
                              "avg_pass_us": round(pass_s * 1e6, 2),
                              "us_per_step": round(sec / steps * 1e6, 3),
                              "site_steps_per_s": p.nx * p.ny * steps / sec,
                              "algorithmic_bytes_per_launch": alg,
                              "frac": round(alg / pass_s / 1e9 / HBM_PEAK_GBS, 4),
                              "eff_frac_one_pass_per_step": round(
                                  p.nx * p.ny * steps / sec * alg / (p.nx * p.ny) / 1e9
                                  / HBM_PEAK_GBS, 3)}), flush=True)
            del psi, plan
    return 0


def run_batch(args) -> dict:
    """512 independent complex64 problems (sides log-uniform in [64, 1024], rounded to
    even; own potential, packets and dt), 500 steps each: one batched call (captured
    HIP graph) against sequential plain tsq_evolve calls on the same GPU."""
    import torch
    import paper_1208_2407_amd as tsq
    from paper_1208_2407_amd import workloads as wl

    probs = wl.batch_problems(512, 4, 500, dtype="c64")
    log(f"batch: generating {len(probs)} problems")
    psi0s, Vs, plans = [], [], []
    for q in probs:
        psi0s.append(wl.initial_state(q, device="cuda", dtype=torch.complex64))
        V = wl.potential(q, device="cuda")
        pl = tsq.Plan(q.nx, q.ny, q.dt, "c64")
        pl.set_potential(V)
        Vs.append(V)
        plans.append(pl)
    steps = [q.steps for q in probs]
    site_steps = sum(q.nx * q.ny * q.steps for q in probs)
    sites = sum(q.nx * q.ny for q in probs)

    def timed(fn, reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    # batch schedule: a short search over steps per pass and phase ring (one pair per lane)
    best = None
    cands = ([tuple(int(v) for v in args.schedule.split(","))] if args.schedule
             else [(S, 0, 1, st) for S in (3, 4, 5, 6) for st in (1, 2)])
    for sched in cands:
        psis = [x.clone() for x in psi0s]
        bt = tsq.Batch(plans, psis, steps, sched)
        bt.launch(use_graph=True)
        t = timed(lambda: bt.launch(use_graph=True), 1)
        log(f"batch: S={sched[0]} store={sched[3]}: {t * 1e3:.1f} ms per call "
            f"({bt.info()[0]} launches)")
        if best is None or t < best[0]:
            best = (t, sched)
        del bt, psis
    sched = best[1]
    psis = [x.clone() for x in psi0s]
    bt = tsq.Batch(plans, psis, steps, sched)
    launches, tiles = bt.info()
    for _ in range(args.warmup):
        bt.launch(use_graph=True)
    t_batch = timed(lambda: bt.launch(use_graph=True), args.steps)
    # sequential plain solves: each problem alone, same kernels and schedule
    seq = [x.clone() for x in psi0s]
    for pl in plans:
        pl.set_schedule(*sched)

    def sequential():
        for pl, x, n in zip(plans, seq, steps):
            pl.evolve(x, n)

    sequential()
    t_seq = timed(sequential, 1)
    # the batched result equals each problem alone (bitwise), spot-checked
    ref = [x.clone() for x in psi0s[:8]]
    for pl, x, n in zip(plans[:8], ref, steps[:8]):
        pl.evolve(x, n)
    one = [x.clone() for x in psi0s]
    bt1 = tsq.Batch(plans, one, steps, sched)
    bt1.launch()
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(one[:8], ref))
    log(f"batch: {t_batch * 1e3:.1f} ms per call, sequential {t_seq * 1e3:.1f} ms, "
        f"speedup {t_seq / t_batch:.2f}x, bitwise equal to alone: {same}")
    return {
        "metric": METRIC, "value": site_steps / t_batch, "unit": "site-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_batch * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "batch512_c64_500steps", "problems": len(probs), "sites": sites,
                   "site_steps_per_call": site_steps, "steps_per_pass": sched[0],
                   "phase_store": "registers" if sched[3] == 1 else "lds",
                   "launches_per_call": launches, "tiles_per_call": tiles,
                   "hip_graph": True},
        "sequential": {"value": site_steps / t_seq, "ms_per_call": t_seq * 1e3},
        "speedup_vs_sequential": t_seq / t_batch,
        "bitwise_equal_to_alone": same,
    }


def run_served(args) -> dict:
    """Poisson arrivals at 200 req/s for --serve-seconds seconds (sides log-uniform
    128-4096, steps 100-2000, 80/20 complex64/complex128) replayed in real time into
    the continuous-batching server; the FIFO one-at-a-time server on the first
    --fifo-seconds of the same trace for comparison."""
    import torch
    from paper_1208_2407_amd import serve
    from paper_1208_2407_amd import workloads as wl

    trace = wl.request_trace(rate=200.0, duration=args.serve_seconds, seed=5)
    offered = sum(r.problem.site_steps for r in trace) / args.serve_seconds
    log(f"served: {len(trace)} requests over {args.serve_seconds} s, offered {offered:.3e} "
        f"site-steps/s")
    # warm the code paths
    serve.Server(block_steps=args.block_steps).run(trace[:16], realtime=False)
    srv = serve.Server(block_steps=args.block_steps)
    st = srv.run(trace, realtime=True).summary()
    log(f"served: {st}")
    fifo_trace = [r for r in trace if r.arrival < args.fifo_seconds]
    batched_prefix = serve.Server(block_steps=args.block_steps).run(fifo_trace).summary()
    fifo = serve.serve_fifo(fifo_trace).summary()
    log(f"served prefix ({args.fifo_seconds} s): batched {batched_prefix}")
    log(f"served prefix ({args.fifo_seconds} s): fifo {fifo}")
    return {
        "metric": METRIC, "value": st["site_steps_per_s"], "unit": "site-steps/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": st["makespan_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64+c128",
        "data": "synthetic",
        "config": {"workload": f"served_poisson200_{args.serve_seconds:g}s",
                   "requests": len(trace), "offered_site_steps_per_s": offered,
                   "block_steps": args.block_steps, "hbm_budget_bytes": srv.budget,
                   "schedules": {k: list(v) for k, v in serve.SCHEDULES.items()}},
        "latency_p50_s": st["p50_s"], "latency_p99_s": st["p99_s"],
        # 1.0 = the server kept up with the offered load (served everything as fast as
        # it arrived); below 1 the queue grew over the trace
        "served_over_offered": st["site_steps_per_s"] / offered if offered else None,
        "served": st,
        "fifo_comparison": {"trace_seconds": args.fifo_seconds, "batched": batched_prefix,
                            "fifo": fifo},
    }


def cpu_baseline(p, psi0_host, V_host, sample_steps: int):
    import oracle
    oracle.build(force=False)
    cores = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.evolve(psi0_host, V_host, p.dt, sample_steps)
    dt = time.perf_counter() - t0
    return {"value": p.nx * p.ny * sample_steps / dt, "unit": "site-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{p.nx}x{p.ny} mesh of the same workload, first {sample_steps} of its "
                      f"{p.steps} steps, FP64 C oracle (OpenMP over lines), {dt:.1f} s"}


def workload_line(res: dict, args, workload: str, mesh, steps: int, dt: float, **extra) -> dict:
    """The JSON line of a workload measured per dtype (`res`: dtype -> run result):
    complex64 at the top level when it was measured, the other dtype nested."""
    head = "c64" if "c64" in res else next(iter(res))
    r = res[head]
    line = {"metric": METRIC, "value": r["value"], "unit": "site-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": head,
            "data": "synthetic",
            "config": {"workload": workload, "mesh": list(mesh), "time_steps_per_solve": steps,
                       "dt": dt, **extra, **r["schedule"]},
            "roofline": r["roofline"], "norm_drift": r["norm_drift"]}
    for d, rr in res.items():
        if d != head:
            line["complex128" if d == "c128" else "complex64"] = {
                "dtype": d, "value": rr["value"], "unit": "site-steps/s",
                "ms_per_step": rr["ms_per_step"], "config": rr["schedule"],
                "roofline": rr["roofline"], "norm_drift": rr["norm_drift"]}
    return line


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed solves")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves")
    ap.add_argument("--schedule", default="",
                    help="S,segment_rows,pairs_per_lane,phase_store (skip tuning)")
    ap.add_argument("--profile-passes", type=int, default=0,
                    help="counter-collection mode: per dtype run exactly this many fused "
                         "passes under --schedule, plus one device copy of 1 GiB (known "
                         "bytes) to scale the HBM counters; prints a short JSON and exits. "
                         "With --schedule sweep: every candidate schedule, each timed")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=400)
    ap.add_argument("--dtypes", default="c64,c128")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--workload", default="mesh4096",
                    choices=["mesh4096", "mesh32768", "batch512", "served", "td4096", "mesh3d512",
                             "order4_4096", "closed4096", "td_closed4096"],
                    help="mesh4096: the benchmark line; mesh32768: 32768^2 complex64, 200 "
                         "steps; batch512: 512 uneven complex64 problems, 500 steps; "
                         "served: Poisson request stream into the batching server; td4096: "
                         "the 4096^2 workload under a time-dependent potential; mesh3d512: "
                         "512^3 packet in a harmonic well, 100 steps; order4_4096: the 4096^2 "
                         "workload under the fourth-order product, 200 steps; closed4096: the 4096^2 "
                         "workload between hard walls; td_closed4096: td4096 between hard walls")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--fifo-seconds", type=float, default=10.0)
    ap.add_argument("--block-steps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        return 2

    import torch
    from paper_1208_2407_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.workload == "batch512":
        print(json.dumps(run_batch(args)), flush=True)
        return 0
    if args.workload == "served":
        print(json.dumps(run_served(args)), flush=True)
        return 0
    if args.workload == "mesh32768":
        p = wl.config("mesh32768_c64")
        log("generating inputs on the device")
        psi0 = wl.initial_state(p, device="cuda", dtype=torch.complex64)
        V = wl.potential(p, device="cuda")
        res = {"c64": run_dtype("c64", p, psi0, V, args)}
        line = workload_line(res, args, "packets_bumps_32768x32768_dt0.05_200steps", (p.nx, p.ny),
                             p.steps, p.dt)
        print(json.dumps(line), flush=True)
        return 0
    if args.workload == "closed4096":
        p = wl.packets_and_bumps(4096, 4096, 2, 0.05, 1000, "c64", name="packets_bumps_4096")
        log("generating inputs on the device")
        psi0 = wl.initial_state(p, device="cuda")
        V = wl.potential(p, device="cuda")
        res = {d: run_dtype(d, p, psi0, V, args, bc="closed") for d in args.dtypes.split(",")}
        line = workload_line(res, args, "packets_bumps_4096x4096_dt0.05_1000steps_closed",
                             (p.nx, p.ny), p.steps, p.dt, boundary="closed")
        print(json.dumps(line), flush=True)
        return 0
    if args.workload == "order4_4096":
        # five second-order sub-steps per fourth-order step (Sec. 2, Eq. fourthorder)
        p = wl.packets_and_bumps(4096, 4096, 2, 0.05, 200, "c64", name="packets_bumps_4096")
        log("generating inputs on the device")
        psi0 = wl.initial_state(p, device="cuda")
        V = wl.potential(p, device="cuda")
        res = {d: run_dtype(d, p, psi0, V, args, order=4) for d in args.dtypes.split(",")}
        line = workload_line(res, args, "packets_bumps_4096x4096_dt0.05_200steps_order4",
                             (p.nx, p.ny), p.steps, p.dt, order=4,
                             second_order_sub_steps_per_step=5)
        print(json.dumps(line), flush=True)
        return 0
    if args.workload == "mesh3d512":
        p = wl.packet_in_well3(512, 6, dt=0.05, steps=100, sigma=16.0, omega=0.005)
        log("generating inputs on the device")
        psi0 = wl.state3(p, device="cuda")
        V = wl.potential3(p, device="cuda")
        res = {d: run_3d(d, p, psi0, V, args) for d in args.dtypes.split(",")}
        line = workload_line(res, args, "packet_well_512x512x512_dt0.05_100steps",
                             (p.nx, p.ny, p.nz), p.steps, p.dt)
        print(json.dumps(line), flush=True)
        return 0
    if args.workload in ("td4096", "td_closed4096"):
        p = wl.packets_and_bumps(4096, 4096, 2, 0.05, 1000, "c64", name="packets_bumps_4096")
        log("generating inputs on the device")
        psi0 = wl.initial_state(p, device="cuda")
        V0 = wl.potential(p, device="cuda")
        W = wl.standing_wave(p, device="cuda")
        f = wl.drive(p.dt, p.steps)
        bc = "closed" if args.workload == "td_closed4096" else "periodic"
        res = {d: run_td(d, p, psi0, V0, W, f, args, bc=bc) for d in args.dtypes.split(",")}
        name = "packets_bumps_4096x4096_dt0.05_1000steps_shaken_standing_wave"
        line = workload_line(res, args, name + ("_closed" if bc == "closed" else ""),
                             (p.nx, p.ny), p.steps, p.dt, boundary=bc,
                             drive="V0 + 0.2 sin(0.5 t) cos(8 pi i / 4096) at column i")
        print(json.dumps(line), flush=True)
        return 0
    p = wl.packets_and_bumps(4096, 4096, 2, 0.05, 1000, "c64", name="packets_bumps_4096")
    log("generating inputs on the device")
    psi0 = wl.initial_state(p, device="cuda")
    V = wl.potential(p, device="cuda")
    torch.cuda.synchronize()

    if args.profile_passes and args.schedule == "sweep":
        return sweep_mode(p, psi0, V, args)
    if args.profile_passes:
        return profile_mode(p, psi0, V, args)

    res = {}
    for d in args.dtypes.split(","):
        res[d] = run_dtype(d, p, psi0, V, args)

    head = "c64" if "c64" in res else next(iter(res))
    r = res[head]
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "site-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": "packets_bumps_4096x4096_dt0.05_1000steps", "mesh": [p.nx, p.ny],
                   "time_steps_per_solve": p.steps, "dt": p.dt, "boundary": "periodic",
                   **r["schedule"]},
        "roofline": r["roofline"],
        "norm_drift": r["norm_drift"],
    }
    for d, rr in res.items():
        if d == head:
            continue
        line[f"{'complex128' if d == 'c128' else 'complex64'}"] = {
            "dtype": d, "value": rr["value"], "unit": "site-steps/s",
            "ms_per_step": rr["ms_per_step"], "config": rr["schedule"],
            "roofline": rr["roofline"], "norm_drift": rr["norm_drift"]}
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        psi_h = wl.initial_state(p).numpy()
        V_h = V.cpu().numpy()
        line["cpu_baseline"] = cpu_baseline(p, psi_h, V_h, args.cpu_sample_steps)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
