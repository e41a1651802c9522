#!/usr/bin/env python3
"""Throughput of the second-order Trotter-Suzuki solve on one MI355X.

Default run (one JSON line on stdout; progress on stderr):
  headline   32768 x 32768 periodic mesh, complex64 (8.6 GB state), four seeded
             Gaussian packets in a harmonic well plus 32 seeded Gaussian bumps
             (recipe scaled to the mesh), dt = 0.05, 200 second-order steps.
             One bench "step" = one whole solve of the hot path: FP64 phase-table
             setup + 200 fused steps + FP64 norm/energy reduction.
  nested     the 4096^2 workload (1000 steps) in complex64 and complex128, the
             256^2 complex128 well (100 steps), the batch of 512 uneven problems,
             the served Poisson stream (p50/p99 latency), and the oracle timed on
             the host cores (cpu_baseline), whose crops also check the headline's
             result.
Inputs are generated on the device before any timed region.  Other workloads:
--workload (see --help).
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


def alg_bytes_per_site(dtype: str, tables: int = 1) -> int:
    """Algorithmic HBM bytes per site of one fused pass: read psi, write psi and
    read the phase factor of each sub-step kind in the pass (one; two for a
    fourth-order pass), each in the working dtype (16 B complex128, 8 B
    complex64)."""
    return (2 + tables) * (16 if dtype == "c128" else 8)


# Bytes per site the library's phase table holds: complex128 exp(-i phi) (16);
# complex64 two 32-bit fixed-point parts (8).
TABLE_BYTES_PER_SITE = {"c128": 16, "c64": 8}


def roofline(dtype: str, sites: int, launch_s: float, site_steps_per_s: float, traffic,
             kernel: str = "march_kernel", tables: int = 1) -> dict:
    """Roofline object of one pass: algorithmic bytes per launch (read and write
    psi, read each phase table, per site, in the working dtype) over the measured
    average launch time, against 8 TB/s."""
    alg = sites * alg_bytes_per_site(dtype, tables)
    achieved = alg / launch_s / 1e9
    elem = 16 if dtype == "c128" else 8
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "kernel": kernel, "avg_launch_us": round(launch_s * 1e6, 2),
           "algorithmic_bytes_per_launch": alg,
           "algorithmic_bytes_per_site": alg_bytes_per_site(dtype, tables),
           # table bytes the pass reads beyond the working dtype's size (0 for both)
           "table_extra_bytes_per_launch": tables * sites * (TABLE_BYTES_PER_SITE[dtype] - elem),
           # one pass per step would move the algorithmic bytes every step: how
           # far fusion takes the solve past that kernel's roofline (> 1)
           "eff_frac_one_pass_per_step": round(site_steps_per_s * alg_bytes_per_site(dtype)
                                               / (HBM_PEAK_GBS * 1e9), 3)}
    if traffic:
        out["traffic_source"] = ("rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel code, mesh "
                                 "and schedule (profiles/traffic.json), not this run")
        out["traffic_over_algorithmic"] = round(traffic / alg, 3)
        out["traffic_GBps"] = round(traffic / launch_s / 1e9, 1)
        out["traffic_frac"] = round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
    return out


def run_dtype(dtype: str, p, psi0, V, args, order: int = 2, bc: str = "periodic",
              keep_result: bool = False):
    """Tune, then time args.steps whole solves (phase table + p.steps fused steps
    + FP64 observables) after args.warmup untimed ones; then one more solve from
    psi0 for the precision figures (norm and energy before and after)."""
    import torch
    import paper_1208_2407_amd as tsq
    from paper_1208_2407_amd import autotune

    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    psi0 = psi0.to(tdt).contiguous()
    psi = psi0.clone()
    plan = tsq.Plan(p.nx, p.ny, p.dt, dtype, order=order, bc=bc, device=psi.device)
    plan.set_potential(V)
    tuning = None
    if args.schedule:
        plan.set_schedule(*[int(v) for v in args.schedule.split(",")])
    elif not args.no_tune:
        sched, table = autotune.tune(plan, psi, log=log if args.verbose else None)
        tuning = {"table_ms": table, "tie": autotune.TIE}
        log(f"{dtype} {p.nx}x{p.ny}: autotuned schedule S={sched[0]} seg={sched[1]} "
            f"ppl={sched[2]} store={sched[3]}")
    sched = plan.schedule()
    passes, copy_back = plan.passes(p.steps)
    stream = torch.cuda.current_stream()

    def solve(events=None):
        plan.set_potential(V)
        if events is not None:
            events[0].record(stream)
        plan.evolve(psi, p.steps)
        if events is not None:
            events[1].record(stream)
        return plan.observables(psi, V)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        solve(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evolve_ms = sum(a.elapsed_time(b) for a, b in evs)
    site_steps = p.nx * p.ny * p.steps * args.steps
    launch_s = evolve_ms * 1e-3 / (args.steps * passes)
    # counters were taken on second-order periodic passes only
    traffic = (committed_traffic(dtype, sched, p.nx, p.ny)
               if order == 2 and bc == "periodic" else None)
    # precision: one solve from the initial state
    psi.copy_(psi0)
    n0, e0 = plan.observables(psi, V)
    n1, e1 = solve()
    log(f"{dtype} {p.nx}x{p.ny}: {wall / args.steps * 1e3:.2f} ms/solve, "
        f"{site_steps / wall:.4e} site-steps/s, pass {launch_s * 1e6:.1f} us, "
        f"norm {n0:.15f} -> {n1:.15f}, energy {e0:.12f} -> {e1:.12f}")
    out = {
        "value": site_steps / wall,
        "ms_per_step": wall / args.steps * 1e3,
        "schedule": {"steps_per_pass": sched[0], "segment_rows": sched[1],
                     "pairs_per_lane": sched[2],
                     "phase_store": {1: "registers", 2: "lds"}[sched[3]],
                     "passes_per_solve": passes, "copy_back": copy_back},
        # a fourth-order pass on a periodic mesh reads both sub-step tables
        "roofline": roofline(dtype, p.nx * p.ny, launch_s, site_steps / wall, traffic,
                             tables=2 if order == 4 and bc == "periodic" else 1),
        "precision": {"norm_start": n0, "norm_end": n1, "norm_drift": n1 - n0,
                      "energy_start": e0, "energy_end": e1, "energy_drift": e1 - e0},
    }
    if tuning:
        out["tuning"] = tuning
    if keep_result:
        out["psi"] = psi
    else:
        del psi
    del plan
    return out


def vs_oracle(prec: dict, ref: dict) -> dict:
    """GPU norm and energy (start and end of one solve) against the oracle's, from
    the same starting values."""
    return {"oracle_norm_drift": ref["norm_end"] - ref["norm_start"],
            "oracle_energy_drift": ref["energy_end"] - ref["energy_start"],
            "norm_end_minus_oracle": prec["norm_end"] - ref["norm_end"],
            "energy_end_rel_diff": abs(prec["energy_end"] - ref["energy_end"])
            / abs(ref["energy_end"]),
            "energy_start_rel_diff": abs(prec["energy_start"] - ref["energy_start"])
            / abs(ref["energy_start"]),
            "oracle_source": "tests/golden/oracle_observables_4096.json (FP64 oracle, "
                             "same workload and starting values)"}


def run_td(dtype: str, p, psi0, V0, W, f, args, bc: str = "periodic"):
    """One solve under the time-dependent potential V0 + f(t) W: table setup,
    len(f) fused steps (the phase formed in FP64 in the march), FP64 observables
    at the final time."""
    import torch
    import paper_1208_2407_amd as tsq

    from paper_1208_2407_amd import autotune

    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    psi = psi0.to(tdt).contiguous()
    plan = tsq.Plan(p.nx, p.ny, p.dt, dtype, bc=bc, device=psi.device)
    plan.set_potential_td(V0, W)
    if args.schedule:
        plan.set_schedule(*[int(v) for v in args.schedule.split(",")])
    else:
        autotune.tune_td(plan, psi, f[:120], log=log if args.verbose else None)
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
    # read psi, write psi, read (theta0, w): the potential's two FP64 parts per site
    alg_bytes = p.nx * p.ny * (2 * elem + 16)
    launch_s = evolve_ms * 1e-3 / (args.steps * passes)
    achieved = alg_bytes / launch_s / 1e9
    log(f"td {dtype}: S={sched[0]} store={sched[3]}: {wall / args.steps * 1e3:.2f} ms/solve, "
        f"{site_steps / wall:.4e} site-steps/s, pass {launch_s * 1e6:.1f} us, norm {norm:.15f}")
    return {
        "value": site_steps / wall, "ms_per_step": wall / args.steps * 1e3,
        "schedule": {"steps_per_pass": sched[0], "pairs_per_lane": sched[2],
                     "phase_store": {1: "registers", 2: "lds"}[sched[3]],
                     "passes_per_solve": passes, "copy_back": copy_back,
                     "picked_by": "given" if args.schedule else "autotune.tune_td"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "algorithmic_bytes_per_site": 2 * elem + 16, "kernel": "march_kernel (td)",
                     "avg_launch_us": round(launch_s * 1e6, 2)},
        "precision": {"norm_drift": norm - n_begin},
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
    launch_s = evolve_ms * 1e-3 / (args.steps * passes)
    traffic = committed_traffic(dtype, (1,), p.nx, p.ny, p.nz)
    log(f"3d {dtype}: {wall / args.steps * 1e3:.2f} ms/solve, {site_steps / wall:.4e} site-steps/s, "
        f"pass {launch_s * 1e6:.1f} us, norm {norm:.15f}")
    return {
        "value": site_steps / wall, "ms_per_step": wall / args.steps * 1e3,
        "schedule": {"steps_per_pass": 1, "passes_per_solve": passes, "copy_back": copy_back},
        "roofline": roofline(dtype, p.sites, launch_s, site_steps / wall, traffic,
                             kernel="march3_kernel"),
        "precision": {"norm_drift": norm - n_begin},
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
                          "algorithmic_bytes_per_launch": p.nx * p.ny * alg_bytes_per_site(d)}
    print(json.dumps(out), flush=True)
    return 0


def sweep_mode(p, psi0, V, args) -> int:
    """Every candidate schedule of the tuner (1-8 steps per pass) for
    exactly --profile-passes passes after a warm-up, each timed with HIP events
    on the current stream, then for twice as many: the difference is the time
    of steady passes alone (the first and the closing pass, which differ, drop
    out).  One JSON line per dtype and schedule.  Run under rocprofv3 --pmc it
    also gives the HBM counters of every schedule."""
    import torch
    import paper_1208_2407_amd as tsq
    from paper_1208_2407_amd import autotune

    cands = list(autotune.DEFAULT_CANDIDATES)
    if ":" in args.schedule:  # sweep:ROWS, every candidate at that segment height
        rows = int(args.schedule.split(":", 1)[1])
        cands = [(c[0], rows, c[2], c[3]) for c in cands]
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
        alg = p.nx * p.ny * alg_bytes_per_site(d)
        for sched in cands:
            psi = psi0.to(tdt).clone()
            plan = tsq.Plan(p.nx, p.ny, p.dt, d, device=psi.device)
            plan.set_potential(V)
            plan.set_schedule(*sched)
            S = sched[0]
            plan.evolve(psi, 2 * S)
            def timed(steps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record(stream)
                plan.evolve(psi, steps)
                e1.record(stream)
                e1.synchronize()
                return e0.elapsed_time(e1) * 1e-3

            steps = S * args.profile_passes
            passes = plan.passes(steps)[0]
            sec = timed(steps)
            pass_s = sec / passes
            # twice the passes: the difference holds steady passes only
            passes2 = plan.passes(2 * steps)[0]
            steady_s = max(timed(2 * steps) - sec, 0.0) / max(passes2 - passes, 1)
            print(json.dumps({"sweep": True, "dtype": d, "schedule": list(sched),
                              "kernel_hash": kernel_hash(), "mesh": [p.nx, p.ny],
                              "steps": steps, "passes": passes,
                              "avg_pass_us": round(pass_s * 1e6, 2),
                              "steady_pass_us": round(steady_s * 1e6, 2),
                              "us_per_step": round(sec / steps * 1e6, 3),
                              "site_steps_per_s": p.nx * p.ny * steps / sec,
                              "steady_site_steps_per_s": (p.nx * p.ny * S / steady_s
                                                          if steady_s > 0 else None),
                              "algorithmic_bytes_per_launch": alg,
                              "frac": round(alg / pass_s / 1e9 / HBM_PEAK_GBS, 4),
                              "steady_frac": (round(alg / steady_s / 1e9 / HBM_PEAK_GBS, 4)
                                              if steady_s > 0 else None),
                              "eff_frac_one_pass_per_step": round(
                                  p.nx * p.ny * steps / sec * alg / (p.nx * p.ny) / 1e9
                                  / HBM_PEAK_GBS, 3)}), flush=True)
            del psi, plan
    return 0


def run_batch(args) -> dict:
    """512 independent complex64 problems (sides log-uniform in [64, 1024], rounded to
    even; own potential, packets and dt), 500 steps each: one batched call (captured
    HIP graph, schedule and tile height from the autotuner) against sequential plain
    tsq_evolve calls on the same GPU."""
    import torch
    import paper_1208_2407_amd as tsq
    from paper_1208_2407_amd import autotune
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

    if args.schedule:
        sched, table = tuple(int(v) for v in args.schedule.split(",")), {}
    else:
        sched, table = autotune.tune_batch(plans, psi0s, steps,
                                           log=log if args.verbose else None)
    log(f"batch: schedule S={sched[0]} tile_rows={sched[1]} store={sched[3]}")
    psis = [x.clone() for x in psi0s]
    bt = tsq.Batch(plans, psis, steps, sched)
    launches, tiles = bt.info()
    for _ in range(args.warmup):
        bt.launch(use_graph=True)
    t_batch = timed(lambda: bt.launch(use_graph=True), args.steps)
    # sequential plain solves: each problem alone, same kernels and steps per pass
    seq = [x.clone() for x in psi0s]
    for pl in plans:
        pl.set_schedule(sched[0], 0, sched[2], sched[3])

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
    # precision: the largest norm drift over the batch (FP64 reductions)
    drift = 0.0
    for pl, x, x0, V in zip(plans, one, psi0s, Vs):
        n1, _ = pl.observables(x, V)
        n0, _ = pl.observables(x0, V)
        drift = max(drift, abs(n1 - n0))
    log(f"batch: {t_batch * 1e3:.1f} ms per call, sequential {t_seq * 1e3:.1f} ms, "
        f"speedup {t_seq / t_batch:.2f}x, bitwise equal to alone: {same}, "
        f"max |norm drift| {drift:.2e}")
    return {
        "workload": "batch512_c64_500steps", "value": site_steps / t_batch,
        "unit": "site-steps/s", "ms_per_call": t_batch * 1e3, "calls_timed": args.steps,
        "problems": len(probs), "sites": sites, "site_steps_per_call": site_steps,
        "schedule": {"steps_per_pass": sched[0], "tile_rows": sched[1] or "auto",
                     "phase_store": "registers" if sched[3] == 1 else "lds",
                     "picked_by": "given" if args.schedule else "autotune.tune_batch"},
        "tuning_table_ms": table,
        "launches_per_call": launches, "tiles_per_call": tiles, "hip_graph": True,
        "sequential": {"value": site_steps / t_seq, "ms_per_call": t_seq * 1e3},
        "speedup_vs_sequential": t_seq / t_batch,
        "bitwise_equal_to_alone": same,
        "precision": {"max_abs_norm_drift": drift},
    }


def run_served(args) -> dict:
    """Poisson arrivals at 200 req/s for --serve-seconds seconds (sides log-uniform
    128-4096, steps 100-2000, 80/20 complex64/complex128) replayed in real time into
    the continuous-batching server; the FIFO one-at-a-time server on the first
    --fifo-seconds of the same trace for comparison."""
    from paper_1208_2407_amd import serve
    from paper_1208_2407_amd import workloads as wl

    trace = wl.request_trace(rate=200.0, duration=args.serve_seconds, seed=5)
    offered = sum(r.problem.site_steps for r in trace) / args.serve_seconds
    log(f"served: {len(trace)} requests over {args.serve_seconds} s, offered {offered:.3e} "
        f"site-steps/s")
    # schedules and block size from the autotuner on the trace's first requests
    srv = serve.Server(block_steps=args.block_steps)
    if not args.block_steps:
        srv.tune(trace[:200], log=log if args.verbose else None)
    log(f"served: schedules {srv.schedules}, block {srv.block} steps")
    # warm the code paths
    serve.Server(block_steps=srv.block, schedules=srv.schedules).run(trace[:16], realtime=False)
    st = srv.run(trace, realtime=True).summary()
    log(f"served: {st}")
    out = {
        "workload": f"served_poisson200_{args.serve_seconds:g}s", "requests": len(trace),
        "offered_site_steps_per_s": offered, "value": st["site_steps_per_s"],
        "unit": "site-steps/s", "latency_p50_s": st["p50_s"], "latency_p99_s": st["p99_s"],
        # 1.0 = the server kept up with the offered load (served everything as fast as
        # it arrived); below 1 the queue grew over the trace
        "served_over_offered": st["site_steps_per_s"] / offered if offered else None,
        "admitted": st["admitted"], "rejected": st["rejected"], "completed": st["completed"],
        "block_steps": srv.block, "hbm_budget_bytes": srv.budget,
        "schedules": srv.schedule_report(), "server": st,
    }
    # utilization rho = offered load / the server's capacity, the capacity being its
    # rate when saturated: the first 5 s of the trace, every request available at once
    sat_trace = [r for r in trace if r.arrival < 5.0]
    sat = serve.Server(block_steps=srv.block, schedules=srv.schedules).run(
        sat_trace, realtime=False).summary()
    out["capacity_site_steps_per_s"] = sat["site_steps_per_s"]
    out["utilization_rho"] = offered / sat["site_steps_per_s"] if sat["site_steps_per_s"] else None
    log(f"served: saturated capacity {sat['site_steps_per_s']:.3e} site-steps/s, "
        f"rho {out['utilization_rho']:.2f}")
    if args.fifo_seconds > 0:
        fifo_trace = [r for r in trace if r.arrival < args.fifo_seconds]
        batched_prefix = serve.Server(block_steps=srv.block,
                                      schedules=srv.schedules).run(fifo_trace).summary()
        fifo = serve.serve_fifo(fifo_trace, schedules=srv.schedules).summary()
        log(f"served prefix ({args.fifo_seconds} s): batched {batched_prefix}")
        log(f"served prefix ({args.fifo_seconds} s): fifo {fifo}")
        out["fifo_comparison"] = {"trace_seconds": args.fifo_seconds,
                                  "batched": batched_prefix, "fifo": fifo}
    return out


def crops_of(p, psi0, V, width: int = 2048):
    """Host copies (complex128 / float64) of `width`^2 windows of the device inputs,
    one centred on each packet (corners on even sites)."""
    n = p.nx
    out = []
    for q in p.packets:
        yc = int(round(q.y0 / p.dy + p.ny / 2)) // 2 * 2
        xc = int(round(q.x0 / p.dx + n / 2)) // 2 * 2
        y0, x0 = yc - width // 2, xc - width // 2
        out.append((y0, x0, psi0[y0:y0 + width, x0:x0 + width].cpu().numpy().astype("complex128"),
                    V[y0:y0 + width, x0:x0 + width].cpu().numpy()))
    return out


def cpu_baseline(p, crops, results, one_core_steps: int) -> dict:
    """The FP64 oracle on the host cores: the four 2048^2 crops of the headline
    mesh (one centred on each packet), p.steps steps each, on every host thread,
    and one crop for `one_core_steps` steps on one thread.  Each crop's interior
    (a margin of the light cone 2N+1 plus one site per side) is compared with the
    GPU's result of the same solve (`results`: the GPU interiors)."""
    import numpy as np
    import oracle

    oracle.build(force=False)
    cores = oracle.max_threads()
    oracle.set_threads(cores)
    t0 = time.perf_counter()
    outs = [oracle.evolve(c, v, p.dt, p.steps) for (_, _, c, v) in crops]
    t_all = time.perf_counter() - t0
    w = crops[0][2].shape[0]
    sites = sum(c.shape[0] * c.shape[1] for (_, _, c, _) in crops)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.evolve(crops[0][2], crops[0][3], p.dt, one_core_steps)
    t_one = time.perf_counter() - t0
    oracle.set_threads(cores)
    m = 2 * p.steps + 2
    errs = []
    for want, got in zip(outs, results):
        wi = want[m:w - m, m:w - m]
        errs.append(float(np.linalg.norm(got - wi) / np.linalg.norm(wi)))
    log(f"oracle: {cores} threads {sites * p.steps / t_all:.3e} site-steps/s ({t_all:.1f} s), "
        f"1 thread {w * w * one_core_steps / t_one:.3e} ({t_one:.1f} s); crop interiors rel L2 "
        + ", ".join(f"{e:.2e}" for e in errs))
    return {
        "baseline": {"value": sites * p.steps / t_all, "unit": "site-steps/s", "cores": cores,
                     "kind": "oracle",
                     "sample": f"the FP64 C oracle (OpenMP over lines) on four {w}x{w} crops of "
                               f"the {p.nx}x{p.ny} mesh, one centred on each packet, {p.steps} "
                               f"steps each ({t_all:.1f} s)",
                     "one_core": {"value": w * w * one_core_steps / t_one, "cores": 1,
                                  "sample": f"one {w}x{w} crop, {one_core_steps} steps "
                                            f"({t_one:.1f} s)"}},
        "crop_rel_l2": errs, "crop_interior": w - 2 * m,
    }


def dtype_entry(r: dict, **extra) -> dict:
    """Nested JSON object of one dtype's run."""
    out = {"value": r["value"], "unit": "site-steps/s", "ms_per_solve": r["ms_per_step"],
           "schedule": r["schedule"], "roofline": r["roofline"], "precision": r["precision"]}
    out.update(extra)
    if "tuning" in r:
        out["tuning"] = r["tuning"]
    return out


def line_head(args, value: float, ms: float, dtype: str, config: dict) -> dict:
    return {"metric": METRIC, "value": value, "unit": "site-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def workload_line(res: dict, args, workload: str, mesh, steps: int, dt: float, **extra) -> dict:
    """The JSON line of a workload measured per dtype (`res`: dtype -> run result):
    complex64 at the top level when it was measured, the other dtype nested."""
    head = "c64" if "c64" in res else next(iter(res))
    r = res[head]
    line = line_head(args, r["value"], r["ms_per_step"], head,
                     {"workload": workload, "mesh": list(mesh), "time_steps_per_solve": steps,
                      "dt": dt, **extra, **r["schedule"]})
    line["roofline"] = r["roofline"]
    line["precision"] = r["precision"]
    for d, rr in res.items():
        if d != head:
            line["complex128" if d == "c128" else "complex64"] = dtype_entry(rr)
    return line


ORACLE_OBSERVABLES = os.path.join(ROOT, "tests", "golden", "oracle_observables_4096.json")


def default_run(args) -> dict:
    """The default benchmark line: the 32768^2 complex64 headline with the 4096^2
    (both dtypes), 256^2, batched and served workloads nested, and the oracle."""
    import torch
    from paper_1208_2407_amd import workloads as wl

    t_start = time.perf_counter()
    p = wl.config("mesh32768_c64")
    log(f"headline: generating the {p.nx}x{p.ny} inputs on the device")
    psi0 = wl.initial_state(p, device="cuda", dtype=torch.complex64)
    V = wl.potential(p, device="cuda")
    torch.cuda.synchronize()
    crops = [] if args.no_cpu_baseline else crops_of(p, psi0, V)
    r = run_dtype("c64", p, psi0, V, args, keep_result=True)
    m = 2 * p.steps + 2
    interiors = []
    for (y0, x0, c, _) in crops:
        w = c.shape[0]
        interiors.append(r["psi"][y0 + m:y0 + w - m, x0 + m:x0 + w - m].cpu().numpy()
                         .astype("complex128"))
    del r["psi"], psi0, V
    torch.cuda.empty_cache()
    line = line_head(args, r["value"], r["ms_per_step"], "c64",
                     {"workload": "packets_bumps_32768x32768_dt0.05_200steps",
                      "mesh": [p.nx, p.ny], "time_steps_per_solve": p.steps, "dt": p.dt,
                      "boundary": "periodic",
                      "step": "one solve: FP64 phase table, 200 fused steps, FP64 norm and "
                              "energy", **r["schedule"]})
    line["roofline"] = r["roofline"]
    line["precision"] = r["precision"]
    if "tuning" in r:
        line["tuning"] = r["tuning"]
    log(f"headline done ({time.perf_counter() - t_start:.0f} s)")

    # the 4096^2 workload, both dtypes, against the oracle's norm and energy
    p2 = wl.packets_and_bumps(4096, 4096, 2, 0.05, 1000, "c64", name="packets_bumps_4096")
    psi02 = wl.initial_state(p2, device="cuda")
    V2 = wl.potential(p2, device="cuda")
    try:
        with open(ORACLE_OBSERVABLES) as f:
            ref = json.load(f)["inputs"]
    except (OSError, ValueError, KeyError):
        ref = {}
    nested = {"workload": "packets_bumps_4096x4096_dt0.05_1000steps", "mesh": [4096, 4096],
              "time_steps_per_solve": p2.steps, "dt": p2.dt}
    for d in ("c64", "c128"):
        rr = run_dtype(d, p2, psi02, V2, args)
        if d in ref:
            rr["precision"]["vs_oracle"] = vs_oracle(rr["precision"], ref[d])
        nested[d] = dtype_entry(rr)
    line["mesh4096"] = nested
    del psi02, V2
    # the 256^2 well, complex128 (its 1 MiB state stays in the caches: no HBM figure)
    p1 = wl.gaussian_in_well(dtype="c128")
    r1 = run_dtype("c128", p1, wl.initial_state(p1, device="cuda"), wl.potential(p1, device="cuda"),
                   args)
    r1["roofline"] = {"note": "1 MiB state held in L2 and the Infinity Cache: no HBM "
                              "roofline", "avg_launch_us": r1["roofline"]["avg_launch_us"]}
    line["mesh256"] = dtype_entry(r1, workload="gaussian_well_256x256_dt0.1_100steps",
                                  dtype="c128")
    torch.cuda.empty_cache()
    log(f"nested meshes done ({time.perf_counter() - t_start:.0f} s)")
    if not args.no_batch:
        line["batch512"] = run_batch(args)
        torch.cuda.empty_cache()
        log(f"batch done ({time.perf_counter() - t_start:.0f} s)")
    if not args.no_served:
        line["served"] = run_served(args)
        torch.cuda.empty_cache()
        log(f"served done ({time.perf_counter() - t_start:.0f} s)")
    if crops:
        log("timing the oracle on the crops of the headline mesh")
        cb = cpu_baseline(p, crops, interiors, args.cpu_one_core_steps)
        line["cpu_baseline"] = cb["baseline"]
        line["precision"]["vs_oracle_crops"] = {
            "rel_l2": cb["crop_rel_l2"], "interior": cb["crop_interior"],
            "note": "GPU complex64 result of the precision solve against the FP64 oracle on "
                    "2048^2 crops centred on the four packets, compared on the interior their "
                    "edges cannot reach in 200 steps"}
    log(f"bench done ({time.perf_counter() - t_start:.0f} s)")
    return line


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed solves (calls) per workload")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves per workload")
    ap.add_argument("--schedule", default="",
                    help="S,segment_rows,pairs_per_lane,phase_store (skip tuning)")
    ap.add_argument("--profile-passes", type=int, default=0,
                    help="counter-collection mode (mesh4096 and mesh32768 workloads): per "
                         "dtype run exactly this many fused passes under --schedule, plus one "
                         "device copy of 1 GiB (known bytes) to scale the HBM counters; prints "
                         "a short JSON and exits.  With --schedule sweep: every candidate "
                         "schedule, each timed (--schedule sweep:ROWS: at segments of ROWS "
                         "rows)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="default run: skip the batch")
    ap.add_argument("--no-served", action="store_true", help="default run: skip the stream")
    ap.add_argument("--cpu-one-core-steps", type=int, default=40)
    ap.add_argument("--dtypes", default="c64,c128")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--workload", default="default",
                    choices=["default", "mesh4096", "mesh32768", "batch512", "served", "td4096",
                             "mesh3d512", "order4_4096", "closed4096", "td_closed4096"],
                    help="default: the 32768^2 complex64 headline with every other benchmark "
                         "workload nested; mesh4096: the 4096^2 workload alone; mesh32768: the "
                         "32768^2 complex64 mesh alone (200 steps); batch512: 512 uneven "
                         "complex64 problems, 500 steps; served: Poisson request stream into the "
                         "batching server; td4096: the 4096^2 workload under a time-dependent "
                         "potential; mesh3d512: 512^3 packet in a harmonic well, 100 steps; "
                         "order4_4096: the 4096^2 workload under the fourth-order product, 200 "
                         "steps; closed4096: the 4096^2 workload between hard walls; "
                         "td_closed4096: td4096 between hard walls")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--fifo-seconds", type=float, default=5.0)
    ap.add_argument("--block-steps", type=int, default=0,
                    help="served: steps per scheduler iteration (0 = the tuned value)")
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
    if args.workload == "default" and not args.profile_passes:
        print(json.dumps(default_run(args)), flush=True)
        return 0
    if args.workload == "batch512":
        r = run_batch(args)
        line = line_head(args, r["value"], r["ms_per_call"], "c64",
                         {"workload": r["workload"], "problems": r["problems"]})
        line.update({k: v for k, v in r.items() if k not in ("value", "workload", "unit")})
        print(json.dumps(line), flush=True)
        return 0
    if args.workload == "served":
        r = run_served(args)
        line = line_head(args, r["value"], r["server"]["makespan_s"] * 1e3, "c64+c128",
                         {"workload": r["workload"], "requests": r["requests"]})
        line.update({k: v for k, v in r.items() if k not in ("value", "workload", "unit")})
        print(json.dumps(line), flush=True)
        return 0
    if args.workload == "mesh32768":
        p = wl.config("mesh32768_c64")
        log("generating inputs on the device")
        psi0 = wl.initial_state(p, device="cuda", dtype=torch.complex64)
        V = wl.potential(p, device="cuda")
        if args.profile_passes and args.schedule.startswith("sweep"):
            return sweep_mode(p, psi0, V, args)
        if args.profile_passes:
            return profile_mode(p, psi0, V, args)
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
    if args.profile_passes and args.schedule.startswith("sweep"):
        return sweep_mode(p, psi0, V, args)
    if args.profile_passes:
        return profile_mode(p, psi0, V, args)
    res = {d: run_dtype(d, p, psi0, V, args) for d in args.dtypes.split(",")}
    line = workload_line(res, args, "packets_bumps_4096x4096_dt0.05_1000steps", (p.nx, p.ny),
                         p.steps, p.dt, boundary="periodic")
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
