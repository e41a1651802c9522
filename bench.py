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


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("tsq_kernels.hip", "tsq_internal.h"):
        with open(os.path.join(ROOT, "paper_1208_2407_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(dtype: str, schedule) -> float | None:
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they were
    taken on this exact kernel source and schedule; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        return None
    e = db.get(kernel_hash(), {}).get(dtype)
    if not e or list(e.get("schedule", [])) != list(schedule):
        return None
    return float(e["bytes_per_launch"])


def run_dtype(dtype: str, p, psi0, V, args):
    import torch
    import paper_1208_2407_amd as tsq
    from paper_1208_2407_amd import autotune

    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    psi = psi0.to(tdt).contiguous()
    plan = tsq.Plan(p.nx, p.ny, p.dt, dtype, device=psi.device)
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
    traffic = committed_traffic(dtype, sched)
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
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "kernel": "march_kernel", "avg_launch_us": round(launch_s * 1e6, 2)},
        "norm_drift": norm - n_begin,
        "energy": energy,
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
                         "bytes) to scale the HBM counters; prints a short JSON and exits")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=400)
    ap.add_argument("--dtypes", default="c64,c128")
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        return 2

    import torch
    from paper_1208_2407_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    p = wl.packets_and_bumps(4096, 4096, 2, 0.05, 1000, "c64", name="packets_bumps_4096")
    log("generating inputs on the device")
    psi0 = wl.initial_state(p, device="cuda")
    V = wl.potential(p, device="cuda")
    torch.cuda.synchronize()

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
