"""Schedule autotuner for the fused step kernel.

A schedule is (steps_per_pass, segment_rows, pairs_per_lane, phase_store) of
``tsq_plan_set_schedule``.  Every schedule gives bitwise identical results, so
the tuner only times: it evolves a scratch copy of the state for a few passes
under each candidate (HIP events on the current stream), keeps the fastest
(among schedules within ``TIE`` of the fastest, the one with the fewest steps
per pass: it computes fewer redundant halo sites for the same speed), and
caches the choice per (device architecture, dtype, mesh) in a JSON file
(``$TSQ_AUTOTUNE_CACHE``, default ``~/.cache/tsq/autotune.json``).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, List, Optional, Tuple

Schedule = Tuple[int, int, int, int]

# segment_rows 0 = one round of resident wavefronts; phase_store 1 = registers, 2 = LDS.
# Not tried by default: 2 pairs per lane (twice the registers, one wavefront
# per SIMD); it stays available through tsq_plan_set_schedule.  7 and 8 steps
# per pass (LDS ring only) are tried: their march loop outgrows the instruction
# cache, which costs complex64 more than it gains, but complex128's 7-step pass
# measured 3% faster than its 6-step one at 4096^2.
DEFAULT_CANDIDATES: List[Schedule] = (
    [(1, 0, 1, 1)]
    + [(S, 0, 1, store) for S in (2, 3, 4, 5, 6) for store in (1, 2)]
    + [(7, 0, 1, 2), (8, 0, 1, 2)]
)


# relative time difference below which two schedules count as equally fast
TIE = 0.02


def cache_path() -> str:
    return os.environ.get("TSQ_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tsq", "autotune.json"))


def _library_stamp() -> str:
    """Size and modification time of the loaded kernel library: a rebuilt
    library invalidates the cached choices."""
    from . import library_path
    try:
        st = os.stat(library_path())
        return f"{st.st_size}:{int(st.st_mtime)}"
    except OSError:
        return "?"


def _key(arch: str, dtype: str, nx: int, ny: int, order: int = 2, bc: int = 0) -> str:
    return f"{arch}|{dtype}|{nx}x{ny}|o{order}|bc{bc}|{_library_stamp()}"


def _load() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db: Dict[str, dict]) -> None:
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def time_schedule(plan, psi, schedule: Schedule, steps: int, repeats: int = 2) -> float:
    """Best-of-`repeats` milliseconds of plan.evolve(psi, steps) under `schedule`."""
    import torch
    plan.set_schedule(*schedule)
    plan.evolve(psi, min(steps, 2 * schedule[0]))  # warm the code path
    best = float("inf")
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.evolve(psi, steps)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def pick(timed: List[Tuple[float, Schedule]], tie: float = TIE) -> Schedule:
    """The schedule to keep from (milliseconds, schedule) pairs: the fewest
    steps per pass among those within `tie` of the fastest (then the fastest)."""
    fastest = min(ms for ms, _ in timed)
    near = [(c[0], ms, c) for ms, c in timed if ms <= fastest * (1.0 + tie)]
    return min(near)[2]


# Segment heights tried around the one-round default (rows; those taller than the
# mesh are skipped).
SEGMENT_ROWS: List[int] = [32, 64, 128, 256, 512, 1024, 2048, 4096, 8192]


def tune(plan, psi, *, candidates: Optional[Iterable[Schedule]] = None, steps: int = 120,
         use_cache: bool = True, segments: bool = True, log=None
         ) -> Tuple[Schedule, Dict[str, float]]:
    """Pick the fastest schedule for this plan's mesh and dtype; set it on the plan.

    Two stages: steps per pass and phase store at the one-round segment height
    (segment_rows 0), then the segment height (SEGMENT_ROWS, tile shape along y)
    for the winner, which keeps 0 unless another height is faster beyond `TIE`.
    `psi` is not modified (a scratch copy is evolved).  Returns the schedule and
    the timing table {"S,seg,ppl,store": ms}."""
    import torch
    arch = torch.cuda.get_device_properties(psi.device).gcnArchName.split(":")[0]
    key = _key(arch, plan.dtype, plan.problem.nx, plan.problem.ny, plan.problem.order,
               plan.problem.bc)
    db = _load() if use_cache else {}
    if use_cache and key in db and len(db[key].get("schedule", [])) == 4:
        sched = tuple(db[key]["schedule"])
        plan.set_schedule(*sched)
        return sched, db[key].get("table", {})
    scratch = psi.clone()
    table: Dict[str, float] = {}
    timed: List[Tuple[float, Schedule]] = []

    def run(cand):
        ms = time_schedule(plan, scratch, cand, steps)
        table[",".join(map(str, cand))] = ms
        timed.append((ms, tuple(cand)))
        if log:
            log(f"autotune {key} S={cand[0]} seg={cand[1]} ppl={cand[2]} store={cand[3]}: "
                f"{ms:.3f} ms")
        return ms

    for cand in (candidates or DEFAULT_CANDIDATES):
        run(cand)
    best = pick(timed)
    if segments and candidates is None:
        base = next(ms for ms, c in timed if c == best)
        seg_timed = [(base, best)]
        for rows in SEGMENT_ROWS:
            if rows >= plan.problem.ny:
                continue
            cand = (best[0], rows, best[2], best[3])
            seg_timed.append((run(cand), cand))
        # another height only if it beats the one-round default beyond the tie
        fastest = min(seg_timed)
        if fastest[0] < base * (1.0 - TIE):
            best = fastest[1]
    del scratch
    plan.set_schedule(*best)
    if use_cache:
        db[key] = {"schedule": list(best), "table": table, "steps": steps}
        _store(db)
    return best, table


# ---------------------------------------------------------------- time-dependent potential

# steps per pass (the time-dependent march fuses at most 6) x phase store
TD_CANDIDATES: List[Schedule] = [(S, 0, 1, store) for S in (1, 2, 3, 4, 5, 6) for store in (1, 2)]


def time_schedule_td(plan, psi, f, schedule: Schedule, repeats: int = 2) -> float:
    """Best-of-`repeats` milliseconds of plan.evolve_td(psi, f) under `schedule`."""
    import torch
    plan.set_schedule(*schedule)
    plan.evolve_td(psi, f[: 2 * schedule[0]])  # warm the code path
    best = float("inf")
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.evolve_td(psi, f)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune_td(plan, psi, f, *, candidates: Optional[Iterable[Schedule]] = None, steps: int = 120,
            use_cache: bool = True, log=None) -> Tuple[Schedule, Dict[str, float]]:
    """Pick the fastest schedule for a plan holding a time-dependent table
    (tsq_set_potential_td) and set it: times `steps` steps of the modulation `f`
    (repeated if shorter) on a scratch copy of `psi` under each candidate; cached
    per device, dtype, mesh, boundary and library, apart from the static choice."""
    import numpy as np
    import torch
    arch = torch.cuda.get_device_properties(psi.device).gcnArchName.split(":")[0]
    key = _key(arch, plan.dtype, plan.problem.nx, plan.problem.ny, plan.problem.order,
               plan.problem.bc) + "|td"
    db = _load() if use_cache else {}
    if use_cache and key in db and len(db[key].get("schedule", [])) == 4:
        sched = tuple(db[key]["schedule"])
        plan.set_schedule(*sched)
        return sched, db[key].get("table", {})
    fs = np.resize(np.asarray(f, dtype=np.float64), steps)
    scratch = psi.clone()
    table: Dict[str, float] = {}
    timed: List[Tuple[float, Schedule]] = []
    for cand in (candidates or TD_CANDIDATES):
        ms = time_schedule_td(plan, scratch, fs, cand)
        table[",".join(map(str, cand))] = ms
        timed.append((ms, tuple(cand)))
        if log:
            log(f"autotune {key} S={cand[0]} store={cand[3]}: {ms:.3f} ms")
    best = pick(timed)
    del scratch
    plan.set_schedule(*best)
    if use_cache:
        db[key] = {"schedule": list(best), "table": table, "steps": steps}
        _store(db)
    return best, table


# ---------------------------------------------------------------- batched form

# steps per pass x phase store (one pair per lane), then the tile height
BATCH_CANDIDATES: List[Schedule] = [(S, 0, 1, store) for S in (3, 4, 5, 6) for store in (1, 2)]
BATCH_TILE_ROWS: List[int] = [32, 64, 128, 256, 512, 1024]


def signature(dtype: str, shapes) -> str:
    """Workload signature of a batch: dtype and a hash of its sorted (nx, ny, steps)."""
    import hashlib
    items = sorted((int(a), int(b), int(c)) for a, b, c in shapes)
    h = hashlib.sha256(repr(items).encode()).hexdigest()[:16]
    return f"{dtype}|n{len(items)}|{h}"


def batch_signature(plans, steps) -> str:
    return signature(plans[0].dtype, [(pl.problem.nx, pl.problem.ny, n)
                                      for pl, n in zip(plans, steps)])


def time_batch(plans, psis, steps, schedule: Schedule, repeats: int = 2) -> float:
    """Best-of-`repeats` milliseconds of one graph-replayed call of a Batch of
    `plans` over `psis` under `schedule` (the first call captures the graph)."""
    import torch
    from . import Batch
    bt = Batch(plans, psis, steps, schedule)
    bt.launch(use_graph=True)
    best = float("inf")
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        bt.launch(use_graph=True)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del bt
    return best


def tune_batch(plans, psi0s, steps, *, candidates: Optional[Iterable[Schedule]] = None,
               tile_rows: Optional[Iterable[int]] = None, use_cache: bool = True, log=None
               ) -> Tuple[Schedule, Dict[str, float]]:
    """Pick the batch schedule (steps per pass, phase store, then tile height in
    segment_rows) for these problems: times graph-replayed batched calls on
    scratch copies of `psi0s`; caches by device, workload signature and library."""
    import torch
    arch = torch.cuda.get_device_properties(psi0s[0].device).gcnArchName.split(":")[0]
    key = f"{arch}|batch|{batch_signature(plans, steps)}|{_library_stamp()}"
    db = _load() if use_cache else {}
    if use_cache and key in db and len(db[key].get("schedule", [])) == 4:
        return tuple(db[key]["schedule"]), db[key].get("table", {})
    psis = [x.clone() for x in psi0s]
    table: Dict[str, float] = {}
    timed: List[Tuple[float, Schedule]] = []

    def run(cand):
        ms = time_batch(plans, psis, steps, cand)
        table[",".join(map(str, cand))] = ms
        timed.append((ms, tuple(cand)))
        if log:
            log(f"autotune batch S={cand[0]} tile_rows={cand[1]} store={cand[3]}: {ms:.3f} ms")
        return ms

    for cand in (candidates or BATCH_CANDIDATES):
        run(cand)
    best = min(timed)[1]
    base = min(timed)[0]
    rows_timed = [(base, best)]
    for rows in (tile_rows if tile_rows is not None else BATCH_TILE_ROWS):
        cand = (best[0], int(rows), best[2], best[3])
        rows_timed.append((run(cand), cand))
    fastest = min(rows_timed)
    if fastest[0] < base * (1.0 - TIE):
        best = fastest[1]
    del psis
    if use_cache:
        db[key] = {"schedule": list(best), "table": table}
        _store(db)
    return best, table


# ---------------------------------------------------------------- served form

SERVE_CANDIDATES: List[Schedule] = [(S, 0, 1, store) for S in (4, 5, 6) for store in (1, 2)]
# Blocks of 10 steps measured slower in the full served stream (p50 0.09 s against
# 0.04 s at 20; the host builds twice as many iterations), which a 16-request
# sample does not show; the search covers 20 and 40.
SERVE_BLOCKS: List[int] = [20, 40]
# a smaller block (finer scheduling, earlier admission) is kept while its
# throughput stays within this fraction of the best block's
SERVE_BLOCK_SLACK = 0.05


def time_block(plans, psis, steps, schedule: Schedule, repeats: int = 2) -> float:
    """Best-of-`repeats` wall milliseconds of one scheduler iteration as the
    server runs it: build a Batch (host work lists, upload), launch it eagerly,
    wait for it."""
    import time as _time
    import torch
    from . import Batch
    best = float("inf")
    for _ in range(repeats + 1):
        torch.cuda.synchronize()
        t0 = _time.perf_counter()
        bt = Batch(plans, psis, steps, schedule)
        bt.launch()
        torch.cuda.synchronize()
        ms = (_time.perf_counter() - t0) * 1e3
        del bt
        best = min(best, ms)
    return best


def tune_serve(sample, device="cuda", *, per_dtype: int = 16, use_cache: bool = True,
               log=None) -> dict:
    """Schedule per dtype and steps per scheduler iteration for the server, from a
    sample of requests (the first `per_dtype` of each dtype): every (schedule,
    block) advances all sampled problems of a dtype together, timed as the server
    runs an iteration; the schedule with the highest site-steps/s wins, and the
    block is the smallest within SERVE_BLOCK_SLACK of the best block's rate."""
    import torch
    from . import Plan
    from . import workloads as wl
    arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    out = {"schedules": {}, "table": {}}
    block_votes: List[int] = []
    for dtype in ("c64", "c128"):
        reqs = [r for r in sample if r.problem.dtype == dtype][:per_dtype]
        if not reqs:
            continue
        sig = signature(dtype, [(r.problem.nx, r.problem.ny, r.problem.steps) for r in reqs])
        key = f"{arch}|serve|{sig}|{_library_stamp()}"
        db = _load() if use_cache else {}
        if use_cache and key in db:
            out["schedules"][dtype] = tuple(db[key]["schedule"])
            out["table"][dtype] = db[key]["table"]
            block_votes.append(int(db[key]["block"]))
            continue
        tdt = torch.complex64 if dtype == "c64" else torch.complex128
        plans, psis = [], []
        for r in reqs:
            p = r.problem
            pl = Plan(p.nx, p.ny, p.dt, dtype, dx=p.dx, dy=p.dy, mass=p.mass, hbar=p.hbar,
                      device=device)
            pl.set_potential(wl.potential(p, device=device))
            plans.append(pl)
            psis.append(wl.initial_state(p, device=device, dtype=tdt))
        rate: Dict[Tuple[Schedule, int], float] = {}
        table: Dict[str, float] = {}
        for cand in SERVE_CANDIDATES:
            for block in SERVE_BLOCKS:
                steps = [min(block, r.problem.steps) for r in reqs]
                ms = time_block(plans, psis, steps, cand)
                work = sum(r.problem.sites * n for r, n in zip(reqs, steps))
                rate[(cand, block)] = work / (ms * 1e-3)
                table[f"{','.join(map(str, cand))}|{block}"] = ms
                if log:
                    log(f"autotune serve {dtype} S={cand[0]} store={cand[3]} block={block}: "
                        f"{ms:.2f} ms, {rate[(cand, block)]:.3e} site-steps/s")
        best_sched = max(SERVE_CANDIDATES,
                         key=lambda c: max(rate[(c, b)] for b in SERVE_BLOCKS))
        top = max(rate[(best_sched, b)] for b in SERVE_BLOCKS)
        block = min(b for b in SERVE_BLOCKS
                    if rate[(best_sched, b)] >= top * (1.0 - SERVE_BLOCK_SLACK))
        out["schedules"][dtype] = best_sched
        out["table"][dtype] = table
        block_votes.append(block)
        if use_cache:
            db[key] = {"schedule": list(best_sched), "block": block, "table": table}
            _store(db)
        del plans, psis
    out["block_steps"] = max(block_votes) if block_votes else 20
    return out
