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
# per SIMD) and 7 or 8 steps per pass (a march loop larger than the
# instruction cache); both stay available through tsq_plan_set_schedule.
DEFAULT_CANDIDATES: List[Schedule] = (
    [(1, 0, 1, 1)]
    + [(S, 0, 1, store) for S in (2, 3, 4, 5, 6) for store in (1, 2)]
)


# relative time difference below which two schedules count as equally fast
TIE = 0.01


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


def tune(plan, psi, *, candidates: Optional[Iterable[Schedule]] = None, steps: int = 120,
         use_cache: bool = True, log=None) -> Tuple[Schedule, Dict[str, float]]:
    """Pick the fastest schedule for this plan's mesh and dtype; set it on the plan.

    `psi` is not modified (a scratch copy is evolved).  Returns the schedule and
    the timing table {"S,seg,ppl": ms}."""
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
    for cand in (candidates or DEFAULT_CANDIDATES):
        ms = time_schedule(plan, scratch, cand, steps)
        table[",".join(map(str, cand))] = ms
        timed.append((ms, tuple(cand)))
        if log:
            log(f"autotune {key} S={cand[0]} seg={cand[1]} ppl={cand[2]} store={cand[3]}: "
                f"{ms:.3f} ms")
    del scratch
    best = pick(timed)
    plan.set_schedule(*best)
    if use_cache:
        db[key] = {"schedule": list(best), "table": table, "steps": steps}
        _store(db)
    return best, table
