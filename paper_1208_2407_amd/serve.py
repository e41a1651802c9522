"""Continuous-batching request server for Trotter-Suzuki solves on one GPU.

A request is one problem statement (mesh, constants, dt, step count, input
recipe) arriving at a given time.  The server keeps every admitted request's
state resident in device memory and advances all of them together:

* admission: a queued request is admitted as soon as its device memory
  (psi, potential, workspace) fits in the HBM budget; a request larger than
  the whole budget is rejected;
* each scheduler iteration advances every resident request by one block of
  `block_steps` steps (or its remainder) with one batched call per dtype
  (``tsq_batch_*``), enqueued on the stream without waiting for the previous
  iteration; an event marks its end;
* a request whose last block's event has completed is retired: its latency is
  completion minus arrival, its memory is released, and queued requests can
  take its place.

A request's blocks depend only on its own step count, so its result is
bitwise identical whether it is served alone or among others.  The FIFO
baseline (:func:`serve_fifo`) solves one request at a time with a plain
``tsq_evolve``.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np
import torch

import paper_1208_2407_amd as tsq
from paper_1208_2407_amd import workloads as wl

# Schedule of each dtype's batched calls before the tuner has run (5 steps per pass,
# register phase ring) and the steps per scheduler iteration; Server.tune replaces
# both with autotune.tune_serve's choice.
SCHEDULES = {"c64": (5, 0, 1, 1), "c128": (5, 0, 1, 1)}
BLOCK_STEPS = 20


def request_bytes(p: wl.Problem) -> int:
    """Device bytes a resident request holds: psi, V and the plan's workspace."""
    elem = 16 if p.dtype == "c128" else 8
    return p.sites * (elem + 8 + elem + 16) + (1 << 16)


@dataclasses.dataclass
class Slot:
    req: wl.Request
    plan: tsq.Plan
    psi: torch.Tensor
    V: torch.Tensor
    remaining: int
    bytes: int
    t_admit: float


@dataclasses.dataclass
class Stats:
    latencies: List[float]
    site_steps: int
    makespan: float
    admitted: int
    rejected: int
    iterations: int
    max_resident: int
    batches_built: int = 0
    graph_replays: int = 0

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.array([np.nan])
        return {"completed": len(self.latencies), "admitted": self.admitted,
                "rejected": self.rejected, "p50_s": float(np.percentile(lat, 50)),
                "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
                "site_steps": self.site_steps, "makespan_s": self.makespan,
                "site_steps_per_s": self.site_steps / self.makespan if self.makespan else 0.0,
                "iterations": self.iterations, "max_resident": self.max_resident,
                "batches_built": self.batches_built, "graph_replays": self.graph_replays}


class Server:
    """`schedules` (dtype -> schedule) and `block_steps` default to the module's
    SCHEDULES and BLOCK_STEPS; :meth:`tune` picks them with the autotuner for a
    sample of the requests to come."""

    def __init__(self, hbm_budget: int = 96 << 30, block_steps: int = 0,
                 max_in_flight: int = 2, keep_results: bool = False, device="cuda",
                 schedules: Optional[Dict[str, tuple]] = None):
        self.budget = int(hbm_budget)
        self.block = int(block_steps) or BLOCK_STEPS
        self.schedules = dict(schedules or SCHEDULES)
        self.tuned: Optional[dict] = None
        self.max_in_flight = max_in_flight
        self.keep_results = keep_results
        self.device = torch.device(device)
        self.results: Dict[int, torch.Tensor] = {}
        self.graph_replays = 0
        self.batches_built = 0

    def tune(self, sample: List[wl.Request], log=None) -> dict:
        """Schedules and block size from autotune.tune_serve on `sample`."""
        from . import autotune
        res = autotune.tune_serve(sample, device=self.device, log=log)
        self.schedules.update(res["schedules"])
        self.block = res["block_steps"]
        self.tuned = res
        return res

    def schedule_report(self) -> dict:
        return {"schedules": {k: list(v) for k, v in self.schedules.items()},
                "block_steps": self.block,
                "picked_by": "autotune.tune_serve" if self.tuned else "module defaults",
                "tuning": self.tuned}

    def _admit(self, r: wl.Request, now: float) -> Slot:
        p = r.problem
        tdt = torch.complex64 if p.dtype == "c64" else torch.complex128
        psi = wl.initial_state(p, device=self.device, dtype=tdt)
        V = wl.potential(p, device=self.device)
        plan = tsq.Plan(p.nx, p.ny, p.dt, p.dtype, dx=p.dx, dy=p.dy, mass=p.mass, hbar=p.hbar,
                        device=self.device)
        plan.set_schedule(*self.schedules[p.dtype])
        plan.set_potential(V)
        return Slot(r, plan, psi, V, p.steps, request_bytes(p), now)

    def run(self, trace: List[wl.Request], realtime: bool = True) -> Stats:
        """Serve `trace`.  realtime: release each request at its arrival time (wall
        clock from the start); otherwise every request is available at time 0."""
        pending = collections.deque(sorted(trace, key=lambda r: r.arrival))
        queue: collections.deque = collections.deque()
        resident: List[Slot] = []
        in_flight: collections.deque = collections.deque()  # (event, batches, finishing)
        used = 0
        latencies: List[float] = []
        site_steps = 0
        admitted = rejected = iterations = max_resident = 0
        side = torch.cuda.Stream(device=self.device)
        last_batch: Dict[str, tuple] = {}
        self.graph_replays = self.batches_built = 0
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()

        def now() -> float:
            return time.perf_counter() - t0

        def arrival(r: wl.Request) -> float:
            return r.arrival if realtime else 0.0

        def retire(entry) -> None:
            nonlocal used, site_steps
            ev, batches, done = entry
            ev.synchronize()
            tdone = now()
            for s in done:
                latencies.append(tdone - arrival(s.req))
                site_steps += s.req.problem.site_steps
                used -= s.bytes
                if self.keep_results:
                    self.results[s.req.rid] = s.psi

        while pending or queue or resident or in_flight:
            t = now()
            while pending and arrival(pending[0]) <= t:
                queue.append(pending.popleft())
            while in_flight and in_flight[0][0].query():
                retire(in_flight.popleft())
            while queue:
                need = request_bytes(queue[0].problem)
                if need > self.budget:
                    queue.popleft()
                    rejected += 1
                    continue
                if used + need > self.budget:
                    break
                resident.append(self._admit(queue.popleft(), now()))
                used += need
                admitted += 1
            max_resident = max(max_resident, len(resident))
            if resident and len(in_flight) < self.max_in_flight:
                # complex64 requests on the current stream, complex128 ones on a side
                # stream (default priority) so the two batched calls overlap
                batches = []
                cur = torch.cuda.current_stream(self.device)
                groups = {dt: [s for s in resident if s.req.problem.dtype == dt]
                          for dt in ("c64", "c128")}
                two = bool(groups["c64"]) and bool(groups["c128"])
                if two:
                    side.wait_stream(cur)
                for dtype, stream in (("c64", cur), ("c128", side if two else cur)):
                    group = groups[dtype]
                    if not group:
                        continue
                    steps = [min(self.block, s.remaining) for s in group]
                    # the same resident set advancing by the same steps as in the
                    # previous iteration: replay that batch's captured graph
                    key = tuple((s.req.rid, n) for s, n in zip(group, steps))
                    with torch.cuda.stream(stream):
                        prev = last_batch.get(dtype)
                        if prev is not None and prev[0] == key:
                            b = prev[1]
                            b.launch(use_graph=True)
                            self.graph_replays += 1
                        else:
                            b = tsq.Batch([s.plan for s in group], [s.psi for s in group], steps,
                                          self.schedules[dtype])
                            b.launch()
                            self.batches_built += 1
                            last_batch[dtype] = (key, b)
                    batches.append(b)
                    for s, n in zip(group, steps):
                        s.remaining -= n
                if two:
                    cur.wait_stream(side)
                ev = torch.cuda.Event()
                ev.record(cur)
                finishing = [s for s in resident if s.remaining == 0]
                resident = [s for s in resident if s.remaining > 0]
                in_flight.append((ev, batches, finishing))
                iterations += 1
            elif in_flight:
                if pending and arrival(pending[0]) - now() < 1e-3:
                    time.sleep(1e-4)
                else:
                    retire(in_flight.popleft())
            elif pending:
                time.sleep(min(2e-3, max(0.0, arrival(pending[0]) - now())))
        torch.cuda.synchronize(self.device)
        return Stats(latencies, site_steps, now(), admitted, rejected, iterations, max_resident,
                     self.batches_built, self.graph_replays)


def serve_fifo(trace: List[wl.Request], device="cuda", time_limit: Optional[float] = None,
               schedules: Optional[Dict[str, tuple]] = None) -> Stats:
    """One request at a time in arrival order, each a plain tsq_evolve, in real time."""
    schedules = schedules or SCHEDULES
    dev = torch.device(device)
    lat, ss = [], 0
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    done = 0
    for r in sorted(trace, key=lambda r: r.arrival):
        t = time.perf_counter() - t0
        if time_limit is not None and t > time_limit:
            break
        if r.arrival > t:
            time.sleep(r.arrival - t)
        p = r.problem
        tdt = torch.complex64 if p.dtype == "c64" else torch.complex128
        psi = wl.initial_state(p, device=dev, dtype=tdt)
        V = wl.potential(p, device=dev)
        plan = tsq.Plan(p.nx, p.ny, p.dt, p.dtype, device=dev)
        plan.set_schedule(*schedules[p.dtype])
        plan.set_potential(V)
        plan.evolve(psi, p.steps)
        torch.cuda.synchronize(dev)
        lat.append(time.perf_counter() - t0 - r.arrival)
        ss += p.site_steps
        done += 1
    makespan = time.perf_counter() - t0
    return Stats(lat, ss, makespan, done, 0, done, 1)
