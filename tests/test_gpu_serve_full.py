"""The request server on requests of its benchmark stream at full size: the first
32 requests of the seeded Poisson trace (sides log-uniform in [128, 4096], 100-2000
steps, complex64/complex128 80/20), served together with the benchmark's block of
20 steps.  Sampled requests equal their solve alone bit for bit and match the
oracle; every request keeps its norm."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_2407_amd import serve
from paper_1208_2407_amd import workloads as wl
from tests.gpu_helpers import TOL, log, rel_l2

pytestmark = pytest.mark.gpu

BLOCK = 20
ORACLE_BUDGET = 1.2e9     # site-steps per sampled request the oracle is asked for


def setup_module(_):
    oracle.build(force=False)


def test_served_stream_prefix_full_size():
    trace = wl.request_trace(rate=200.0, duration=60.0, seed=5)[:32]
    assert max(max(r.problem.nx, r.problem.ny) for r in trace) > 3000
    mix = serve.Server(keep_results=True, block_steps=BLOCK)
    st = mix.run(trace, realtime=False)
    assert st.admitted == len(trace) and len(st.latencies) == len(trace)
    assert st.max_resident > 1

    for r in trace:
        p = r.problem
        psi0 = wl.initial_state(p, device="cuda",
                                dtype=torch.complex64 if p.dtype == "c64" else torch.complex128)
        n0 = psi0.abs().double().square().sum().item()
        n1 = mix.results[r.rid].abs().double().square().sum().item()
        assert abs(n1 - n0) <= TOL[p.dtype] * n0, (r.rid, p.dtype, n1 - n0)

    cost = {r.rid: r.problem.nx * r.problem.ny * r.problem.steps for r in trace}
    by_cost = sorted(trace, key=lambda r: cost[r.rid])
    small = [r for r in by_cost if cost[r.rid] <= ORACLE_BUDGET]
    c128 = [r for r in small if r.problem.dtype == "c128"]
    checked = {r.rid: r for r in small[:2] + small[-2:] + c128[-2:]}
    alone_only = {r.rid: r for r in by_cost[-2:]}
    for rid, r in sorted({**checked, **alone_only}.items()):
        p = r.problem
        alone = serve.Server(keep_results=True, block_steps=BLOCK)
        alone.run([r], realtime=False)
        assert torch.equal(mix.results[rid], alone.results[rid]), rid
        if rid not in checked:
            continue
        psi0 = wl.initial_state(p).numpy()
        if p.dtype == "c64":
            psi0 = psi0.astype(np.complex64).astype(np.complex128)
        want = oracle.evolve(psi0, wl.potential(p).numpy(), p.dt, p.steps)
        got = mix.results[rid].cpu().numpy().astype(np.complex128)
        err = rel_l2(got, want)
        log(f"  served request {rid} ({p.nx}x{p.ny}, {p.steps} steps, {p.dtype}) vs oracle {err:.3e}")
        assert err <= TOL[p.dtype], (rid, p.dtype, err)
