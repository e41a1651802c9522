"""GPU tests of the continuous-batching server: every request's result is the
same alone and in the mix (bitwise), within tolerance of the oracle, and the
admission by memory budget keeps the queue moving."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_2407_amd import serve
from paper_1208_2407_amd import workloads as wl
from tests.gpu_helpers import TOL, rel_l2

pytestmark = pytest.mark.gpu


def small_trace(n=24, seed=11):
    tr = wl.request_trace(rate=100.0, duration=1.0, seed=seed, lo=16, hi=160, steps_lo=5,
                          steps_hi=60, p_c64=0.6)
    return tr[:n]


def test_served_results_equal_alone_and_match_oracle():
    oracle.build(force=False)
    trace = small_trace()
    mix = serve.Server(keep_results=True, block_steps=8)
    st = mix.run(trace, realtime=False)
    assert st.admitted == len(trace) and len(st.latencies) == len(trace)
    assert st.max_resident > 1                      # requests really shared the device
    for r in trace:
        alone = serve.Server(keep_results=True, block_steps=8)
        alone.run([r], realtime=False)
        assert torch.equal(mix.results[r.rid], alone.results[r.rid]), r.rid
    for r in trace[:5]:
        p = r.problem
        psi0 = wl.initial_state(p).numpy()
        if p.dtype == "c64":
            psi0 = psi0.astype(np.complex64).astype(np.complex128)
        want = oracle.evolve(psi0, wl.potential(p).numpy(), p.dt, p.steps)
        got = mix.results[r.rid].cpu().numpy().astype(np.complex128)
        assert rel_l2(got, want) <= TOL[p.dtype], (r.rid, p.dtype)


def test_budget_admission_and_rejection():
    trace = small_trace(12, seed=12)
    sizes = [serve.request_bytes(r.problem) for r in trace]
    budget = max(max(sizes), sum(sizes) // 3)
    assert sum(sizes) > budget          # the budget really limits what is resident at once
    s = serve.Server(hbm_budget=budget, block_steps=8)
    huge = wl.Request(999, 0.0, wl.packets_and_bumps(4096, 4096, 1, 0.05, 10, "c128"))
    st = s.run(trace + [huge], realtime=False)
    assert st.rejected == 1 and st.admitted == len(trace)
    assert len(st.latencies) == len(trace)
    assert 1 <= st.max_resident < len(trace)
