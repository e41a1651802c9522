"""The batched form at the full size of its benchmark workload: 512 independent
complex64 problems, sides log-uniform in [64, 1024] rounded to even, each with its
own packets-and-bumps recipe and dt, 500 steps, replayed from a captured HIP graph.

Every schedule the benchmark chooses among gives the same bits for all 512
problems; sampled problems match the oracle (relative L2 <= 1e-5) and their solve
alone (bitwise); every problem keeps its norm.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1208_2407_amd as tsq
from paper_1208_2407_amd import workloads as wl
from tests.gpu_helpers import TOL, log, rel_l2

pytestmark = pytest.mark.gpu

# the candidates the batched benchmark times: steps per pass x phase ring, one pair per lane
SCHEDULES = [(S, 0, 1, store) for S in (3, 4, 5, 6) for store in (1, 2)]


def setup_module(_):
    oracle.build(force=False)
    tsq.load_library()


def test_batch512_full_size():
    probs = wl.batch_problems(512, 4, 500, dtype="c64")
    log(f"  batch512: generating {len(probs)} problems on the device")
    psi0s, Vs, plans = [], [], []
    for q in probs:
        psi0s.append(wl.initial_state(q, device="cuda", dtype=torch.complex64))
        V = wl.potential(q, device="cuda")
        pl = tsq.Plan(q.nx, q.ny, q.dt, "c64")
        pl.set_potential(V)
        Vs.append(V)
        plans.append(pl)
    steps = [q.steps for q in probs]
    assert sum(q.nx * q.ny for q in probs) > 5e7

    ref = None
    for sched in SCHEDULES:
        log(f"  batch512: schedule {sched}")
        psis = [x.clone() for x in psi0s]
        bt = tsq.Batch(plans, psis, steps, sched)
        bt.launch(use_graph=True)
        torch.cuda.synchronize()
        if ref is None:
            ref, ref_sched = psis, sched
        else:
            for i, (a, b) in enumerate(zip(psis, ref)):
                assert torch.equal(a, b), (sched, i, probs[i].name)
        del bt

    n0 = torch.stack([x.abs().double().square().sum() for x in psi0s])
    n1 = torch.stack([x.abs().double().square().sum() for x in ref])
    drift = (n1 - n0).abs().max().item()
    log(f"  batch512: largest norm drift over 512 problems {drift:.3e}")
    assert drift <= TOL["c64"]

    sizes = np.array([q.nx * q.ny for q in probs])
    rng = np.random.Generator(np.random.PCG64(44))
    sample = sorted(set(np.argsort(sizes)[:3].tolist() + [int(np.argmax(sizes))]
                        + rng.choice(len(probs), 3, replace=False).tolist()))
    for i in sample:
        q = probs[i]
        psi0 = psi0s[i].cpu().numpy().astype(np.complex128)
        got = ref[i].cpu().numpy().astype(np.complex128)
        alone = psi0s[i].clone()
        plans[i].set_schedule(*ref_sched)
        plans[i].evolve(alone, steps[i])
        torch.cuda.synchronize()
        assert torch.equal(alone, ref[i]), (i, q.name)
        want = oracle.evolve(psi0, Vs[i].cpu().numpy(), q.dt, q.steps)
        err = rel_l2(got, want)
        log(f"  batch512: problem {i} ({q.nx}x{q.ny}, dt {q.dt}) vs oracle {err:.3e}")
        assert err <= TOL["c64"], (i, q.name, err)
