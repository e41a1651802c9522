"""GPU tests of the batched form: many uneven problems per launch.

The batch must reproduce, bit for bit, each problem evolved alone with the
same schedule (every site sees the same operations in the same order), and
through the oracle stay within the dtype's tolerance.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1208_2407_amd as tsq
from paper_1208_2407_amd import workloads as wl
from tests.gpu_helpers import TOL, TORCH_DT, as_input, gpu_evolve, log, rel_l2

pytestmark = pytest.mark.gpu

SIDES = [2, 4, 6, 40, 66, 130, 258, 300]


def setup_module(_):
    oracle.build(force=False)
    tsq.load_library()


def make_problems(n, seed, dtype, max_steps=13):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        nx, ny = int(rng.choice(SIDES)), int(rng.choice(SIDES))
        dt = float(rng.choice([0.02, 0.05, 0.1, -0.07]))
        steps = int(rng.integers(0, max_steps + 1))
        psi0 = as_input(wl.random_state(nx, ny, 1000 + i), dtype)
        V = wl.random_potential(nx, ny, 2000 + i, scale=0.5)
        out.append((psi0, V, dt, steps))
    return out


def build_batch(problems, dtype, schedule):
    plans, psis, Vs = [], [], []
    for psi0, V, dt, steps in problems:
        ny, nx = psi0.shape
        psi = torch.from_numpy(psi0).to(TORCH_DT[dtype]).cuda()
        Vd = torch.from_numpy(V).cuda()
        pl = tsq.Plan(nx, ny, dt, dtype, device=psi.device)
        pl.set_potential(Vd)
        plans.append(pl)
        psis.append(psi)
        Vs.append(Vd)
    batch = tsq.Batch(plans, psis, [p[3] for p in problems], schedule)
    return batch, plans, psis, Vs


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("schedule", [(1, 0, 1, 1), (3, 0, 1, 2), (4, 0, 2, 1), (6, 0, 1, 2)])
def test_batch_equals_each_problem_alone(dtype, schedule):
    problems = make_problems(24, 7 + schedule[0], dtype)
    batch, plans, psis, Vs = build_batch(problems, dtype, schedule)
    batch.launch()
    torch.cuda.synchronize()
    S, _, ppl, store = schedule
    for i, (psi0, V, dt, steps) in enumerate(problems):
        got = psis[i].cpu().numpy().astype(np.complex128)
        alone = gpu_evolve(psi0, V, dt, steps, dtype, steps_per_pass=S, pairs_per_lane=ppl,
                           phase_store=store)
        assert np.array_equal(got, alone), (i, psi0.shape, steps)
        if i < 6:
            want = oracle.evolve(psi0, V, dt, steps)
            if steps:
                assert rel_l2(got, want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_graph_replays(dtype):
    """The captured graph is replayed several times with eager work and synchronisations
    in between; every replay must match evolving each problem alone again."""
    problems = make_problems(16, 99, dtype, max_steps=9)
    batch, plans, psis, Vs = build_batch(problems, dtype, (4, 0, 1, 2))
    refs = [torch.from_numpy(p[0]).to(TORCH_DT[dtype]).cuda() for p in problems]
    ref_plans = []
    for (psi0, V, dt, steps), Vd in zip(problems, Vs):
        ny, nx = psi0.shape
        pl = tsq.Plan(nx, ny, dt, dtype)
        pl.set_schedule(4, 0, 1, 2)
        pl.set_potential(Vd)
        ref_plans.append(pl)
    scratch = torch.randn(1 << 20, device="cuda")
    for replay in range(3):
        batch.launch(use_graph=True)
        scratch.mul_(1.0001)                      # unrelated eager work between replays
        torch.cuda.synchronize()
        for pl, r, p in zip(ref_plans, refs, problems):
            pl.evolve(r, p[3])
        torch.cuda.synchronize()
        for i in range(len(problems)):
            assert torch.equal(psis[i], refs[i]), (replay, i)


def test_batch_rejects_bad_input():
    p = make_problems(2, 5, "c64")
    batch, plans, psis, Vs = build_batch(p, "c64", (2, 0, 1, 1))
    other = tsq.Plan(8, 8, 0.1, "c128")
    psi = torch.zeros(8, 8, dtype=torch.complex128, device="cuda")
    other.set_potential(torch.zeros(8, 8, dtype=torch.float64, device="cuda"))
    with pytest.raises(tsq.TsqError) as ei:            # mixed dtypes
        tsq.tsq_batch_create([plans[0].handle, other.handle], [psis[0].data_ptr(), psi.data_ptr()],
                             [plans[0]._ws.data_ptr(), other._ws.data_ptr()], [1, 1])
    assert ei.value.status == -3
    with pytest.raises(tsq.TsqError) as ei:            # workspace not bound by set_potential
        tsq.tsq_batch_create([plans[0].handle], [psis[0].data_ptr()], [plans[1]._ws.data_ptr()], [1])
    assert ei.value.status == -6
    with pytest.raises(tsq.TsqError) as ei:            # negative steps
        tsq.tsq_batch_create([plans[0].handle], [psis[0].data_ptr()], [plans[0]._ws.data_ptr()], [-1])
    assert ei.value.status == -1
    h = tsq.tsq_batch_create([plans[0].handle], [psis[0].data_ptr()], [plans[0]._ws.data_ptr()], [3])
    try:
        with pytest.raises(tsq.TsqError) as ei:        # launch before upload
            tsq.tsq_batch_launch(h, False, 0)
        assert ei.value.status == -6
    finally:
        tsq.tsq_batch_destroy(h)
