"""The 32768^2 complex64 mesh (8.6 GB state): 200 steps at dt = 0.05 with the
packets-and-bumps recipe scaled to the mesh; spot checks against the FP64
oracle on 2048^2 crops centred on the packets, compared on the interior the
crop's own (periodic) edges cannot reach in 200 steps: the light cone is
2N+1 = 401 sites, so a 402-site margin per side leaves a 1244^2 interior."""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_1208_2407_amd as tsq
from paper_1208_2407_amd import workloads as wl
from tests.gpu_helpers import TOL, log, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.mark.timeout(600)
def test_mesh32768_complex64_crops():
    oracle.build(force=False)
    p = wl.config("mesh32768_c64")
    n = p.nx
    log(f"  generating the {n}^2 inputs on the device")
    psi = wl.initial_state(p, device="cuda", dtype=torch.complex64)
    V = wl.potential(p, device="cuda")
    W, m = 2048, 2 * p.steps + 2
    crops = []
    for q in p.packets:
        yc = int(round(q.y0 / p.dy + n / 2)) // 2 * 2
        xc = int(round(q.x0 / p.dx + n / 2)) // 2 * 2
        y0, x0 = yc - W // 2, xc - W // 2
        crops.append((y0, x0,
                      psi[y0:y0 + W, x0:x0 + W].cpu().numpy().astype(np.complex128),
                      V[y0:y0 + W, x0:x0 + W].cpu().numpy()))
    plan = tsq.Plan(n, n, p.dt, "c64")
    plan.set_potential(V)
    psi0 = psi.clone()
    # the schedules the tuner picks between for this mesh in bench.py: 6 steps per
    # pass, 512-row segments, register or LDS phase ring (bitwise equal)
    plan.set_schedule(6, 512, 1, 2)
    plan.evolve(psi0, p.steps)
    plan.set_schedule(6, 512, 1, 1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan.evolve(psi, p.steps)
    e1.record()
    norm, energy = plan.observables(psi, V)
    ms = e0.elapsed_time(e1)
    log(f"  {n}^2 c64 x {p.steps} steps: {ms:.1f} ms, {n * n * p.steps / (ms * 1e-3):.3e} site-steps/s, "
        f"schedule {plan.schedule()}, norm {norm:.9f}")
    assert torch.equal(psi, psi0)
    del psi0
    assert abs(norm - 1.0) < 1e-5
    errs = []
    for (y0, x0, cin, cV) in crops:
        want = oracle.evolve(cin, cV, p.dt, p.steps)[m:W - m, m:W - m]
        got = psi[y0 + m:y0 + W - m, x0 + m:x0 + W - m].cpu().numpy().astype(np.complex128)
        errs.append(rel_l2(got, want))
    log(f"  crop interiors ({W - 2 * m}^2): rel L2 {', '.join(f'{e:.2e}' for e in errs)}")
    assert max(errs) <= TOL["c64"]
