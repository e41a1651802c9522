"""GPU parity of the time-dependent potential V(t) = V0 + f(t) W against the
FP64 oracle (each step frozen at its midpoint; the oracle's pins are in
test_oracle_pins.py).  Tolerances as for the static path: complex128 <= 1e-12,
complex64 <= 1e-5 relative L2."""
import numpy as np
import pytest
import torch

import oracle
import paper_1208_2407_amd as tsq
from paper_1208_2407_amd import workloads as wl
from tests.gpu_helpers import TOL, TORCH_DT, as_input, gpu_evolve, light_cone_windows, log, rel_l2

pytestmark = pytest.mark.gpu

ANISO = dict(dx=1.3, dy=0.8, mass=1.7, hbar=0.9)


def setup_module(_):
    oracle.build(force=False)
    tsq.load_library()


def gpu_evolve_td(psi0, V0, W, f, dt, dtype, steps_per_pass=0, segment_rows=0, phase_store=0,
                  chunks=1, **consts):
    ny, nx = psi0.shape
    psi = torch.from_numpy(np.ascontiguousarray(psi0)).to(TORCH_DT[dtype]).cuda()
    plan = tsq.Plan(nx, ny, dt, dtype, device=psi.device, **consts)
    plan.set_schedule(steps_per_pass, segment_rows, 1, phase_store)
    plan.set_potential_td(torch.from_numpy(np.ascontiguousarray(V0, dtype=np.float64)).cuda(),
                          torch.from_numpy(np.ascontiguousarray(W, dtype=np.float64)).cuda())
    for part in np.array_split(np.asarray(f, dtype=np.float64), chunks):
        plan.evolve_td(psi, part)
    torch.cuda.synchronize()
    return psi.cpu().numpy().astype(np.complex128)


SHAPES = [(2, 2), (4, 6), (130, 66), (258, 300), (66, 1030)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("S", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("shape", SHAPES)
def test_td_ragged_meshes(shape, S, dtype):
    nx, ny = shape
    psi0 = wl.random_state(nx, ny, 17 + nx)
    V0 = wl.random_potential(nx, ny, 18 + ny, scale=0.5)
    W = wl.random_potential(nx, ny, 19 + nx, scale=0.7)
    for steps in (1, 7, 2 * S + 1):
        f = np.random.default_rng(steps).uniform(-1.5, 1.5, steps)
        want = oracle.evolve_td(as_input(psi0, dtype), V0, W, f, 0.11, **ANISO)
        for store in (1, 2):
            got = gpu_evolve_td(psi0, V0, W, f, 0.11, dtype, steps_per_pass=S, segment_rows=16,
                                phase_store=store, **ANISO)
            err = rel_l2(got, want)
            assert err <= TOL[dtype], (shape, S, store, steps, err)


CLOSED_SHAPES = [(2, 2), (3, 5), (131, 67), (257, 301)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("S", [1, 3, 4, 6])
@pytest.mark.parametrize("shape", CLOSED_SHAPES)
def test_td_closed_meshes(shape, S, dtype):
    """The time-dependent potential between hard walls (odd sides allowed) against the
    oracle's closed mesh, both phase rings."""
    nx, ny = shape
    psi0 = wl.random_state(nx, ny, 70 + nx)
    V0 = wl.random_potential(nx, ny, 71 + ny, scale=0.5)
    W = wl.random_potential(nx, ny, 72 + nx, scale=0.7)
    for steps in (1, 2 * S + 1):
        f = np.random.default_rng(90 + steps).uniform(-1.5, 1.5, steps)
        want = oracle.evolve_td(as_input(psi0, dtype), V0, W, f, 0.11, bc="closed", **ANISO)
        for store in (1, 2):
            got = gpu_evolve_td(psi0, V0, W, f, 0.11, dtype, steps_per_pass=S, segment_rows=16,
                                phase_store=store, bc="closed", **ANISO)
            err = rel_l2(got, want)
            assert err <= TOL[dtype], (shape, S, store, steps, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_td_closed_odd_sides_long_run(dtype):
    """Odd width and height between walls: the shared factors carry the
    interior's even-factor cosines and the march rescales the last column and
    row (no even partner there).  A wrong scale would grow step after step:
    240 driven steps against the oracle, and the norm."""
    nx, ny = 77, 45
    psi0 = wl.random_state(nx, ny, 73)
    V0 = wl.random_potential(nx, ny, 74, scale=0.5)
    W = wl.random_potential(nx, ny, 75, scale=0.7)
    f = np.sin(0.05 * np.arange(240)) * 1.3
    want = oracle.evolve_td(as_input(psi0, dtype), V0, W, f, 0.11, bc="closed", **ANISO)
    got = gpu_evolve_td(psi0, V0, W, f, 0.11, dtype, steps_per_pass=4, bc="closed", **ANISO)
    err = rel_l2(got, want)
    n0 = float(np.sum(np.abs(as_input(psi0, dtype).astype(np.complex128)) ** 2))
    n1 = float(np.sum(np.abs(got.astype(np.complex128)) ** 2))
    log(f"  td closed odd sides 240 steps {dtype}: rel L2 {err:.3e}, norm drift {n1 - n0:.3e}")
    assert err <= (1e-11 if dtype == "c128" else 2e-5)
    assert abs(n1 - n0) <= (1e-12 if dtype == "c128" else 1e-5) * n0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_td_closed_schedule_does_not_change_a_bit(dtype):
    nx, ny = 131, 67
    psi0 = wl.random_state(nx, ny, 80)
    V0 = wl.random_potential(nx, ny, 81)
    W = wl.random_potential(nx, ny, 82)
    f = np.random.default_rng(83).uniform(-1, 1, 9)
    ref = gpu_evolve_td(psi0, V0, W, f, 0.09, dtype, steps_per_pass=1, segment_rows=2,
                        phase_store=1, bc="closed")
    for S in (2, 4, 8):
        for seg in (2, 10, 0):
            for store in ((1, 2) if S <= 6 else (2,)):
                got = gpu_evolve_td(psi0, V0, W, f, 0.09, dtype, steps_per_pass=S,
                                    segment_rows=seg, phase_store=store, bc="closed")
                assert np.array_equal(got, ref), (S, seg, store)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_td_closed_constant_modulation_equals_static_potential(dtype):
    nx, ny = 129, 95
    psi0 = wl.random_state(nx, ny, 84)
    V0 = wl.random_potential(nx, ny, 85, scale=3.0)
    W = wl.random_potential(nx, ny, 86, scale=2.0)
    c = -0.41
    got = gpu_evolve_td(psi0, V0, W, np.full(30, c), 0.2, dtype, bc="closed", **ANISO)
    want = gpu_evolve(psi0, V0 + c * W, 0.2, 30, dtype, bc="closed", **ANISO)
    err = rel_l2(got, want)
    log(f"  td closed constant f vs static {dtype}: {err:.3e}")
    assert err <= (1e-13 if dtype == "c128" else 2e-6)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_td_schedule_and_call_split_do_not_change_a_bit(dtype):
    """Every schedule gives the same bits (a schedule deeper than the
    time-dependent march fuses runs 6).  Splitting the modulation over several
    calls continues the evolution: each call closes and reopens the odd half
    factors that one call merges, so the split agrees to rounding."""
    nx, ny = 258, 130
    psi0 = wl.random_state(nx, ny, 3)
    V0 = wl.random_potential(nx, ny, 4)
    W = wl.random_potential(nx, ny, 5)
    f = np.random.default_rng(6).uniform(-1, 1, 13)
    ref = gpu_evolve_td(psi0, V0, W, f, 0.09, dtype, steps_per_pass=1, segment_rows=2, phase_store=1)
    for S in range(1, 9):
        for seg in (2, 6, 0):
            for store in ((1, 2) if S <= 6 else (2,)):
                got = gpu_evolve_td(psi0, V0, W, f, 0.09, dtype, steps_per_pass=S, segment_rows=seg,
                                    phase_store=store)
                assert np.array_equal(got, ref), (S, seg, store)
    split = gpu_evolve_td(psi0, V0, W, f, 0.09, dtype, chunks=4)
    assert rel_l2(split, ref) <= (1e-14 if dtype == "c128" else 1e-6)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_td_constant_modulation_equals_static_potential(dtype):
    """f_n = c for every step is the static potential V0 + c W: the in-kernel FP64
    phase (sine and cosine written for the march) against the table of the static
    path (the HIP math library's sincos)."""
    nx, ny = 256, 192
    psi0 = wl.random_state(nx, ny, 8)
    V0 = wl.random_potential(nx, ny, 9, scale=3.0)
    W = wl.random_potential(nx, ny, 10, scale=2.0)
    c = 0.73
    got = gpu_evolve_td(psi0, V0, W, np.full(40, c), 0.2, dtype, **ANISO)
    want = gpu_evolve(psi0, V0 + c * W, 0.2, 40, dtype, **ANISO)
    err = rel_l2(got, want)
    log(f"  td constant f vs static {dtype}: {err:.3e}")
    assert err <= (1e-13 if dtype == "c128" else 2e-6)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_td_large_phases(dtype):
    """Phase angles of a few hundred radians per step (the range reduction of the
    in-kernel sine and cosine; an FP64 angle of size a carries a rounding of
    about a * 1e-16 whoever computes it, which bounds the sizes a 1e-12 parity
    can be asked at)."""
    nx, ny = 128, 96
    psi0 = wl.random_state(nx, ny, 11)
    V0 = wl.random_potential(nx, ny, 12, scale=300.0)
    W = wl.random_potential(nx, ny, 13, scale=100.0)
    f = np.random.default_rng(14).uniform(-2, 2, 9)
    want = oracle.evolve_td(as_input(psi0, dtype), V0, W, f, 0.3)
    got = gpu_evolve_td(psi0, V0, W, f, 0.3, dtype)
    err = rel_l2(got, want)
    log(f"  td large phases {dtype}: {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_td_phase_factor_alone(dtype):
    """With a mass so large that every kinetic rotation rounds to the identity, a
    step is its phase factor alone: psi_n = psi_0 exp(-i sum_k (theta0 + f_k w)).
    Checked site by site against that closed form over angles of up to ~1e3 rad
    of either sign (the angle-addition reduction, the factor table with
    negative indices, the short series) and against the oracle."""
    nx, ny = 130, 34
    rng = np.random.default_rng(51)
    psi0 = as_input(wl.random_state(nx, ny, 52), dtype)
    V0 = rng.uniform(-2000.0, 2000.0, (ny, nx))
    W = rng.uniform(-300.0, 300.0, (ny, nx))
    f = rng.uniform(-2.0, 2.0, 7)
    dt, mass = 0.5, 1e30
    eps0 = 2.0 / mass
    theta0 = dt * (V0 + eps0)
    w = dt * W
    want = psi0 * np.exp(-1j * (len(f) * theta0 + f.sum() * w))
    oracle_run = oracle.evolve_td(psi0, V0, W, f, dt, mass=mass)
    tol = 1e-11 if dtype == "c128" else 1e-6  # complex64: 7 roundings of 2^-24
    assert np.max(np.abs(oracle_run - want)) <= 1e-11
    for S in (1, 3, 5):
        got = gpu_evolve_td(psi0, V0, W, f, dt, dtype, steps_per_pass=S, mass=mass)
        err = np.max(np.abs(got - want) / np.abs(want))
        log(f"  td phase alone {dtype} S={S}: max site rel error {err:.3e}")
        assert err <= tol, (S, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_td_forward_then_backward(dtype):
    p = wl.packets_and_bumps(512, 384, 21, 0.05, 150, dtype)
    psi0 = as_input(wl.initial_state(p).numpy(), dtype)
    V0 = wl.potential(p).numpy()
    W = wl.standing_wave(p).numpy()
    f = wl.drive(p.dt, p.steps)
    fwd = gpu_evolve_td(psi0, V0, W, f, p.dt, dtype)
    back = gpu_evolve_td(fwd, V0, W, f[::-1], -p.dt, dtype)
    err = rel_l2(back, psi0)
    log(f"  td forward/backward {dtype}: {err:.3e}")
    assert err <= (1e-13 if dtype == "c128" else 5e-6)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_td_driven_mesh_1024(dtype):
    """1024^2 packets and bumps under the shaken standing wave, 200 steps, against
    one oracle run; norm stays put."""
    p = wl.packets_and_bumps(1024, 1024, 22, 0.05, 200, dtype)
    psi0 = as_input(wl.initial_state(p).numpy(), dtype)
    V0 = wl.potential(p).numpy()
    W = wl.standing_wave(p).numpy()
    f = wl.drive(p.dt, p.steps)
    got = gpu_evolve_td(psi0, V0, W, f, p.dt, dtype)
    want = oracle.evolve_td(psi0, V0, W, f, p.dt)
    err = rel_l2(got, want)
    n0, n1 = np.sum(np.abs(psi0) ** 2), np.sum(np.abs(got) ** 2)
    log(f"  td driven 1024^2 {dtype}: rel L2 {err:.3e}, norm drift {n1 - n0:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("bc", ["periodic", "closed"])
def test_td_tuner_picks_a_candidate_and_keeps_the_bits(bc):
    """autotune.tune_td times the candidates on a scratch copy, sets its choice on the
    plan and leaves the state alone; the tuned evolution equals the one-step-per-pass one."""
    from paper_1208_2407_amd import autotune
    nx, ny = 256, 130
    psi0 = wl.random_state(nx, ny, 31)
    V0 = wl.random_potential(nx, ny, 32)
    W = wl.random_potential(nx, ny, 33)
    f = np.random.default_rng(34).uniform(-1, 1, 23)
    psi = torch.from_numpy(psi0).to(torch.complex64).cuda()
    plan = tsq.Plan(nx, ny, 0.07, "c64", bc=bc, device=psi.device)
    plan.set_potential_td(torch.from_numpy(V0).cuda(), torch.from_numpy(W).cuda())
    before = psi.clone()
    sched, table = autotune.tune_td(plan, psi, f, steps=24, use_cache=False)
    assert torch.equal(psi, before)
    assert sched in autotune.TD_CANDIDATES and plan.schedule() == sched
    assert len(table) == len(autotune.TD_CANDIDATES)
    plan.evolve_td(psi, f)
    torch.cuda.synchronize()
    ref = gpu_evolve_td(psi0, V0, W, f, 0.07, "c64", steps_per_pass=1, bc=bc)
    assert np.array_equal(psi.cpu().numpy().astype(np.complex128), ref)


def test_td_state_errors():
    nx, ny = 64, 32
    plan = tsq.Plan(nx, ny, 0.1, "c128")
    psi = torch.zeros((ny, nx), dtype=torch.complex128, device="cuda")
    V = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    plan.set_potential(V)
    with pytest.raises(tsq.TsqError) as ei:
        plan.evolve_td(psi, [0.1])
    assert ei.value.status == -6
    plan.set_potential_td(V, V)
    with pytest.raises(tsq.TsqError) as ei:
        plan.evolve(psi, 1)
    assert ei.value.status == -6
    with pytest.raises(tsq.TsqError) as ei:
        plan.evolve_td(psi, [0.1, float("nan")])
    assert ei.value.status == -1
    with pytest.raises(tsq.TsqError) as ei:
        tsq.Batch([plan], [psi], [3])
    assert ei.value.status == -7
    plan.set_schedule(2, 0, 2, 1)
    with pytest.raises(tsq.TsqError) as ei:
        plan.evolve_td(psi, [0.1])
    assert ei.value.status == -1
    plan.set_schedule(8, 0, 1, 2)
    assert plan.passes(8) == (2, False)   # runs 6 steps per pass, then 2
    assert plan.passes(12) == (2, False)


@pytest.mark.parametrize("bc", ["periodic", "closed"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_td4096_sampled_windows(dtype, bc):
    """The 4096^2 driven workload (packets and bumps under the shaken standing wave)
    at full size in the schedules its tuner picks among (4, 5 and 6 steps per pass, both
    phase rings; all bitwise equal), 50 steps; 256^2 windows on the packets and at the
    mesh corner (and, between walls, along an edge) against oracle runs on the window
    plus its light cone."""
    p = wl.packets_and_bumps(4096, 4096, 2, 0.05, 50, dtype)
    # the packets plus seeded noise over the whole mesh: every window, the walls'
    # included, holds a state
    psi0 = wl.initial_state(p).numpy() + 0.5 * wl.random_state(4096, 4096, 61)
    V0 = wl.potential(p).numpy()
    W = wl.standing_wave(p).numpy()
    f = wl.drive(p.dt, p.steps)
    runs = [gpu_evolve_td(psi0, V0, W, f, p.dt, dtype, steps_per_pass=S, phase_store=st, bc=bc)
            for S in (4, 5, 6) for st in (1, 2)]
    for r in runs[1:]:
        assert np.array_equal(r, runs[0])
    h = w = 256
    wins = [((int(q.y0 + 2048) - h // 2) // 2 * 2, (int(q.x0 + 2048) - w // 2) // 2 * 2)
            for q in p.packets]
    wins += [(0, 0), (4096 - h // 2, 4096 - w // 2)] if bc == "periodic" else [(0, 0), (2048, 4096 - w)]
    errs = light_cone_windows(runs[0], [as_input(psi0, dtype), V0, W],
                              lambda s, v, ww, bc: oracle.evolve_td(s, v, ww, f, p.dt, bc=bc),
                              wins, h, w, 2 * p.steps + 2, bc)
    log(f"  td4096 {bc} windows {dtype}: max rel L2 {max(errs):.3e} over {len(errs)}")
    assert len(errs) == len(wins) and max(errs) <= TOL[dtype]
