"""GPU parity of three-dimensional meshes (the seven-part split, one step per
pass) against the FP64 oracle, whose 3D pins are in test_oracle_pins.py.
Tolerances: complex128 <= 1e-12, complex64 <= 1e-5 relative L2."""
import numpy as np
import pytest
import torch

import oracle
import paper_1208_2407_amd as tsq
from paper_1208_2407_amd import workloads as wl
from tests.gpu_helpers import TOL, TORCH_DT, as_input, log, rel_l2

pytestmark = pytest.mark.gpu

ANISO3 = dict(dx=1.3, dy=0.8, dz=1.1, mass=1.7, hbar=0.9)


def setup_module(_):
    oracle.build(force=False)
    tsq.load_library()


def rand3(n3, seed, scale=1.0):
    nx, ny, nz = n3
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    return psi / np.linalg.norm(psi), scale * rng.standard_normal((nz, ny, nx))


def gpu_evolve3(psi0, V, dt, steps, dtype, segment_planes=0, **consts):
    nz, ny, nx = psi0.shape
    psi = torch.from_numpy(np.ascontiguousarray(psi0)).to(TORCH_DT[dtype]).cuda()
    plan = tsq.Plan(nx, ny, dt, dtype, nz=nz, device=psi.device, **consts)
    plan.set_schedule(0, segment_planes, 0, 0)
    plan.set_potential(torch.from_numpy(np.ascontiguousarray(V, dtype=np.float64)).cuda())
    plan.evolve(psi, steps)
    torch.cuda.synchronize()
    return psi.cpu().numpy().astype(np.complex128)


SHAPES3 = [(2, 2, 2), (4, 6, 8), (130, 18, 10), (66, 34, 12), (258, 6, 4), (6, 50, 6)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n3", SHAPES3)
def test_3d_ragged_meshes(n3, dtype):
    """Sides that are not multiples of the strip, the slab or the segment; odd and
    even step counts; anisotropic constants."""
    psi0, V = rand3(n3, 31 + n3[0], scale=0.5)
    for steps in (1, 2, 5):
        want = oracle.evolve3(as_input(psi0, dtype), V, 0.11, steps, **ANISO3)
        got = gpu_evolve3(psi0, V, 0.11, steps, dtype, **ANISO3)
        err = rel_l2(got, want)
        assert err <= TOL[dtype], (n3, steps, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_3d_segments_do_not_change_a_bit(dtype):
    """Segment height and march direction change nothing: bitwise equal results."""
    psi0, V = rand3((130, 34, 24), 41)
    ref = gpu_evolve3(psi0, V, 0.09, 5, dtype, segment_planes=24)
    for seg in (4, 6, 10, 0):
        assert np.array_equal(gpu_evolve3(psi0, V, 0.09, 5, dtype, segment_planes=seg), ref), seg


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_3d_packet_128(dtype):
    """128^3 packet in a harmonic well, 60 steps, against the oracle; norm and
    energy of the GPU reductions against the oracle's."""
    p = wl.packet_in_well3(128, 51, dt=0.05, steps=60)
    psi0 = as_input(wl.state3(p).numpy(), dtype)
    V = wl.potential3(p).numpy()
    got = gpu_evolve3(psi0, V, p.dt, p.steps, dtype)
    want = oracle.evolve3(psi0, V, p.dt, p.steps)
    err = rel_l2(got, want)
    psi_d = torch.from_numpy(got).to(TORCH_DT[dtype]).cuda()
    n, e = tsq.observables(psi_d, torch.from_numpy(V).cuda())
    n_o, e_o = oracle.observables3(as_input(got, dtype), V)
    log(f"  3d packet 128^3 {dtype}: rel L2 {err:.3e}, norm {n:.15f}, |dE|/|E| {abs(e - e_o) / abs(e_o):.2e}")
    assert err <= TOL[dtype]
    assert abs(n - n_o) < 1e-12 and abs(e - e_o) <= 1e-12 * abs(e_o)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_3d_forward_then_backward(dtype):
    psi0, V = rand3((66, 34, 20), 52)
    psi0 = as_input(psi0, dtype)
    fwd = gpu_evolve3(psi0, V, 0.2, 30, dtype, **ANISO3)
    back = gpu_evolve3(fwd, V, -0.2, 30, dtype, **ANISO3)
    err = rel_l2(back, psi0)
    log(f"  3d forward/backward {dtype}: {err:.3e}")
    assert err <= (1e-13 if dtype == "c128" else 5e-6)


def test_3d_observables_match_oracle():
    psi0, V = rand3((130, 34, 12), 53)
    psi = torch.from_numpy(psi0).cuda()
    n, e = tsq.observables(psi, torch.from_numpy(V).cuda(), **ANISO3)
    n_o, e_o = oracle.observables3(psi0, V, **ANISO3)
    assert abs(n - n_o) < 1e-13 and abs(e - e_o) <= 1e-12 * abs(e_o)


def _oracle_1d(n, k, p):
    """One axis of the separable packet-in-a-well problem through the oracle: a mesh
    of n x 2 x 2 sites with the state and potential constant across the two thin
    axes (there every pair joins equal values, a pure phase that cancels the thin
    axes' share of the diagonal constant), so each line evolves as the 1D mesh."""
    x = np.arange(n) - n / 2
    f = np.exp(-x * x / (4 * p.sigma ** 2) + 1j * k * x)
    f /= np.linalg.norm(f)
    v = 0.5 * p.mass * p.omega ** 2 * x * x
    out = oracle.evolve3(np.broadcast_to(f, (2, 2, n)).copy(), np.broadcast_to(v, (2, 2, n)).copy(),
                         p.dt, p.steps)
    return torch.from_numpy(out[0, 0].copy()).cuda()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_3d_packet_in_well_512_full_size(dtype):
    """The 512^3 benchmark problem (one packet in an isotropic harmonic well, 100
    steps, the benchmark's launch configuration) at full size: state and potential
    are separable, so the exact result of the split is the tensor product of three
    1D oracle runs, compared over every site."""
    p = wl.packet_in_well3(512, 6, dt=0.05, steps=100, sigma=16.0, omega=0.005)
    psi = wl.state3(p, device="cuda", dtype=TORCH_DT[dtype])
    plan = tsq.Plan(p.nx, p.ny, p.dt, dtype, nz=p.nz, device=psi.device)
    V = wl.potential3(p, device="cuda")
    plan.set_potential(V)
    plan.evolve(psi, p.steps)
    torch.cuda.synchronize()
    del V
    fx, fy, fz = (_oracle_1d(n, k, p) for n, k in zip((p.nx, p.ny, p.nz), p.k))
    want = fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    err = (torch.linalg.vector_norm(psi.to(torch.complex128) - want)
           / torch.linalg.vector_norm(want)).item()
    log(f"  3d 512^3 packet {dtype}: rel L2 vs tensor product of 1D oracle runs {err:.3e}")
    assert err <= TOL[dtype]
