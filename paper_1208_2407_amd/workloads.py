"""Seeded synthetic inputs for the Trotter-Suzuki solver: meshes, potentials, states.

This module holds input generation only (no step of the method).  The tests,
the benchmark and the oracle-side checks all draw their inputs from here, so
the HIP path and the oracle always see the same arrays.

The paper benchmarks "a synthetic state" on a flat potential (Sec. 2 last
paragraph; Sec. 4).  The workloads below follow that spirit with richer
potentials so that the diagonal phase is exercised:

* coordinates  x_i = (i - nx/2) dx,  y_j = (j - ny/2) dy  (origin at the centre);
* Gaussian packet  exp(-((x-x0)^2 + (y-y0)^2) / (4 sigma^2) + i (kx x + ky y));
  a superposition takes unit amplitudes with seeded phases and is normalised so
  that sum |psi|^2 = 1 (the normalisation uses exact 1D Gram sums, so any
  window of the mesh can be generated on its own with the global constant);
* harmonic well  V = m omega^2 (x^2 + y^2) / 2;
* bump  A exp(-|r - c|^2 / (2 w^2)),  A ~ U[-0.5, 0.5],  c uniform over the mesh.

Every field is a sum of separable terms, so a mesh of any size is built from
1D vectors with outer products (and one small matrix product for the bumps).
Random numbers come from numpy PCG64(seed) in a fixed draw order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch


@dataclasses.dataclass
class Packet:
    x0: float
    y0: float
    kx: float
    ky: float
    theta: float
    sigma: float


@dataclasses.dataclass
class Bump:
    amp: float
    cx: float
    cy: float
    width: float


@dataclasses.dataclass
class Problem:
    """One solve: mesh, constants, time step, step count and the input recipe."""
    name: str
    nx: int
    ny: int
    dt: float
    steps: int
    dtype: str = "c128"          # "c128" or "c64"
    dx: float = 1.0
    dy: float = 1.0
    mass: float = 1.0
    hbar: float = 1.0
    bc: str = "periodic"
    omega: float = 0.0
    packets: List[Packet] = dataclasses.field(default_factory=list)
    bumps: List[Bump] = dataclasses.field(default_factory=list)
    v0: float = 0.0              # constant offset added to the potential

    @property
    def sites(self) -> int:
        return self.nx * self.ny

    @property
    def site_steps(self) -> int:
        return self.nx * self.ny * self.steps


# ---------------------------------------------------------------- recipe draws

def _even(v: float, lo: int) -> int:
    n = int(round(v / 2.0)) * 2
    return max(lo, n)


def _draw_packets(rng: np.random.Generator, n: int, Lx: float, Ly: float, frac: float,
                  sigma: float) -> List[Packet]:
    out = []
    for _ in range(n):
        x0 = rng.uniform(-frac * Lx, frac * Lx)
        y0 = rng.uniform(-frac * Ly, frac * Ly)
        kx = rng.uniform(-0.5, 0.5)
        ky = rng.uniform(-0.5, 0.5)
        th = rng.uniform(0.0, 2.0 * math.pi)
        out.append(Packet(x0, y0, kx, ky, th, sigma))
    return out


def _draw_bumps(rng: np.random.Generator, n: int, Lx: float, Ly: float,
                width: float) -> List[Bump]:
    out = []
    for _ in range(n):
        a = rng.uniform(-0.5, 0.5)
        cx = rng.uniform(-0.5 * Lx, 0.5 * Lx)
        cy = rng.uniform(-0.5 * Ly, 0.5 * Ly)
        out.append(Bump(a, cx, cy, width))
    return out


def gaussian_in_well(n: int = 256, seed: int = 1, dt: float = 0.1, steps: int = 100,
                     dtype: str = "c128") -> Problem:
    """One packet (sigma = 16 sites, centred, seeded momentum in [-0.5, 0.5]^2)
    in a harmonic well omega = 0.01; hbar = m = dx = 1.  Default: 256^2,
    dt = 0.1, 100 steps, complex128."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kx, ky = rng.uniform(-0.5, 0.5, size=2)
    p = Packet(0.0, 0.0, float(kx), float(ky), 0.0, 16.0)
    return Problem(f"gaussian_in_well_{n}", n, n, dt, steps, dtype, omega=0.01, packets=[p])


def packets_and_bumps(nx: int, ny: int, seed: int, dt: float, steps: int, dtype: str,
                      n_packets: int = 4, scale: float = 1.0, name: str = "") -> Problem:
    """Four seeded packets (sigma = 16, centres in the central [-L/8, L/8]^2,
    momenta in [-0.5, 0.5]^2) in a harmonic well plus 32 seeded Gaussian bumps.
    `scale` stretches the recipe's lengths: omega = 0.01 / scale, bump width
    64 * scale (scale = L / 4096 reproduces the 4096^2 recipe on another mesh)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    packets = _draw_packets(rng, n_packets, float(nx), float(ny), 0.125, 16.0)
    bumps = _draw_bumps(rng, 32, float(nx), float(ny), 64.0 * scale)
    return Problem(name or f"packets_bumps_{nx}x{ny}", nx, ny, dt, steps, dtype,
                   omega=0.01 / scale, packets=packets, bumps=bumps)


def config(name: str) -> Problem:
    """The named single-mesh workloads."""
    if name == "well256":
        return gaussian_in_well()
    if name == "mesh4096_c128":
        return packets_and_bumps(4096, 4096, 2, 0.05, 1000, "c128", name=name)
    if name == "mesh4096_c64":
        return packets_and_bumps(4096, 4096, 2, 0.05, 1000, "c64", name=name)
    if name == "mesh32768_c64":
        return packets_and_bumps(32768, 32768, 3, 0.05, 200, "c64", scale=32768 / 4096,
                                 name=name)
    raise KeyError(name)


def batch_problems(count: int = 512, seed: int = 4, steps: int = 500, lo: int = 64,
                   hi: int = 1024, dtype: str = "c64") -> List[Problem]:
    """Independent problems with sides log-uniform in [lo, hi] rounded to even
    (square with probability 1/2, else two independent draws), each with its
    own packets-and-bumps recipe and dt drawn from {0.02, 0.05, 0.1}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        square = rng.uniform() < 0.5
        a = _even(math.exp(rng.uniform(math.log(lo), math.log(hi))), lo)
        b = a if square else _even(math.exp(rng.uniform(math.log(lo), math.log(hi))), lo)
        dt = float(rng.choice([0.02, 0.05, 0.1]))
        sub_seed = int(rng.integers(0, 2**31 - 1))
        p = packets_and_bumps(a, b, sub_seed, dt, steps, dtype, name=f"batch{i}_{a}x{b}")
        out.append(p)
    return out


# ---------------------------------------------------------------- fields

def _dev(a: np.ndarray, device) -> torch.Tensor:
    """A host array on `device`: to a GPU through pinned memory, asynchronously on the
    current stream (the request loop of the server generates inputs between launches)."""
    t = torch.from_numpy(np.ascontiguousarray(a))
    if torch.device(device).type != "cuda":
        return t.to(device)
    return t.pin_memory().to(device, non_blocking=True)


def _coords(n: int, d: float, lo: int, hi: int) -> np.ndarray:
    return (np.arange(lo, hi, dtype=np.float64) - n / 2) * d


def _packet_1d(x: np.ndarray, x0: float, k: float, sigma: float) -> np.ndarray:
    return np.exp(-((x - x0) ** 2) / (4.0 * sigma * sigma) + 1j * k * x)


def state_norm2(p: Problem) -> float:
    """sum |sum_k a_k f_k(x) g_k(y)|^2 over the full mesh, from 1D Gram sums."""
    xs = _coords(p.nx, p.dx, 0, p.nx)
    ys = _coords(p.ny, p.dy, 0, p.ny)
    F = np.stack([_packet_1d(xs, q.x0, q.kx, q.sigma) for q in p.packets])  # (K, nx)
    G = np.stack([_packet_1d(ys, q.y0, q.ky, q.sigma) for q in p.packets])
    a = np.array([np.exp(1j * q.theta) for q in p.packets])
    Gx = np.conj(F) @ F.T       # Gx[k, l] = sum_x conj(f_k) f_l
    Gy = np.conj(G) @ G.T
    n2 = np.einsum("k,l,kl,kl->", np.conj(a), a, Gx, Gy)
    return float(n2.real)


def initial_state(p: Problem, device="cpu", dtype=torch.complex128,
                  rows: Optional[Tuple[int, int]] = None,
                  cols: Optional[Tuple[int, int]] = None,
                  chunk_rows: int = 2048) -> torch.Tensor:
    """psi_0 on rows [r0, r1) x cols [c0, c1) of the mesh (default: all), normalised
    over the whole mesh, as a contiguous tensor of `dtype` on `device`."""
    r0, r1 = rows if rows is not None else (0, p.ny)
    c0, c1 = cols if cols is not None else (0, p.nx)
    inv = 1.0 / math.sqrt(state_norm2(p))
    xs = _coords(p.nx, p.dx, c0, c1)
    ys = _coords(p.ny, p.dy, r0, r1)
    F = np.stack([_packet_1d(xs, q.x0, q.kx, q.sigma) for q in p.packets])
    a = np.array([np.exp(1j * q.theta) * inv for q in p.packets])
    G = np.stack([_packet_1d(ys, q.y0, q.ky, q.sigma) for q in p.packets]) * a[:, None]
    F = _dev(F, device)
    G = _dev(G.T, device)                                    # (rows, K)
    out = torch.empty((r1 - r0, c1 - c0), dtype=dtype, device=device)
    for s in range(0, r1 - r0, chunk_rows):
        e = min(r1 - r0, s + chunk_rows)
        out[s:e] = (G[s:e] @ F).to(dtype)
    return out


def potential(p: Problem, device="cpu", rows: Optional[Tuple[int, int]] = None,
              cols: Optional[Tuple[int, int]] = None, chunk_rows: int = 2048) -> torch.Tensor:
    """V on rows [r0, r1) x cols [c0, c1) as contiguous float64 on `device`."""
    r0, r1 = rows if rows is not None else (0, p.ny)
    c0, c1 = cols if cols is not None else (0, p.nx)
    xs = _coords(p.nx, p.dx, c0, c1)
    ys = _coords(p.ny, p.dy, r0, r1)
    k = 0.5 * p.mass * p.omega * p.omega
    vx = _dev(k * xs * xs + p.v0, device)
    vy = _dev(k * ys * ys, device)
    nb = len(p.bumps)
    out = torch.empty((r1 - r0, c1 - c0), dtype=torch.float64, device=device)
    if nb:
        U = np.stack([np.exp(-((xs - b.cx) ** 2) / (2 * b.width ** 2)) for b in p.bumps])
        W = np.stack([b.amp * np.exp(-((ys - b.cy) ** 2) / (2 * b.width ** 2))
                      for b in p.bumps])
        U = _dev(U, device)
        W = _dev(W.T, device)
    for s in range(0, r1 - r0, chunk_rows):
        e = min(r1 - r0, s + chunk_rows)
        blk = vy[s:e, None] + vx[None, :]
        if nb:
            blk = blk + W[s:e] @ U
        out[s:e] = blk
    return out


# Time-dependent potential V(t) = V0 + f(t) W: the static potential of a
# problem plus a standing wave along x whose strength oscillates in time (a
# "shaken" lattice), periodic on the mesh.

def standing_wave(p: Problem, periods: int = 4, device="cpu",
                  rows: Optional[Tuple[int, int]] = None,
                  cols: Optional[Tuple[int, int]] = None) -> torch.Tensor:
    """W(x, y) = cos(2 pi periods i / nx) at column i, on rows [r0, r1) x cols [c0, c1)."""
    r0, r1 = rows if rows is not None else (0, p.ny)
    c0, c1 = cols if cols is not None else (0, p.nx)
    wx = torch.from_numpy(np.cos(2.0 * math.pi * periods * np.arange(c0, c1) / p.nx)).to(device)
    return wx[None, :].expand(r1 - r0, c1 - c0).contiguous()


def drive(dt: float, steps: int, amplitude: float = 0.2, omega: float = 0.5,
          phase: float = 0.0, t0: float = 0.0) -> np.ndarray:
    """f(t) = amplitude sin(omega t + phase) at the step midpoints t0 + (n + 1/2) dt."""
    t = t0 + (np.arange(steps) + 0.5) * dt
    return amplitude * np.sin(omega * t + phase)


# Three-dimensional meshes (nz, ny, nx): one Gaussian packet in a harmonic
# well, both separable, so the fields are outer products of 1D vectors.

@dataclasses.dataclass
class Problem3:
    nx: int
    ny: int
    nz: int
    dt: float
    steps: int
    sigma: float
    k: Tuple[float, float, float]
    omega: float
    mass: float = 1.0
    hbar: float = 1.0

    @property
    def sites(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def site_steps(self) -> int:
        return self.sites * self.steps


def packet_in_well3(n: int, seed: int, dt: float = 0.05, steps: int = 200, sigma: float = 8.0,
                    omega: float = 0.02, nz: int = 0, ny: int = 0) -> Problem3:
    """One packet at the centre of an n x ny x nz mesh, momentum drawn U[-0.5, 0.5]^3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = tuple(float(v) for v in rng.uniform(-0.5, 0.5, 3))
    return Problem3(n, ny or n, nz or n, dt, steps, sigma, k, omega)


def state3(p: Problem3, device="cpu", dtype=torch.complex128) -> torch.Tensor:
    """Unit-norm packet exp(-r^2/(4 sigma^2) + i k.r) as (nz, ny, nx)."""
    vecs = []
    for n, kk in ((p.nx, p.k[0]), (p.ny, p.k[1]), (p.nz, p.k[2])):
        x = np.arange(n) - n / 2
        v = np.exp(-x * x / (4 * p.sigma ** 2) + 1j * kk * x)
        vecs.append(torch.from_numpy(v / np.linalg.norm(v)).to(device))
    fx, fy, fz = vecs
    return (fz[:, None, None] * fy[None, :, None] * fx[None, None, :]).to(dtype).contiguous()


def potential3(p: Problem3, device="cpu") -> torch.Tensor:
    """V = m omega^2 r^2 / 2 as (nz, ny, nx) float64."""
    k = 0.5 * p.mass * p.omega ** 2
    v = [torch.from_numpy(k * (np.arange(n) - n / 2) ** 2).to(device) for n in (p.nx, p.ny, p.nz)]
    return (v[2][:, None, None] + v[1][None, :, None] + v[0][None, None, :]).contiguous()


def random_state(nx: int, ny: int, seed: int) -> np.ndarray:
    """Unit-norm complex Gaussian noise: a state with every wavenumber present."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    return a / np.linalg.norm(a)


def random_potential(nx: int, ny: int, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return scale * rng.standard_normal((ny, nx))


@dataclasses.dataclass
class Request:
    """One solve request of a served trace: arrival time (s) and its problem."""
    rid: int
    arrival: float
    problem: Problem


def request_trace(rate: float = 200.0, duration: float = 60.0, seed: int = 5, lo: int = 128,
                  hi: int = 4096, steps_lo: int = 100, steps_hi: int = 2000,
                  p_c64: float = 0.8) -> List[Request]:
    """Poisson arrivals at `rate` per second for `duration` seconds.  Sides
    log-uniform in [lo, hi] rounded to even (square with probability 1/2),
    steps uniform in [steps_lo, steps_hi], complex64 with probability p_c64
    else complex128, 1-4 seeded packets in a harmonic well plus bumps, dt from
    {0.02, 0.05, 0.1}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out: List[Request] = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        square = rng.uniform() < 0.5
        a = _even(math.exp(rng.uniform(math.log(lo), math.log(hi))), lo)
        b = a if square else _even(math.exp(rng.uniform(math.log(lo), math.log(hi))), lo)
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        dtype = "c64" if rng.uniform() < p_c64 else "c128"
        dt = float(rng.choice([0.02, 0.05, 0.1]))
        npk = int(rng.integers(1, 5))
        sub = int(rng.integers(0, 2**31 - 1))
        prob = packets_and_bumps(a, b, sub, dt, steps, dtype, n_packets=npk,
                                 name=f"req{len(out)}_{a}x{b}")
        out.append(Request(len(out), t, prob))
    return out
