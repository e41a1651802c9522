"""Closed-form solutions of the Trotter-Suzuki step that pin the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Bloch form.  For a flat potential V = V0 on a periodic mesh with even sides,
every factor of the second-order step (Sec. 2, Eq. "secondorder", five-part
split in 2D) commutes with translations by two sites.  Along one axis write
A_j = psi_{2j}, B_j = psi_{2j+1} and take the discrete Fourier transform over
j (wavenumber q = 2 pi m / (L/2)).  Then, with c = cos(alpha),
s = sin(alpha), alpha = tau J / hbar, J = hbar^2 / (2 m a^2):

  even pairs (2j, 2j+1):    E    = [[c, i s], [i s, c]]
  odd pairs (2j+1, 2j+2):   O(q) = [[c, i s e^{-iq}], [i s e^{+iq}, c]]

(the odd pair couples B_{j-1} into A_j and A_{j+1} into B_j, which the
transform turns into the phases e^{-iq}, e^{+iq}).  One step applies O, E, E,
O along each axis (rightmost first in matrix order: M = O E E O) and the
potential factor, which for flat V is the global phase
exp(-i dt (V0 + hbar^2/(m dx^2) + hbar^2/(m dy^2)) / hbar).  N steps are
therefore  psi_N = IFFT[ (M_x^N kron M_y^N) FFT psi_0 ] * exp(-i N phi).
This is exact, any size, and uses no rotation routine of the oracle.
"""
from __future__ import annotations

import numpy as np


def _axis_step_matrices(L: int, tau_half: float, J: float, hbar: float) -> np.ndarray:
    """Stack (L/2, 2, 2) of the one-step matrices M(q) = O E E O along one axis."""
    alpha = tau_half * J / hbar
    c, s = np.cos(alpha), np.sin(alpha)
    m = np.arange(L // 2)
    q = 2.0 * np.pi * m / (L // 2)
    E = np.array([[c, 1j * s], [1j * s, c]], dtype=np.complex128)
    O = np.empty((L // 2, 2, 2), dtype=np.complex128)
    O[:, 0, 0] = c
    O[:, 1, 1] = c
    O[:, 0, 1] = 1j * s * np.exp(-1j * q)
    O[:, 1, 0] = 1j * s * np.exp(1j * q)
    return O @ E @ E @ O


def bloch_evolve(psi0, V0: float, dt: float, steps: int, *, dx=1.0, dy=1.0, mass=1.0,
                 hbar=1.0) -> np.ndarray:
    """psi after `steps` second-order steps on a periodic mesh with flat V = V0."""
    psi0 = np.asarray(psi0, dtype=np.complex128)
    ny, nx = psi0.shape
    if nx % 2 or ny % 2:
        raise ValueError("Bloch form needs even sides")
    h = 0.5 * dt
    Jx = hbar * hbar / (2.0 * mass * dx * dx)
    Jy = hbar * hbar / (2.0 * mass * dy * dy)
    Mx = np.linalg.matrix_power(_axis_step_matrices(nx, h, Jx, hbar), int(steps))
    My = np.linalg.matrix_power(_axis_step_matrices(ny, h, Jy, hbar), int(steps))
    # psi[jy, sy, jx, sx]
    a = psi0.reshape(ny // 2, 2, nx // 2, 2)
    ah = np.fft.fft(np.fft.fft(a, axis=0), axis=2)
    ah = _apply(Mx, My, ah)
    out = np.fft.ifft(np.fft.ifft(ah, axis=0), axis=2).reshape(ny, nx)
    eps0 = hbar * hbar / (mass * dx * dx) + hbar * hbar / (mass * dy * dy)
    phi = dt * (V0 + eps0) / hbar
    return out * np.exp(-1j * phi * steps)


def _apply(Mx: np.ndarray, My: np.ndarray, ah: np.ndarray) -> np.ndarray:
    # ah[my, sy, mx, sx]; out[my, sy', mx, sx'] = sum My[my, sy', sy] Mx[mx, sx', sx] ah[...]
    t = np.einsum("yab,ybxc->yaxc", My, ah)
    return np.einsum("xcd,yaxd->yaxc", Mx, t)


def plane_wave(nx: int, ny: int, mx: int, my: int) -> np.ndarray:
    """Normalised lattice plane wave exp(i (kx x + ky y)), k = 2 pi m / L."""
    y, x = np.mgrid[0:ny, 0:nx]
    kx, ky = 2 * np.pi * mx / nx, 2 * np.pi * my / ny
    return np.exp(1j * (kx * x + ky * y)) / np.sqrt(nx * ny)


def plane_wave_energy(nx: int, ny: int, mx: int, my: int, V0: float, *, dx=1.0, dy=1.0,
                      mass=1.0, hbar=1.0) -> float:
    """<H> of a lattice plane wave on a periodic mesh with flat V0:
    V0 + sum_a hbar^2/(m da^2) (1 - cos(k_a)), the tight-binding dispersion."""
    kx, ky = 2 * np.pi * mx / nx, 2 * np.pi * my / ny
    return (V0 + hbar * hbar / (mass * dx * dx) * (1 - np.cos(kx))
            + hbar * hbar / (mass * dy * dy) * (1 - np.cos(ky)))
