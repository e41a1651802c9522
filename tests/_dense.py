"""Dense-matrix forms of the lattice Hamiltonian and its Trotter factors, for pins.

The mesh site (x, y) is basis vector l = y * nx + x.  The pieces follow the
split of Sec. 2: a diagonal H0 = V + hbar^2/(m dx^2) + hbar^2/(m dy^2) and, per
axis, a block-diagonal hopping matrix on the even pairs and one on the odd
pairs, each block [[0, -J], [-J, 0]] with J = hbar^2 / (2 m a^2).  Exponentials
are scipy's expm / numpy's eigh, independent of the oracle's rotation code.
"""
import numpy as np
import scipy.linalg


def hop_matrix(nx, ny, axis, parity, J, bc):
    n = nx * ny
    H = np.zeros((n, n))
    L = nx if axis == "x" else ny
    for y in range(ny):
        for x in range(nx):
            c = x if axis == "x" else y
            if c % 2 != parity:
                continue
            c2 = c + 1
            if c2 == L:
                if bc == "closed":
                    continue
                c2 = 0
            if axis == "x":
                l1, l2 = y * nx + x, y * nx + c2
            else:
                l1, l2 = y * nx + x, c2 * nx + x
            H[l1, l2] += -J
            H[l2, l1] += -J
    return H


def parts(nx, ny, V, dx=1.0, dy=1.0, mass=1.0, hbar=1.0, bc="periodic"):
    Jx = hbar * hbar / (2 * mass * dx * dx)
    Jy = hbar * hbar / (2 * mass * dy * dy)
    H0 = np.diag(np.asarray(V, dtype=float).reshape(-1) + 2 * Jx + 2 * Jy)
    return {
        "H0": H0,
        "Ex": hop_matrix(nx, ny, "x", 0, Jx, bc),
        "Ox": hop_matrix(nx, ny, "x", 1, Jx, bc),
        "Ey": hop_matrix(nx, ny, "y", 0, Jy, bc),
        "Oy": hop_matrix(nx, ny, "y", 1, Jy, bc),
    }


def full_h(nx, ny, V, **kw):
    p = parts(nx, ny, V, **kw)
    return p["H0"] + p["Ex"] + p["Ox"] + p["Ey"] + p["Oy"]


def factor(Hk, tau, hbar=1.0):
    return scipy.linalg.expm(-1j * tau * Hk / hbar)


def u2_dense(nx, ny, V, dt, dx=1.0, dy=1.0, mass=1.0, hbar=1.0, bc="periodic"):
    p = parts(nx, ny, V, dx=dx, dy=dy, mass=mass, hbar=hbar, bc=bc)
    h = dt / 2
    f = {k: factor(p[k], h, hbar) for k in ("Ex", "Ox", "Ey", "Oy")}
    P = factor(p["H0"], dt, hbar)
    # applied first = rightmost: Ox Oy Ex Ey P Ey Ex Oy Ox (palindromic)
    seq = [f["Ox"], f["Oy"], f["Ex"], f["Ey"], P, f["Ey"], f["Ex"], f["Oy"], f["Ox"]]
    U = np.eye(nx * ny, dtype=complex)
    for M in seq:
        U = M @ U
    return U


def exact_evolution(nx, ny, V, t, hbar=1.0, **kw):
    H = full_h(nx, ny, V, hbar=hbar, **kw)
    w, Q = np.linalg.eigh(H)
    return (Q * np.exp(-1j * w * t / hbar)) @ Q.conj().T
