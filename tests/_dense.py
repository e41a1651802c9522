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


# ---------------------------------------------------------------- three dimensions
# Site (x, y, z) is basis vector l = (z * ny + y) * nx + x; the split has seven
# parts: the diagonal and the even and odd pairs along each of the three axes.

def hop_matrix3(n3, axis, parity, J, bc):
    nx, ny, nz = n3
    n = nx * ny * nz
    H = np.zeros((n, n))
    L = n3[axis]
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                c = [x, y, z]
                if c[axis] % 2 != parity:
                    continue
                c2 = list(c)
                c2[axis] += 1
                if c2[axis] == L:
                    if bc == "closed":
                        continue
                    c2[axis] = 0
                l1 = (c[2] * ny + c[1]) * nx + c[0]
                l2 = (c2[2] * ny + c2[1]) * nx + c2[0]
                H[l1, l2] += -J
                H[l2, l1] += -J
    return H


def parts3(n3, V, dx=1.0, dy=1.0, dz=1.0, mass=1.0, hbar=1.0, bc="periodic"):
    J = [hbar * hbar / (2 * mass * d * d) for d in (dx, dy, dz)]
    out = {"H0": np.diag(np.asarray(V, dtype=float).reshape(-1) + 2 * sum(J))}
    for a, name in enumerate("xyz"):
        out["E" + name] = hop_matrix3(n3, a, 0, J[a], bc)
        out["O" + name] = hop_matrix3(n3, a, 1, J[a], bc)
    return out


def full_h3(n3, V, **kw):
    p = parts3(n3, V, **kw)
    return sum(p.values())


def u2_dense3(n3, V, dt, hbar=1.0, **kw):
    p = parts3(n3, V, hbar=hbar, **kw)
    h = dt / 2
    f = {k: factor(p[k], h, hbar) for k in p if k != "H0"}
    P = factor(p["H0"], dt, hbar)
    seq = [f["Ox"], f["Oy"], f["Oz"], f["Ex"], f["Ey"], f["Ez"], P,
           f["Ez"], f["Ey"], f["Ex"], f["Oz"], f["Oy"], f["Ox"]]
    U = np.eye(P.shape[0], dtype=complex)
    for M in seq:
        U = M @ U
    return U


def u2_dense1(L, V1, dt, d=1.0, mass=1.0, hbar=1.0):
    """One axis alone: Oa(h) Ea(h) P_a(dt) Ea(h) Oa(h) with the diagonal V1 + hbar^2/(m d^2)."""
    J = hbar * hbar / (2 * mass * d * d)
    E = hop_matrix(L, 1, "x", 0, J, "periodic")
    O = hop_matrix(L, 1, "x", 1, J, "periodic")
    P = factor(np.diag(np.asarray(V1, dtype=float) + 2 * J), dt, hbar)
    fe, fo = factor(E, dt / 2, hbar), factor(O, dt / 2, hbar)
    return fo @ fe @ P @ fe @ fo
