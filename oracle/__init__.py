"""FP64 CPU oracle for the second-order Trotter-Suzuki step (Sec. 2 of the paper).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product package.  It
shares no code with the HIP library.  ``tso_oracle.c`` holds the arithmetic;
this module only marshals NumPy arrays into it.  ``closed_form.py`` holds the
independent closed-form solutions used to pin it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tso_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libtso_oracle.so")

BC = {"periodic": 0, "closed": 1}


def compile_library(src: str, out: str) -> str:
    """gcc -O2 -fopenmp a C oracle source into a shared library."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the C oracle into oracle/_build/libtso_oracle.so (portable -O2, OpenMP)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    return compile_library(_SRC, _LIB)


_lib = None


def load_library(path: str):
    """A configured handle on an oracle library at `path` (the default build, or a
    variant compiled by a test)."""
    lib = ctypes.CDLL(path)
    d, i, ll, p = ctypes.c_double, ctypes.c_int, ctypes.c_longlong, ctypes.c_void_p
    lib.tso_evolve.argtypes = [i, i, i, d, d, d, d, d, p, p, ll, i]
    lib.tso_evolve.restype = i
    lib.tso_evolve_td.argtypes = [i, i, i, d, d, d, d, d, p, p, p, p, ll]
    lib.tso_evolve_td.restype = i
    lib.tso_evolve3.argtypes = [i, i, i, i, d, d, d, d, d, d, p, p, ll]
    lib.tso_evolve3.restype = i
    lib.tso_observables3.argtypes = [i, i, i, i, d, d, d, d, d, p, p,
                                     ctypes.POINTER(d), ctypes.POINTER(d)]
    lib.tso_observables3.restype = i
    lib.tso_apply_factor.argtypes = [i, i, i, d, d, d, d, i, i, d, p, p]
    lib.tso_apply_factor.restype = i
    lib.tso_observables.argtypes = [i, i, i, d, d, d, d, p, p,
                                    ctypes.POINTER(d), ctypes.POINTER(d)]
    lib.tso_observables.restype = i
    lib.tso_set_threads.argtypes = [i]
    lib.tso_set_threads.restype = None
    lib.tso_max_threads.argtypes = []
    lib.tso_max_threads.restype = i
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = load_library(_LIB)
    return _lib


def set_threads(n: int) -> None:
    _load().tso_set_threads(int(n))


def max_threads() -> int:
    return int(_load().tso_max_threads())


def _as_psi(psi) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    if a.ndim != 2:
        raise ValueError("psi must be (ny, nx)")
    return a.copy()


def _as_v(V, shape) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(V, dtype=np.float64))
    if v.shape != shape:
        raise ValueError(f"V shape {v.shape} != psi shape {shape}")
    return v


def evolve(psi0, V, dt, steps, *, dx=1.0, dy=1.0, mass=1.0, hbar=1.0,
           bc="periodic", order=2) -> np.ndarray:
    """Return psi after `steps` steps of U2(dt) (order=2) or U4(dt) (order=4)."""
    psi = _as_psi(psi0)
    v = _as_v(V, psi.shape)
    ny, nx = psi.shape
    rc = _load().tso_evolve(nx, ny, BC[bc], dx, dy, mass, hbar, dt,
                            v.ctypes.data, psi.ctypes.data, int(steps), int(order))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return psi


def evolve_td(psi0, V0, W, f, dt, *, dx=1.0, dy=1.0, mass=1.0, hbar=1.0,
              bc="periodic") -> np.ndarray:
    """Return psi after len(f) steps of U2(dt) under V(t) = V0 + f(t) W, step n
    using f[n] = f(t_n + dt/2) (the potential at the step's midpoint)."""
    psi = _as_psi(psi0)
    v0 = _as_v(V0, psi.shape)
    w = _as_v(W, psi.shape)
    fv = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
    ny, nx = psi.shape
    rc = _load().tso_evolve_td(nx, ny, BC[bc], dx, dy, mass, hbar, dt, v0.ctypes.data,
                               w.ctypes.data, fv.ctypes.data if fv.size else None,
                               psi.ctypes.data, int(fv.size))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return psi


def _as_psi3(psi) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    if a.ndim != 3:
        raise ValueError("psi must be (nz, ny, nx)")
    return a.copy()


def evolve3(psi0, V, dt, steps, *, dx=1.0, dy=1.0, dz=1.0, mass=1.0, hbar=1.0,
            bc="periodic") -> np.ndarray:
    """Three-dimensional mesh (nz, ny, nx): `steps` second-order steps."""
    psi = _as_psi3(psi0)
    v = _as_v(V, psi.shape)
    nz, ny, nx = psi.shape
    rc = _load().tso_evolve3(nx, ny, nz, BC[bc], dx, dy, dz, mass, hbar, dt, v.ctypes.data,
                             psi.ctypes.data, int(steps))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return psi


def observables3(psi, V, *, dx=1.0, dy=1.0, dz=1.0, mass=1.0, hbar=1.0, bc="periodic"):
    a = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    v = _as_v(V, a.shape)
    nz, ny, nx = a.shape
    n, e = ctypes.c_double(), ctypes.c_double()
    rc = _load().tso_observables3(nx, ny, nz, BC[bc], dx, dy, dz, mass, hbar, v.ctypes.data,
                                  a.ctypes.data, ctypes.byref(n), ctypes.byref(e))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return n.value, e.value


def apply_factor(psi0, V, which, parity, tau, *, dx=1.0, dy=1.0, mass=1.0, hbar=1.0,
                 bc="periodic") -> np.ndarray:
    """Apply one factor: which in {"x", "y", "P"}; parity 0 = even pairs, 1 = odd."""
    psi = _as_psi(psi0)
    ny, nx = psi.shape
    v = _as_v(V if V is not None else np.zeros((ny, nx)), psi.shape)
    w = {"x": 0, "y": 1, "P": 2}[which]
    rc = _load().tso_apply_factor(nx, ny, BC[bc], dx, dy, mass, hbar, w, int(parity),
                                  float(tau), v.ctypes.data, psi.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return psi


def observables(psi, V, *, dx=1.0, dy=1.0, mass=1.0, hbar=1.0, bc="periodic"):
    """Return (norm, energy) = (sum |psi|^2, <psi|H|psi>/norm)."""
    a = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    v = _as_v(V, a.shape)
    ny, nx = a.shape
    n, e = ctypes.c_double(), ctypes.c_double()
    rc = _load().tso_observables(nx, ny, BC[bc], dx, dy, mass, hbar, v.ctypes.data,
                                 a.ctypes.data, ctypes.byref(n), ctypes.byref(e))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return n.value, e.value
