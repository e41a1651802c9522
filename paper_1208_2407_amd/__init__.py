"""Second-order Trotter-Suzuki solver for one particle on a 2D mesh, for AMD MI355X.

Thin Python binding of ``libtsq.so`` (C ABI in ``include/tsq.h``): every
function named ``tsq_*`` here marshals its arguments into the C call of the
same name and raises :class:`TsqError` on a non-zero status.  All arithmetic
runs in the HIP kernels; torch is used only to own device memory and to hand
over the current HIP stream.  There is no CPU fallback: if the library is not
built, or no GPU is present, the calls fail loudly.

Convenience layer: :class:`Plan` (one problem statement) and the functions
:func:`evolve` and :func:`observables`.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libtsq.so")

TSQ_OK = 0
STATUS = {0: "TSQ_OK", -1: "TSQ_ERR_ARG", -2: "TSQ_ERR_SHAPE", -3: "TSQ_ERR_DTYPE",
          -4: "TSQ_ERR_WORKSPACE", -5: "TSQ_ERR_DEVICE", -6: "TSQ_ERR_STATE",
          -7: "TSQ_ERR_UNSUPPORTED"}
DTYPES = {"c64": 0, "c128": 1}
BCS = {"periodic": 0, "closed": 1}

EXPORTED = ("tsq_abi_version", "tsq_last_error", "tsq_plan_create", "tsq_plan_destroy",
            "tsq_workspace_size", "tsq_plan_set_schedule", "tsq_plan_get_schedule",
            "tsq_evolve_passes", "tsq_set_potential", "tsq_evolve", "tsq_set_potential_td",
            "tsq_evolve_td", "tsq_observables",
            "tsq_batch_create", "tsq_batch_destroy", "tsq_batch_workspace_size", "tsq_batch_info",
            "tsq_batch_upload", "tsq_batch_launch", "tsq_batch_evolve_workspace_size",
            "tsq_batch_evolve", "tsq_batch_evolve_noalloc")


class TsqError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class tsq_schedule(ctypes.Structure):
    _fields_ = [("steps_per_pass", ctypes.c_int32), ("segment_rows", ctypes.c_int32),
                ("pairs_per_lane", ctypes.c_int32), ("phase_store", ctypes.c_int32)]

    def as_tuple(self) -> Tuple[int, int, int, int]:
        return (self.steps_per_pass, self.segment_rows, self.pairs_per_lane, self.phase_store)


PHASE_STORE = {"default": 0, "registers": 1, "lds": 2}


class tsq_problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("mass", ctypes.c_double), ("hbar", ctypes.c_double),
                ("dt", ctypes.c_double), ("bc", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("order", ctypes.c_int32), ("nz", ctypes.c_int32), ("dz", ctypes.c_double)]


_lib = None


def library_path() -> str:
    """Path of the kernel library this module loads."""
    return LIB_PATH


def load_library(path: Optional[str] = None) -> ctypes.CDLL:
    """Load libtsq.so (built in-tree by ``python -m paper_1208_2407_amd.build``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libtsq.so is not built ({p}); run `python -m paper_1208_2407_amd.build`")
    lib = ctypes.CDLL(p)
    vp, sz, i32, i64, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.tsq_abi_version.argtypes = []
    lib.tsq_abi_version.restype = ctypes.c_int
    lib.tsq_last_error.argtypes = []
    lib.tsq_last_error.restype = ctypes.c_char_p
    lib.tsq_plan_create.argtypes = [ctypes.POINTER(tsq_problem), ctypes.POINTER(vp)]
    lib.tsq_plan_destroy.argtypes = [vp]
    lib.tsq_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.tsq_plan_set_schedule.argtypes = [vp, ctypes.POINTER(tsq_schedule)]
    lib.tsq_plan_get_schedule.argtypes = [vp, ctypes.POINTER(tsq_schedule)]
    lib.tsq_evolve_passes.argtypes = [vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.tsq_set_potential.argtypes = [vp, vp, vp, sz, vp]
    lib.tsq_evolve.argtypes = [vp, vp, i64, vp, sz, vp]
    lib.tsq_set_potential_td.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.tsq_evolve_td.argtypes = [vp, vp, i64, ctypes.POINTER(d), vp, sz, vp]
    lib.tsq_observables.argtypes = [vp, vp, vp, ctypes.POINTER(d), ctypes.POINTER(d), vp, sz, vp]
    vpp = ctypes.POINTER(vp)
    lib.tsq_batch_create.argtypes = [vpp, vpp, vpp, ctypes.POINTER(i64), i32,
                                     ctypes.POINTER(tsq_schedule), vpp]
    lib.tsq_batch_destroy.argtypes = [vp]
    lib.tsq_batch_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.tsq_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.tsq_batch_upload.argtypes = [vp, vp, sz, vp]
    lib.tsq_batch_launch.argtypes = [vp, i32, vp]
    lib.tsq_batch_evolve_workspace_size.argtypes = [vpp, vpp, vpp, ctypes.POINTER(i64), i32,
                                                    ctypes.POINTER(tsq_schedule),
                                                    ctypes.POINTER(sz)]
    lib.tsq_batch_evolve.argtypes = [vpp, vpp, vpp, ctypes.POINTER(i64), i32,
                                     ctypes.POINTER(tsq_schedule), vp, sz, vp]
    lib.tsq_batch_evolve_noalloc.argtypes = [vpp, vpp, vpp, ctypes.POINTER(i64), i32,
                                             ctypes.POINTER(tsq_schedule), vp]
    for name in EXPORTED[2:]:
        getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != TSQ_OK:
        raise TsqError(rc, load_library().tsq_last_error().decode())


# ---------------------------------------------------------------- C-ABI mirrors

def tsq_abi_version() -> int:
    return load_library().tsq_abi_version()


def tsq_last_error() -> str:
    return load_library().tsq_last_error().decode()


def tsq_plan_create(problem: tsq_problem) -> int:
    h = ctypes.c_void_p()
    _check(load_library().tsq_plan_create(ctypes.byref(problem), ctypes.byref(h)))
    return h.value


def tsq_plan_destroy(plan: int) -> None:
    _check(load_library().tsq_plan_destroy(plan))


def tsq_workspace_size(plan: int) -> int:
    n = ctypes.c_size_t()
    _check(load_library().tsq_workspace_size(plan, ctypes.byref(n)))
    return n.value


def tsq_plan_set_schedule(plan: int, schedule: tsq_schedule) -> None:
    _check(load_library().tsq_plan_set_schedule(plan, ctypes.byref(schedule)))


def tsq_plan_get_schedule(plan: int) -> tsq_schedule:
    sc = tsq_schedule()
    _check(load_library().tsq_plan_get_schedule(plan, ctypes.byref(sc)))
    return sc


def tsq_evolve_passes(plan: int, steps: int) -> Tuple[int, bool]:
    n, c = ctypes.c_int64(), ctypes.c_int32()
    _check(load_library().tsq_evolve_passes(plan, int(steps), ctypes.byref(n), ctypes.byref(c)))
    return n.value, bool(c.value)


def tsq_set_potential(plan: int, V_dev: int, ws: int, ws_bytes: int, stream: int) -> None:
    _check(load_library().tsq_set_potential(plan, V_dev, ws, ws_bytes, stream))


def tsq_evolve(plan: int, psi_dev: int, steps: int, ws: int, ws_bytes: int, stream: int) -> None:
    _check(load_library().tsq_evolve(plan, psi_dev, int(steps), ws, ws_bytes, stream))


def tsq_set_potential_td(plan: int, V0_dev: int, W_dev: int, ws: int, ws_bytes: int,
                         stream: int) -> None:
    _check(load_library().tsq_set_potential_td(plan, V0_dev, W_dev, ws, ws_bytes, stream))


def tsq_evolve_td(plan: int, psi_dev: int, f, ws: int, ws_bytes: int, stream: int) -> None:
    """`f`: the modulation of each step at its midpoint (len(f) steps)."""
    import numpy as np
    fv = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
    ptr = fv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if fv.size else None
    _check(load_library().tsq_evolve_td(plan, psi_dev, int(fv.size), ptr, ws, ws_bytes, stream))


def tsq_observables(plan: int, psi_dev: int, V_dev: int, ws: int, ws_bytes: int,
                    stream: int) -> Tuple[float, float]:
    n, e = ctypes.c_double(), ctypes.c_double()
    _check(load_library().tsq_observables(plan, psi_dev, V_dev, ctypes.byref(n), ctypes.byref(e),
                                          ws, ws_bytes, stream))
    return n.value, e.value


def tsq_batch_create(plans, psi_devs, wss, steps, schedule: Optional[tsq_schedule] = None) -> int:
    n = len(plans)
    arr = lambda xs: (ctypes.c_void_p * n)(*xs)
    st = (ctypes.c_int64 * n)(*[int(v) for v in steps])
    h = ctypes.c_void_p()
    _check(load_library().tsq_batch_create(arr(plans), arr(psi_devs), arr(wss), st, n,
                                           ctypes.byref(schedule) if schedule is not None else None,
                                           ctypes.byref(h)))
    return h.value


def tsq_batch_destroy(batch: int) -> None:
    _check(load_library().tsq_batch_destroy(batch))


def tsq_batch_workspace_size(batch: int) -> int:
    n = ctypes.c_size_t()
    _check(load_library().tsq_batch_workspace_size(batch, ctypes.byref(n)))
    return n.value


def tsq_batch_info(batch: int) -> Tuple[int, int]:
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().tsq_batch_info(batch, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def tsq_batch_upload(batch: int, bws: int, nbytes: int, stream: int) -> None:
    _check(load_library().tsq_batch_upload(batch, bws, nbytes, stream))


def tsq_batch_launch(batch: int, use_graph: bool, stream: int) -> None:
    _check(load_library().tsq_batch_launch(batch, 1 if use_graph else 0, stream))


def _batch_args(plans, psi_devs, wss, steps):
    n = len(plans)
    arr = lambda xs: (ctypes.c_void_p * n)(*xs)
    return arr(plans), arr(psi_devs), arr(wss), (ctypes.c_int64 * n)(*[int(v) for v in steps]), n


def tsq_batch_evolve_workspace_size(plans, psi_devs, wss, steps,
                                    schedule: Optional[tsq_schedule] = None) -> int:
    a, b, c, st, n = _batch_args(plans, psi_devs, wss, steps)
    out = ctypes.c_size_t()
    _check(load_library().tsq_batch_evolve_workspace_size(
        a, b, c, st, n, ctypes.byref(schedule) if schedule is not None else None,
        ctypes.byref(out)))
    return out.value


def tsq_batch_evolve(plans, psi_devs, wss, steps, schedule: Optional[tsq_schedule], bws: int,
                     bws_bytes: int, stream: int) -> None:
    a, b, c, st, n = _batch_args(plans, psi_devs, wss, steps)
    _check(load_library().tsq_batch_evolve(
        a, b, c, st, n, ctypes.byref(schedule) if schedule is not None else None, bws, bws_bytes,
        stream))


def tsq_batch_evolve_noalloc(plans, psi_devs, wss, steps, schedule: Optional[tsq_schedule],
                             stream: int) -> None:
    a, b, c, st, n = _batch_args(plans, psi_devs, wss, steps)
    _check(load_library().tsq_batch_evolve_noalloc(
        a, b, c, st, n, ctypes.byref(schedule) if schedule is not None else None, stream))


# ---------------------------------------------------------------- convenience layer

def _torch():
    import torch
    return torch


def _stream_handle(device) -> int:
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


class Plan:
    """One problem statement (mesh, spacing, mass, hbar, dt, dtype) with its workspace.

    The workspace (second psi buffer, phase table, reduction scratch) is a
    torch uint8 tensor on the plan's device; :meth:`set_potential` must be
    called before :meth:`evolve`.
    """

    def __init__(self, nx: int, ny: int, dt: float, dtype: str = "c128", *, dx=1.0, dy=1.0,
                 mass=1.0, hbar=1.0, bc="periodic", order: int = 2, nz: int = 0, dz=1.0,
                 device="cuda"):
        """nz >= 2 makes a 3D mesh: psi and V are then (nz, ny, nx) tensors."""
        self.problem = tsq_problem(int(nx), int(ny), float(dx), float(dy), float(mass),
                                   float(hbar), float(dt), BCS[bc], DTYPES[dtype], int(order),
                                   int(nz), float(dz))
        self.dtype = dtype
        self.handle = tsq_plan_create(self.problem)
        self.device = device
        self._ws = None
        self._V = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                tsq_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def shape(self) -> Tuple[int, ...]:
        """(ny, nx) of a 2D mesh, (nz, ny, nx) of a 3D one."""
        p = self.problem
        return (p.nz, p.ny, p.nx) if p.nz >= 2 else (p.ny, p.nx)

    @property
    def workspace_bytes(self) -> int:
        return tsq_workspace_size(self.handle)

    def set_schedule(self, steps_per_pass: int = 0, segment_rows: int = 0,
                     pairs_per_lane: int = 0, phase_store: int = 0) -> None:
        """Zero fields take the library defaults; phase_store 1 = registers, 2 = LDS."""
        tsq_plan_set_schedule(self.handle, tsq_schedule(int(steps_per_pass), int(segment_rows),
                                                        int(pairs_per_lane), int(phase_store)))

    def schedule(self) -> Tuple[int, int, int, int]:
        """(steps_per_pass, segment_rows, pairs_per_lane, phase_store) in force."""
        return tsq_plan_get_schedule(self.handle).as_tuple()

    def passes(self, steps: int) -> Tuple[int, bool]:
        """(kernel launches, trailing copy) that evolve(psi, steps) makes."""
        return tsq_evolve_passes(self.handle, steps)

    def workspace(self):
        torch = _torch()
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def set_potential(self, V) -> None:
        torch = _torch()
        if V.dtype != torch.float64 or not V.is_contiguous() or tuple(V.shape) != self.shape:
            raise ValueError(f"V must be a contiguous float64 {self.shape} device tensor")
        ws = self.workspace()
        tsq_set_potential(self.handle, V.data_ptr(), ws.data_ptr(), ws.numel(),
                          _stream_handle(V.device))
        self._V = V

    def set_potential_td(self, V0, W) -> None:
        """Time-dependent potential V0 + f(t) W (modulations given to evolve_td)."""
        torch = _torch()
        for name, a in (("V0", V0), ("W", W)):
            if a.dtype != torch.float64 or not a.is_contiguous() or tuple(a.shape) != self.shape:
                raise ValueError(f"{name} must be a contiguous float64 {self.shape} device tensor")
        ws = self.workspace()
        tsq_set_potential_td(self.handle, V0.data_ptr(), W.data_ptr(), ws.data_ptr(), ws.numel(),
                             _stream_handle(V0.device))
        self._V = None

    def evolve_td(self, psi, f):
        """Apply len(f) steps to psi in place, step n under V0 + f[n] W (f[n] taken
        at the step's midpoint), and return it."""
        self._check_psi(psi)
        ws = self.workspace()
        tsq_evolve_td(self.handle, psi.data_ptr(), f, ws.data_ptr(), ws.numel(),
                      _stream_handle(psi.device))
        return psi

    def _check_psi(self, psi) -> None:
        torch = _torch()
        want = torch.complex128 if self.dtype == "c128" else torch.complex64
        if psi.dtype != want or not psi.is_contiguous() or tuple(psi.shape) != self.shape:
            raise ValueError(f"psi must be a contiguous {want} {self.shape} device tensor")

    def evolve(self, psi, steps: int):
        """Apply U2(dt)^steps to psi in place and return it."""
        self._check_psi(psi)
        ws = self.workspace()
        tsq_evolve(self.handle, psi.data_ptr(), steps, ws.data_ptr(), ws.numel(),
                   _stream_handle(psi.device))
        return psi

    def observables(self, psi, V=None) -> Tuple[float, float]:
        """(norm, energy) of psi in FP64; synchronises the current stream."""
        self._check_psi(psi)
        V = self._V if V is None else V
        if V is None:
            raise ValueError("no potential given")
        torch = _torch()
        if V.dtype != torch.float64 or not V.is_contiguous() or tuple(V.shape) != self.shape:
            raise ValueError(f"V must be a contiguous float64 {self.shape} device tensor")
        ws = self.workspace()
        return tsq_observables(self.handle, psi.data_ptr(), V.data_ptr(), ws.data_ptr(),
                               ws.numel(), _stream_handle(psi.device))


class Batch:
    """Many independent problems advanced together (``tsq_batch_*``).

    ``plans[i]`` (with its potential set) evolves ``psis[i]`` by ``steps[i]``;
    all plans share one dtype.  :meth:`launch` enqueues every pass of every
    problem on the current stream, optionally through a HIP graph (captured on
    the first such call on a side stream ordered with the current one, replayed
    by later calls on the current stream).
    """

    def __init__(self, plans, psis, steps, schedule=(0, 0, 0, 0)):
        torch = _torch()
        if not (len(plans) == len(psis) == len(steps)) or not plans:
            raise ValueError("plans, psis and steps must be non-empty and of equal length")
        for pl, psi in zip(plans, psis):
            pl._check_psi(psi)
            if pl._ws is None:
                raise ValueError("every plan needs set_potential() before batching")
        self.plans, self.psis = list(plans), list(psis)
        self.device = psis[0].device
        sc = tsq_schedule(*[int(v) for v in schedule])
        self.handle = tsq_batch_create([p.handle for p in plans], [t.data_ptr() for t in psis],
                                       [p._ws.data_ptr() for p in plans], steps, sc)
        self.bws = torch.empty(tsq_batch_workspace_size(self.handle), dtype=torch.uint8,
                               device=self.device)
        tsq_batch_upload(self.handle, self.bws.data_ptr(), self.bws.numel(),
                         _stream_handle(self.device))
        self._side = None
        self._captured = False

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                tsq_batch_destroy(h)
            except Exception:
                pass
            self.handle = None

    def info(self) -> Tuple[int, int]:
        """(kernel launches per call, tiles per call)."""
        return tsq_batch_info(self.handle)

    def launch(self, use_graph: bool = False) -> None:
        torch = _torch()
        if not use_graph:
            tsq_batch_launch(self.handle, False, _stream_handle(self.device))
            return
        if self._captured:  # replay on the current stream
            tsq_batch_launch(self.handle, True, _stream_handle(self.device))
            return
        # capture on a side stream (the current one may be the null stream, which
        # cannot capture), ordered with the current one
        if self._side is None:
            self._side = torch.cuda.Stream(device=self.device)
        cur = torch.cuda.current_stream(self.device)
        self._side.wait_stream(cur)
        tsq_batch_launch(self.handle, True, self._side.cuda_stream)
        cur.wait_stream(self._side)
        self._captured = True


def _dtype_name(t) -> str:
    torch = _torch()
    if t.dtype == torch.complex128:
        return "c128"
    if t.dtype == torch.complex64:
        return "c64"
    raise ValueError(f"psi dtype {t.dtype} is not complex64/complex128")


def evolve(psi, V, dt: float, steps: int, *, dx=1.0, dy=1.0, dz=1.0, mass=1.0, hbar=1.0,
           bc="periodic", order: int = 2, steps_per_pass: int = 0, segment_rows: int = 0,
           pairs_per_lane: int = 0, phase_store: int = 0):
    """Evolve the device tensor psi (ny, nx), or (nz, ny, nx) for a 3D mesh, in place by
    `steps` steps of U2 (order 2) or U4 (order 4)."""
    nz, ny, nx = psi.shape if psi.dim() == 3 else (0,) + tuple(psi.shape)
    plan = Plan(nx, ny, dt, _dtype_name(psi), dx=dx, dy=dy, mass=mass, hbar=hbar, bc=bc,
                order=order, nz=nz, dz=dz, device=psi.device)
    plan.set_schedule(steps_per_pass, segment_rows, pairs_per_lane, phase_store)
    plan.set_potential(V)
    plan.evolve(psi, steps)
    return psi


def evolve_td(psi, V0, W, f, dt: float, *, dx=1.0, dy=1.0, mass=1.0, hbar=1.0,
              steps_per_pass: int = 0, segment_rows: int = 0, phase_store: int = 0):
    """Evolve psi in place by len(f) steps under V(t) = V0 + f(t) W, step n using
    f[n] = f(t_n + dt/2) (periodic mesh, order 2)."""
    ny, nx = psi.shape
    plan = Plan(nx, ny, dt, _dtype_name(psi), dx=dx, dy=dy, mass=mass, hbar=hbar,
                device=psi.device)
    plan.set_schedule(steps_per_pass, segment_rows, 1, phase_store)
    plan.set_potential_td(V0, W)
    plan.evolve_td(psi, f)
    return psi


def observables(psi, V, *, dx=1.0, dy=1.0, dz=1.0, mass=1.0, hbar=1.0,
                bc="periodic") -> Tuple[float, float]:
    nz, ny, nx = psi.shape if psi.dim() == 3 else (0,) + tuple(psi.shape)
    plan = Plan(nx, ny, 0.0, _dtype_name(psi), dx=dx, dy=dy, mass=mass, hbar=hbar, bc=bc,
                nz=nz, dz=dz, device=psi.device)
    return plan.observables(psi, V)
