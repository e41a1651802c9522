"""Shared helpers of the GPU tests: run the HIP path through the C ABI binding,
and run the oracle on the same host arrays."""
import sys
import time

import numpy as np
import torch

import oracle
import paper_1208_2407_amd as tsq

TOL = {"c128": 1e-12, "c64": 1e-5}
TORCH_DT = {"c128": torch.complex128, "c64": torch.complex64}


def log(msg: str) -> None:
    print(msg, file=sys.__stderr__, flush=True)


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def as_input(psi0: np.ndarray, dtype: str) -> np.ndarray:
    """The exact complex128 values the GPU starts from (complex64 rounds psi0)."""
    if dtype == "c64":
        return psi0.astype(np.complex64).astype(np.complex128)
    return np.asarray(psi0, dtype=np.complex128)


def gpu_evolve(psi0: np.ndarray, V: np.ndarray, dt: float, steps: int, dtype: str,
               steps_per_pass: int = 0, segment_rows: int = 0, pairs_per_lane: int = 0,
               phase_store: int = 0, **consts) -> np.ndarray:
    ny, nx = psi0.shape
    psi = torch.from_numpy(np.ascontiguousarray(psi0)).to(TORCH_DT[dtype]).cuda()
    Vd = torch.from_numpy(np.ascontiguousarray(V, dtype=np.float64)).cuda()
    plan = tsq.Plan(nx, ny, dt, dtype, device=psi.device, **consts)
    plan.set_schedule(steps_per_pass, segment_rows, pairs_per_lane, phase_store)
    plan.set_potential(Vd)
    plan.evolve(psi, steps)
    torch.cuda.synchronize()
    return psi.cpu().numpy().astype(np.complex128)


def oracle_evolve(psi0: np.ndarray, V: np.ndarray, dt: float, steps: int, dtype: str,
                  chunk: int = 0, label: str = "", **consts) -> np.ndarray:
    """Oracle run on the GPU's starting values; long runs go in chunks with a log line each."""
    psi = as_input(psi0, dtype)
    if chunk <= 0 or chunk >= steps:
        return oracle.evolve(psi, V, dt, steps, **consts)
    done = 0
    t0 = time.time()
    while done < steps:
        n = min(chunk, steps - done)
        psi = oracle.evolve(psi, V, dt, n, **consts)
        done += n
        log(f"  oracle {label}: {done}/{steps} steps, {time.time() - t0:.1f} s")
    return psi


def crop_periodic(a: np.ndarray, y0: int, x0: int, h: int, w: int) -> np.ndarray:
    ys = np.arange(y0, y0 + h) % a.shape[0]
    xs = np.arange(x0, x0 + w) % a.shape[1]
    return a[np.ix_(ys, xs)]
