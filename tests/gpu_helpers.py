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


def light_cone_windows(got: np.ndarray, fields, run_oracle, windows, h: int, w: int, m: int,
                       bc: str):
    """Relative L2 of `h` x `w` windows of a full-mesh result `got` against oracle
    runs on each window plus a margin of `m` sites (at least the light cone of the
    run).  `fields` are the full-mesh input arrays the oracle needs (state first);
    `run_oracle(*crops, bc=...)` evolves the cropped arrays.  Periodic meshes crop
    with wrap-around and run the crop periodic; closed meshes clip the crop at the
    mesh walls and run it closed, so true walls stay walls and every cut edge lies
    at least `m` sites from the window.  Pairs are fixed by site parity, so a
    crop must start on an even site: windows start on even sites and the margin is
    rounded up to even."""
    ny, nx = got.shape
    m += m & 1
    errs = []
    for y0, x0 in windows:
        if (y0 | x0) & 1:
            raise ValueError(f"window ({y0}, {x0}) does not start on an even site")
        if bc == "periodic":
            crops = [crop_periodic(f, y0 - m, x0 - m, h + 2 * m, w + 2 * m) for f in fields]
            oy, ox = m, m
        else:
            ya, yb = max(0, y0 - m), min(ny, y0 + h + m)
            xa, xb = max(0, x0 - m), min(nx, x0 + w + m)
            crops = [np.ascontiguousarray(f[ya:yb, xa:xb]) for f in fields]
            oy, ox = y0 - ya, x0 - xa
        want = run_oracle(*crops, bc=bc)[oy:oy + h, ox:ox + w]
        g = crop_periodic(got, y0, x0, h, w)
        if np.linalg.norm(want) > 0:
            errs.append(rel_l2(g, want))
    return errs
