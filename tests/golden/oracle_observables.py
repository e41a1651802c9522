"""Writes oracle_observables_4096.json: the FP64 oracle's norm and energy before
and after the 4096 x 4096 packets-and-bumps workload (four packets in a harmonic
well plus 32 bumps, dt = 0.05, 1000 second-order steps), once from the
complex128 initial state and once from that state rounded to complex64 (the
values a complex64 run starts from).  The benchmark reports its GPU results'
norm and energy against these.  Calls only the oracle.

    python tests/golden/oracle_observables.py        (about 2 minutes on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1208_2407_amd import workloads as wl  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_observables_4096.json")


def main() -> None:
    oracle.build(force=False)
    p = wl.packets_and_bumps(4096, 4096, 2, 0.05, 1000, "c64", name="packets_bumps_4096")
    psi0 = wl.initial_state(p).numpy()
    V = wl.potential(p).numpy()
    out = {"workload": "packets_bumps_4096x4096_dt0.05_1000steps", "steps": p.steps,
           "dt": p.dt, "mesh": [p.nx, p.ny], "inputs": {}}
    for name, start in (("c128", psi0.astype(np.complex128)),
                        ("c64", psi0.astype(np.complex64).astype(np.complex128))):
        n0, e0 = oracle.observables(start, V)
        t0 = time.time()
        end = oracle.evolve(start, V, p.dt, p.steps)
        n1, e1 = oracle.observables(end, V)
        print(f"{name}: norm {n0!r} -> {n1!r}, energy {e0!r} -> {e1!r} "
              f"({time.time() - t0:.0f} s)", flush=True)
        out["inputs"][name] = {"norm_start": n0, "energy_start": e0, "norm_end": n1,
                               "energy_end": e1}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
