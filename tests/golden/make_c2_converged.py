"""Write tests/golden/c2_converged.npz: the oracle's moments of the two shock-structure runs
(Mach 2 and 3, E_l = 0.3, Nx = 2048, Q = 48) after 2000 and after the full 20000 steps.

The GPU tests compare the long FP64 and FP32 runs with these.  Calls only oracle/ (and the
seeded inputs of workloads/).  About four minutes per run on 8 host threads.  Run from the
repository root:  python tests/golden/make_c2_converged.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle.run import solver_from_workload  # noqa: E402
import workloads  # noqa: E402

CHECKPOINTS = (2000, 20000)


def main():
    oracle.set_threads(min(8, os.cpu_count() or 1))
    out = {}
    for mach in (2, 3):
        w = workloads.config2(mach)
        o = solver_from_workload(w)
        done = 0
        for cp in CHECKPOINTS:
            t0 = time.time()
            o.step(cp - done)
            done = cp
            n, u, T, q, pxx = o.moments()
            out[f"M{mach}_s{cp}"] = np.stack([n, u, T, q, pxx])
            print(f"Mach {mach}: step {cp} in {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "c2_converged.npz"), **out)


if __name__ == "__main__":
    main()
