"""Shared helpers of the parity tests: run a workload through the HIP library and through
the oracle, and compare."""
import sys

import numpy as np

import oracle
from oracle.run import solver_from_workload


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b, floor=0.0):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den = max(np.linalg.norm(b), floor * np.sqrt(b.size))
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def gpu_solver(w, precision, n_herm=0, moment_fixup=0):
    import paper_2211_16933_amd as elb
    s = elb.Solver(elb.params_from_workload(w, precision=precision, n_herm=n_herm,
                                            moment_fixup=moment_fixup))
    s.set_state_moments(w["n"], w["u"], w["T"])
    return s


def oracle_solver(w, nh=None):
    return solver_from_workload(w, nh=nh)


def field_errors(gm, om, n_scale=1.0, T_scale=1.0):
    """Relative L2 of (n, u, T, q, Pxx); u and q are measured against floors set by the
    scale of the flow (sound speed and n T^{3/2}) so near-zero fields stay meaningful."""
    n, u, T, q, pxx = om
    cs = np.sqrt(np.mean(T))
    return {"n": rel_l2(gm[0], n), "u": rel_l2(gm[1], u, floor=1e-3 * cs),
            "T": rel_l2(gm[2], T), "q": rel_l2(gm[3], q, floor=1e-3 * np.mean(n) * cs ** 3),
            "pxx": rel_l2(gm[4], pxx)}
