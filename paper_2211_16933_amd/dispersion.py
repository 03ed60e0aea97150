"""Sound-wave dispersion from batched GPU runs: the speed of sound and the damping rates of
small periodic waves over a range of denseness (the comparison of Sec. IV.A).

Host driver and analysis.  The waves run in one libelb batch; at regular times the library
projects the density of every instance on the shape of its initial perturbation (sin or
cos of k x; the paper projects on cos; elb_batch_get_amplitudes), and this module fits the
linear modes of a small perturbation of a uniform state:
    A(t) = c_t e^{-a_t t} + e^{-a_a t} (c_c cos w t + c_s sin w t)
(thermal mode a_t, acoustic pair with damping a_a and frequency w = c_s k).  For a start at
rest with uniform temperature the linearised solution has c_s = 0, c_c = P_n / c_s^2 and
c_t = 1 - c_c (the paper's solution of the density amplitude, Sec. IV.A).
"""
import math

import numpy as np

from . import binding as B


def run(workloads, periods=4.0, samples=300, omega_guess=None, precision=B.FP64,
        device="cuda:0"):
    """Run the sound waves (periodic workloads on [0, L), initial sin or cos profile of
    amplitude w['amplitude'], w['phase']) together for `periods` acoustic periods of the
    slowest wave and return per instance (t, A(t)) with A normalised by the initial
    amplitude.  omega_guess: expected angular frequency of each wave (sets the duration)."""
    params = [B.params_from_workload(w, precision=precision) for w in workloads]
    batch = B.BatchSolver(params, device=device)
    for i, w in enumerate(workloads):
        batch.set_state_moments(i, w["n"], w["u"], w["T"])
    dts = [B.derived(p)["dt"] for p in params]
    omega = omega_guess or [2.0 * math.pi * math.sqrt(5.0 / 3.0) / w["length"] for w in workloads]
    t_end = max(periods * 2.0 * math.pi / o for o in omega)
    nsteps = max(int(t_end / dt) for dt in dts)
    every = max(1, nsteps // samples)
    series = [([], []) for _ in workloads]
    for s in range(0, nsteps + 1, every):
        for i, w in enumerate(workloads):
            a_sin, a_cos = batch.amplitudes(i, 2.0 * math.pi / w["length"])
            series[i][0].append(s * dts[i])
            series[i][1].append((a_cos if w.get("phase") == "cos" else a_sin) / w["amplitude"])
        batch.step(every)
    batch.close()
    return [(np.array(t), np.array(a)) for t, a in series]


def fit(t, amp, guess):
    """Least-squares fit of the three-mode model; guess = (a_t, a_a, w).  Returns
    (a_t, a_a, w, c_t, c_c, c_s)."""
    from scipy.optimize import curve_fit

    def model(tt, a_t, a_a, om, ct, cc, cs):
        return ct * np.exp(-a_t * tt) + np.exp(-a_a * tt) * (cc * np.cos(om * tt) + cs * np.sin(om * tt))

    p0 = [guess[0], guess[1], guess[2], 0.3, 0.7, 0.0]
    popt, _ = curve_fit(model, t, amp, p0=p0, maxfev=50000)
    return popt
