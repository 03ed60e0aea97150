"""The Sod problem of Sec. IV.B on the GPU (needs an MI355X): parity with the oracle on a
coarse tube, and a near-inviscid run against the oracle's exact dense-gas Riemann solution
(the comparison of Fig. 7, where the kinetic profile overlaps the inviscid one as the
molecular diameter goes to zero)."""
import time

import numpy as np
import pytest

from oracle import physics
import workloads
from helpers import say, gpu_solver, oracle_solver, field_errors

pytestmark = pytest.mark.gpu

FP64, FP32, FP32_MIXED = 0, 1, 2
ETA_I = 0.05


def sod(sigma, nx, q=8):
    """Sod tube at eta_i = 0.05 with molecular diameter sigma: E_l from eta_i and the mean
    free path l = sigma / E_l as the Knudsen number on unit length."""
    El = physics.denseness(ETA_I)
    return workloads.sod_tube(El, sigma / El, nx=nx, q=q, name=f"sod_sigma{sigma:g}_nx{nx}")


def inviscid_errors(w, moments, t):
    n, u, T = moments[:3]
    b = physics.units(w["denseness"], w["kn"])["b"]
    r = physics.riemann(1.0, 1.0, 0.125, 1.0, b)
    L = w["length"]
    dx = L / w["nx"]
    x = (np.arange(w["nx"]) + 0.5) * dx
    ex = np.array([r["sample"]((xx - 0.5 * L) / t) for xx in x])
    l1 = {k: float(np.mean(np.abs(a - ex[:, j]))) for j, (k, a) in enumerate((("n", n), ("u", u), ("T", T)))}
    plateaus = []
    for xi in (0.5 * (r["xi_tail"] + r["uc"]), 0.5 * (r["uc"] + r["xi_shock"])):
        i = int((0.5 * L + xi * t) / dx)
        e = r["sample"](xi)
        plateaus.append(max(abs(n[i] / e[0] - 1), abs(u[i] / e[1] - 1), abs(T[i] / e[2] - 1)))
    # shock position: the last cell whose density exceeds the mean of n2 and n_R
    half = 0.5 * (r["n2"] + 0.125)
    i_s = int(np.flatnonzero(n > half)[-1])
    shock_shift = (x[i_s] + 0.5 * dx - (0.5 * L + r["xi_shock"] * t)) / dx
    return l1, plateaus, shock_shift


def test_sod_parity_fp64():
    """Coarse tube (sigma = 0.01, Nx = 800, Q = 8) to t ~ 2.4: GPU FP64 against the oracle
    to 1e-12 relative L2, or 100x the oracle's own spread under a 1e-16 perturbation of its
    start if the step start amplifies round-off more than that."""
    w = sod(0.01, 800)
    steps = 200
    say(f"case {w['name']} steps={steps} precision=FP64")
    a, b = oracle_solver(w), oracle_solver(w)
    rng = np.random.default_rng(0)
    b.phi[3:-3] *= 1 + 1e-16 * rng.standard_normal(b.phi[3:-3].shape)
    b.theta[3:-3] *= 1 + 1e-16 * rng.standard_normal(b.theta[3:-3].shape)
    a.step(steps)
    b.step(steps)
    spread = field_errors(b.moments(), a.moments())
    g = gpu_solver(w, FP64)
    g.step(steps)
    err = field_errors(g.moments(), a.moments())
    say("  errors", {k: f"{v:.2e}" for k, v in err.items()},
        "spread", {k: f"{v:.2e}" for k, v in spread.items()})
    for f in ("n", "u", "T", "q", "pxx"):
        assert err[f] <= max(1e-12, 100 * spread[f]), (f, err, spread)


@pytest.mark.parametrize("precision", [FP64, FP32_MIXED])
def test_sod_near_inviscid(precision):
    """sigma = 1e-4 on Nx = 80000 cells of L = 80 (dx = 1e-3, the paper's resolution for
    Fig. 7), Q = 8, to t = 10: the profile matches the exact inviscid solution: L1 errors
    of a few 1e-4, the plateaus to 3e-4 and the shock within 3 cells."""
    w = sod(1e-4, 80000)
    g = gpu_solver(w, precision)
    dt = g.info["dt"]
    steps = int(round(10.0 / dt))
    say(f"case {w['name']} steps={steps} precision={precision}")
    t0 = time.time()
    g.step(steps)
    m = g.moments()
    say(f"  {steps} steps in {time.time() - t0:.1f} s")
    l1, plateaus, shift = inviscid_errors(w, m, steps * dt)
    say("  L1", {k: f"{v:.2e}" for k, v in l1.items()}, "plateaus",
        [f"{p:.2e}" for p in plateaus], f"shock shift {shift:+.2f} cells")
    assert l1["n"] < 1e-3 and l1["u"] < 1e-3 and l1["T"] < 2e-3
    assert max(plateaus) < 3e-4
    assert abs(shift) <= 3.0


@pytest.mark.parametrize("eta_i", [0.05, 0.15, 0.25])
def test_sod_dense_plateaus(eta_i):
    """The denseness series of the paper's shock runs (Sec. IV.B, Fig. 4: sigma = 0.01,
    eta_i = 0.05, 0.15, 0.25, L = 80, Nx = 800, Q = 8, dt = 1e-3, chi_RET-FM), to t = 9 in
    FP64: both plateaus within 5e-3 of the exact dense-gas Riemann solution.  The dense
    solutions differ from the ideal-gas one far more than that (P_c 0.348, 0.427, 0.530
    against 0.317)."""
    El = physics.denseness(eta_i)
    w = workloads.sod_tube(El, 0.01 / El, nx=800, q=8, name=f"sod_dense_eta{eta_i:g}")
    w["chi"], w["dt"] = "ret", 1e-3
    g = gpu_solver(w, FP64)
    say(f"case {w['name']} steps=9000 FP64 chi=ret")
    g.step(9000)
    l1, plateaus, shift = inviscid_errors(w, g.moments(), 9.0)
    b = physics.units(w["denseness"], w["kn"])["b"]
    dense, ideal = physics.riemann(1.0, 1.0, 0.125, 1.0, b), physics.riemann(1.0, 1.0, 0.125, 1.0, 0.0)
    say("  L1", {k: f"{v:.2e}" for k, v in l1.items()}, "plateaus", [f"{p:.2e}" for p in plateaus],
        f"shock shift {shift:+.2f} cells; P_c dense {dense['Pc']:.4f} ideal {ideal['Pc']:.4f}")
    assert max(plateaus) < 5e-3
    if eta_i >= 0.15:
        assert abs(dense["Pc"] / ideal["Pc"] - 1.0) > 0.3
    assert abs(shift) <= 3.0
