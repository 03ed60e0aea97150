"""Large velocity sets (Sec. IV.B, near-ballistic regime) on the GPU (needs an MI355X): the
Sod tube at molecular diameter sigma = 1 (eta_i = 0.05, L = 80, Nx = 160, dt = 1e-3,
chi_RET-FM), where the paper needs Q = 200 for smooth profiles.  Parity with the oracle at
Q = 200, and the profiles at Q = 8, 40, 200 converging with Q."""
import numpy as np
import pytest

from oracle import physics
import workloads
from helpers import say, rel_l2, gpu_solver, oracle_solver, field_errors

pytestmark = pytest.mark.gpu

FP64, FP32, FP32_MIXED = 0, 1, 2


def ballistic_sod(q, nx=160):
    El = physics.denseness(0.05)
    w = workloads.sod_tube(El, 1.0 / El, nx=nx, q=q, name=f"ballistic_sod_q{q}")
    w["chi"] = "ret"
    w["dt"] = 1e-3
    return w


def test_q200_parity():
    w = ballistic_sod(200)
    steps = 300
    say(f"case {w['name']} steps={steps} FP64 and FP32_MIXED")
    a, b = oracle_solver(w), oracle_solver(w)
    rng = np.random.default_rng(0)
    b.phi[3:-3] *= 1 + 1e-16 * rng.standard_normal(b.phi[3:-3].shape)
    b.theta[3:-3] *= 1 + 1e-16 * rng.standard_normal(b.theta[3:-3].shape)
    a.step(steps)
    b.step(steps)
    om = a.moments()
    spread = field_errors(b.moments(), om)
    g = gpu_solver(w, FP64)
    g.step(steps)
    err = field_errors(g.moments(), om)
    say("  FP64 errors", {k: f"{v:.2e}" for k, v in err.items()},
        "spread", {k: f"{v:.2e}" for k, v in spread.items()})
    for f in ("n", "u", "T", "q", "pxx"):
        assert err[f] <= max(1e-12, 100 * spread[f]), (f, err, spread)
    phi, th = g.dist()
    assert rel_l2(phi, a.phi[3:-3]) <= max(1e-12, 100 * spread["n"])
    m = gpu_solver(w, FP32_MIXED)
    m.step(steps)
    err32 = field_errors(m.moments(), om)
    say("  FP32_MIXED errors", {k: f"{v:.2e}" for k, v in err32.items()})
    for f in ("n", "u", "T"):
        assert err32[f] <= 1e-5, (f, err32)


def roughness(v):
    """Sum of the absolute second differences: the kinks of a staircase profile."""
    return float(np.sum(np.abs(np.diff(v, 2))))


def test_profiles_converge_with_q():
    """At t = 9 the Q = 8 profile is a staircase of free-streaming fronts: Q = 40 is much
    closer to Q = 200 than Q = 8 is, and the roughness of n, u and T falls as Q grows (the
    oracle gives 0.196, 0.121, 0.055 for n at Q = 8, 40, 200)."""
    steps = 9000
    prof = {}
    for q in (8, 40, 200):
        w = ballistic_sod(q)
        say(f"case {w['name']} steps={steps} FP64")
        g = gpu_solver(w, FP64)
        g.step(steps)
        n, u, T, _, _ = g.moments()
        prof[q] = (n, u, T)
        c1 = g.conserved()
        # the flux through the fixed end states moves mass, so only finiteness is checked
        assert np.all(np.isfinite(c1)) and np.all(n > 0) and np.all(T > 0)
    d8 = [float(np.mean(np.abs(prof[8][j] - prof[200][j]))) for j in range(3)]
    d40 = [float(np.mean(np.abs(prof[40][j] - prof[200][j]))) for j in range(3)]
    rough = {q: [roughness(v) for v in prof[q]] for q in prof}
    say("  L1 to Q=200 (n, u, T): Q=8", [f"{v:.2e}" for v in d8], "Q=40",
        [f"{v:.2e}" for v in d40], "roughness", {q: [f"{v:.3f}" for v in r] for q, r in rough.items()})
    for a, b in zip(d40, d8):
        assert a < b / 3
    for j in range(3):
        assert rough[8][j] > 1.25 * rough[40][j] > 1.25 ** 2 * rough[200][j]


@pytest.mark.parametrize("eta_i,nx", [(0.05, 400), (0.25, 200)])
def test_initial_shock_structure_setup_parity(eta_i, nx):
    """The set-up of the paper's early-time shock structure (Sec. IV.B, Fig. 6): sigma = 1,
    L = 10, Q = 200, chi_RET-FM with sigma / dx = 40 or 20, to t = 0.2 in FP64 against the
    oracle (1e-12, or 100x the oracle's own spread under a 1e-16 perturbation)."""
    El = physics.denseness(eta_i)
    w = workloads.sod_tube(El, 1.0 / El, nx=nx, q=200, length=10.0,
                           name=f"shock_structure_eta{eta_i:g}_nx{nx}_q200")
    w["chi"] = "ret"
    a = oracle_solver(w)
    steps = int(round(0.2 / a.dt))
    say(f"case {w['name']} steps={steps} FP64")
    b = oracle_solver(w)
    rng = np.random.default_rng(0)
    b.phi[3:-3] *= 1 + 1e-16 * rng.standard_normal(b.phi[3:-3].shape)
    b.theta[3:-3] *= 1 + 1e-16 * rng.standard_normal(b.theta[3:-3].shape)
    a.step(steps)
    b.step(steps)
    om = a.moments()
    spread = field_errors(b.moments(), om)
    g = gpu_solver(w, FP64)
    g.step(steps)
    err = field_errors(g.moments(), om)
    say("  errors", {k: f"{v:.2e}" for k, v in err.items()},
        "spread", {k: f"{v:.2e}" for k, v in spread.items()})
    for f in ("n", "u", "T", "q", "pxx"):
        assert err[f] <= max(1e-12, 100 * spread[f]), (f, err, spread)
