"""chi_RET-FM (Sec. II.A, eq. chi_ret) on the GPU against the oracle (needs an MI355X):
the ball average of the density feeds chi, tau, Pr and the J1 source of every cell."""
import numpy as np
import pytest

from oracle import physics
import workloads
from helpers import say, rel_l2, gpu_solver, oracle_solver, field_errors

pytestmark = pytest.mark.gpu

FP64, FP32, FP32_MIXED = 0, 1, 2
TOL64, TOL32 = 1e-12, 1e-5


def ret_wave(nx, ratio, El=0.4, q=16, amplitude=2e-2):
    """Periodic wave on [0, 1) with sigma = ratio * dx."""
    sigma = ratio / nx
    w = workloads.sound_wave(nx=nx, q=q, denseness=El, kn=sigma / El, amplitude=amplitude,
                             pr_mode="enskog", name=f"ret_wave_nx{nx}_S{ratio:g}")
    w["chi"] = "ret"
    return w


def ret_sod(nx=160, q=32, sigma=1.0, eta_i=0.05):
    """Sod tube of Sec. IV.B (L = 80) at molecular diameter sigma (sigma / dx = 2 here)."""
    El = physics.denseness(eta_i)
    w = workloads.sod_tube(El, sigma / El, nx=nx, q=q, name=f"ret_sod_nx{nx}_q{q}")
    w["chi"] = "ret"
    return w


def _spread(w, steps):
    a, b = oracle_solver(w), oracle_solver(w)
    rng = np.random.default_rng(0)
    b.phi[3:-3] *= 1 + 1e-16 * rng.standard_normal(b.phi[3:-3].shape)
    b.theta[3:-3] *= 1 + 1e-16 * rng.standard_normal(b.theta[3:-3].shape)
    a.step(steps)
    b.step(steps)
    return a, field_errors(b.moments(), a.moments())


CASES = [("wave_S5.5_ragged", lambda: ret_wave(101, 5.5), 300),
         ("wave_S40", lambda: ret_wave(256, 40.0), 100),
         ("wave_S0.4", lambda: ret_wave(64, 0.4), 300),
         ("sod_S2", lambda: ret_sod(), 200)]


@pytest.mark.parametrize("name,make,steps", CASES, ids=[c[0] for c in CASES])
def test_ret_parity_fp64(name, make, steps):
    w = make()
    say(f"case {w['name']} steps={steps} precision=FP64 chi=ret")
    o, spread = _spread(w, steps)
    g = gpu_solver(w, FP64)
    g.step(steps)
    err = field_errors(g.moments(), o.moments())
    say("  errors", {k: f"{v:.2e}" for k, v in err.items()},
        "spread", {k: f"{v:.2e}" for k, v in spread.items()})
    for f in ("n", "u", "T", "q", "pxx"):
        assert err[f] <= max(TOL64, 100 * spread[f]), (f, err, spread)
    phi, th = g.dist()
    assert rel_l2(phi, o.phi[3:-3]) <= max(TOL64, 100 * spread["n"])


@pytest.mark.parametrize("precision", [FP32, FP32_MIXED, 3])
@pytest.mark.parametrize("name,make,steps", CASES[:1] + CASES[3:], ids=["wave", "sod"])
def test_ret_parity_fp32(name, make, steps, precision):
    """FP32, FP32 with bookkeeping, and (3) the latter with the moment fix-up."""
    w = make()
    say(f"case {w['name']} steps={steps} precision={precision} chi=ret")
    o = oracle_solver(w)
    o.step(steps)
    g = gpu_solver(w, FP32_MIXED, moment_fixup=1) if precision == 3 else gpu_solver(w, precision)
    g.step(steps)
    err = field_errors(g.moments(), o.moments())
    say("  errors", {k: f"{v:.2e}" for k, v in err.items()})
    for f in ("n", "u", "T"):
        assert err[f] <= TOL32, (f, err)


def test_ret_conserves_mass_and_differs_from_set():
    w = ret_wave(101, 5.5)
    g = gpu_solver(w, FP64)
    c0 = g.conserved()
    g.step(300)
    c1 = g.conserved()
    assert abs(c1[0] - c0[0]) <= 1e-12 * abs(c0[0])
    w_set = dict(w)
    w_set["chi"] = "set"
    s = gpu_solver(w_set, FP64)
    s.step(300)
    d = rel_l2(g.moments()[0] - 1.0, s.moments()[0] - 1.0)
    say(f"  RET vs SET density deviation: {d:.2e}")
    assert d > 1e-4


def test_ret_dilute_gas_equals_set_bitwise():
    """b = 0: chi = 1 and ln chi = 0 in both modes, so the runs agree bit for bit."""
    w = workloads.sound_wave(nx=64, q=16, denseness=0.0, kn=0.1, amplitude=1e-2,
                             pr_mode="enskog")
    a = gpu_solver(dict(w, chi="ret"), FP64)
    b = gpu_solver(w, FP64)
    a.step(100)
    b.step(100)
    pa, ta = a.dist()
    pb, tb = b.dist()
    assert np.array_equal(pa, pb) and np.array_equal(ta, tb)
