"""Physics pins of the oracle run as a whole solver (CPU): the hydrodynamic limit of small
sound waves and the Rankine-Hugoniot structure of a converged dense-gas shock."""
import math

import numpy as np
import pytest
from scipy.optimize import curve_fit

from oracle import physics
from oracle.run import solver_from_workload
import workloads


def _fit_sound(El, kn, nx=64, q=8, periods=4):
    """Run a small periodic wave and fit the density amplitude with
    c_t e^{-a_t t} + e^{-a_a t}(c_c cos w t + c_s sin w t)."""
    amp = 1e-4
    w = workloads.sound_wave(nx=nx, q=q, denseness=El, kn=kn, amplitude=amp, pr_mode="enskog")
    s = solver_from_workload(w)
    k = 2 * math.pi
    at, aa, as_ = physics.linear_modes(1.0, 1.0, s.units["b"], s.units["mu_ref"], k)
    x = workloads.cell_centres(nx, 1.0)
    nsteps = int(periods * 2 * math.pi / as_ / s.dt)
    every = max(1, nsteps // 400)
    ts, amps = [], []
    for i in range(0, nsteps, every):
        n = s.moments()[0]
        ts.append(i * s.dt)
        amps.append(physics.sin_amplitude(n, x, k) / amp)
        s.step(every)

    def model(t, a_t, a_a, om, ct, cc, cs):
        return ct * np.exp(-a_t * t) + np.exp(-a_a * t) * (cc * np.cos(om * t) + cs * np.sin(om * t))

    popt, _ = curve_fit(model, np.array(ts), np.array(amps), p0=[at, aa, as_, 0.3, 0.7, 0.0],
                        maxfev=20000)
    return popt, (at, aa, as_), s.units


def test_sound_dilute_limit():
    """b = 0: speed, acoustic and thermal damping match the linearised Navier-Stokes-Fourier
    modes of a monatomic gas with Pr = 2/3 within 1 %."""
    popt, (at, aa, as_), _ = _fit_sound(0.0, 0.01)
    assert popt[2] == pytest.approx(as_, rel=2e-3)
    assert popt[1] == pytest.approx(aa, rel=1e-2)
    assert popt[0] == pytest.approx(at, rel=1e-2)


@pytest.mark.parametrize("El,q", [(0.3, 8), (0.5, 12)])
def test_sound_speed_dense(El, q):
    """The speed of sound follows the dense-gas c_s^2 = d_rho P + P d_T P/(rho^2 c_V)
    (eq. sw_cs) within 0.5 %; damping stays within 15 % of the Enskog hydrodynamic modes
    (the model's damping departs from them as the denseness grows, as the paper reports)."""
    popt, (at, aa, as_), u = _fit_sound(El, 0.01, q=q)
    cs = math.sqrt(physics.cs2(1.0, 1.0, u["b"]))
    assert popt[2] / (2 * math.pi) == pytest.approx(cs, rel=5e-3)
    assert popt[1] == pytest.approx(aa, rel=0.15)
    assert popt[0] == pytest.approx(at, rel=0.15)


def test_sound_damping_error_grows_with_denseness():
    errs = []
    for El in (0.0, 0.1, 0.3):
        popt, (at, aa, as_), _ = _fit_sound(El, 0.01)
        errs.append(abs(popt[1] / aa - 1.0))
    assert errs[0] < errs[1] < errs[2]


@pytest.mark.parametrize("M,q", [(1.5, 16), (2.0, 24)])
def test_converged_dense_shock_fluxes(M, q):
    """A standing dense-gas shock (E_l = 0.3, Kn = 1, 256 cells over 40 mean free paths)
    converges to uniform fluxes of mass n u, momentum n u^2 + P_xx + b n^2 chi T and energy
    sum p (p^2 phi + theta)/2 + u b n^2 chi T (the non-ideal parts are the collisional
    transfer carried by J1), with plateaus at the Rankine-Hugoniot states."""
    El = 0.3
    st = physics.shock_states(M, El)
    table = {"states": {f"M{M:g}_El{El:g}": st}}
    w = workloads.shock_structure(M, seed=7, nx=256, q=q, denseness=El, table=table)
    s = solver_from_workload(w)
    s.step(8000)
    n, u, T, qx, pxx = s.moments()
    b = s.par.b
    y = b * n * physics.chi_set(0.25 * b * n)
    p = s.p
    mass = n * u
    mom = n * u * u + pxx + y * n * T
    ef = np.einsum("k,ik->i", p, 0.5 * (p * p * s.phi[3:-3] + s.theta[3:-3])) + u * y * n * T

    def spread(a):
        return (a.max() - a.min()) / abs(a.mean())

    assert spread(mass) < 1e-3 and spread(mom) < 1e-3 and spread(ef) < 1e-3
    assert n[0] == pytest.approx(st["n1"], rel=1e-4) and n[-1] == pytest.approx(st["n2"], rel=1e-3)
    assert T[-1] == pytest.approx(st["T2"], rel=1e-3)
