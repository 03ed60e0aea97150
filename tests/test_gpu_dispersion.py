"""Sound speed and damping of small waves over a range of denseness, from one batched GPU
run (needs an MI355X), against the dense-gas hydrodynamics of the oracle's physics module:
the speed of sound follows c_s^2 = T [Z + n Z' + (2/3) Z^2] (Sec. III.A), and the acoustic
damping approaches the linearised Navier-Stokes-Fourier value of the Enskog transport
coefficients, with departures that grow with the denseness (as Sec. III.A reports): the
speed to 0.5 % up to E_l = 1 (1.9 % at E_l = 2), the damping from 2 % to 22 %."""
import math

import numpy as np
import pytest

from oracle import physics
import workloads
from helpers import say

pytestmark = pytest.mark.gpu

DENSENESS = (0.0, 0.05, 0.1, 0.2, 0.3, 0.5, 1.0, 2.0)


def test_dispersion_over_denseness():
    from paper_2211_16933_amd import dispersion
    k = 2.0 * math.pi
    ws, modes, cs = [], [], []
    for El in DENSENESS:
        w = workloads.sound_wave(nx=64, q=8, denseness=El, kn=0.01, amplitude=1e-4,
                                 pr_mode="enskog", name=f"dispersion_El{El:g}")
        u = physics.units(El, 0.01)
        modes.append(physics.linear_modes(1.0, 1.0, u["b"], u["mu_ref"], k))
        cs.append(math.sqrt(physics.cs2(1.0, 1.0, u["b"])))
        ws.append(w)
    say(f"case dispersion: {len(ws)} waves, E_l {DENSENESS}")
    series = dispersion.run(ws, periods=4.0, omega_guess=[m[2] for m in modes])
    errs_c, errs_a = [], []
    for El, (t, a), m, c in zip(DENSENESS, series, modes, cs):
        popt = dispersion.fit(t, a, m)
        ec = popt[2] / k / c - 1.0
        ea = popt[1] / m[1] - 1.0
        et = popt[0] / m[0] - 1.0
        errs_c.append(ec)
        errs_a.append(ea)
        say(f"  E_l={El:4.2f}: c_s {popt[2] / k:.5f} (dense EOS {c:.5f}, {ec:+.2e}); "
            f"a_a {popt[1]:.4f} ({ea:+.2e}); a_t {popt[0]:.4f} ({et:+.2e})")
        assert abs(ec) <= (5e-3 if El <= 1.0 else 3e-2)
    # the dilute gas matches the Navier-Stokes-Fourier speed and damping closely; the
    # departures then grow with the denseness
    assert abs(errs_a[0]) <= 1e-2
    assert all(abs(b) >= abs(a) for a, b in zip(errs_c[1:], errs_c[2:]))
    assert all(abs(b) >= abs(a) for a, b in zip(errs_a, errs_a[1:]))
    assert all(abs(e) <= 0.3 for e in errs_a)
