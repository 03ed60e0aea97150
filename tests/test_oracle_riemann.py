"""Pins of the oracle's dense-gas Riemann solver (Sec. IV.B, inviscid limit) against
results fixed independently of it:
  - b -> 0: the closed-form Riemann solution of an ideal monatomic gas (gamma = 5/3), with
    the textbook pressure function of a rarefaction and a shock;
  - the fan lies on one isentrope, whose invariant has a closed form for P = n T Z(n) with
    e = 3T/2 (not the ODE in c_s^2 that the solver integrates);
  - the shock, seen in its own frame, is the standing shock of the separate Newton solver
    of the jump conditions;
  - the self-similar solution conserves mass and energy and gains momentum at the rate
    P_L - P_R, integrated numerically over xi.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

from oracle import physics

GAMMA = 5.0 / 3.0


def ideal_riemann(rl, pl, rr, pr):
    """Closed-form ideal-gas Riemann solution (left rarefaction, right shock), both sides at
    rest: returns (p*, u*, rho*L, rho*R, S_shock, sample(xi) -> (rho, u, p))."""
    g = GAMMA
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)

    def f_raref(p):
        return 2.0 * cl / (g - 1.0) * ((p / pl) ** ((g - 1.0) / (2.0 * g)) - 1.0)

    def f_shock(p):
        A, Bk = 2.0 / ((g + 1.0) * rr), (g - 1.0) / (g + 1.0) * pr
        return (p - pr) * math.sqrt(A / (p + Bk))

    ps = brentq(lambda p: f_raref(p) + f_shock(p), pr, pl, xtol=1e-16, rtol=1e-15)
    us = 0.5 * (f_shock(ps) - f_raref(ps))
    rsl = rl * (ps / pl) ** (1.0 / g)
    m = (g - 1.0) / (g + 1.0)
    rsr = rr * (ps / pr + m) / (m * ps / pr + 1.0)
    S = cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
    cs_star = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))

    def sample(xi):
        if xi <= -cl:
            return rl, 0.0, pl
        if xi < us - cs_star:
            c = 2.0 / (g + 1.0) * (cl - 0.5 * (g - 1.0) * xi)
            u = 2.0 / (g + 1.0) * (cl + xi)
            return rl * (c / cl) ** (2.0 / (g - 1.0)), u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
        if xi < us:
            return rsl, us, ps
        if xi < S:
            return rsr, us, ps
        return rr, 0.0, pr

    return ps, us, rsl, rsr, S, sample


def sod(eta_i):
    """Sod initial state of Sec. IV.B: eta_R = eta_L / 8, T = 1 on both sides; n_L = 1 so
    that b = 4 eta_i."""
    return 1.0, 1.0, 0.125, 1.0, 4.0 * eta_i


def test_dilute_limit_matches_ideal_closed_form():
    nL, TL, nR, TR, _ = sod(0.05)
    r = physics.riemann(nL, TL, nR, TR, 0.0)
    ps, us, rsl, rsr, S, sample = ideal_riemann(nL, nL * TL, nR, nR * TR)
    assert abs(r["Pc"] / ps - 1.0) < 1e-11
    assert abs(r["uc"] / us - 1.0) < 1e-11
    assert abs(r["n1"] / rsl - 1.0) < 1e-11
    assert abs(r["n2"] / rsr - 1.0) < 1e-11
    assert abs(r["xi_shock"] / S - 1.0) < 1e-11
    for xi in np.linspace(-2.5, 2.5, 41):
        n, u, T = r["sample"](xi)
        rho, ue, p = sample(xi)
        assert abs(n - rho) < 1e-10 and abs(u - ue) < 1e-10 and abs(n * T - p) < 1e-10, xi


@pytest.mark.parametrize("eta_i", [0.05, 0.15, 0.25])
def test_fan_is_one_isentrope(eta_i):
    nL, TL, nR, TR, b = sod(eta_i)
    r = physics.riemann(nL, TL, nR, TR, b)
    s0 = physics.isentrope_invariant(nL, TL, b)
    for xi in np.linspace(r["xi_head"], r["xi_tail"], 12):
        n, u, T = r["sample"](xi)
        assert abs(physics.isentrope_invariant(n, T, b) - s0) < 1e-10, xi
        # inside the fan the flow leaves with u - c_s = xi
        assert abs(u - math.sqrt(physics.cs2(n, T, b)) - xi) < 1e-10
    assert abs(physics.isentrope_invariant(r["n1"], r["T1"], b) - s0) < 1e-10


@pytest.mark.parametrize("eta_i", [0.05, 0.15, 0.25])
def test_shock_is_the_standing_shock_in_its_frame(eta_i):
    nL, TL, nR, TR, b = sod(eta_i)
    r = physics.riemann(nL, TL, nR, TR, b)
    # in the frame moving with xi_s, the gas ahead enters at speed xi_s
    n2, u2, T2 = physics.rankine_hugoniot(nR, TR, r["xi_shock"], b)
    assert abs(n2 / r["n2"] - 1.0) < 1e-9
    assert abs(T2 / r["T2"] - 1.0) < 1e-9
    assert abs((r["xi_shock"] - u2) / r["uc"] - 1.0) < 1e-9
    # the contact: equal pressure and velocity on its two sides
    assert abs(physics.pressure(r["n1"], r["T1"], b) / r["Pc"] - 1.0) < 1e-12
    assert abs(physics.pressure(r["n2"], r["T2"], b) / r["Pc"] - 1.0) < 1e-12
    assert abs(r["uc"] - r["uc_shock"]) < 1e-11


@pytest.mark.parametrize("eta_i", [0.0, 0.05, 0.25])
def test_global_balance_of_the_similarity_solution(eta_i):
    nL, TL, nR, TR, b = sod(eta_i)
    r = physics.riemann(nL, TL, nR, TR, b)
    f = r["sample"]
    lo, hi = r["xi_head"] - 0.5, r["xi_shock"] + 0.5
    pts = [r["xi_head"], r["xi_tail"], 0.0, r["uc"], r["xi_shock"]]
    EL, ER = 1.5 * nL * TL, 1.5 * nR * TR

    def integral(g):
        return quad(g, lo, hi, points=pts, limit=200, epsabs=1e-13, epsrel=1e-12)[0]

    mass = integral(lambda x: f(x)[0] - (nL if x < 0 else nR))
    mom = integral(lambda x: f(x)[0] * f(x)[1])
    energy = integral(lambda x: 1.5 * f(x)[0] * f(x)[2] + 0.5 * f(x)[0] * f(x)[1] ** 2
                      - (EL if x < 0 else ER))
    PL, PR = physics.pressure(nL, TL, b), physics.pressure(nR, TR, b)
    assert abs(mass) < 1e-9
    assert abs(mom - (PL - PR)) < 1e-9
    assert abs(energy) < 1e-9


def test_rejects_a_tube_without_a_pressure_drop():
    with pytest.raises(ValueError):
        physics.riemann(0.125, 1.0, 1.0, 1.0, 0.2)


# ---------------------------------------------------------------------------------------
# the kinetic oracle approaches the inviscid solution as sigma -> 0 (Sec. IV.B, Fig. 5)
# ---------------------------------------------------------------------------------------
def kinetic_sod(sigma, nx, eta_i=0.05, t_end=10.0):
    import workloads
    from oracle.run import solver_from_workload
    El = physics.denseness(eta_i)
    w = workloads.sod_tube(El, sigma / El, nx=nx, q=8)
    s = solver_from_workload(w)
    steps = int(round(t_end / s.dt))
    s.step(steps)
    t = steps * s.dt
    n, u, T, _, _ = s.moments()
    r = physics.riemann(1.0, 1.0, 0.125, 1.0, s.units["b"])
    x = (np.arange(nx) + 0.5) * w["length"] / nx
    ex = np.array([r["sample"]((xx - 0.5 * w["length"]) / t) for xx in x])
    l1 = [float(np.mean(np.abs(a - ex[:, j]))) for j, a in enumerate((n, u, T))]
    plateaus = []
    for xi in (0.5 * (r["xi_tail"] + r["uc"]), 0.5 * (r["uc"] + r["xi_shock"])):
        i = int((0.5 * w["length"] + xi * t) / (w["length"] / nx))
        e = r["sample"](xi)
        plateaus.append(max(abs(n[i] / e[0] - 1), abs(u[i] / e[1] - 1), abs(T[i] / e[2] - 1)))
    return l1, plateaus


def test_kinetic_sod_converges_to_the_inviscid_solution():
    coarse, pc = kinetic_sod(0.02, 400)
    fine, pf = kinetic_sod(0.01, 800)
    print("L1 (n, u, T):", coarse, fine, "plateaus:", pc, pf)
    # the contact spreads by diffusion (width ~ sqrt(t sigma)), the shock and the fan edges
    # by ~ sigma: halving sigma cuts the L1 error by a factor between sqrt 2 and 2
    for c, f in zip(coarse, fine):
        assert f < c / 1.35
    assert max(pf) < 4e-3 and max(pf) < max(pc)
    assert max(fine) < 0.02
