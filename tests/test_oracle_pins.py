"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  Each pins one part of the oracle to something other
than the oracle itself: printed numbers, closed forms, library routines, invariants.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import physics
from oracle.run import solver_from_workload, rows_with_ghosts
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")
GOLDEN_VALUES = json.load(open(GOLD))


# --------------------------------------------------------------------------------------
# closures and units
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("pair", GOLDEN_VALUES["denseness_pairs"])
def test_denseness_printed_pairs(pair):
    """E_l = 6 sqrt(2) eta chi_SET(eta) reproduces every (eta, E_l) pair the paper prints."""
    el = physics.denseness(pair["eta"])
    assert round(el, pair["digits"]) == pytest.approx(pair["El"], abs=0.6 * 10 ** -pair["digits"])
    # and the C oracle's chi agrees with the Python closure
    assert oracle.chi(pair["eta"]) == pytest.approx(physics.chi_set(pair["eta"]), rel=1e-15)
    # inverse map
    assert physics.eta_from_denseness(el) == pytest.approx(pair["eta"], rel=1e-12)


@pytest.mark.parametrize("eta", [0.0, 0.01, 0.1, 0.3, 0.49])
def test_carnahan_starling_identity(eta):
    """chi_SET = (P^hs/(n k T) - 1)/(n b) with the Carnahan-Starling P^hs (eq. chi)."""
    z_cs = physics.compressibility_cs(eta)
    assert 1.0 + 4.0 * eta * oracle.chi(eta) == pytest.approx(z_cs, rel=1e-14, abs=1e-15)


@pytest.mark.parametrize("eta", [0.001, 0.05, 0.2, 0.45])
def test_dlnchi_chain_rule(eta):
    """d ln chi / d ln n against a central difference of ln chi_SET in ln eta."""
    h = 1e-5
    fd = (math.log(physics.chi_set(eta * math.exp(h))) -
          math.log(physics.chi_set(eta * math.exp(-h)))) / (2 * h)
    assert oracle.dlnchi_dlnn(eta) == pytest.approx(fd, rel=1e-8)


@pytest.mark.parametrize("y", [0.0, 1e-3, 0.5, 2.0, 10.0])
def test_prandtl_is_cp_mu_over_lambda(y):
    """Pr(b rho chi) (Sec. II.B) equals c_P mu / lambda built from the printed mu and
    lambda with lambda_ref/mu_ref = (75/64)/(5/16); its dilute limit is 2/3."""
    # choose n, b giving this y: n = 1, solve b n chi(bn/4) = y by bisection
    lo, hi = 0.0, 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid * physics.chi_set(0.25 * mid) < y:
            lo = mid
        else:
            hi = mid
    b = 0.5 * (lo + hi)
    mu = physics.viscosity(1.0, 1.3, b, 0.7)
    lam = physics.conductivity(1.0, 1.3, b, 0.7)
    assert oracle.prandtl_enskog(y) == pytest.approx(2.5 * mu / lam, rel=1e-12)
    if y == 0.0:
        assert oracle.prandtl_enskog(y) == 2.0 / 3.0


@pytest.mark.parametrize("n,T,El", [(1.0, 1.0, 0.1), (1.7, 0.6, 0.4), (0.3, 1.9, 0.02)])
def test_tau_is_mu_over_Pi(n, T, El):
    """The oracle's tau equals mu/(n T) with the printed mu (Sec. II.B)."""
    u = physics.units(El, 0.1)
    t = oracle.tau(u["mu_ref"], u["b"], n, T)
    assert t == pytest.approx(physics.viscosity(n, T, u["b"], u["mu_ref"]) / (n * T), rel=1e-14)


def test_tau_sigma_form_and_dilute_limit():
    """tau = sigma g[eta] with sigma = E_l l (eq. tau_sigma) reproduces the oracle's tau;
    in the dilute limit tau -> (5/16) sqrt(2 pi) l / sqrt(T) (hard-sphere relation)."""
    for El in (0.1, 0.4, 2.0):
        u = physics.units(El, 0.05)
        sigma = u["sigma"]
        eta = u["eta0"]
        y = 4 * eta * physics.chi_set(eta)
        g = 5 * math.sqrt(math.pi) / 24 * (1 / y + 0.8 + physics.C_MU * y)
        assert oracle.tau(u["mu_ref"], u["b"], 1.0, 1.0) == pytest.approx(sigma * g, rel=1e-13)
    u = physics.units(1e-9, 0.3)
    assert oracle.tau(u["mu_ref"], u["b"], 1.0, 2.0) == pytest.approx(
        5 / 16 * math.sqrt(2 * math.pi) * 0.3 / math.sqrt(2.0), rel=1e-7)


def test_config1_units():
    """E_l = 0.1 and Kn = 0.1 at n = 1: eta0, chi0 and tau0 of the sound-wave case."""
    u = physics.units(0.1, 0.1)
    assert physics.denseness(u["eta0"]) == pytest.approx(0.1, rel=1e-13)
    assert u["eta0"] == pytest.approx(0.0114505, rel=1e-5)
    assert oracle.tau(u["mu_ref"], u["b"], 1.0, 1.0) == pytest.approx(0.081420, rel=1e-4)


# --------------------------------------------------------------------------------------
# quadrature and Hermite equilibrium
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("Q", [7, 8, 12, 16, 20, 24, 32, 40, 48, 64, 96, 200])
def test_quadrature_matches_numpy_hermegauss(Q):
    p, w = oracle.quadrature(Q)
    pn, wn = np.polynomial.hermite_e.hermegauss(Q)
    wn = wn / math.sqrt(2 * math.pi)
    assert np.max(np.abs(p - pn)) < 1e-13 * max(1.0, np.max(np.abs(pn)))
    assert np.max(np.abs(w - wn) / wn) < 1e-12
    assert np.all(np.diff(p) > 0)


@pytest.mark.parametrize("Q", [7, 16, 20, 40, 48, 96])
def test_quadrature_exactness(Q):
    """sum_k w_k p_k^j = (j-1)!! for even j and 0 for odd j, up to j = 2Q - 1."""
    p, w = oracle.quadrature(Q)
    for j in range(0, 2 * Q):
        exact = 0.0 if j % 2 else float(np.prod(np.arange(j - 1, 0, -2, dtype=float))) if j else 1.0
        val = float(np.sum(w * p ** j))
        scale = float(np.sum(w * np.abs(p) ** j))
        assert abs(val - exact) <= 1e-12 * scale + 1e-300, (j, val, exact)


@pytest.mark.parametrize("Q", [8, 40, 96, 200])
def test_quadrature_orthonormality(Q):
    """Gauss exactness in a form that does not overflow at Q = 200 (p_max = 27, so p^(2Q-1)
    leaves FP64): the normalised Hermite polynomials h_l = He_l / sqrt(l!), l < Q, are
    orthonormal under the weight exp(-p^2/2)/sqrt(2 pi), and the rule is exact for every
    product h_l h_m (degree <= 2Q - 2), so sum_k w_k h_l(p_k) h_m(p_k) = delta_lm.  h_l comes
    from its own three-term recurrence h_{l+1} = (p h_l - sqrt(l) h_{l-1}) / sqrt(l+1), not
    from the oracle.  Also h_Q vanishes at every node (the nodes are the roots of He_Q)."""
    p, w = oracle.quadrature(Q)
    H = np.zeros((Q + 1, Q))
    H[0] = 1.0
    H[1] = p
    for l in range(1, Q):
        H[l + 1] = (p * H[l] - math.sqrt(l) * H[l - 1]) / math.sqrt(l + 1)
    gram = (H[:Q] * w) @ H[:Q].T
    assert np.max(np.abs(gram - np.eye(Q))) < 1e-12, np.max(np.abs(gram - np.eye(Q)))
    # |h_Q(p_k)| relative to the size of the terms of its recurrence at that node
    scale = np.abs(p * H[Q - 1]) + math.sqrt(Q - 1) * np.abs(H[Q - 2])
    assert np.max(np.abs(H[Q]) / scale) < 1e-12
    assert abs(np.sum(w) - 1.0) < 1e-14 and np.all(w > 0)


def _maxwellian_raw_moment(j, u, T):
    """E[p^j] for p ~ N(u, T): sum over even m of C(j, m) u^(j-m) T^(m/2) (m-1)!!."""
    s = 0.0
    for m in range(0, j + 1, 2):
        dfact = float(np.prod(np.arange(m - 1, 0, -2, dtype=float))) if m else 1.0
        s += math.comb(j, m) * u ** (j - m) * T ** (m / 2) * dfact
    return s


@pytest.mark.parametrize("Q", [8, 16, 48])
@pytest.mark.parametrize("u,T", [(0.0, 1.0), (0.3, 1.2), (-1.1, 0.5), (2.4, 0.42), (0.7, 1.8)])
def test_equilibrium_reproduces_maxwellian_moments(Q, u, T):
    """sum_k g_k p_k^j equals the Maxwellian moments for j <= N = Q - 1 (Sec. II.D)."""
    p, w = oracle.quadrature(Q)
    g = oracle.equilibrium(p, w, u, T)
    # every moment up to N holds in exact arithmetic; in FP64 the high ones are dominated by
    # rounding of the (tiny) outer-node values times p^j, so check j <= min(N, 12): up to 6
    # (the moments the model uses) tightly, the rest loosely
    for j in range(min(Q, 13)):
        exact = _maxwellian_raw_moment(j, u, T)
        val = float(np.sum(g * p ** j))
        scale = float(np.sum(np.abs(g) * np.abs(p) ** j)) + abs(exact)
        tol = 2e-13 if j <= 6 else 1e-11
        assert abs(val - exact) <= tol * scale, (j, val, exact)


@pytest.mark.parametrize("u,T", [(0.4, 1.3), (-0.8, 0.7)])
def test_equilibrium_coefficients_by_integration(u, T):
    """Independent route to the expansion: a_l = (1/l!) int He_l(p) N(p; u, T) dp computed by
    adaptive quadrature, then g_k = w_k sum_l He_l(p_k) a_l."""
    Q = 8
    p, w = oracle.quadrature(Q)
    g = oracle.equilibrium(p, w, u, T)
    a = []
    for l in range(Q):
        f = lambda x, l=l: (np.polynomial.hermite_e.hermeval(x, [0] * l + [1]) *
                            math.exp(-(x - u) ** 2 / (2 * T)) / math.sqrt(2 * math.pi * T))
        val, _ = integrate.quad(f, u - 30 * math.sqrt(T), u + 30 * math.sqrt(T),
                                epsabs=1e-15, epsrel=1e-13, limit=400)
        a.append(val / math.factorial(l))
    g_ref = np.array([w[k] * sum(np.polynomial.hermite_e.hermeval(p[k], [0] * l + [1]) * a[l]
                                 for l in range(Q)) for k in range(Q)])
    assert np.max(np.abs(g - g_ref)) < 1e-12


def test_equilibrium_lower_order_truncation():
    """With N < Q - 1 the expansion reproduces moments only up to N (order is honoured)."""
    Q, N = 16, 6
    p, w = oracle.quadrature(Q)
    g = oracle.equilibrium(p, w, 0.5, 1.4, nh=N)
    for j in range(N + 1):
        assert float(np.sum(g * p ** j)) == pytest.approx(_maxwellian_raw_moment(j, 0.5, 1.4),
                                                          rel=1e-12, abs=1e-13)
    assert abs(float(np.sum(g * p ** (N + 2))) - _maxwellian_raw_moment(N + 2, 0.5, 1.4)) > 1e-6


# --------------------------------------------------------------------------------------
# Shakhov target and Enskog source
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("Q", [16, 48])
def test_shakhov_target_moments(Q):
    """phi_S, theta_S carry n, n u, n T (= sum xi^2 phi_S), (3/2) n T and the heat flux
    (1 - Pr) q (Sec. II.C)."""
    p, w = oracle.quadrature(Q)
    n, u, T, qx, Pr = 1.3, 0.4, 1.1, 0.07, 0.61
    phS, thS, _, _ = oracle.cell_sources(p, w, n, u, T, qx, Pr, 0.0, 0, 0, 0, 0)
    xi = p - u
    assert phS.sum() == pytest.approx(n, rel=1e-14)
    assert (p * phS).sum() == pytest.approx(n * u, rel=1e-14)
    assert (xi ** 2 * phS).sum() == pytest.approx(n * T, rel=1e-13)
    e = 0.5 * xi ** 2 * phS + 0.5 * thS
    assert e.sum() == pytest.approx(1.5 * n * T, rel=1e-13)
    assert (xi * e).sum() == pytest.approx((1 - Pr) * qx, rel=1e-12)
    nn, uu, TT, qq, pxx = oracle.moments_row(p, phS, thS)
    assert (nn, uu, TT) == pytest.approx((n, u, T), rel=1e-13)
    assert qq == pytest.approx((1 - Pr) * qx, rel=1e-12)


@pytest.mark.parametrize("Q", [16, 48])
def test_enskog_source_moments(Q):
    """Moments of J1 (eq. j1_expanded with the common prefactor -b rho chi):
      mass 0; momentum -y n T (dlnchi + 2 dlnn + dlnT), the gradient of the non-ideal
      pressure b n^2 chi T; energy u * momentum - y n T du."""
    p, w = oracle.quadrature(Q)
    n, u, T, y = 1.2, -0.3, 0.9, 0.37
    dlnn, du, dlnT, dlnchi = 0.21, -0.13, 0.08, 0.05
    _, _, J1p, J1t = oracle.cell_sources(p, w, n, u, T, 0.0, 2 / 3, y, dlnn, du, dlnT, dlnchi)
    mom = -y * n * T * (dlnchi + 2 * dlnn + dlnT)
    assert abs(J1p.sum()) < 1e-15
    assert (p * J1p).sum() == pytest.approx(mom, rel=1e-13)
    en = (0.5 * p ** 2 * J1p + 0.5 * J1t).sum()
    assert en == pytest.approx(u * mom - y * n * T * du, rel=1e-13)


def test_enskog_source_matches_3d_reduction():
    """The reduced J1 brackets equal the 3-D J1(f_MB) (Sec. II.B) integrated over p_y, p_z,
    done here by 2-D Gauss-Hermite quadrature in the transverse momenta."""
    Q = 16
    p, w = oracle.quadrature(Q)
    n, u, T, y = 1.0, 0.2, 1.3, 0.5
    dlnn, du, dlnT, dlnchi = 0.3, 0.1, -0.2, 0.07
    g = oracle.equilibrium(p, w, u, T)
    _, _, J1p, J1t = oracle.cell_sources(p, w, n, u, T, 0.0, 2 / 3, y, dlnn, du, dlnT, dlnchi)
    zt, wt = np.polynomial.hermite_e.hermegauss(20)
    wt = wt / math.sqrt(2 * math.pi)
    for k in range(Q):
        xi_x = p[k] - u
        acc_phi = acc_th = 0.0
        for a in range(20):
            for c in range(20):
                vy, vz = math.sqrt(T) * zt[a], math.sqrt(T) * zt[c]
                xi2 = xi_x ** 2 + vy ** 2 + vz ** 2
                zeta2 = xi2 / (2 * T)
                br = (xi_x * (dlnchi + 2 * dlnn + dlnT + 0.6 * (zeta2 - 2.5) * dlnT)
                      + 0.4 * (2 * xi_x ** 2 / (2 * T) * du + (zeta2 - 2.5) * du))
                wgt = wt[a] * wt[c]
                acc_phi += wgt * br
                acc_th += wgt * br * (vy ** 2 + vz ** 2)
        assert J1p[k] == pytest.approx(-y * n * g[k] * acc_phi, rel=1e-11, abs=1e-16)
        assert J1t[k] == pytest.approx(-y * n * g[k] * acc_th, rel=1e-11, abs=1e-16)


# --------------------------------------------------------------------------------------
# finite differences and WENO
# --------------------------------------------------------------------------------------
def test_central6_coefficients_and_polynomials():
    """The stencil weights printed in App. A.3; exact for polynomials of degree <= 6."""
    dx = 0.37
    for j in range(7):
        imp = np.zeros(7)
        imp[j] = 1.0  # unit value at offset j - 3
        assert oracle.central6(imp, 1.0)[0] == pytest.approx(GOLDEN_VALUES["central6"]["coeffs"][j],
                                                             abs=1e-16)
    x = np.arange(-3, 4) * dx + 0.81
    for deg in range(7):
        f = x ** deg
        exact = deg * 0.81 ** (deg - 1) if deg else 0.0
        assert oracle.central6(f, dx)[0] == pytest.approx(exact, rel=1e-12, abs=1e-12)


def test_central6_modified_wavenumber():
    k, dx = 2 * math.pi, 1 / 32
    x = (np.arange(-3, 40) + 0.5) * dx
    d = oracle.central6(np.sin(k * x), dx)
    kmod = (1.5 * math.sin(k * dx) - 0.3 * math.sin(2 * k * dx) + math.sin(3 * k * dx) / 30) / dx
    assert np.max(np.abs(d - kmod * np.cos(k * x[3:-3]))) < 1e-12


@pytest.mark.parametrize("row", GOLDEN_VALUES["weno_table"]["rows"])
def test_weno_table_III(row):
    ind = np.array([0.3, 0.7, 1.9])
    for z in row["zero"]:
        ind[z - 1] = 0.0
    assert np.max(np.abs(oracle.weno_weights(ind) - np.array(row["wbar"]))) <= 2.3e-16


def test_weno_weights_formula_and_limits():
    """wbar_q = (delta_q/varphi_q^2)/sum (eq. weno5_omega); tiny indicators do not overflow and
    approach the Table III limit."""
    ind = np.array([2.0, 0.5, 1.0])
    wt = np.array([0.1, 0.6, 0.3]) / ind ** 2
    assert np.allclose(oracle.weno_weights(ind), wt / wt.sum(), rtol=1e-15)
    tiny = oracle.weno_weights(np.array([1e-300, 1.0, 1.0]))
    assert np.all(np.isfinite(tiny)) and tiny[0] == pytest.approx(1.0)
    both = oracle.weno_weights(np.array([1.0, 1e-200, 1e-200]))
    assert both == pytest.approx([0.0, 2 / 3, 1 / 3], abs=1e-15)


def test_weno_indicators_formula_points():
    """Smoothness indicators (eq. weno5_sigma) on quadratics: the second-difference part is
    (13/12)(2a)^2 for f = a x^2 on unit spacing."""
    a = 0.7
    v = a * (np.arange(5) - 2.0) ** 2
    ind = oracle.weno_indicators(v)
    d2 = (2 * a) ** 2 * 13 / 12
    assert ind[0] == pytest.approx(d2 + 0.25 * (v[0] - 4 * v[1] + 3 * v[2]) ** 2, rel=1e-14)
    assert ind[1] == pytest.approx(d2 + 0.25 * (v[1] - v[3]) ** 2, rel=1e-14)


def test_weno_linear_data_exact():
    v = 0.3 + 1.7 * (np.arange(5) - 2.0)
    assert oracle.weno5(v) == pytest.approx(0.3 + 1.7 * 0.5, rel=1e-15)


def test_weno_fifth_order_monotone():
    """Finite-difference WENO: (F_{i+1/2} - F_{i-1/2})/dx approximates f' at 5th order in
    smooth monotone data (f = exp(x))."""
    errs = []
    for h in (0.2, 0.1, 0.05):
        x = 1.0 + h * np.arange(-3, 4)
        f = np.exp(x)
        fp = oracle.weno5(f[1:6])   # interface i+1/2 with i at x=1
        fm = oracle.weno5(f[0:5])   # interface i-1/2
        errs.append(abs((fp - fm) / h - math.exp(1.0)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert math.log2(r1) > 4.5 and math.log2(r2) > 4.5, errs


# --------------------------------------------------------------------------------------
# time stepping and whole-solver invariants
# --------------------------------------------------------------------------------------
def _butcher_R(z):
    A = np.array(GOLDEN_VALUES["rk3_butcher"]["A"])
    b = np.array(GOLDEN_VALUES["rk3_butcher"]["b"])
    return 1.0 + z * b @ np.linalg.solve(np.eye(3) - z * A, np.ones(3))


def test_rk3_uniform_relaxation_closed_form():
    """A uniform state with q != 0 and P_xx != n T: J1 and advection vanish, so each step
    maps q -> R(-Pr dt/tau) q and (P_xx - n T) -> R(-dt/tau)(P_xx - n T), with R the
    stability function of the Table II tableau."""
    Q, nx = 16, 8
    n, T, Pr = 1.3, 1.0, 0.61
    p, w = oracle.quadrature(Q)
    He = lambda l, x: np.polynomial.hermite_e.hermeval(x, [0] * l + [1])
    g = oracle.equilibrium(p, w, 0.0, T)
    phi = n * g + 0.02 * w * He(3, p) + 0.03 * w * He(2, p)
    theta = 2 * T * n * g + 0.01 * w * He(1, p) - 0.06 * w
    u = physics.units(0.3, 0.2)
    s = oracle.Solver(nx, Q, 0.1, 0.0, u["b"], u["mu_ref"], pr=Pr)
    tau = oracle.tau(u["mu_ref"], u["b"], n, T)
    s.par.dt = 0.37 * tau
    s.phi[:] = phi
    s.theta[:] = theta
    n0, u0, T0, q0, pxx0 = oracle.moments_row(p, phi, theta)
    s.step(3)
    n1, u1, T1, q1, pxx1 = s.moments()
    assert np.allclose(n1, n0, rtol=1e-14) and np.allclose(T1, T0, rtol=1e-14)
    Rq = _butcher_R(-Pr * 0.37) ** 3
    Rp = _butcher_R(-0.37) ** 3
    assert np.allclose(q1, Rq * q0, rtol=1e-12)
    assert np.allclose(pxx1 - n0 * T0, Rp * (pxx0 - n0 * T0), rtol=1e-11)


@pytest.mark.parametrize("bc", [oracle.BC_PERIODIC, oracle.BC_EQUILIBRIUM])
def test_uniform_equilibrium_is_stationary(bc):
    Q, nx = 16, 24
    u = physics.units(0.4, 0.05)
    s = oracle.Solver(nx, Q, 1 / nx, 0.0, u["b"], u["mu_ref"], pr_mode=oracle.PR_ENSKOG, bc=bc)
    s.par.dt = 0.5 / nx / np.max(s.p)
    R = nx + 6
    s.init_equilibrium(np.full(R, 1.4), np.full(R, 0.35), np.full(R, 1.25))
    phi0, th0 = s.phi.copy(), s.theta.copy()
    s.step(1000)
    assert np.max(np.abs(s.phi - phi0)) <= 1e-14 * np.max(np.abs(phi0))
    assert np.max(np.abs(s.theta - th0)) <= 1e-14 * np.max(np.abs(th0))


def _random_periodic(nx, Q, El, seed, kn=0.05):
    rng = np.random.default_rng(seed)
    w = workloads.sound_wave(nx=nx, q=Q, denseness=El, kn=kn, amplitude=0.05, pr_mode="enskog")
    x = workloads.cell_centres(nx, 1.0)
    w["u"] = 0.1 * np.sin(2 * math.pi * x + rng.uniform(0, 6))
    w["T"] = 1.0 + 0.1 * np.cos(4 * math.pi * x + rng.uniform(0, 6))
    return w


def test_mass_conservation_periodic_dense():
    w = _random_periodic(40, 12, 0.5, 1)
    s = solver_from_workload(w)
    c0 = s.conserved()
    s.step(200)
    c1 = s.conserved()
    assert abs(c1[0] - c0[0]) <= 1e-12 * abs(c0[0])


def test_full_conservation_periodic_dilute():
    """b = 0: mass, momentum and energy are conserved to round-off."""
    w = _random_periodic(40, 12, 0.0, 2)
    s = solver_from_workload(w)
    c0 = s.conserved()
    s.step(200)
    c1 = s.conserved()
    scale = [abs(c0[0]), abs(c0[0]), abs(c0[2])]
    for j in range(3):
        assert abs(c1[j] - c0[j]) <= 1e-12 * scale[j], (j, c0, c1)


def test_mirror_symmetry():
    """x -> -x with p_k -> -p_k maps a solution to a solution."""
    w = _random_periodic(32, 12, 0.3, 3)
    s = solver_from_workload(w)
    m = solver_from_workload(w)
    m.phi[:] = s.phi[::-1, ::-1]
    m.theta[:] = s.theta[::-1, ::-1]
    s.step(50)
    m.step(50)
    scale = np.max(np.abs(s.phi))
    assert np.max(np.abs(m.phi[::-1, ::-1] - s.phi)) <= 1e-13 * scale
    assert np.max(np.abs(m.theta[::-1, ::-1] - s.theta)) <= 1e-13 * np.max(np.abs(s.theta))


def test_sound_wave_reflection_symmetry():
    """n = 1 + A sin(2 pi x) is symmetric under x -> 1/2 - x, and stays so; u is odd."""
    w = workloads.config1()
    s = solver_from_workload(w)
    s.step(100)
    n, u, T, q, pxx = s.moments()
    # cells i and nx-1-i' with x_j = 1/2 - x_i: j = (nx/2 - 1 - i) mod nx
    nx = w["nx"]
    j = (nx // 2 - 1 - np.arange(nx)) % nx
    assert np.max(np.abs(n[j] - n)) < 1e-14
    assert np.max(np.abs(u[j] + u)) < 1e-14 * max(1.0, np.max(np.abs(u))) + 1e-17


def test_scale_invariance():
    """(n, b, mu_ref) -> (c n, b/c, c mu_ref) leaves y and tau unchanged and scales phi,
    theta by c (Sec. II.B: only eta = b n / 4 enters, plus sigma through tau)."""
    w = _random_periodic(24, 12, 0.4, 4)
    s = solver_from_workload(w)
    c = 3.0
    t = oracle.Solver(w["nx"], w["q"], s.par.dx, s.par.dt, s.par.b / c, s.par.mu_ref * c,
                      pr_mode=oracle.PR_ENSKOG)
    t.phi[:] = c * s.phi
    t.theta[:] = c * s.theta
    s.step(30)
    t.step(30)
    assert np.max(np.abs(t.phi - c * s.phi)) <= 1e-13 * np.max(np.abs(t.phi))


# --------------------------------------------------------------------------------------
# Rankine-Hugoniot and sound speed
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("M", [1.2, 2.0, 3.0, 5.0])
def test_rh_ideal_gas_limit(M):
    """b = 0: n2/n1 = 4 M^2/(M^2 + 3), T2/T1 = (5 M^2 - 1)(M^2 + 3)/(16 M^2) (gamma = 5/3)."""
    u1 = M * math.sqrt(5.0 / 3.0)
    n2, u2, T2 = physics.rankine_hugoniot(1.0, 1.0, u1, 0.0)
    assert n2 == pytest.approx(4 * M * M / (M * M + 3), rel=1e-12)
    assert T2 == pytest.approx((5 * M * M - 1) * (M * M + 3) / (16 * M * M), rel=1e-12)


@pytest.mark.parametrize("M,El", [(2.0, 0.3), (3.0, 0.3), (1.5, 0.05)])
def test_rh_dense_fluxes_and_scaling(M, El):
    st = physics.shock_states(M, El)
    b = st["b"]
    for n1, u1, T1, n2, u2, T2 in [(st["n1"], st["u1"], st["T1"], st["n2"], st["u2"], st["T2"])]:
        assert n1 * u1 == pytest.approx(n2 * u2, rel=1e-13)
        assert n1 * u1 ** 2 + physics.pressure(n1, T1, b) == pytest.approx(
            n2 * u2 ** 2 + physics.pressure(n2, T2, b), rel=1e-13)
        h1 = 2.5 * T1 + physics.pressure(n1, T1, b) / n1 - T1 + 0.5 * u1 ** 2
        h2 = 2.5 * T2 + physics.pressure(n2, T2, b) / n2 - T2 + 0.5 * u2 ** 2
        assert h1 == pytest.approx(h2, rel=1e-13)
    assert st["T1"] + st["T2"] == pytest.approx(2.0, rel=1e-14)
    assert st["u1"] / math.sqrt(physics.cs2(st["n1"], st["T1"], b)) == pytest.approx(M, rel=1e-13)


@pytest.mark.parametrize("n,T,El", [(1.0, 1.0, 0.3), (0.1, 1.0, 4.0), (2.0, 0.5, 1.0)])
def test_sound_speed_two_forms(n, T, El):
    """c_s^2 from eq. sw_cs equals the (rho, P) form used for the rarefaction; dilute 5T/3."""
    b = 4 * physics.eta_from_denseness(El)
    assert physics.cs2(n, T, b) == pytest.approx(
        physics.cs2_rho_P(n, physics.pressure(n, T, b), b), rel=1e-13)
    assert physics.cs2(n, T, 0.0) == pytest.approx(5 * T / 3, rel=1e-15)


def test_linear_modes_dilute_limits():
    """b = 0, Pr = 2/3: alpha_a -> (k^2 mu/rho)(2/3 + (gamma - 1)/(2 Pr) ...) small-k forms:
    alpha_t = k^2 lambda/(rho c_P), alpha_s = k c_s (leading order in k)."""
    k = 2 * math.pi
    mu_ref = 1e-4
    at, aa, as_ = physics.linear_modes(1.0, 1.0, 0.0, mu_ref, k, pr=2 / 3)
    mu = mu_ref
    lam = 2.5 * mu / (2 / 3)
    assert at == pytest.approx(k * k * lam / 2.5, rel=1e-3)
    gamma = 5 / 3
    assert aa == pytest.approx(0.5 * k * k * (4 * mu / 3 + (gamma - 1) * lam / 2.5), rel=1e-3)
    assert as_ == pytest.approx(k * math.sqrt(5 / 3), rel=1e-6)
