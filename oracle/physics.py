"""Analytic side of the oracle: units, dense-gas equation of state, Rankine-Hugoniot
states, linearised hydrodynamics and the sound-wave amplitude diagnostic.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Units m = k_B = 1, T_ref = 1.
"""
import math

import numpy as np

C_MU = (4.0 / 25.0) * (1.0 + 12.0 / math.pi)          # viscosity y^2 coefficient (Sec. II.B)
C_LAMBDA = (9.0 / 25.0) * (1.0 + 32.0 / (9.0 * math.pi))  # conductivity y^2 coefficient


# ---------------------------------------------------------------------------------------
# hard-sphere closures (Sec. II.A-B)
# ---------------------------------------------------------------------------------------
def chi_set(eta):
    """Carnahan-Starling contact value chi_SET = (1/2)(2 - eta)/(1 - eta)^3 (eq. chi)."""
    return 0.5 * (2.0 - eta) / (1.0 - eta) ** 3


def compressibility_cs(eta):
    """Carnahan-Starling P^hs/(n k T) = (1 + eta + eta^2 - eta^3)/(1 - eta)^3."""
    return (1.0 + eta + eta ** 2 - eta ** 3) / (1.0 - eta) ** 3


def denseness(eta):
    """E_l = sigma / l = (3/sqrt 2) b n chi with b n = 4 eta (Sec. II.B)."""
    return 3.0 / math.sqrt(2.0) * 4.0 * eta * chi_set(eta)


def eta_from_denseness(El, tol=1e-15):
    """Invert E_l(eta) on [0, 0.5) by bisection (E_l is increasing there)."""
    if El == 0.0:
        return 0.0
    lo, hi = 0.0, 0.5
    while denseness(hi) < El:
        raise ValueError("denseness out of range")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if denseness(mid) < El:
            lo = mid
        else:
            hi = mid
        if hi - lo < tol:
            break
    return 0.5 * (lo + hi)


def units(El, kn, kn_length=1.0, n_ref=1.0):
    """Map denseness E_l (at n_ref, T = 1) and Knudsen number kn = l / kn_length to the
    model's covolume b and dilute reference viscosity mu_ref.

    eta0 solves E_l = 6 sqrt(2) eta chi(eta); b = 4 eta0 / n_ref.  The Enskog mean free path
    l = 1/(sqrt 2 pi sigma^2 n chi) (Sec. II.B) gives the dilute hard-sphere viscosity
    mu_ref = (5/16) sqrt(2 pi) n_ref (chi0 l), the relation of mu_ref (Sec. II.B, reference
    values) to the dilute mean free path chi0 l.  Setting sigma to the relaxation scale
    sigma = E_l l (eq. tau_sigma) is the same statement.
    """
    eta0 = eta_from_denseness(El)
    chi0 = chi_set(eta0)
    b = 4.0 * eta0 / n_ref
    l = kn * kn_length
    mu_ref = 5.0 / 16.0 * math.sqrt(2.0 * math.pi) * n_ref * chi0 * l
    return {"eta0": eta0, "chi0": chi0, "b": b, "mu_ref": mu_ref, "mfp": l,
            "sigma": El * l}


def y_of(n, b):
    """y = b rho chi at density n."""
    return b * n * chi_set(0.25 * b * n)


def prandtl_enskog(y):
    return (2.0 / 3.0) * (1.0 + 0.8 * y + C_MU * y * y) / (1.0 + 1.2 * y + C_LAMBDA * y * y)


def viscosity(n, T, b, mu_ref):
    """Dense-gas shear viscosity mu = mu_0 b rho [1/(b rho chi) + 0.8 + C b rho chi],
    mu_0 = mu_ref sqrt(T) (Sec. II.B), written for b -> 0 as (mu_0/chi)(1 + 0.8 y + C y^2)."""
    chi = chi_set(0.25 * b * n)
    y = b * n * chi
    return mu_ref * math.sqrt(T) / chi * (1.0 + 0.8 * y + C_MU * y * y)


def bulk_viscosity(n, T, b, mu_ref):
    """mu_v = (16/(5 pi)) mu_0 b^2 rho^2 chi (Sec. II.B)."""
    return 16.0 / (5.0 * math.pi) * mu_ref * math.sqrt(T) * b * b * n * n * chi_set(0.25 * b * n)


def conductivity(n, T, b, mu_ref):
    """lambda = lambda_0 b rho [1/(b rho chi) + 1.2 + C' b rho chi] with
    lambda_ref = (15/4) mu_ref (ratio of the two reference values, Sec. II.B)."""
    chi = chi_set(0.25 * b * n)
    y = b * n * chi
    return 15.0 / 4.0 * mu_ref * math.sqrt(T) / chi * (1.0 + 1.2 * y + C_LAMBDA * y * y)


def tau(n, T, b, mu_ref):
    """tau = mu / P_i, P_i = n T (Sec. II.B)."""
    return viscosity(n, T, b, mu_ref) / (n * T)


# ---------------------------------------------------------------------------------------
# equation of state and sound speed
# ---------------------------------------------------------------------------------------
def Z(n, b):
    """Compressibility P/(n T) = 1 + b rho chi (Sec. II.B)."""
    return 1.0 + b * n * chi_set(0.25 * b * n)


def dZ_dn(n, b):
    eta = 0.25 * b * n
    chi = chi_set(eta)
    dchi_deta = chi * (3.0 / (1.0 - eta) - 1.0 / (2.0 - eta))
    return b * (chi + eta * dchi_deta)


def pressure(n, T, b):
    return n * T * Z(n, b)


def cs2(n, T, b):
    """c_s^2 = d_rho P + P/(rho^2 c_V) d_T P with c_V = 3/2 (eq. sw_cs); for P = n T Z(n)
    this is T [Z + n Z' + (2/3) Z^2]."""
    z = Z(n, b)
    return T * (z + n * dZ_dn(n, b) + 2.0 / 3.0 * z * z)


def cs2_rho_P(n, P, b):
    """The form of c_s^2 in terms of rho and P used for the rarefaction (Sec. IV.B.2)."""
    eta = 0.25 * b * n
    chi = chi_set(eta)
    dchi_dn = 0.25 * b * chi * (3.0 / (1.0 - eta) - 1.0 / (2.0 - eta))
    return (P / n + 2.0 * P * (1.0 + b * n * chi) / (3.0 * n)
            + b * P * (chi + n * dchi_dn) / (1.0 + b * n * chi))


# ---------------------------------------------------------------------------------------
# Rankine-Hugoniot for a steady normal shock with the dense equation of state
# ---------------------------------------------------------------------------------------
def rankine_hugoniot(n1, T1, u1, b, tol=1e-14, maxit=100):
    """Downstream (n2, u2, T2) of a standing normal shock with upstream (n1, u1 > 0, T1).

    Jumps of mass n u, momentum n u^2 + P and energy flux u (e + n u^2/2 + P), with
    e = (3/2) n T and P = n T Z(n) (eq. rankine_hugoniot written in the shock frame).
    Newton iteration on (n2, T2) from the ideal-gas solution.
    """
    j = n1 * u1
    P1 = pressure(n1, T1, b)
    mom = j * u1 + P1
    H1 = 1.5 * T1 + P1 / n1 + 0.5 * u1 * u1
    M2 = u1 * u1 / cs2(n1, T1, b)
    if M2 <= 1.0:
        raise ValueError("upstream flow must be supersonic")
    # ideal-gas starting point (gamma = 5/3)
    r = 4.0 * M2 / (M2 + 3.0)
    tr = (5.0 * M2 - 1.0) * (M2 + 3.0) / (16.0 * M2)
    x = np.array([n1 * r, T1 * tr])

    def F(v):
        n2, T2 = v
        u2 = j / n2
        P2 = pressure(n2, T2, b)
        return np.array([j * u2 + P2 - mom, 1.5 * T2 + P2 / n2 + 0.5 * u2 * u2 - H1])

    for _ in range(maxit):
        f = F(x)
        h = 1e-7
        Jm = np.zeros((2, 2))
        for c in range(2):
            dx = np.zeros(2)
            dx[c] = h * max(1.0, abs(x[c]))
            Jm[:, c] = (F(x + dx) - F(x - dx)) / (2 * dx[c])
        step = np.linalg.solve(Jm, f)
        x = x - step
        if np.max(np.abs(step) / np.abs(x)) < tol:
            break
    n2, T2 = float(x[0]), float(x[1])
    return n2, j / n2, T2


def shock_states(mach, El, n1=1.0):
    """Upstream/downstream states of a standing shock at Mach `mach`, denseness E_l at n1.

    Reading: the Hermite expansion of the equilibrium converges only for |T - 1| < 1 in
    T_ref units, so the temperature unit is chosen such that T1 + T2 = 2.  The jump
    ratios do not depend on T1 (P = n T Z(n) is linear in T), so the solution at T1 = 1
    is rescaled: T -> s T, u -> sqrt(s) u with s = 2 / (1 + T2/T1).
    """
    b = 4.0 * eta_from_denseness(El) / n1
    u1 = mach * math.sqrt(cs2(n1, 1.0, b))
    n2, u2, T2 = rankine_hugoniot(n1, 1.0, u1, b)
    s = 2.0 / (1.0 + T2)
    return {"n1": n1, "u1": u1 * math.sqrt(s), "T1": s,
            "n2": n2, "u2": u2 * math.sqrt(s), "T2": T2 * s, "b": b}


# ---------------------------------------------------------------------------------------
# linearised Navier-Stokes-Fourier modes of a sound wave
# ---------------------------------------------------------------------------------------
def linear_modes(n0, T0, b, mu_ref, k, pr=None):
    """Eigenvalues alpha of the linearised NSF system for perturbations exp(i k x - alpha t):

      alpha dn = i k n0 du
      alpha n0 du = i k (P_n dn + P_T dT) + k^2 (4 mu/3 + mu_v) du
      alpha n0 c_V dT = i k T0 P_T du + k^2 lambda dT

    with P = n T Z(n), c_V = 3/2, mu = tau P_i, mu_v (Sec. II.B) and lambda = (5/2) mu / Pr.
    Reading: the printed damping coefficients are not dimensionally consistent, so the
    reference is the spectrum of this system.  Returns (alpha_t, alpha_a, alpha_s).
    """
    mu = viscosity(n0, T0, b, mu_ref)
    muv = bulk_viscosity(n0, T0, b, mu_ref)
    if pr is None:
        pr = prandtl_enskog(y_of(n0, b))
    lam = 2.5 * mu / pr
    cV = 1.5
    Pn = T0 * (Z(n0, b) + n0 * dZ_dn(n0, b))
    PT = n0 * Z(n0, b)
    M = np.array([
        [0.0, 1j * k * n0, 0.0],
        [1j * k * Pn / n0, k * k * (4.0 * mu / 3.0 + muv) / n0, 1j * k * PT / n0],
        [0.0, 1j * k * T0 * PT / (n0 * cV), k * k * lam / (n0 * cV)],
    ], dtype=complex)
    ev = np.linalg.eigvals(M)
    real = [e for e in ev if abs(e.imag) < 1e-12 * max(1.0, abs(e))]
    cplx = [e for e in ev if abs(e.imag) >= 1e-12 * max(1.0, abs(e))]
    if len(real) != 1 or len(cplx) != 2:
        raise ValueError(f"unexpected spectrum {ev}")
    alpha_t = real[0].real
    alpha_a = 0.5 * (cplx[0].real + cplx[1].real)
    alpha_s = abs(cplx[0].imag)
    return alpha_t, alpha_a, alpha_s


def sin_amplitude(n, x, k):
    """(2/N_x) sum_i n(x_i) sin(k x_i): the paper's projection (Sec. IV.A.3) taken on
    sin(k x), the shape of the initial perturbation used here."""
    return 2.0 / n.size * float(np.sum(n * np.sin(k * x)))


# ---------------------------------------------------------------------------------------
# Riemann problem of the dense-gas Euler equations (Sec. IV.B, inviscid limit)
# ---------------------------------------------------------------------------------------
def _rarefaction(nL, PL, uL, b, n_end):
    """Left-facing rarefaction from (nL, PL, uL): the similarity equations reduce along the
    wave to dP/dn = c_s^2(n, P) and du/dn = -c_s(n, P)/n (Sec. IV.B, with u = xi + c_s);
    integrated from nL down to n_end.  Returns the ODE solution (dense output) in n."""
    from scipy.integrate import solve_ivp

    def rhs(n, y):
        c2 = cs2_rho_P(n, y[0], b)
        return [c2, -math.sqrt(c2) / n]

    return solve_ivp(rhs, (nL, n_end), [PL, uL], method="DOP853", rtol=1e-13, atol=1e-15,
                     dense_output=True)


def _shock_right(nR, TR, Pc, b):
    """Post-shock state behind a right-facing shock into (nR, TR, u = 0) with pressure Pc:
    from the jumps of mass, momentum and energy (eq. rankine_hugoniot), the Hugoniot
    relation e2 - eR = (Pc + PR)/2 (1/nR - 1/n2) per particle with e = 3T/2 and
    T2 = Pc / (n2 Z(n2)) fixes n2; then the mass flux m^2 = (Pc - PR)/(1/nR - 1/n2) gives
    u_c = m (1/nR - 1/n2) and the shock speed xi_s = m / nR.  Returns (n2, T2, u_c, xi_s)."""
    from scipy.optimize import brentq
    PR = pressure(nR, TR, b)

    def hug(n2):
        T2 = Pc / (n2 * Z(n2, b))
        return 1.5 * (T2 - TR) - 0.5 * (Pc + PR) * (1.0 / nR - 1.0 / n2)

    nmax = 0.999 * 4.0 / b if b > 0 else 4.0 * nR * 1e3
    lo, hi = nR * (1.0 + 1e-12), nR * 1.01
    while hug(hi) > 0.0 and hi < nmax:
        hi = min(2.0 * hi, nmax)
    n2 = brentq(hug, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    T2 = Pc / (n2 * Z(n2, b))
    dv = 1.0 / nR - 1.0 / n2
    m = math.sqrt((Pc - PR) / dv)
    return n2, T2, m * dv, m / nR


def riemann(nL, TL, nR, TR, b):
    """Exact solution of the dense-gas Riemann problem with both sides at rest and
    P_L > P_R (the shock-tube configuration of Sec. IV.B): a left rarefaction, a contact
    and a right shock.  Returns a dict with the star pressure P_c, velocity u_c, densities
    n1 (left of the contact), n2 (right), temperatures T1, T2, the wave speeds and a
    function sample(xi) -> (n, u, T) of the similarity variable xi = (x - x0)/t."""
    from scipy.optimize import brentq
    PL, PR = pressure(nL, TL, b), pressure(nR, TR, b)
    if not PL > PR:
        raise ValueError("expects P_L > P_R")
    # the rarefaction branch: u along the wave as a function of P, down to below PR
    n_lo = nR * 1e-3
    sol = _rarefaction(nL, PL, 0.0, b, n_lo)

    def n_of_P(P):
        return brentq(lambda n: sol.sol(n)[0] - P, n_lo, nL, xtol=1e-15, rtol=1e-15, maxiter=500)

    def mismatch(P):
        u_raref = sol.sol(n_of_P(P))[1]
        u_shock = _shock_right(nR, TR, P, b)[2]
        return u_raref - u_shock

    Pc = brentq(mismatch, PR * (1.0 + 1e-9), PL * (1.0 - 1e-12), xtol=1e-15, rtol=1e-15,
                maxiter=500)
    n1 = n_of_P(Pc)
    uc = float(sol.sol(n1)[1])
    T1 = Pc / (n1 * Z(n1, b))
    n2, T2, uc2, xis = _shock_right(nR, TR, Pc, b)
    cL = math.sqrt(cs2(nL, TL, b))
    c1 = math.sqrt(cs2(n1, T1, b))
    xi_head, xi_tail = -cL, float(uc - c1)

    def sample(xi):
        if xi <= xi_head:
            return nL, 0.0, TL
        if xi < xi_tail:
            # inside the fan u - c_s = xi
            def f(n):
                P, u = sol.sol(n)
                return u - math.sqrt(cs2_rho_P(n, P, b)) - xi
            n = brentq(f, n1, nL, xtol=1e-15, rtol=1e-15, maxiter=500)
            P, u = sol.sol(n)
            return n, float(u), float(P / (n * Z(n, b)))
        if xi < uc:
            return n1, uc, T1
        if xi < xis:
            return n2, uc, T2
        return nR, 0.0, TR

    return {"Pc": Pc, "uc": float(uc), "uc_shock": uc2, "n1": n1, "T1": T1, "n2": n2,
            "T2": T2, "xi_head": xi_head, "xi_tail": xi_tail, "xi_shock": xis,
            "sample": sample}


def isentrope_invariant(n, T, b):
    """ln T - (2/3) [ln n + 1/(1 - eta)^2 + 2/(1 - eta)], eta = b n/4: constant along an
    isentrope of P = n T Z(n) with e = 3T/2 (T ds = (3/2) dT - T Z(n) dn/n and
    int 4 chi_SET(eta) d eta = 1/(1 - eta)^2 + 2/(1 - eta))."""
    eta = 0.25 * b * n
    return math.log(T) - (2.0 / 3.0) * (math.log(n) + 1.0 / (1.0 - eta) ** 2 + 2.0 / (1.0 - eta))
