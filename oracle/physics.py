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
