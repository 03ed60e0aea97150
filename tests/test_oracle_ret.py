"""Pins of the oracle's chi_RET-FM (Sec. II.A, eq. chi_ret): the Fischer-Methfessel ball
average of the density and its use in the right-hand side.

  - a uniform density averages to itself;
  - a cubic profile averages to n + sigma^2 n''/10 exactly (the moments of the disc-area
    weight 3/(4 sigma^3)(sigma^2 - s^2) are 1 and sigma^2/5, and the interpolant is exact
    for cubics);
  - a plane wave averages to 3 j_1(k sigma)/(k sigma) times itself, the Fourier transform
    of the ball indicator in three dimensions, to the interpolation error O(dx^4);
  - sigma -> 0 gives chi_SET, and the right-hand side then matches the chi_SET one to the
    difference between the central difference of ln chi and the chain rule;
  - a uniform state stays an exact equilibrium.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import physics

NG = oracle.NG


def rows_from(fn, nx, periodic, left=None, right=None):
    """Row densities (ghosts included) from a function of the cell index."""
    i = np.arange(-NG, nx + NG, dtype=np.float64)
    n = fn(i)
    if not periodic:
        n[:NG] = fn(np.array([-NG], dtype=float))[0] if left is None else left
        n[-NG:] = fn(np.array([nx + NG - 1], dtype=float))[0] if right is None else right
    return n


@pytest.mark.parametrize("S", [0.0, 0.3, 1.0, 2.5, 7.2])
@pytest.mark.parametrize("periodic", [True, False])
def test_uniform_density_is_its_own_average(S, periodic):
    nx = 40
    n = np.full(nx + 2 * NG, 0.731)
    for i in (-3, 0, 5, nx - 1, nx + 2):
        assert abs(oracle.fm_density(n, nx, periodic, S, i) / 0.731 - 1.0) < 1e-14


@pytest.mark.parametrize("S", [0.3, 1.0, 2.5, 7.2])
def test_cubic_profile_average_is_exact(S):
    a, b, c, d = 1.0, 2e-3, -3e-5, 4e-7
    nx = 80
    fn = lambda t: a + b * t + c * t * t + d * t ** 3
    n = rows_from(fn, nx, periodic=False)
    # interior cells whose interpolation stencils stay inside the grid
    reach = int(math.ceil(S)) + 2
    for i in range(reach, nx - reach, 7):
        exact = fn(float(i)) + S * S * (2 * c + 6 * d * i) / 10.0
        got = oracle.fm_density(n, nx, False, S, i)
        assert abs(got / exact - 1.0) < 1e-14, (S, i)


@pytest.mark.parametrize("sigma,nx", [(0.1, 400), (0.003, 100), (0.3, 800)])
def test_plane_wave_average_is_the_ball_transform(sigma, nx):
    """Periodic wave on [0, 1): n = 1 + A sin(2 pi x)."""
    A, k = 1e-2, 2.0 * math.pi
    dx = 1.0 / nx
    x = lambda i: (i + 0.5) * dx
    n = rows_from(lambda i: 1.0 + A * np.sin(k * x(i)), nx, periodic=True)
    z = k * sigma
    factor = 3.0 * (math.sin(z) - z * math.cos(z)) / z ** 3
    for i in (0, 1, nx // 3, nx - 1):   # boundary cells use the periodic images
        exact = 1.0 + A * math.sin(k * x(i)) * factor
        got = oracle.fm_density(n, nx, True, sigma / dx, i)
        assert abs(got - exact) < 2.0 * A * (k * dx) ** 4 + 1e-15, (sigma, i, got - exact)


def test_beyond_the_domain_the_average_sees_the_end_states():
    """Equilibrium ghosts: a step between two end states; the cell next to the left edge
    averages the left end state over the part of the ball outside the domain."""
    nx, S = 40, 5.0
    n = np.concatenate([np.full(NG, 2.0), np.full(nx, 1.0), np.full(NG, 0.5)])
    # cell -3 (a ghost row): the ball reaches cells -8 .. 2 with interpolation nodes down to
    # -9 and up to 3: only the interior cells 0..3 differ from the left end state 2.0
    got = oracle.fm_density(n, nx, False, S, -3)
    assert 1.0 < got < 2.0
    # far from both edges the average is the interior value
    assert abs(oracle.fm_density(n, nx, False, S, nx // 2) - 1.0) < 1e-15
    # symmetric in the data: reflecting the row reflects the result
    nr = n[::-1].copy()
    assert abs(oracle.fm_density(nr, nx, False, S, nx + 2) - got) < 1e-15


def _smooth_solver(chi_mode, sigma, nx=64, q=16):
    El, kn = 0.3, 0.05
    u = physics.units(El, kn)
    p, _ = oracle.quadrature(q)
    dx = 1.0 / nx
    s = oracle.Solver(nx, q, dx, 0.5 * dx / np.max(np.abs(p)), u["b"], u["mu_ref"],
                      pr_mode=oracle.PR_ENSKOG, bc=oracle.BC_PERIODIC, chi_mode=chi_mode,
                      sigma=sigma)
    x = (np.arange(-NG, nx + NG) + 0.5) * dx
    s.init_equilibrium(1.0 + 0.1 * np.sin(2 * np.pi * x), 0.05 * np.cos(2 * np.pi * x),
                       1.0 + 0.05 * np.sin(4 * np.pi * x))
    return s


def test_vanishing_sigma_gives_chi_set():
    s = _smooth_solver(oracle.CHI_RETFM, 1e-12)
    n, u, T, _, _ = s.moments()
    rows = np.concatenate([n[-NG:], n, n[:NG]])
    chi = s.chi_rows(rows)
    for r in range(len(rows)):
        assert abs(chi[r] / oracle.chi(0.25 * s.par.b * rows[r]) - 1.0) < 1e-12
    Lp_ret, Lt_ret = s.rhs()
    Lp_set, Lt_set = _smooth_solver(oracle.CHI_SET, 0.0).rhs()
    # the two differ only by d ln chi: central difference of ln chi vs the chain rule,
    # a 6th-order truncation error on 64 cells per period
    scale = np.max(np.abs(Lp_set))
    assert np.max(np.abs(Lp_ret - Lp_set)) < 1e-7 * scale
    assert np.max(np.abs(Lt_ret - Lt_set)) < 1e-7 * np.max(np.abs(Lt_set))
    # and the gap is not round-off only: d ln chi does enter the result
    assert np.max(np.abs(Lp_ret - Lp_set)) > 1e-14 * scale


def test_finite_sigma_changes_only_the_chi_terms():
    """At sigma = 2 dx the RET right-hand side differs from the SET one, and the difference
    has no mass moment (chi enters through tau, Pr and J1, none of which moves mass)."""
    s_ret = _smooth_solver(oracle.CHI_RETFM, 2.0 / 64)
    s_set = _smooth_solver(oracle.CHI_SET, 0.0)
    Lp_r, _ = s_ret.rhs()
    Lp_s, _ = s_set.rhs()
    d = Lp_r - Lp_s
    assert np.max(np.abs(d)) > 1e-6 * np.max(np.abs(Lp_s))
    assert np.max(np.abs(d.sum(axis=1))) < 1e-12 * np.max(np.abs(Lp_s))


def test_uniform_state_stays_in_equilibrium():
    nx, q = 32, 16
    u = physics.units(0.4, 0.05)
    p, _ = oracle.quadrature(q)
    dx = 1.0 / nx
    s = oracle.Solver(nx, q, dx, 0.5 * dx / np.max(np.abs(p)), u["b"], u["mu_ref"],
                      pr_mode=oracle.PR_ENSKOG, bc=oracle.BC_PERIODIC,
                      chi_mode=oracle.CHI_RETFM, sigma=3.5 * dx)
    R = nx + 2 * NG
    s.init_equilibrium(np.full(R, 1.2), np.full(R, 0.1), np.full(R, 0.9))
    Lp, Lt = s.rhs()
    assert np.max(np.abs(Lp)) < 1e-13 and np.max(np.abs(Lt)) < 1e-13
