"""FP64 CPU oracle for the FDLB step of the simplified Enskog-Shakhov model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this module; only the
test suite, the smoke check and the benchmark's CPU-baseline leg use it.  It shares no
code with the HIP library.  The numerical core is oracle.c (compiled to liboracle.so by
oracle/build.py); physics.py holds the analytic references (units, equation of state,
Rankine-Hugoniot, linear hydrodynamics).

Storage convention: a distribution is an array of shape (nx + 6, q); row r holds cell
r - 3, and the first and last three rows are ghost cells.
"""
import ctypes
import os

import numpy as np

from . import build as _build

NG = 3
PR_CONST, PR_ENSKOG = 0, 1
BC_PERIODIC, BC_EQUILIBRIUM = 0, 1
CHI_SET, CHI_RETFM = 0, 1

_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("q", ctypes.c_int), ("nh", ctypes.c_int),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("b", ctypes.c_double), ("mu_ref", ctypes.c_double),
                ("pr_mode", ctypes.c_int), ("pr", ctypes.c_double), ("bc", ctypes.c_int),
                ("chi_mode", ctypes.c_int), ("sigma", ctypes.c_double)]


_D = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load liboracle.so, compiling it first if it is missing or stale."""
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        L.or_hermite.restype = ctypes.c_double
        L.or_hermite.argtypes = [ctypes.c_int, ctypes.c_double]
        L.or_quadrature.restype = ctypes.c_int
        L.or_quadrature.argtypes = [ctypes.c_int, _D, _D]
        L.or_equilibrium.restype = None
        L.or_equilibrium.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_double,
                                     ctypes.c_double, _D]
        for name in ("or_chi", "or_dlnchi_dlnn", "or_prandtl_enskog"):
            f = getattr(L, name)
            f.restype = ctypes.c_double
            f.argtypes = [ctypes.c_double]
        L.or_tau.restype = ctypes.c_double
        L.or_tau.argtypes = [ctypes.c_double] * 4
        L.or_tau_chi.restype = ctypes.c_double
        L.or_tau_chi.argtypes = [ctypes.c_double] * 5
        L.or_fm_density.restype = ctypes.c_double
        L.or_fm_density.argtypes = [_D, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.or_fm_chi.restype = ctypes.c_int
        L.or_fm_chi.argtypes = [ctypes.POINTER(_Params), _D, _D]
        L.or_moments_row.restype = None
        L.or_moments_row.argtypes = [ctypes.c_int, _D, _D, _D, _D, _D, _D, _D, _D]
        L.or_moments.restype = None
        L.or_moments.argtypes = [ctypes.POINTER(_Params), _D, _D, _D, _D, _D, _D, _D, _D]
        L.or_central6.restype = ctypes.c_double
        L.or_central6.argtypes = [_D, ctypes.c_double]
        L.or_weno_weights.restype = None
        L.or_weno_weights.argtypes = [_D, _D]
        L.or_weno_indicators.restype = None
        L.or_weno_indicators.argtypes = [_D, _D]
        L.or_weno5.restype = ctypes.c_double
        L.or_weno5.argtypes = [_D]
        L.or_cell_sources.restype = None
        L.or_cell_sources.argtypes = ([ctypes.c_int, ctypes.c_int, _D, _D] +
                                      [ctypes.c_double] * 10 + [_D, _D, _D, _D])
        L.or_rhs.restype = ctypes.c_int
        L.or_rhs.argtypes = [ctypes.POINTER(_Params), _D, _D, _D, _D, _D, _D]
        L.or_step.restype = ctypes.c_int
        L.or_step.argtypes = [ctypes.POINTER(_Params), _D, _D, _D, _D, ctypes.c_int]
        L.or_init_equilibrium.restype = None
        L.or_init_equilibrium.argtypes = [ctypes.POINTER(_Params), _D, _D, _D, _D, _D, _D, _D]
        L.or_conserved.restype = None
        L.or_conserved.argtypes = [ctypes.POINTER(_Params), _D, _D, _D, _D]
        _lib = L
    return _lib


def _ptr(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def set_threads(n: int) -> None:
    """Set the OpenMP thread count used by the oracle's per-cell loops."""
    os.environ["OMP_NUM_THREADS"] = str(int(n))
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(int(n))
    except OSError:
        pass


# ---------------------------------------------------------------------------------------
# thin wrappers of the C entry points
# ---------------------------------------------------------------------------------------
def hermite(l: int, x: float) -> float:
    """Probabilists' Hermite polynomial He_l(x) (Sec. II.D)."""
    return lib().or_hermite(int(l), float(x))


def quadrature(q: int):
    """Nodes (roots of He_Q, ascending) and weights w_k = Q!/He_{Q+1}(p_k)^2 (Sec. II.D)."""
    p = np.zeros(q)
    w = np.zeros(q)
    rc = lib().or_quadrature(int(q), _ptr(p), _ptr(w))
    if rc != 0:
        raise RuntimeError(f"oracle quadrature failed for Q={q} (code {rc})")
    return p, w


def equilibrium(p, w, u: float, T: float, nh: int = None):
    """Hermite-expanded equilibrium g_k[u,T] (Sec. II.D, eq. g_alpha), literal double sum."""
    p = _f64(p)
    w = _f64(w)
    q = p.size
    nh = q - 1 if nh is None else nh
    g = np.zeros(q)
    lib().or_equilibrium(q, int(nh), _ptr(p), _ptr(w), float(u), float(T), _ptr(g))
    return g


def chi(eta: float) -> float:
    return lib().or_chi(float(eta))


def dlnchi_dlnn(eta: float) -> float:
    return lib().or_dlnchi_dlnn(float(eta))


def prandtl_enskog(y: float) -> float:
    return lib().or_prandtl_enskog(float(y))


def tau(mu_ref: float, b: float, n: float, T: float) -> float:
    return lib().or_tau(float(mu_ref), float(b), float(n), float(T))


def fm_density(n_rows, nx, periodic, S, i):
    """Fischer-Methfessel ball average of the density at cell i (S = sigma / dx); n_rows
    holds nx + 6 row densities (ghost rows included)."""
    n_rows = _f64(n_rows)
    assert n_rows.size == nx + 2 * NG
    return lib().or_fm_density(_ptr(n_rows), int(nx), int(bool(periodic)), float(S), int(i))


def cell_sources(p, w, n, u, T, qx, pr, y, dlnn, du, dlnT, dlnchi, nh=None):
    """Shakhov targets phi_S, theta_S and Enskog sources J1^phi, J1^theta of one cell."""
    p, w = _f64(p), _f64(w)
    q = p.size
    nh = q - 1 if nh is None else nh
    outs = [np.zeros(q) for _ in range(4)]
    lib().or_cell_sources(q, int(nh), _ptr(p), _ptr(w), *[float(v) for v in (
        n, u, T, qx, pr, y, dlnn, du, dlnT, dlnchi)], *[_ptr(o) for o in outs])
    return tuple(outs)


def moments_row(p, phi, theta):
    """(n, u, T, q, Pxx) of one cell from its quadrature-weighted phi, theta."""
    p, phi, theta = _f64(p), _f64(phi), _f64(theta)
    out = [ctypes.c_double() for _ in range(5)]
    lib().or_moments_row(p.size, _ptr(p), _ptr(phi), _ptr(theta),
                         *[ctypes.byref(o) for o in out])
    return tuple(o.value for o in out)


def central6(f, dx: float) -> np.ndarray:
    """Sixth-order central derivative at every point of f[3:-3] (App. A.3)."""
    f = _f64(f)
    out = np.zeros(f.size - 6)
    base = f.ctypes.data
    for i in range(out.size):
        ptr = ctypes.cast(base + 8 * (i + 3), _D)
        out[i] = lib().or_central6(ptr, float(dx))
    return out


def weno_weights(ind):
    ind = _f64(ind)
    out = np.zeros(3)
    lib().or_weno_weights(_ptr(ind), _ptr(out))
    return out


def weno_indicators(v):
    v = _f64(v)
    out = np.zeros(3)
    lib().or_weno_indicators(_ptr(v), _ptr(out))
    return out


def weno5(v) -> float:
    """WENO-5 reconstruction at i+1/2 from (f_{i-2}, ..., f_{i+2}) for positive velocity."""
    return lib().or_weno5(_ptr(_f64(v)))


# ---------------------------------------------------------------------------------------
# whole-domain solver
# ---------------------------------------------------------------------------------------
class Solver:
    """The FDLB solver on nx cells with Q nodes, advanced by or_step in FP64.

    b, mu_ref: covolume and dilute reference viscosity (see physics.units()).
    bc: BC_PERIODIC or BC_EQUILIBRIUM (ghost rows hold a fixed equilibrium).
    chi_mode: CHI_SET, or CHI_RETFM with molecular diameter sigma.
    """

    def __init__(self, nx, q, dx, dt, b, mu_ref, pr_mode=PR_CONST, pr=2.0 / 3.0,
                 bc=BC_PERIODIC, nh=None, chi_mode=CHI_SET, sigma=0.0):
        self.p, self.w = quadrature(q)
        self.par = _Params(int(nx), int(q), int(q - 1 if nh is None else nh), float(dx),
                           float(dt), float(b), float(mu_ref), int(pr_mode), float(pr),
                           int(bc), int(chi_mode), float(sigma))
        self.nx, self.q = nx, q
        self.phi = np.zeros((nx + 2 * NG, q))
        self.theta = np.zeros((nx + 2 * NG, q))

    def init_equilibrium(self, n_rows, u_rows, T_rows):
        """Set every row (ghosts included, nx + 6 entries each) to its local equilibrium."""
        n_rows, u_rows, T_rows = _f64(n_rows), _f64(u_rows), _f64(T_rows)
        R = self.nx + 2 * NG
        assert n_rows.size == R and u_rows.size == R and T_rows.size == R
        lib().or_init_equilibrium(ctypes.byref(self.par), _ptr(self.p), _ptr(self.w),
                                  _ptr(n_rows), _ptr(u_rows), _ptr(T_rows), _ptr(self.phi),
                                  _ptr(self.theta))

    def chi_rows(self, n_rows):
        """chi_RET-FM of every row from the row densities (nx + 6 entries)."""
        n_rows = _f64(n_rows)
        out = np.zeros(self.nx + 2 * NG)
        rc = lib().or_fm_chi(ctypes.byref(self.par), _ptr(n_rows), _ptr(out))
        if rc != 0:
            raise ValueError(f"or_fm_chi failed (code {rc})")
        return out

    def step(self, nsteps=1):
        rc = lib().or_step(ctypes.byref(self.par), _ptr(self.p), _ptr(self.w), _ptr(self.phi),
                           _ptr(self.theta), int(nsteps))
        if rc != 0:
            raise RuntimeError(f"oracle step failed (code {rc})")

    def rhs(self):
        """L[phi], L[theta] for the interior cells (ghost rows must already be filled)."""
        Lp = np.zeros((self.nx, self.q))
        Lt = np.zeros((self.nx, self.q))
        rc = lib().or_rhs(ctypes.byref(self.par), _ptr(self.p), _ptr(self.w), _ptr(self.phi),
                          _ptr(self.theta), _ptr(Lp), _ptr(Lt))
        if rc != 0:
            raise RuntimeError(f"oracle rhs failed (code {rc})")
        return Lp, Lt

    def moments(self):
        """Per interior cell: n, u, T, q_x, P_xx."""
        outs = [np.zeros(self.nx) for _ in range(5)]
        lib().or_moments(ctypes.byref(self.par), _ptr(self.p), _ptr(self.phi),
                         _ptr(self.theta), *[_ptr(o) for o in outs])
        return tuple(outs)

    def conserved(self):
        out = np.zeros(3)
        lib().or_conserved(ctypes.byref(self.par), _ptr(self.p), _ptr(self.phi),
                           _ptr(self.theta), _ptr(out))
        return out
