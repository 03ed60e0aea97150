"""FP64 reference of the learned closure: projection between quadratures, closure features
and targets, the MLP with its gradients, Adam, and the corrected RK3 step.

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may use this module.  It shares no code with the GPU library.

The closure is an addition to the method.  The paper's parts are the moments, the Hermite
expansion and the Gauss-Hermite quadrature it is built on (Sec. II.D).  A coarse
"student" quadrature with Q_s nodes carries Hermite moments 0..Q_s-1 of the distribution.
A small network predicts, from local moments and their gradients, the part of the
right-hand side L[phi] that a fine "teacher" quadrature sees but the student misses:

  r = Pi L_T[f_T] - L_s[Pi f_T]                      (phi component only)

where Pi maps teacher values to student values with the same Hermite moments 0..Q_s-1.
The correction added to the student's L[phi] is projected so that it carries no mass,
momentum or energy: sum_k c_k {1, p_k, p_k^2} = 0.

Network: 12 inputs -> 64 -> 64 -> 64 (SiLU) -> Q_s outputs.  Weights and the inputs of
every layer are rounded to bfloat16 (round to nearest even), products are accumulated
exactly here (FP32 on the GPU) and biases are added unrounded.  `emulate=False` turns the
rounding off (for finite-difference checks of the gradients).
"""
import math

import numpy as np

from . import NG, quadrature, hermite, moments_row, central6, tau as or_tau

N_IN = 12
HIDDEN = 64


# ---------------------------------------------------------------------------------------
# projection between quadratures (Sec. II.D: Hermite moments on Gauss-Hermite nodes)
# ---------------------------------------------------------------------------------------
def projection_matrix(q_from, q_to):
    """Pi[j][k] such that f_s = Pi f_T has the same Hermite moments
    M_l = sum_k He_l(p_k) f_k, l = 0..q_to-1, as f_T.  The student values are the
    truncated Hermite series f_s,j = w_j sum_{l<q_to} He_l(p_j) M_l / l!."""
    pT, _ = quadrature(q_from)
    ps, ws = quadrature(q_to)
    HT = np.array([[hermite(l, x) for x in pT] for l in range(q_to)])        # [l][k]
    Hs = np.array([[hermite(l, x) for x in ps] for l in range(q_to)])        # [l][j]
    fact = np.array([math.factorial(l) for l in range(q_to)], dtype=np.float64)
    return (ws[:, None] * Hs.T / fact[None, :]) @ HT


def lift_matrix(q_from, q_to):
    """Lam[k][j]: the values on the q_to nodes P_k of the truncated Hermite series
    W_k sum_{l<q_from} He_l(P_k) M_l / l! whose moments M_l, l = 0..q_from-1, are those of a
    state on the q_from nodes p_j (the lift of a coarse state onto finer nodes)."""
    ps, _ = quadrature(q_from)
    pT, wT = quadrature(q_to)
    Hs = np.array([[hermite(l, x) for x in ps] for l in range(q_from)])      # [l][j]
    HT = np.array([[hermite(l, x) for x in pT] for l in range(q_from)])      # [l][k]
    fact = np.array([math.factorial(l) for l in range(q_from)], dtype=np.float64)
    return (wT[:, None] * HT.T / fact[None, :]) @ Hs


def conservative_projector(p):
    """I - V (V^T V)^{-1} V^T with V = [1, p, p^2]: removes every component that carries
    mass, momentum or energy."""
    p = np.asarray(p, dtype=np.float64)
    V = np.stack([np.ones_like(p), p, p * p], axis=1)
    return np.eye(p.size) - V @ np.linalg.solve(V.T @ V, V.T)


# ---------------------------------------------------------------------------------------
# features and target
# ---------------------------------------------------------------------------------------
def row_moments(p, phi_rows, theta_rows):
    """(n, u, T, q, Pxx) of every row (ghost rows included)."""
    return np.array([moments_row(p, phi_rows[r], theta_rows[r])
                     for r in range(phi_rows.shape[0])]).T


def features(p, phi_rows, theta_rows, dx, b, mu_ref, denseness, kn):
    """The 12 closure inputs of every interior cell from rows that include the 3 ghost
    rows per side:  n, u, T, q/(n T^1.5), Pxx/(n T) - 1, then the sixth-order central
    x-derivatives (App. A.3) of n, u, T, q, Pxx scaled by the local relaxation length
    lambda = tau sqrt(T) and by n, sqrt(T), T, n T^1.5, n T respectively, then E_l and
    log10(Kn).  Also returns n / tau per cell (the scale of the target)."""
    n, u, T, q, pxx = row_moments(p, phi_rows, theta_rows)
    s = slice(NG, n.size - NG)
    ni, ui, Ti, qi, pi = n[s], u[s], T[s], q[s], pxx[s]
    tau = np.array([or_tau(mu_ref, b, a, c) for a, c in zip(ni, Ti)])
    lam = tau * np.sqrt(Ti)
    qs = ni * Ti ** 1.5
    x = np.zeros((ni.size, N_IN))
    x[:, 0], x[:, 1], x[:, 2] = ni, ui, Ti
    x[:, 3] = qi / qs
    x[:, 4] = pi / (ni * Ti) - 1.0
    x[:, 5] = lam * central6(n, dx) / ni
    x[:, 6] = lam * central6(u, dx) / np.sqrt(Ti)
    x[:, 7] = lam * central6(T, dx) / Ti
    x[:, 8] = lam * central6(q, dx) / qs
    x[:, 9] = lam * central6(pxx, dx) / (ni * Ti)
    x[:, 10] = denseness
    x[:, 11] = math.log10(kn)
    return x, ni / tau


def project_rows(Pi, rows):
    return rows @ Pi.T


def sample(teacher, student, denseness, kn):
    """Closure inputs and scaled targets of every interior cell for the teacher's current
    state (an oracle Solver with filled ghost rows).  The student Solver (same grid and
    physics, Q_s nodes) is set to the projected state.  Target: y = r tau / n with
    r = Pi L_T[phi_T] - L_s[Pi f_T]."""
    Pi = projection_matrix(teacher.q, student.q)
    student.phi = np.ascontiguousarray(project_rows(Pi, teacher.phi))
    student.theta = np.ascontiguousarray(project_rows(Pi, teacher.theta))
    LT, _ = teacher.rhs()
    Ls, _ = student.rhs()
    r = project_rows(Pi, LT) - Ls
    par = student.par
    x, sc = features(student.p, student.phi, student.theta, par.dx, par.b, par.mu_ref,
                     denseness, kn)
    return x, r / sc[:, None]


# ---------------------------------------------------------------------------------------
# bfloat16 rounding and the network
# ---------------------------------------------------------------------------------------
def bf16(x):
    """Round to the nearest bfloat16 (ties to even) after rounding to FP32, as the GPU
    rounds its FP32 values; returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(q_out, seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and zero biases."""
    rng = np.random.default_rng(seed)
    dims = [N_IN, HIDDEN, HIDDEN, HIDDEN, q_out]
    out = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = 1.0 / math.sqrt(a)
        out.append(rng.uniform(-lim, lim, size=(b, a)))
        out.append(np.zeros(b))
    return out


def _r(x, emulate):
    return bf16(x) if emulate else np.asarray(x, dtype=np.float64)


def mlp_forward(params, x, emulate=True):
    """y = W4 a3 + b4 with a_l = SiLU(W_l a_{l-1} + b_l); x is [batch][12].  Returns y and
    the cache (rounded layer inputs and pre-activations) used by mlp_backward."""
    W = [_r(params[2 * i], emulate) for i in range(4)]
    bias = [np.asarray(params[2 * i + 1], dtype=np.float64) for i in range(4)]
    a = _r(x, emulate)
    acts, zs = [a], []
    for l in range(4):
        z = a @ W[l].T + bias[l]
        zs.append(z)
        if l < 3:
            a = _r(silu(z), emulate)
            acts.append(a)
    return zs[3], {"W": W, "acts": acts, "zs": zs, "emulate": emulate}


def mlp_backward(cache, dy):
    """Gradients of sum(dy * y) with respect to every weight and bias (the same order as
    the parameter list).  Layer gradients flow through the rounded weights; the
    back-propagated signal is rounded before each product, as on the GPU."""
    W, acts, zs, em = cache["W"], cache["acts"], cache["zs"], cache["emulate"]
    grads = [None] * 8
    dz = np.asarray(dy, dtype=np.float64)
    for l in range(3, -1, -1):
        dzr = _r(dz, em)
        grads[2 * l] = dzr.T @ acts[l]
        grads[2 * l + 1] = dz.sum(axis=0)
        if l > 0:
            da = dzr @ W[l]
            dz = da * dsilu(zs[l - 1])
    return grads


def mse_grad(y, t):
    """Loss mean((y - t)^2) over batch and outputs, and its gradient with respect to y."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) of w with gradient g at step t >= 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------------------
# the corrected student step
# ---------------------------------------------------------------------------------------
class Closure:
    """A trained network with its normalisation: inputs x -> (x - in_mean) / in_std, outputs
    y -> y * out_std + out_mean, correction c = P (n/tau) y on cells whose normalised
    inputs lie inside [lo, hi], zero elsewhere."""

    def __init__(self, params, in_mean, in_std, out_mean, out_std, lo, hi, p_student):
        self.params = params
        self.in_mean, self.in_std = np.asarray(in_mean), np.asarray(in_std)
        self.out_mean, self.out_std = np.asarray(out_mean), np.asarray(out_std)
        self.lo, self.hi = np.asarray(lo), np.asarray(hi)
        self.P = conservative_projector(p_student)

    def correction(self, x, scale):
        xn = (x - self.in_mean) / self.in_std
        inside = np.all((xn >= self.lo) & (xn <= self.hi), axis=1)
        y, _ = mlp_forward(self.params, xn)
        y = y * self.out_std + self.out_mean
        c = (scale[:, None] * y) @ self.P.T
        c[~inside] = 0.0
        return c, int((~inside).sum())


def corrected_step(solver, closure, denseness, kn, nsteps=1, periodic=True):
    """SSP-RK3 (App. A.1) of an oracle Solver whose L[phi] gets the closure correction of
    its current stage state.  Ghost rows: periodic copies, or held fixed."""
    p = solver.p
    par = solver.par

    def fill(a):
        if periodic:
            a[:NG] = a[-2 * NG:-NG]
            a[-NG:] = a[NG:2 * NG]

    def L(phi, th):
        fill(phi)
        fill(th)
        solver.phi, solver.theta = phi, th
        Lp, Lt = solver.rhs()
        x, sc = features(p, phi, th, par.dx, par.b, par.mu_ref, denseness, kn)
        c, _ = closure.correction(x, sc)
        return Lp + c, Lt

    dt = par.dt
    s = slice(NG, solver.nx + NG)
    for _ in range(nsteps):
        f0p, f0t = solver.phi.copy(), solver.theta.copy()
        Lp, Lt = L(f0p.copy(), f0t.copy())
        f1p, f1t = f0p.copy(), f0t.copy()
        f1p[s] += dt * Lp
        f1t[s] += dt * Lt
        Lp, Lt = L(f1p.copy(), f1t.copy())
        f2p, f2t = f0p.copy(), f0t.copy()
        f2p[s] = 0.75 * f0p[s] + 0.25 * f1p[s] + 0.25 * dt * Lp
        f2t[s] = 0.75 * f0t[s] + 0.25 * f1t[s] + 0.25 * dt * Lt
        Lp, Lt = L(f2p.copy(), f2t.copy())
        outp, outt = f0p.copy(), f0t.copy()
        outp[s] = f0p[s] / 3.0 + 2.0 * f2p[s] / 3.0 + 2.0 * dt * Lp / 3.0
        outt[s] = f0t[s] / 3.0 + 2.0 * f2t[s] / 3.0 + 2.0 * dt * Lt / 3.0
        fill(outp)
        fill(outt)
        solver.phi, solver.theta = outp, outt
