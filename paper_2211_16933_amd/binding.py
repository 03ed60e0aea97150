"""ctypes binding of libelb.so with the names of include/elb.h (argument marshalling only)."""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

ELB_OK, ELB_EINVAL, ELB_ENOMEM, ELB_EHIP, ELB_ENONFINITE, ELB_ESTATE, ELB_EUNSUPPORTED = range(7)
BC_PERIODIC, BC_EQUILIBRIUM = 0, 1
PR_CONST, PR_ENSKOG = 0, 1
FP64, FP32, FP32_MIXED = 0, 1, 2
CHI_SET, CHI_RETFM = 0, 1
_STATUS = ["ELB_OK", "ELB_EINVAL", "ELB_ENOMEM", "ELB_EHIP", "ELB_ENONFINITE", "ELB_ESTATE",
           "ELB_EUNSUPPORTED"]


class ElbError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        name = _STATUS[code] if 0 <= code < len(_STATUS) else str(code)
        super().__init__(f"{name}: {msg}" if msg else name)


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("q", ctypes.c_int32), ("n_herm", ctypes.c_int32),
                ("length", ctypes.c_double), ("x0", ctypes.c_double),
                ("cfl", ctypes.c_double), ("dt", ctypes.c_double),
                ("denseness", ctypes.c_double), ("kn", ctypes.c_double),
                ("kn_length", ctypes.c_double), ("n_ref", ctypes.c_double),
                ("pr_mode", ctypes.c_int32), ("pr", ctypes.c_double), ("bc", ctypes.c_int32),
                ("ghost_left", ctypes.c_double * 3), ("ghost_right", ctypes.c_double * 3),
                ("precision", ctypes.c_int32), ("closure", ctypes.c_int32),
                ("chi_mode", ctypes.c_int32), ("moment_fixup", ctypes.c_int32)]


_D = ctypes.POINTER(ctypes.c_double)
_lib = None


def library_path():
    return os.path.join(HERE, "libelb.so")


def lib():
    """Load libelb.so.  Raises if it has not been built: there is no fallback path.

    PyTorch is imported first: its HIP runtime then serves libelb.so too.  Loaded the other
    way round, the process holds two HIP runtimes and the one initialised second finds no
    device."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (see above)
        path = library_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing; build it with python -m paper_2211_16933_amd.build")
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(Params)
        vp = ctypes.c_void_p
        sig = {
            "elb_derived": (ctypes.c_int, [P, _D]),
            "elb_supported_q": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
            "elb_quadrature": (ctypes.c_int, [ctypes.c_int32, _D, _D]),
            "elb_workspace_bytes": (ctypes.c_int64, [P]),
            "elb_create": (ctypes.c_int, [P, vp, ctypes.c_int64, vp, ctypes.POINTER(vp)]),
            "elb_set_state_moments": (ctypes.c_int, [vp, _D, _D, _D]),
            "elb_set_state_dist": (ctypes.c_int, [vp, _D, _D]),
            "elb_step": (ctypes.c_int, [vp, ctypes.c_int64]),
            "elb_set_graph": (ctypes.c_int, [vp, ctypes.c_int32]),
            "elb_get_moments": (ctypes.c_int, [vp, _D, _D, _D, _D, _D]),
            "elb_get_amplitudes": (ctypes.c_int, [vp, ctypes.c_double, _D]),
            "elb_get_dist": (ctypes.c_int, [vp, _D, _D]),
            "elb_get_conserved": (ctypes.c_int, [vp, _D]),
            "elb_get_time": (ctypes.c_int, [vp, _D, ctypes.POINTER(ctypes.c_int64)]),
            "elb_last_error": (ctypes.c_char_p, [vp]),
            "elb_destroy": (ctypes.c_int, [vp]),
            "elb_batch_workspace_bytes": (ctypes.c_int64, [P, ctypes.c_int32]),
            "elb_batch_create": (ctypes.c_int, [P, ctypes.c_int32, vp, ctypes.c_int64, vp,
                                                ctypes.POINTER(vp)]),
            "elb_batch_set_state_moments": (ctypes.c_int, [vp, ctypes.c_int32, _D, _D, _D]),
            "elb_batch_step": (ctypes.c_int, [vp, ctypes.c_int64]),
            "elb_batch_set_graph": (ctypes.c_int, [vp, ctypes.c_int32]),
            "elb_batch_get_moments": (ctypes.c_int, [vp, ctypes.c_int32, _D, _D, _D, _D, _D]),
            "elb_batch_get_amplitudes": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_double, _D]),
            "elb_batch_get_dist": (ctypes.c_int, [vp, ctypes.c_int32, _D, _D]),
            "elb_batch_tune": (ctypes.c_int, [vp, ctypes.c_char_p, ctypes.c_int32]),
            "elb_batch_groups": (ctypes.c_int, [vp] + [ctypes.POINTER(ctypes.c_int32)] * 4 +
                                 [ctypes.c_int32]),
            "elb_batch_last_error": (ctypes.c_char_p, [vp]),
            "elb_batch_destroy": (ctypes.c_int, [vp]),
            "elb_mlp_param_count": (ctypes.c_int64, []),
            "elb_mlp_norm_count": (ctypes.c_int64, []),
            "elb_mlp_workspace_bytes": (ctypes.c_int64, [ctypes.c_int64]),
            "elb_mlp_forward": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.c_int64, vp, vp, vp]),
            "elb_mlp_loss": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_int64, ctypes.c_int32, vp,
                                            vp, vp, vp]),
            "elb_mlp_backward": (ctypes.c_int, [vp, vp, ctypes.c_int64, vp, vp, vp]),
            "elb_mlp_loss_noalloc": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_int64, ctypes.c_int32,
                                                    vp, vp, vp]),
            "elb_mlp_adam": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]),
            "elb_mlp_round": (ctypes.c_int, [vp, vp, vp]),
            "elb_mlp_normaliser": (ctypes.c_int, [vp, ctypes.c_int64, ctypes.c_int32,
                                                  ctypes.c_double, vp, vp, vp, vp]),
            "elb_projection": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _D]),
            "elb_rhs": (ctypes.c_int, [vp, _D, _D]),
            "elb_lift": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _D]),
            "elb_closure_lift": (ctypes.c_int, [vp, vp]),
            "elb_closure_sample": (ctypes.c_int, [vp, vp, vp, vp]),
            "elb_set_closure": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32]),
            "elb_closure_outside": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int64),
                                                   ctypes.c_int32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _ptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


def supported_q():
    buf = (ctypes.c_int32 * 32)()
    n = lib().elb_supported_q(buf, 32)
    return [buf[i] for i in range(min(n, 32))]


def quadrature(q):
    """Gauss-Hermite nodes and weights (normalised to sum 1) computed by the library."""
    p = np.zeros(q)
    w = np.zeros(q)
    rc = lib().elb_quadrature(int(q), _ptr(p), _ptr(w))
    if rc:
        raise ElbError(rc, "elb_quadrature")
    return p, w


def derived(params):
    out = np.zeros(7)
    rc = lib().elb_derived(ctypes.byref(params), _ptr(out))
    if rc:
        msg = lib().elb_last_error(None)
        raise ElbError(rc, f"elb_derived: {msg.decode() if msg else ''}")
    keys = ["dx", "dt", "b", "mu_ref", "eta0", "chi0", "n_herm"]
    return dict(zip(keys, out.tolist()))


def workspace_bytes(params):
    return int(lib().elb_workspace_bytes(ctypes.byref(params)))


def params_from_workload(w, precision=FP64, dt=0.0, n_herm=0, closure=0, moment_fixup=0):
    """elb_params of a workload dict (see workloads/__init__.py)."""
    P = Params()
    P.closure = int(closure)
    P.moment_fixup = int(moment_fixup)
    P.nx, P.q, P.n_herm = int(w["nx"]), int(w["q"]), int(n_herm)
    P.length, P.x0 = float(w["length"]), float(w["x0"])
    P.cfl, P.dt = float(w["cfl"]), float(w.get("dt", dt) or dt)
    P.denseness, P.kn = float(w["denseness"]), float(w["kn"])
    P.kn_length, P.n_ref = float(w["kn_length"]), float(w["n_ref"])
    P.pr_mode = PR_ENSKOG if w["pr_mode"] == "enskog" else PR_CONST
    P.pr = float(w["pr"])
    P.bc = BC_PERIODIC if w["bc"] == "periodic" else BC_EQUILIBRIUM
    if P.bc == BC_EQUILIBRIUM:
        for j in range(3):
            P.ghost_left[j] = float(w["left"][j])
            P.ghost_right[j] = float(w["right"][j])
    P.precision = int(precision)
    P.chi_mode = CHI_RETFM if w.get("chi", "set") == "ret" else CHI_SET
    return P


class Solver:
    """One libelb context.  The device workspace is a torch uint8 tensor on `device`, and
    work is enqueued on torch's current stream for that device (or `stream`)."""

    def __init__(self, params, device="cuda:0", stream=None):
        import torch

        self.P = params
        self.nx, self.q = params.nx, params.q
        nbytes = workspace_bytes(params)
        if nbytes < 0:
            derived(params)  # raises with the library's reason
            raise ElbError(ELB_EINVAL, "invalid parameters")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = ctypes.c_void_p()
        rc = lib().elb_create(ctypes.byref(params), ctypes.c_void_p(aligned), nbytes,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._ctx))
        if rc:
            msg = lib().elb_last_error(None)
            raise ElbError(rc, f"elb_create: {msg.decode() if msg else ''}")
        self.info = derived(params)

    def _check(self, rc, what):
        if rc:
            msg = lib().elb_last_error(self._ctx)
            raise ElbError(rc, f"{what}: {msg.decode() if msg else ''}")

    def set_state_moments(self, n, u, T):
        nx = self.nx
        n, u, T = _f64(n, nx), _f64(u, nx), _f64(T, nx)
        self._check(lib().elb_set_state_moments(self._ctx, _ptr(n), _ptr(u), _ptr(T)),
                    "elb_set_state_moments")

    def rhs(self):
        """L[phi], L[theta] of the current state ([nx][q] each; FP64 contexts)."""
        Lp = np.zeros((self.nx, self.q))
        Lt = np.zeros((self.nx, self.q))
        self._check(lib().elb_rhs(self._ctx, _ptr(Lp), _ptr(Lt)), "elb_rhs")
        return Lp, Lt

    def set_closure(self, params, norm, enabled=True):
        if not enabled:
            self._check(lib().elb_set_closure(self._ctx, None, None, 0), "elb_set_closure")
            return
        params = np.ascontiguousarray(params, dtype=np.float32)
        norm = np.ascontiguousarray(norm, dtype=np.float32)
        if params.size != mlp_param_count() or norm.size != mlp_norm_count():
            raise ValueError("closure parameters or normalisation block of the wrong size")
        # True or 1: evaluated inside the stage kernel; 2: by two kernels before each stage
        self._check(lib().elb_set_closure(self._ctx, params.ctypes.data, norm.ctypes.data,
                                          int(enabled)), "elb_set_closure")

    def closure_outside(self, reset=True):
        v = ctypes.c_int64()
        self._check(lib().elb_closure_outside(self._ctx, ctypes.byref(v), int(bool(reset))),
                    "elb_closure_outside")
        return v.value

    def set_state_dist(self, phi, theta):
        n = self.nx * self.q
        phi, theta = _f64(phi, n), _f64(theta, n)
        self._check(lib().elb_set_state_dist(self._ctx, _ptr(phi), _ptr(theta)),
                    "elb_set_state_dist")

    def step(self, nsteps=1):
        self._check(lib().elb_step(self._ctx, int(nsteps)), "elb_step")

    def set_graph(self, enabled):
        self._check(lib().elb_set_graph(self._ctx, int(bool(enabled))), "elb_set_graph")

    def moments(self):
        outs = [np.zeros(self.nx) for _ in range(5)]
        self._check(lib().elb_get_moments(self._ctx, *[_ptr(o) for o in outs]),
                    "elb_get_moments")
        return tuple(outs)

    def amplitudes(self, k):
        """(sin, cos) Fourier amplitudes of the density at wavenumber k (elb_get_amplitudes)."""
        out = np.zeros(2)
        self._check(lib().elb_get_amplitudes(self._ctx, float(k), _ptr(out)), "elb_get_amplitudes")
        return float(out[0]), float(out[1])

    def dist(self):
        phi = np.zeros((self.nx, self.q))
        theta = np.zeros((self.nx, self.q))
        self._check(lib().elb_get_dist(self._ctx, _ptr(phi), _ptr(theta)), "elb_get_dist")
        return phi, theta

    def conserved(self):
        out = np.zeros(3)
        self._check(lib().elb_get_conserved(self._ctx, _ptr(out)), "elb_get_conserved")
        return out

    def time(self):
        dt = ctypes.c_double()
        steps = ctypes.c_int64()
        self._check(lib().elb_get_time(self._ctx, ctypes.byref(dt), ctypes.byref(steps)),
                    "elb_get_time")
        return dt.value, steps.value

    def close(self):
        if self._ctx:
            lib().elb_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """A libelb batch: many independent problems stepped together.  `params_list` holds one
    Params per instance (all with the same precision)."""

    def __init__(self, params_list, device="cuda:0", stream=None):
        import torch

        self.count = len(params_list)
        self.params = (Params * self.count)(*params_list)
        self.nx = [p.nx for p in params_list]
        self.q = [p.q for p in params_list]
        nbytes = int(lib().elb_batch_workspace_bytes(self.params, self.count))
        if nbytes < 0:
            msg = lib().elb_batch_last_error(None)
            raise ElbError(ELB_EINVAL, f"invalid batch parameters: {msg.decode() if msg else ''}")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._b = ctypes.c_void_p()
        rc = lib().elb_batch_create(self.params, self.count, ctypes.c_void_p(aligned), nbytes,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._b))
        if rc:
            msg = lib().elb_batch_last_error(None)
            raise ElbError(rc, f"elb_batch_create: {msg.decode() if msg else ''}")

    def _check(self, rc, what):
        if rc:
            msg = lib().elb_batch_last_error(self._b)
            raise ElbError(rc, f"{what}: {msg.decode() if msg else ''}")

    def set_state_moments(self, inst, n, u, T):
        nx = self.nx[inst]
        n, u, T = _f64(n, nx), _f64(u, nx), _f64(T, nx)
        self._check(lib().elb_batch_set_state_moments(self._b, int(inst), _ptr(n), _ptr(u),
                                                      _ptr(T)), "elb_batch_set_state_moments")

    def step(self, nsteps=1):
        self._check(lib().elb_batch_step(self._b, int(nsteps)), "elb_batch_step")

    def set_graph(self, enabled):
        self._check(lib().elb_batch_set_graph(self._b, int(bool(enabled))), "elb_batch_set_graph")

    def moments(self, inst):
        outs = [np.zeros(self.nx[inst]) for _ in range(5)]
        self._check(lib().elb_batch_get_moments(self._b, int(inst), *[_ptr(o) for o in outs]),
                    "elb_batch_get_moments")
        return tuple(outs)

    def amplitudes(self, inst, k):
        """(sin, cos) Fourier amplitudes of instance inst's density at wavenumber k."""
        out = np.zeros(2)
        self._check(lib().elb_batch_get_amplitudes(self._b, int(inst), float(k), _ptr(out)),
                    "elb_batch_get_amplitudes")
        return float(out[0]), float(out[1])

    def dist(self, inst):
        phi = np.zeros((self.nx[inst], self.q[inst]))
        theta = np.zeros((self.nx[inst], self.q[inst]))
        self._check(lib().elb_batch_get_dist(self._b, int(inst), _ptr(phi), _ptr(theta)),
                    "elb_batch_get_dist")
        return phi, theta

    def tune(self, cache_path=None, force=False):
        path = cache_path.encode() if cache_path else None
        self._check(lib().elb_batch_tune(self._b, path, int(bool(force))), "elb_batch_tune")

    def groups(self):
        cap = max(self.count, 1)             # every group holds at least one instance
        arrs = [(ctypes.c_int32 * cap)() for _ in range(4)]
        n = lib().elb_batch_groups(self._b, *arrs, cap)
        return [{"q": arrs[0][i], "strips": arrs[1][i], "strip_len": arrs[2][i],
                 "items": arrs[3][i]} for i in range(min(n, cap))]

    def close(self):
        if self._b:
            lib().elb_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------------------
# learned closure
# ---------------------------------------------------------------------------------------
def mlp_param_count():
    return int(lib().elb_mlp_param_count())


def mlp_norm_count():
    return int(lib().elb_mlp_norm_count())


def mlp_workspace_bytes(batch):
    return int(lib().elb_mlp_workspace_bytes(int(batch)))


def projection(q_from, q_to):
    P = np.zeros((q_to, q_from))
    rc = lib().elb_projection(int(q_from), int(q_to), _ptr(P))
    if rc:
        raise ElbError(rc, "elb_projection")
    return P


def lift(q_from, q_to):
    """Lift matrix [q_to][q_from] of elb_lift."""
    L = np.zeros((q_to, q_from))
    rc = lib().elb_lift(int(q_from), int(q_to), _ptr(L))
    if rc:
        raise ElbError(rc, "elb_lift")
    return L


def closure_lift(student, teacher):
    """elb_closure_lift: the teacher's interior state becomes the lift of the student's."""
    rc = lib().elb_closure_lift(student._ctx, teacher._ctx)
    if rc:
        raise ElbError(rc, "elb_closure_lift: " + lib().elb_last_error(teacher._ctx).decode())


def mlp_normaliser(x, margin=0.0):
    """(mean, std, lo, hi) of the columns of x [n][dim] (FP32), as elb_mlp_normaliser."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    n, dim = x.shape
    outs = [np.zeros(dim, dtype=np.float32) for _ in range(4)]
    rc = lib().elb_mlp_normaliser(x.ctypes.data, n, dim, float(margin),
                                  *[o.ctypes.data for o in outs])
    if rc:
        raise ElbError(rc, "elb_mlp_normaliser")
    return tuple(outs)


def closure_sample(teacher, student):
    """x [nx][12], y [nx][q_student] for the teacher's current state (both FP64 Solvers)."""
    x = np.zeros((student.nx, 12), dtype=np.float32)
    y = np.zeros((student.nx, student.q), dtype=np.float32)
    rc = lib().elb_closure_sample(teacher._ctx, student._ctx, x.ctypes.data, y.ctypes.data)
    if rc:
        msg = lib().elb_last_error(student._ctx)
        raise ElbError(rc, f"elb_closure_sample: {msg.decode() if msg else ''}")
    return x, y


def _dp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def mlp_forward(params, wb, norm, x, index, batch, y, ws, stream=None):
    rc = lib().elb_mlp_forward(_dp(params), _dp(wb), _dp(norm), _dp(x), _dp(index), int(batch),
                               _dp(y), _dp(ws), _stream(stream))
    if rc:
        raise ElbError(rc, "elb_mlp_forward")


def mlp_loss(y, t, index, norm, batch, q_out, dy, loss, ws, stream=None):
    rc = lib().elb_mlp_loss(_dp(y), _dp(t), _dp(index), _dp(norm), int(batch), int(q_out),
                            _dp(dy), _dp(loss), _dp(ws), _stream(stream))
    if rc:
        raise ElbError(rc, "elb_mlp_loss")


def mlp_loss_noalloc(y, t, index, norm, batch, q_out, dy, loss, stream=None):
    """elb_mlp_loss without a workspace (the library's static device scratch)."""
    rc = lib().elb_mlp_loss_noalloc(_dp(y), _dp(t), _dp(index), _dp(norm), int(batch), int(q_out),
                                    _dp(dy), _dp(loss), _stream(stream))
    if rc:
        raise ElbError(rc, "elb_mlp_loss_noalloc: " + lib().elb_last_error(None).decode())


def mlp_backward(wb, dy, batch, grad, ws, stream=None):
    rc = lib().elb_mlp_backward(_dp(wb), _dp(dy), int(batch), _dp(grad), _dp(ws),
                                _stream(stream))
    if rc:
        raise ElbError(rc, "elb_mlp_backward")


def mlp_adam(params, wb, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
             stream=None):
    rc = lib().elb_mlp_adam(_dp(params), _dp(wb), _dp(m), _dp(v), _dp(grad), int(step),
                            float(lr), float(beta1), float(beta2), float(eps), _stream(stream))
    if rc:
        raise ElbError(rc, "elb_mlp_adam")


def mlp_round(params, wb, stream=None):
    rc = lib().elb_mlp_round(_dp(params), _dp(wb), _stream(stream))
    if rc:
        raise ElbError(rc, "elb_mlp_round")
