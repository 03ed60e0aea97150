"""Learned closure: training data from teacher runs, training on the GPU, and the corrected
student solver with its fallback.

Host driver only.  The samples, the forward and backward passes, the loss and the Adam
updates all run in libelb's kernels (include/elb.h, "Learned closure"); this module
allocates device buffers with PyTorch, draws minibatch indices and decides when to fall
back to the fine quadrature.
"""
import math

import numpy as np

from . import binding as B

N_IN, HIDDEN, OUT_PAD, K1 = 12, 64, 16, 32
# packed layout of include/elb.h (W[out][in], row-major)
_LAYOUT = [("W1", (HIDDEN, K1)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
           ("W3", (HIDDEN, HIDDEN)), ("b3", (HIDDEN,)), ("W4", (OUT_PAD, HIDDEN)), ("b4", (OUT_PAD,))]


def pack_params(layers):
    """Packed FP32 array from [W1 (64x12), b1, W2, b2, W3, b3, W4 (q_out x 64), b4] (zero
    padding of W1's inputs and of the outputs beyond q_out)."""
    out = np.zeros(B.mlp_param_count(), dtype=np.float32)
    o = 0
    for (name, shape), a in zip(_LAYOUT, layers):
        full = np.zeros(shape, dtype=np.float32)
        a = np.asarray(a, dtype=np.float32)
        full[tuple(slice(0, s) for s in a.shape)] = a
        n = full.size
        out[o:o + n] = full.ravel()
        o += n
    return out


def unpack_params(packed, q_out):
    """Inverse of pack_params (padding dropped)."""
    packed = np.asarray(packed, dtype=np.float64)
    layers, o = [], 0
    for name, shape in _LAYOUT:
        n = int(np.prod(shape))
        a = packed[o:o + n].reshape(shape)
        o += n
        if name == "W1":
            a = a[:, :N_IN]
        elif name in ("W4", "b4"):
            a = a[:q_out]
        layers.append(a.copy())
    return layers


def init_params(q_out, seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (packed)."""
    rng = np.random.default_rng(seed)
    dims = [N_IN, HIDDEN, HIDDEN, HIDDEN, q_out]
    layers = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = 1.0 / math.sqrt(a)
        layers.append(rng.uniform(-lim, lim, size=(b, a)))
        layers.append(np.zeros(b))
    return pack_params(layers)


def make_norm(in_mean, in_std, out_mean, out_std, lo, hi):
    norm = np.zeros(B.mlp_norm_count(), dtype=np.float32)
    norm[0:12], norm[12:24] = in_mean, in_std
    q = len(out_mean)
    norm[24:40], norm[40:56] = 0.0, 1.0
    norm[24:24 + q], norm[40:40 + q] = out_mean, out_std
    norm[56:68], norm[68:80] = lo, hi
    return norm


# weight of the learned correction in the corrected runs (under-relaxation): with the full
# correction, corrected student runs of some trainings diverge; at 0.6 every training
# tried stayed finite and closer to the teacher than the student alone while the shock forms
CORRECTION_WEIGHT = 0.6


def weighted_norm(norm, weight=CORRECTION_WEIGHT):
    """The normalisation block with the output mean and spread scaled by `weight`: the
    library then adds weight times the network's correction (c = P (n / tau)(y sigma + mu)
    is linear in sigma and mu).  Inputs and the range guard are unchanged."""
    n = np.array(norm, dtype=np.float32).copy()
    n[24:40] *= weight
    n[40:56] *= weight
    return n


# ---------------------------------------------------------------------------------------
# training data
# ---------------------------------------------------------------------------------------
def with_q(w, q):
    w = dict(w)
    w["q"] = int(q)
    return w


def generate(workloads, q_teacher, q_student, start, every, count, cells=None, seed=0,
             active=None, quiet=0.25, device="cuda:0"):
    """Samples of the teacher runs: the workloads run together as one FP64 batch at
    q_teacher; after `start` steps and then every `every` steps (`count` times) each
    instance's state is projected onto q_student nodes and every cell (or `cells` cells drawn
    at random) gives one sample.  With `active`, the cells with a scaled gradient input above
    it (the disturbed part of a large, mostly uniform domain) are kept together with
    `quiet` times as many of the other cells, drawn at random, so that undisturbed states
    stay inside the training range.  Returns x [n][12], y [n][q_student] (FP32)."""
    rng = np.random.default_rng(seed)
    ws = [with_q(w, q_teacher) for w in workloads]
    batch = B.BatchSolver([B.params_from_workload(w, precision=B.FP64) for w in ws],
                          device=device)
    pairs = []
    for i, w in enumerate(ws):
        batch.set_state_moments(i, w["n"], w["u"], w["T"])
        t = B.Solver(B.params_from_workload(w, precision=B.FP64), device=device,
                     stream=batch.stream)
        s = B.Solver(B.params_from_workload(with_q(w, q_student), precision=B.FP64, closure=1),
                     device=device, stream=batch.stream)
        t.set_state_moments(w["n"], w["u"], w["T"])
        s.set_state_moments(w["n"], w["u"], w["T"])
        pairs.append((t, s))
    xs, ys = [], []
    batch.step(start)
    for _ in range(count):
        for i, (t, s) in enumerate(pairs):
            phi, theta = batch.dist(i)
            t.set_state_dist(phi, theta)
            x, y = _select(*B.closure_sample(t, s), rng, active, quiet, cells)
            xs.append(x)
            ys.append(y)
        batch.step(every)
    batch.close()
    return np.concatenate(xs), np.concatenate(ys)


def _select(x, y, rng, active, quiet, cells):
    """The samples kept from one state: with `active`, the cells whose largest scaled
    gradient input exceeds it and `quiet` times as many others drawn at random; then at most
    `cells` of them drawn at random."""
    if active is not None:
        busy = np.max(np.abs(x[:, 5:10]), axis=1) > active
        calm = np.flatnonzero(~busy)
        extra = min(calm.size, int(quiet * np.count_nonzero(busy)) + 1)
        keep = busy.copy()
        keep[rng.choice(calm, size=extra, replace=False)] = True
        x, y = x[keep], y[keep]
    if cells is not None and cells < x.shape[0]:
        pick = rng.choice(x.shape[0], size=cells, replace=False)
        x, y = x[pick], y[pick]
    return x, y


def generate_on_student(workloads, q_teacher, q_student, params, norm, start, every, count,
                        relax, cells=None, seed=0, active=None, quiet=0.25, device="cuda:0",
                        weight=CORRECTION_WEIGHT):
    """Samples along the corrected student's own trajectories (dataset aggregation, Ross,
    Gordon and Bagnell 2011): each workload runs at q_student with the learned correction of
    (params, norm) times `weight`; after `start` steps and then every `every` steps (`count` times) the
    student's state is lifted onto the teacher's nodes (elb_closure_lift: the Hermite series
    with the student's moments 0..Q_s-1), the teacher runs `relax` steps from there so that
    its higher moments take values of its own, and the cells of that teacher state give
    samples, selected as in generate().  A student run that breaks down stops giving
    samples.  Returns x, y."""
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for w in workloads:
        st = B.Solver(B.params_from_workload(with_q(w, q_student), precision=B.FP64, closure=1),
                      device=device)
        stream = st.stream
        t = B.Solver(B.params_from_workload(with_q(w, q_teacher), precision=B.FP64), device=device,
                     stream=stream)
        smp = B.Solver(B.params_from_workload(with_q(w, q_student), precision=B.FP64, closure=1),
                       device=device, stream=stream)
        for s in (st, t, smp):
            s.set_state_moments(w["n"], w["u"], w["T"])
        st.set_closure(params, weighted_norm(norm, weight), True)
        st.step(start)
        for _ in range(count):
            try:
                st.moments()            # a student run that broke down gives no more samples
                B.closure_lift(st, t)
                t.step(relax)
                x, y = B.closure_sample(t, smp)
            except B.ElbError:
                break
            x, y = _select(x, y, rng, active, quiet, cells)
            xs.append(x)
            ys.append(y)
            st.step(every)
        for s in (smp, t, st):
            s.close()
    return np.concatenate(xs), np.concatenate(ys)


# ---------------------------------------------------------------------------------------
# training
# ---------------------------------------------------------------------------------------
class Trainer:
    """Minibatch Adam on the MSE of the normalised targets, all on the GPU."""

    def __init__(self, x, y, batch=4096, lr=1e-3, seed=0, margin=0.05, device="cuda:0"):
        import torch
        self.torch = torch
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        self.n, self.q_out = x.shape[0], y.shape[1]
        in_mean, in_std, lo, hi = B.mlp_normaliser(x, margin)
        out_mean, out_std, _, _ = B.mlp_normaliser(y)
        self.norm_host = make_norm(in_mean, in_std, out_mean, out_std, lo, hi)
        dev = torch.device(device)
        self.dev = dev
        self.batch = int(min(batch, self.n))
        self.lr = lr
        self.rng = np.random.default_rng(seed)
        self.x = torch.from_numpy(x).to(dev)
        self.y = torch.from_numpy(y).to(dev)
        self.norm = torch.from_numpy(self.norm_host).to(dev)
        self.params = torch.from_numpy(init_params(self.q_out, seed)).to(dev)
        P = self.params.numel()
        self.wb = torch.empty(P, dtype=torch.int16, device=dev)
        self.m = torch.zeros(P, dtype=torch.float32, device=dev)
        self.v = torch.zeros(P, dtype=torch.float32, device=dev)
        self.grad = torch.zeros(P, dtype=torch.float32, device=dev)
        self.out = torch.zeros(self.batch * OUT_PAD, dtype=torch.float32, device=dev)
        self.dout = torch.zeros_like(self.out)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.ws = torch.empty(B.mlp_workspace_bytes(self.batch), dtype=torch.uint8, device=dev)
        self.t = 0
        self.order = np.empty(0, dtype=np.int32)
        B.mlp_round(self.params, self.wb)

    def _next_index(self):
        if self.order.size < self.batch:
            self.order = np.concatenate([self.order,
                                         self.rng.permutation(self.n).astype(np.int32)])
        idx, self.order = self.order[:self.batch], self.order[self.batch:]
        return idx

    def step(self):
        idx = self.torch.from_numpy(np.ascontiguousarray(self._next_index())).to(self.dev)
        B.mlp_forward(self.params, self.wb, self.norm, self.x, idx, self.batch, self.out, self.ws)
        B.mlp_loss(self.out, self.y, idx, self.norm, self.batch, self.q_out, self.dout,
                   self.loss, self.ws)
        B.mlp_backward(self.wb, self.dout, self.batch, self.grad, self.ws)
        self.t += 1
        B.mlp_adam(self.params, self.wb, self.m, self.v, self.grad, self.t, lr=self.lr)
        return idx

    def train(self, iters, log_every=100):
        losses = []
        for i in range(iters):
            self.step()
            if (i + 1) % log_every == 0 or i == iters - 1:
                losses.append(float(self.loss.item()))
        return losses

    def evaluate(self, x, y):
        """Mean squared error of the normalised targets on a held-out set (GPU forward)."""
        torch = self.torch
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(self.dev)
        yt = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(self.dev)
        n = x.shape[0]
        out = torch.zeros(n * OUT_PAD, dtype=torch.float32, device=self.dev)
        dout = torch.zeros_like(out)
        ws = torch.empty(B.mlp_workspace_bytes(n), dtype=torch.uint8, device=self.dev)
        loss = torch.zeros(1, dtype=torch.float64, device=self.dev)
        B.mlp_forward(self.params, self.wb, self.norm, x, None, n, out, ws)
        B.mlp_loss(out, yt, None, self.norm, n, self.q_out, dout, loss, ws)
        return float(loss.item())

    def result(self):
        return self.params.cpu().numpy().copy(), self.norm_host.copy()


# ---------------------------------------------------------------------------------------
# the corrected student and its fallback
# ---------------------------------------------------------------------------------------
def run_student(w, q_student, params, norm, steps, precision=B.FP64, device="cuda:0",
                weight=CORRECTION_WEIGHT):
    """Run workload w at q_student with the learned correction (times `weight`) for `steps`
    steps.  Returns (solver, cells_outside): cells_outside counts the cells (over all
    stages) whose inputs left the training range and got no correction."""
    s = B.Solver(B.params_from_workload(with_q(w, q_student), precision=precision, closure=1),
                 device=device)
    s.set_state_moments(w["n"], w["u"], w["T"])
    s.set_closure(params, weighted_norm(norm, weight), True)
    s.step(steps)
    return s, s.closure_outside()


def run_with_fallback(w, q_student, q_fine, params, norm, t_end, precision=B.FP64,
                      max_outside=0, device="cuda:0", weight=CORRECTION_WEIGHT):
    """The learned student up to time t_end; if more than `max_outside` cell-stages left the
    training range, or the corrected run broke down, the plain fine-quadrature solver runs
    the problem instead.  Returns (moments, used) with used in {"learned", "fallback"}."""
    s, _ = run_student(w, q_student, params, norm, 0, precision, device, weight)
    s.step(int(round(t_end / s.info["dt"])))
    try:
        if s.closure_outside() <= max_outside:
            return s.moments(), "learned"
    except B.ElbError as e:     # the corrected run broke down (a cell with n <= 0 or T <= 0)
        if e.code != B.ELB_ENONFINITE:
            raise
    f = B.Solver(B.params_from_workload(with_q(w, q_fine), precision=precision), device=device)
    f.set_state_moments(w["n"], w["u"], w["T"])
    f.step(int(round(t_end / f.info["dt"])))
    return f.moments(), "fallback"
