"""Learned closure on the GPU against the FP64 oracle (needs an MI355X).

The network runs on bfloat16 matrix cores with FP32 accumulation; the oracle rounds the
weights and every layer input to bfloat16 at the same points and accumulates exactly.  The
two then differ by the FP32 accumulation order and by the rare activations whose FP32
value sits so close to a bfloat16 rounding boundary that the two sides round it to
neighbouring values (2^-8 relative).  The tolerances below bound those effects."""
import numpy as np
import pytest

import oracle
from oracle import closure as cl
from oracle.run import solver_from_workload
import workloads
from helpers import say, rel_l2, gpu_solver

pytestmark = pytest.mark.gpu

FP64, FP32, FP32_MIXED = 0, 1, 2


def _net(q_out, seed, scale=0.15):
    rng = np.random.default_rng(seed)
    layers = cl.init_params(q_out, seed)
    return [(a + scale * rng.normal(size=a.shape)).astype(np.float32).astype(np.float64)
            for a in layers]


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda:0") if dtype is None else t.to("cuda:0", dtype)


def _norm(rng, q_out):
    from paper_2211_16933_amd import learned
    return learned.make_norm(rng.uniform(-0.5, 0.5, 12), rng.uniform(0.5, 2.0, 12),
                             rng.uniform(-0.2, 0.2, q_out), rng.uniform(0.5, 2.0, q_out),
                             -np.full(12, 50.0), np.full(12, 50.0))


@pytest.mark.parametrize("q_out,batch", [(8, 300), (12, 1000)])
def test_mlp_forward_loss_backward_match_oracle(q_out, batch):
    import torch
    import paper_2211_16933_amd as elb
    from paper_2211_16933_amd import learned
    rng = np.random.default_rng(q_out)
    layers = _net(q_out, seed=q_out)
    norm = _norm(rng, q_out)
    rows = batch + 37
    x = rng.normal(size=(rows, 12)).astype(np.float32)
    t = rng.normal(size=(rows, q_out)).astype(np.float32)
    index = rng.permutation(rows)[:batch].astype(np.int32)
    say(f"case mlp q_out={q_out} batch={batch}")

    params = _dev(learned.pack_params(layers))
    wb = torch.empty(params.numel(), dtype=torch.int16, device="cuda:0")
    elb.mlp_round(params, wb)
    y = torch.zeros(batch * 16, dtype=torch.float32, device="cuda:0")
    dy = torch.zeros_like(y)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    grad = torch.zeros_like(params)
    ws = torch.empty(elb.mlp_workspace_bytes(batch), dtype=torch.uint8, device="cuda:0")
    xd, td, nd, idd = _dev(x), _dev(t), _dev(norm), _dev(index)
    elb.mlp_forward(params, wb, nd, xd, idd, batch, y, ws)
    elb.mlp_loss(y, td, idd, nd, batch, q_out, dy, loss, ws)
    elb.mlp_backward(wb, dy, batch, grad, ws)
    torch.cuda.synchronize()

    # the bfloat16 copy is the round-to-nearest-even of the FP32 parameters
    wb_h = wb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    assert np.array_equal(wb_h.view(np.float32).astype(np.float64),
                          cl.bf16(learned.pack_params(layers)))

    # oracle: the same normalisation in FP32, then the bfloat16-emulating network
    xn = ((x[index] - norm[:12]) / norm[12:24]).astype(np.float64)
    yo, cache = cl.mlp_forward(layers, xn)
    tn = ((t[index] - norm[24:24 + q_out]) / norm[40:40 + q_out]).astype(np.float64)
    lo, go = cl.mse_grad(yo, tn)
    grads = cl.mlp_backward(cache, go)

    yg = y.cpu().numpy().reshape(batch, 16)
    e_y = rel_l2(yg[:, :q_out], yo)
    assert np.all(yg[:, q_out:] == 0.0)
    e_loss = abs(loss.item() - lo) / lo
    dyg = dy.cpu().numpy().reshape(batch, 16)
    e_dy = rel_l2(dyg[:, :q_out], go)
    gg = learned.unpack_params(grad.cpu().numpy(), q_out)
    e_g = [rel_l2(a, b) for a, b in zip(gg, grads)]
    say(f"  y {e_y:.1e} loss {e_loss:.1e} dy {e_dy:.1e} grads " + " ".join(f"{v:.1e}" for v in e_g))
    # measured: y 3-7e-5, loss <= 1e-6, dy <= 2e-5, gradients <= 5e-5.  A flip moves one
    # activation by 2^-8 of itself; 5e-4 relative L2 allows flips in about 1 % of the
    # activations, several times what bfloat16 boundary cases produce
    assert e_y <= 5e-4 and e_loss <= 1e-4 and e_dy <= 5e-4
    assert max(e_g) <= 5e-4
    # padded parameters get no gradient
    full = grad.cpu().numpy()
    assert np.all(full[0:64 * 32].reshape(64, 32)[:, 12:] == 0.0)


def test_adam_matches_oracle():
    import torch
    import paper_2211_16933_amd as elb
    rng = np.random.default_rng(9)
    P = elb.mlp_param_count()
    w0 = rng.normal(size=P).astype(np.float32)
    g = (rng.normal(size=P) * 10.0 ** rng.uniform(-6, 1, P)).astype(np.float32)
    w, m, v = _dev(w0), torch.zeros(P, device="cuda:0"), torch.zeros(P, device="cuda:0")
    wb = torch.empty(P, dtype=torch.int16, device="cuda:0")
    gd = _dev(g)
    wo, mo, vo = w0.astype(np.float64), np.zeros(P), np.zeros(P)
    for step in range(1, 4):
        elb.mlp_adam(w, wb, m, v, gd, step, lr=1e-3)
        wo, mo, vo = cl.adam_step(wo, mo, vo, g.astype(np.float64), step, lr=1e-3)
    torch.cuda.synchronize()
    wg = w.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(wg - wo)) <= 1e-6 * np.max(np.abs(wo))
    assert np.max(np.abs((wg - w0) - (wo - w0))) <= 1e-3 * np.max(np.abs(wo - w0))
    wb_h = (wb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(wb_h.astype(np.float64), cl.bf16(wg))


def _pair(w, q_teacher, q_student):
    import paper_2211_16933_amd as elb
    wt = dict(w, q=q_teacher)
    ws = dict(w, q=q_student)
    t = elb.Solver(elb.params_from_workload(wt, precision=FP64))
    s = elb.Solver(elb.params_from_workload(ws, precision=FP64, closure=1), stream=t.stream)
    t.set_state_moments(w["n"], w["u"], w["T"])
    s.set_state_moments(w["n"], w["u"], w["T"])
    return wt, ws, t, s


@pytest.mark.parametrize("kind", ["sound", "shock"])
def test_closure_sample_matches_oracle(kind):
    import paper_2211_16933_amd as elb
    if kind == "sound":
        w = workloads.sound_wave(nx=40, q=16, denseness=0.3, kn=0.05, amplitude=2e-2,
                                 pr_mode="enskog")
        qt, qs = 16, 8
    else:
        d = workloads.closure_draws()[40]
        d = dict(d, nx=48)
        w = workloads.closure_instance(d, 24)
        qt, qs = 24, 12
    say(f"case sample {kind} nx={w['nx']} teacher {qt} student {qs}")
    wt, ws, t, s = _pair(w, qt, qs)
    t.step(5)
    x, y = elb.closure_sample(t, s)
    ot = solver_from_workload(wt)
    ot.step(5)
    os_ = solver_from_workload(ws)
    xo, yo = cl.sample(ot, os_, w["denseness"], w["kn"])
    ex = [float(np.max(np.abs(x[:, c] - xo[:, c])) / max(np.max(np.abs(xo[:, c])), 1e-300))
          for c in range(12)]
    ey = rel_l2(y, yo)
    say("  x " + " ".join(f"{v:.0e}" for v in ex) + f"  y {ey:.1e}  |y| {np.max(np.abs(yo)):.2e}")
    assert max(ex) <= 1e-5 and ey <= 1e-5
    # the student now holds the projected teacher state
    phi, theta = s.dist()
    P = elb.projection(qt, qs)
    tp, tt = t.dist()
    assert rel_l2(phi, tp @ P.T) <= 1e-13 and rel_l2(theta, tt @ P.T) <= 1e-13


def test_rhs_matches_oracle():
    d = dict(workloads.closure_draws()[40], nx=64)
    w = workloads.closure_instance(d, 48)
    g = gpu_solver(w, FP64)
    Lp, Lt = g.rhs()
    Op, Ot = solver_from_workload(w).rhs()
    say(f"case rhs shock nx=64 q=48: {rel_l2(Lp, Op):.1e} {rel_l2(Lt, Ot):.1e}")
    assert rel_l2(Lp, Op) <= 1e-12 and rel_l2(Lt, Ot) <= 1e-12


@pytest.mark.parametrize("precision", [FP64, FP32_MIXED])
def test_corrected_step_matches_oracle(precision):
    """10 corrected steps of a Q = 8 sound wave.  Compared: the change the correction makes
    to phi (corrected minus plain run), GPU against oracle.  Each network evaluation agrees
    to ~1e-4 relative (bfloat16 rounding flips); over 30 stage evaluations such differences
    add up to a few 1e-4, hence the 2e-3 bound."""
    import paper_2211_16933_amd as elb
    from paper_2211_16933_amd import learned
    w = workloads.sound_wave(nx=40, q=8, denseness=0.3, kn=0.05, amplitude=2e-2,
                             pr_mode="enskog")
    layers = _net(8, seed=3, scale=0.3)
    norm = learned.make_norm(np.zeros(12), np.ones(12), np.zeros(8), np.full(8, 1e-3),
                             -np.full(12, 1e3), np.full(12, 1e3))
    # inputs around the sound wave's values
    norm[:12] = [1.0, 0.0, 1.0, 0, 0, 0, 0, 0, 0, 0, 0.3, np.log10(0.05)]
    norm[12:24] = [0.02, 0.02, 0.02, 0.01, 0.01, 0.05, 0.05, 0.05, 0.05, 0.05, 1.0, 1.0]
    say(f"case corrected step precision {precision}")
    s = elb.Solver(elb.params_from_workload(w, precision=precision, closure=1))
    s.set_state_moments(w["n"], w["u"], w["T"])
    c0 = s.conserved()
    s.set_closure(learned.pack_params(layers), norm, True)
    s.step(10)
    g = gpu_solver(w, precision)
    g.step(10)
    o = solver_from_workload(w)
    oc = cl.Closure(layers, norm[:12], norm[12:24], norm[24:32], norm[40:48], norm[56:68],
                    norm[68:80], o.p)
    cl.corrected_step(o, oc, w["denseness"], w["kn"], nsteps=10, periodic=True)
    plain = solver_from_workload(w)
    plain.step(10)
    d_gpu = s.dist()[0] - g.dist()[0]
    d_or = o.phi[3:-3] - plain.phi[3:-3]
    err = rel_l2(d_gpu, d_or)
    effect = np.linalg.norm(d_or) / np.linalg.norm(plain.phi[3:-3])
    say(f"  effect on phi {effect:.1e}, GPU vs oracle {err:.1e}, outside {s.closure_outside()}")
    assert effect >= 1e-3                      # the correction does something
    assert err <= 2e-3
    c1 = s.conserved()
    assert abs(c1[0] - c0[0]) <= 1e-12 * abs(c0[0])
    assert abs(c1[2] - c0[2]) <= 1e-9 * abs(c0[2])


@pytest.mark.parametrize("precision,q", [(FP64, 12), (FP32_MIXED, 12), (FP32_MIXED, 16),
                                         (FP32, 8)])
def test_fused_closure_matches_separate_kernels(precision, q):
    """The correction evaluated inside the stage kernel (enabled = 1) against the same
    correction from the two kernels before each stage (enabled = 2; that form is the one
    compared with the oracle above), on a standing shock of several tiles with a ragged last
    one.  Same network arithmetic in the same order; the inputs come from row moments
    summed in a different order, which can move a bfloat16 rounding of an input or an
    activation (each such flip moves the output by ~1e-3 of its size).  Compared: the
    change the correction makes to phi over 20 steps, and the cells outside the range."""
    import paper_2211_16933_amd as elb
    from paper_2211_16933_amd import learned
    table = workloads.load_shock_table()
    d = [d for d in workloads.closure_draws(128) if d["kind"] == "shock"][3]
    w = workloads.closure_instance(d, q, table)
    layers = _net(q, seed=7, scale=0.3)
    norm = learned.make_norm(np.zeros(12), np.ones(12), np.zeros(q), np.full(q, 1e-2),
                             -np.full(12, 1e3), np.full(12, 1e3))
    norm[:12] = [1.0, 0.0, 1.0, 0, 0, 0, 0, 0, 0, 0, w["denseness"], np.log10(w["kn"])]
    norm[12:24] = [0.3, 0.3, 0.3, 0.05, 0.05, 0.5, 0.5, 0.5, 0.5, 0.5, 1.0, 1.0]
    # a range that cuts through the shock, so that both forms mask and count cells
    norm[68] = 1.15
    say(f"case fused closure precision {precision} q {q} nx {w['nx']}")
    runs = {}
    for enabled in (1, 2):
        s = elb.Solver(elb.params_from_workload(w, precision=precision, closure=1))
        s.set_state_moments(w["n"], w["u"], w["T"])
        s.set_closure(learned.pack_params(layers), norm, enabled)
        s.step(20)
        runs[enabled] = (s.dist()[0], s.closure_outside())
    g = elb.Solver(elb.params_from_workload(w, precision=precision, closure=1))
    g.set_state_moments(w["n"], w["u"], w["T"])
    g.step(20)
    plain = g.dist()[0]
    effect = np.linalg.norm(runs[2][0] - plain) / np.linalg.norm(plain)
    err = rel_l2(runs[1][0] - plain, runs[2][0] - plain)
    say(f"  effect {effect:.1e}, fused vs separate {err:.1e}, outside {runs[1][1]} / {runs[2][1]}")
    assert effect >= 1e-4
    assert err <= 5e-3
    assert runs[2][1] > 0 and abs(runs[1][1] - runs[2][1]) <= 0.01 * runs[2][1] + 3


def test_closure_inputs_out_of_range_are_masked_and_counted():
    import paper_2211_16933_amd as elb
    from paper_2211_16933_amd import learned
    w = workloads.sound_wave(nx=64, q=8, denseness=0.3, kn=0.05, amplitude=2e-2,
                             pr_mode="enskog")
    layers = _net(8, seed=5, scale=0.3)
    norm = learned.make_norm(np.zeros(12), np.ones(12), np.zeros(8), np.ones(8),
                             -np.full(12, 1e3), np.full(12, 1e3))
    norm[56] = 1.0 + 1e-3    # n below this: outside (the wave's trough)
    s = elb.Solver(elb.params_from_workload(w, precision=FP64, closure=1))
    s.set_state_moments(w["n"], w["u"], w["T"])
    s.set_closure(learned.pack_params(layers), norm, True)
    s.step(1)
    out = s.closure_outside()
    say(f"case hull: {out} cell-stages outside")
    assert 3 * 20 <= out <= 3 * 44
    assert s.closure_outside() == 0            # reset by the read
    s.set_closure(None, None, False)
    s.step(1)
    assert s.closure_outside() == 0
    # enabled: 0 off, 1 inside the stage kernel, 2 separate kernels; nothing else
    for bad in (3, -1):
        with pytest.raises(elb.ElbError) as e:
            s.set_closure(learned.pack_params(layers), norm, bad)
        assert e.value.code == elb.ELB_EINVAL
