"""What the trained closure gains (needs an MI355X).

A Q = 8 student is trained on the GPU, by the library's own kernels, against a Q = 64
teacher on standing shocks (Mach 1.1-1.8, E_l in [0.05, 0.5], Kn in [0.01, 1]), with
Mach 1.5 +- 0.05 and E_l 0.25 +- 0.05, 0.45 +- 0.05 held out, in two rounds:
  * round 0 on the teacher's own states projected onto the student's nodes;
  * round 1 on those samples together with samples along the corrected student's own runs
    (dataset aggregation): the round-0 student is run with its correction, its states are
    lifted onto the teacher's nodes, the teacher relaxes 20 steps from each, and the
    samples are taken there.
It is then run on the held-out Mach 1.5, E_l = 0.25 shock and compared with the teacher at
equal physical time.  The corrected runs (and the student runs that give the round-1
samples) add the correction times learned.CORRECTION_WEIGHT = 0.6: with the full
correction, two of three trainings that differ only in their seed diverged; at 0.6 all three
stayed finite and inside the training range.
  * a priori: the round-0 network explains most of the held-out right-hand-side defect;
  * a posteriori, while the shock forms (t = 0.039, 0.13 and 0.39, 0.4 to 4 upstream
    relaxation times), the corrected student is closer to the teacher than the student
    alone in each of n, u, T, with every cell inside the training range, so the fallback is
    not taken (measured over three seeds: 0.48-0.95 of the student alone's error per field);
  * near the steady state (t = 1.2) the student alone is within 0.4 % of the teacher and the
    correction adds error (2-4x); the test requires the answer of run_with_fallback (the
    corrected run, else the fine quadrature) to be finite.
"""
import numpy as np
import pytest

import workloads
from helpers import say

pytestmark = pytest.mark.gpu

Q_T, Q_S = 64, 8


def _errors(m, mt):
    return [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(m[:3], mt[:3])]


def _fit(learned, X, Y, seed=0):
    tr = learned.Trainer(X, Y, batch=4096, lr=1e-3, seed=seed, margin=0.1)
    tr.train(2000)
    tr.lr = 3e-4
    tr.train(2000)
    return tr


def test_learned_closure_gain_on_held_out_shock():
    import paper_2211_16933_amd as elb
    from paper_2211_16933_amd import learned
    table = workloads.load_shock_table()
    draws = [d for d in workloads.closure_draws(128) if d["kind"] == "shock"]
    train = [workloads.closure_instance(d, Q_T, table) for d in draws]
    say(f"case closure gain: {len(train)} teacher shocks, Q {Q_T} -> {Q_S}")
    X, Y = learned.generate(train, Q_T, Q_S, start=20, every=25, count=40, cells=128)
    hd = workloads.closure_held_out()[0]
    held = workloads.closure_instance(hd, Q_T, table, key="closure_held_out")
    Xh, Yh = learned.generate([held], Q_T, Q_S, start=20, every=25, count=40)
    tr0 = _fit(learned, X, Y)
    l0 = tr0.evaluate(Xh, Yh)
    p0, n0 = tr0.result()
    say(f"  round 0: {X.shape[0]} samples; held-out a-priori loss {l0:.4f}")
    # the untrained network's held-out loss, for the a-priori check
    tr_init = learned.Trainer(X, Y, batch=4096, lr=1e-3, seed=0, margin=0.1)
    assert l0 <= 0.2 * tr_init.evaluate(Xh, Yh)

    Xs, Ys = learned.generate_on_student(train, Q_T, Q_S, p0, n0, start=20, every=25, count=40,
                                         relax=20, cells=128, seed=1)
    tr1 = _fit(learned, np.concatenate([X, Xs]), np.concatenate([Y, Ys]))
    params, norm = tr1.result()
    say(f"  round 1: {Xs.shape[0]} samples on the student's own states added")

    wt = held
    ws = workloads.closure_instance(hd, Q_S, table, key="closure_held_out")
    for steps_t in (300, 1000, 3000, 9000):
        T = elb.Solver(elb.params_from_workload(wt, precision=elb.FP64))
        T.set_state_moments(wt["n"], wt["u"], wt["T"])
        T.step(steps_t)
        t_end = steps_t * T.info["dt"]
        mt = T.moments()
        S = elb.Solver(elb.params_from_workload(ws, precision=elb.FP64))
        S.set_state_moments(ws["n"], ws["u"], ws["T"])
        ns = int(round(t_end / S.info["dt"]))
        S.step(ns)
        e_alone = _errors(S.moments(), mt)
        m, used = learned.run_with_fallback(ws, Q_S, Q_T, params, norm, t_end)
        assert all(np.all(np.isfinite(v)) for v in m)
        if steps_t == 9000:
            # near the steady state the corrected run may leave the range or break down; the
            # fallback must then answer with the fine quadrature
            say(f"  t={t_end:.3f}: student alone n,u,T {np.round(e_alone, 4)}; returned {used}, "
                f"n,u,T {np.round(_errors(m, mt), 4)}")
            continue
        L, outside = learned.run_student(ws, Q_S, params, norm, ns)
        e_learned = _errors(L.moments(), mt)
        say(f"  t={t_end:.3f}: student alone n,u,T {np.round(e_alone, 4)}; corrected "
            f"{np.round(e_learned, 4)} (cells outside {outside}); returned {used}")
        assert outside == 0 and used == "learned"
        assert all(a < b for a, b in zip(e_learned, e_alone)), (t_end, e_learned, e_alone)
