"""Batched stepping of many heterogeneous instances (needs an MI355X).

A batch runs the same per-tile arithmetic as a single context, so with the default tile
shapes every instance must come out bitwise identical to stepping it alone, whether the
steps run through the captured HIP graph or by direct launches.  A tile shape picked by the
tuner changes only where strips start; results then agree to rounding."""
import json
import os

import numpy as np
import pytest

import workloads
from helpers import say, gpu_solver, oracle_solver, field_errors

pytestmark = pytest.mark.gpu

FP64, FP32, FP32_MIXED = 0, 1, 2


def _small_sweep(count=16, nx_cap=None, seed=3):
    """Instances spread over the sweep's draws (both kinds, every Q)."""
    draws = workloads.batch_draws(512, seed)
    picks = [draws[i] for i in range(0, 256, 256 // (count // 2))][: count // 2] + \
            [draws[i] for i in range(256, 512, 256 // (count // 2))][: count // 2]
    table = workloads.load_shock_table()
    ws = []
    for d in picks:
        d = dict(d)
        if nx_cap:
            d["nx"] = min(d["nx"], nx_cap)
        ws.append(workloads.batch_instance(d, table))
    return ws


def _batch(ws, precision):
    import paper_2211_16933_amd as elb
    b = elb.BatchSolver([elb.params_from_workload(w, precision=precision) for w in ws])
    for i, w in enumerate(ws):
        b.set_state_moments(i, w["n"], w["u"], w["T"])
    return b


@pytest.mark.parametrize("precision", [FP64, FP32_MIXED])
def test_batch_bitwise_equals_single(precision):
    ws = _small_sweep(16)
    say(f"case batch of {len(ws)} (Q {sorted(set(w['q'] for w in ws))}) precision {precision}")
    b = _batch(ws, precision)
    b.step(20)
    for i, w in enumerate(ws):
        s = gpu_solver(w, precision)
        s.step(20)
        pb, tb = b.dist(i)
        ps, ts = s.dist()
        assert np.array_equal(pb, ps) and np.array_equal(tb, ts), (i, w["name"])


def test_batch_graph_replays_match_direct_launches():
    """Several replays of the captured graph, with host reads in between, against direct
    launches of the same steps."""
    ws = _small_sweep(8)
    g = _batch(ws, FP32_MIXED)
    d = _batch(ws, FP32_MIXED)
    d.set_graph(False)
    for rep in range(4):
        g.step(50)      # one chunk: one graph replay
        d.step(50)
        for i in range(len(ws)):
            mg, md = g.moments(i), d.moments(i)
            for a, c in zip(mg, md):
                assert np.array_equal(a, c), (rep, i)
    g.step(123)         # two replays and 23 direct steps
    d.step(123)
    for i in range(len(ws)):
        assert np.array_equal(g.dist(i)[0], d.dist(i)[0])


def _rel_max(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_batch_tuner_keeps_results_and_caches(tmp_path):
    ws = _small_sweep(8)
    ref = _batch(ws, FP32_MIXED)
    ref.step(10)
    b = _batch(ws, FP32_MIXED)
    cache = str(tmp_path / "tune.json")
    b.tune(cache)
    say("  tuned groups", b.groups())
    entries = json.load(open(cache))
    assert len(entries) == len(b.groups())
    b.step(10)
    worst = 0.0
    for i in range(len(ws)):
        mb, mr = b.moments(i), ref.moments(i)
        for a, c in zip(mb[:3], mr[:3]):
            worst = max(worst, _rel_max(a, c))
    say(f"  tuned vs default shapes, 10 steps: max relative difference {worst:.1e}")
    assert worst <= 1e-6
    b2 = _batch(ws, FP32_MIXED)
    b2.tune(cache)          # read back from the cache
    assert b2.groups() == b.groups()


def test_batch_against_oracle():
    """Batched FP32-with-bookkeeping instances against the FP64 oracle, 50 steps."""
    ws = _small_sweep(8, nx_cap=96)
    b = _batch(ws, FP32_MIXED)
    b.step(50)
    for i, w in enumerate(ws):
        o = oracle_solver(w)
        o.step(50)
        err = field_errors(b.moments(i), o.moments())
        say(f"  {w['name']} q={w['q']} nx={w['nx']}", {k: f"{v:.1e}" for k, v in err.items()})
        for f in ("n", "u", "T"):
            assert err[f] <= 1e-5, (w["name"], f, err)


def test_full_sweep_runs_and_matches_single_instances():
    """All 512 instances of the batched sweep in one batch: a sample against single contexts
    (bitwise with the default shapes), then tuned and stepped on, every instance valid."""
    ws = workloads.config3()
    b = _batch(ws, FP32_MIXED)
    b.step(20)
    sample = (0, 77, 255, 256, 400, 511)
    singles = {}
    for i in sample:
        s = gpu_solver(ws[i], FP32_MIXED)
        s.step(20)
        assert np.array_equal(b.dist(i)[0], s.dist()[0]), i
        singles[i] = s
    b.tune()
    say("  groups", b.groups())
    b.step(20)
    for i in range(len(ws)):
        b.moments(i)  # raises on a non-finite cell
    for i in sample:
        singles[i].step(20)
        mb, ms = b.moments(i), singles[i].moments()
        for a, c in zip(mb[:3], ms[:3]):
            assert _rel_max(a, c) <= 1e-6, i


@pytest.mark.parametrize("precision", [FP64, FP32_MIXED])
def test_batch_with_large_velocity_sets(precision):
    """Q = 40 and Q = 200 instances (the near-ballistic node counts; Q = 200 blocks are
    padded to whole waves) batched with a Q = 16 one: bitwise equal to stepping each alone."""
    ws = [workloads.shock_tube(nx=101, q=200, denseness=0.3, kn=0.5, name="tube_q200"),
          workloads.sound_wave(nx=77, q=40, denseness=0.2, kn=0.1, amplitude=1e-2,
                               pr_mode="enskog", name="wave_q40"),
          workloads.shock_tube(nx=130, q=40, denseness=0.4, kn=0.2, name="tube_q40"),
          workloads.sound_wave(nx=64, q=16, denseness=0.1, kn=0.05, amplitude=1e-3,
                               pr_mode="enskog", name="wave_q16")]
    say(f"case batch with Q 200/40/16, precision {precision}")
    b = _batch(ws, precision)
    b.step(60)
    for i, w in enumerate(ws):
        s = gpu_solver(w, precision)
        s.step(60)
        pb, tb = b.dist(i)
        ps, ts = s.dist()
        assert np.array_equal(pb, ps) and np.array_equal(tb, ts), (i, w["name"])


@pytest.mark.parametrize("precision", [FP64, FP32_MIXED])
def test_batch_with_chi_ret(precision):
    """chi_RET-FM instances (different sigma / dx, so different stencil half-widths in one
    group) batched with chi_SET ones of the same Q: bitwise equal to stepping each alone."""
    def ret(w):
        w["chi"] = "ret"
        return w
    ws = [ret(workloads.shock_tube(nx=160, q=32, denseness=0.48, kn=0.026, name="tube_ret_S2")),
          ret(workloads.sound_wave(nx=101, q=32, denseness=0.4, kn=0.136, amplitude=2e-2,
                                   pr_mode="enskog", name="wave_ret_S5.5")),
          workloads.sound_wave(nx=101, q=32, denseness=0.4, kn=0.136, amplitude=2e-2,
                               pr_mode="enskog", name="wave_set"),
          ret(workloads.sound_wave(nx=64, q=16, denseness=0.3, kn=0.01, amplitude=1e-2,
                                   pr_mode="enskog", name="wave_ret_S0.2"))]
    say(f"case batch with chi_RET-FM, precision {precision}")
    b = _batch(ws, precision)
    b.step(60)
    for i, w in enumerate(ws):
        s = gpu_solver(w, precision)
        s.step(60)
        pb, tb = b.dist(i)
        ps, ts = s.dist()
        assert np.array_equal(pb, ps) and np.array_equal(tb, ts), (i, w["name"])
