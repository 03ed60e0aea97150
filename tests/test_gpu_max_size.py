"""A problem past 2^31 distribution values per level (needs an MI355X with ~60 GB free): every
index of the stage, initialisation and readout kernels must be 64-bit safe there.

A 64-cell periodic pattern repeated 360,000 times (Nx = 23,040,000, Q = 96, FP32 with FP64
bookkeeping; 2.2e9 values per distribution level) evolves exactly as the 64-cell problem
alone, so every cell of the large run is checked against the small run, and the small run
against the oracle."""
import math

import numpy as np
import pytest

import workloads
from helpers import say, gpu_solver, oracle_solver, field_errors

pytestmark = pytest.mark.gpu

FP32_MIXED = 2
PATTERN, REPEATS = 64, 360000


def pattern_wave():
    w = workloads.sound_wave(nx=PATTERN, q=96, denseness=0.4, kn=0.05, amplitude=0.05,
                             pr_mode="enskog", name="max_size_pattern")
    x = workloads.cell_centres(PATTERN, 1.0)
    w["u"] = 0.1 * np.sin(2 * math.pi * x + 0.3)
    w["T"] = 1.0 + 0.1 * np.cos(2 * math.pi * x)
    return w


def test_repeated_pattern_past_2_31_values():
    import torch
    small = pattern_wave()
    big = dict(small)
    big["nx"], big["length"] = PATTERN * REPEATS, float(REPEATS)   # same dx, same Kn length
    big["name"] = f"max_size_nx{big['nx']}_q96"
    for f in ("n", "u", "T"):
        big[f] = np.tile(small[f], REPEATS)
    assert (big["nx"] + 6) * 96 > 2 ** 31
    steps = 2
    say(f"case {big['name']} steps={steps} FP32_MIXED ({(big['nx'] + 6) * 96 * 2:.3e} values per level)")
    torch.cuda.empty_cache()
    g = gpu_solver(big, FP32_MIXED)
    g.step(steps)
    mb = g.moments()
    cb = g.conserved()
    del g
    torch.cuda.empty_cache()
    s = gpu_solver(small, FP32_MIXED)
    s.step(steps)
    ms = s.moments()
    cs = s.conserved()
    worst = 0.0
    for j, name in enumerate(("n", "u", "T", "q", "pxx")):
        ref = np.tile(ms[j], REPEATS)
        scale = max(np.max(np.abs(ms[j])), 1e-3)
        d = float(np.max(np.abs(mb[j] - ref))) / scale
        worst = max(worst, d if name in ("n", "u", "T") else 0.0)
        say(f"  {name}: max |large - tiled small| / max |small| = {d:.2e}")
    assert worst <= 1e-6
    # totals: the large problem holds REPEATS copies of the small one (up to the rounding of
    # a 2.3e7-term FP64 sum, bounded by N eps = 2.6e-9)
    say(f"  mass: large / (copies x small) - 1 = {cb[0] / (REPEATS * cs[0]) - 1.0:.2e}")
    assert abs(cb[0] / (REPEATS * cs[0]) - 1.0) <= 1e-9
    o = oracle_solver(small)
    o.step(steps)
    err = field_errors(ms, o.moments())
    say("  small run vs oracle", {k: f"{v:.2e}" for k, v in err.items()})
    for f in ("n", "u", "T"):
        assert err[f] <= 1e-5
