"""Seeded synthetic inputs shaped like the paper's sound-wave and shock problems.

This module is shared by the tests, the benchmark and the oracle-side scripts.  It holds
none of the method's arithmetic: it only lays out grids, draws seeded random parameters
and builds primitive (n, u, T) profiles.  Shock end states come as data (a JSON table
written by tests/golden/make_shock_states.py), never computed here.

A workload is a plain dict:
  nx, q            cells and Gauss-Hermite nodes
  length, x0       domain [x0, x0 + length), cell-centred grid
  bc               "periodic" | "equilibrium"
  denseness, kn, kn_length, n_ref
                   E_l at n_ref (T = 1) and Kn = mean free path / kn_length
  pr_mode, pr      "const" with pr, or "enskog"
  cfl, steps       time step dt = cfl * dx / max|p_k| and the number of RK3 steps
  n, u, T          float64 arrays of nx primitive values (interior cells)
  left, right      (n, u, T) of the ghost-cell equilibrium for bc == "equilibrium"
"""
import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
SHOCK_TABLE = os.path.join(REPO, "tests", "golden", "shock_states.json")


def cell_centres(nx, length, x0=0.0):
    dx = length / nx
    return x0 + (np.arange(nx) + 0.5) * dx


def _base(nx, q, length, x0, bc, denseness, kn, kn_length, pr_mode, pr, cfl, steps, name):
    return {"name": name, "nx": int(nx), "q": int(q), "length": float(length), "x0": float(x0),
            "bc": bc, "denseness": float(denseness), "kn": float(kn),
            "kn_length": float(kn_length), "n_ref": 1.0, "pr_mode": pr_mode, "pr": float(pr),
            "cfl": float(cfl), "steps": int(steps)}


def sound_wave(nx=128, q=16, denseness=0.1, kn=0.1, amplitude=1e-3, pr_mode="const",
               pr=2.0 / 3.0, cfl=0.5, steps=1000, name="sound_wave", phase="sin"):
    """Periodic longitudinal wave on [0, 1): n = 1 + A sin(2 pi x) (or cos with
    phase="cos"), u = 0, T = 1."""
    w = _base(nx, q, 1.0, 0.0, "periodic", denseness, kn, 1.0, pr_mode, pr, cfl, steps, name)
    x = cell_centres(nx, 1.0)
    shape = np.cos if phase == "cos" else np.sin
    w["n"] = 1.0 + amplitude * shape(2.0 * math.pi * x)
    w["phase"] = phase
    w["u"] = np.zeros(nx)
    w["T"] = np.ones(nx)
    w["amplitude"] = float(amplitude)
    return w


def config1():
    """Plain FP64 sound wave: Nx = 128, Q = 16, E_l = 0.1, Kn = 0.1, Pr = 2/3, CFL 0.5,
    1000 steps."""
    return sound_wave(name="sound_wave_nx128_q16")


def _tanh_profile(x, left, right, width):
    s = 0.5 * (1.0 + np.tanh(x / width))
    return [left[j] + (right[j] - left[j]) * s for j in range(3)]


def load_shock_table(path=SHOCK_TABLE):
    with open(path) as f:
        return json.load(f)


def shock_structure(mach, seed, nx=2048, q=48, denseness=0.3, steps=20000, table=None,
                    name=None):
    """Standing normal shock over 40 upstream mean free paths, [-20, 20), Kn = 1 on the
    upstream mean free path.  Primitive fields are upstream + (downstream - upstream)
    * (1 + tanh(x / w)) / 2 with w = 2 dx (1 + 0.25 U(-1, 1)) drawn from
    numpy.random.default_rng(seed).  End states are read from the shock-state table."""
    table = load_shock_table() if table is None else table
    key = f"M{mach:g}_El{denseness:g}"
    st = table["states"][key]
    length = 40.0
    w = _base(nx, q, length, -20.0, "equilibrium", denseness, 1.0, 1.0, "enskog", 0.0, 0.5,
              steps, name or f"shock_M{mach:g}_nx{nx}_q{q}")
    rng = np.random.default_rng(seed)
    dx = length / nx
    width = 2.0 * dx * (1.0 + 0.25 * rng.uniform(-1.0, 1.0))
    x = cell_centres(nx, length, -20.0)
    left = (st["n1"], st["u1"], st["T1"])
    right = (st["n2"], st["u2"], st["T2"])
    w["n"], w["u"], w["T"] = _tanh_profile(x, left, right, width)
    w["left"], w["right"] = left, right
    w["width"] = width
    w["mach"] = float(mach)
    return w


def config2(mach=2):
    """FP32-vs-FP64 shock structure, Mach 2 (seed 2) or Mach 3 (seed 3)."""
    return shock_structure(mach, seed=int(mach))


def shock_tube(nx=65536, q=96, denseness=0.4, kn=0.05, left=(1.5, 0.0, 1.2),
               right=(1.0, 0.0, 1.0), steps=10000, cfl=0.5, name=None):
    """Riemann problem on [0, 1) with the membrane at x = 0.5 and equilibrium ghosts of the
    two end states."""
    w = _base(nx, q, 1.0, 0.0, "equilibrium", denseness, kn, 1.0, "enskog", 0.0, cfl, steps,
              name or f"shock_tube_nx{nx}_q{q}")
    x = cell_centres(nx, 1.0)
    lm = x < 0.5
    w["n"] = np.where(lm, left[0], right[0]).astype(np.float64)
    w["u"] = np.where(lm, left[1], right[1]).astype(np.float64)
    w["T"] = np.where(lm, left[2], right[2]).astype(np.float64)
    w["left"], w["right"] = tuple(left), tuple(right)
    return w


def sod_tube(denseness, kn, nx=1600, q=8, length=80.0, steps=0, cfl=0.5, name=None):
    """The Sod problem of Sec. IV.B: membrane at the middle of [0, length), left state
    (n, u, T) = (1, 0, 1), right state (1/8, 0, 1), so that eta_R = eta_L / 8 at T = 1;
    equilibrium ghosts of the two end states.  E_l is taken at the left density."""
    w = _base(nx, q, length, 0.0, "equilibrium", denseness, kn, 1.0, "enskog", 0.0, cfl,
              steps, name or f"sod_tube_nx{nx}_q{q}")
    x = cell_centres(nx, length)
    lm = x < 0.5 * length
    w["n"] = np.where(lm, 1.0, 0.125)
    w["u"] = np.zeros(nx)
    w["T"] = np.ones(nx)
    w["left"], w["right"] = (1.0, 0.0, 1.0), (0.125, 0.0, 1.0)
    return w


def config5(nx=65536, q=96):
    """Large single shock tube: Nx = 65536, Q = 96, E_l = 0.4, Kn = 0.05,
    left (1.5, 0, 1.2), right (1, 0, 1), 10000 steps."""
    return shock_tube(nx=nx, q=q)


# Highest Mach number of a standing shock started from a tanh profile that the scheme
# carries stably with Q nodes over the whole E_l, Kn range of the sweep (checked with the
# oracle); a coarser velocity grid cannot hold the wider upstream/downstream spread.
MACH_MAX = {16: 2.0, 24: 2.4, 32: 2.7, 48: 3.0}


def batch_draws(count=512, seed=3):
    """Seeded parameters of the batched sweep: the first half sound waves, the second half
    standing shocks.  N_x ~ U{64..2048}, Q ~ U{16, 24, 32, 48}, E_l ~ U[0.05, 0.5],
    Kn ~ logU[0.01, 1], amplitude ~ logU[1e-4, 1e-2], Mach ~ U[1.2, MACH_MAX[Q]]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        d = {"index": i, "kind": "sound" if i < count // 2 else "shock",
             "nx": int(rng.integers(64, 2049)), "q": int(rng.choice([16, 24, 32, 48])),
             "denseness": float(rng.uniform(0.05, 0.5)),
             "kn": float(10.0 ** rng.uniform(-2.0, 0.0)),
             "amplitude": float(10.0 ** rng.uniform(-4.0, -2.0))}
        d["mach"] = 1.2 + (MACH_MAX[d["q"]] - 1.2) * float(rng.uniform(0.0, 1.0))
        d["seed"] = int(rng.integers(0, 2 ** 31))
        out.append(d)
    return out


def batch_instance(d, table=None):
    """Workload of one batched instance from its draw (see batch_draws): a periodic sound
    wave on [0, 1) of amplitude d['amplitude'], or a standing shock on [-1/2, 1/2) with
    Kn on the upstream mean free path, end states read from the shock-state table and a
    tanh start over 2 dx (1 + 0.25 U(-1, 1)) drawn from default_rng(d['seed'])."""
    if d["kind"] == "sound":
        return sound_wave(nx=d["nx"], q=d["q"], denseness=d["denseness"], kn=d["kn"],
                          amplitude=d["amplitude"], pr_mode="enskog", steps=5000,
                          name=f"batch{d['index']}_sound")
    table = load_shock_table() if table is None else table
    st = table["batch"][str(d["index"])]
    nx, length = d["nx"], 1.0
    w = _base(nx, d["q"], length, -0.5, "equilibrium", d["denseness"], d["kn"], 1.0, "enskog",
              0.0, 0.5, 5000, f"batch{d['index']}_shock")
    rng = np.random.default_rng(d["seed"])
    dx = length / nx
    width = 2.0 * dx * (1.0 + 0.25 * rng.uniform(-1.0, 1.0))
    x = cell_centres(nx, length, -0.5)
    left = (st["n1"], st["u1"], st["T1"])
    right = (st["n2"], st["u2"], st["T2"])
    w["n"], w["u"], w["T"] = _tanh_profile(x, left, right, width)
    w["left"], w["right"] = left, right
    w["mach"] = d["mach"]
    return w


def config3(count=512, seed=3):
    """The batched sweep: `count` instances (first half sound waves, second half standing
    shocks) with uneven N_x, Q, denseness and Kn."""
    table = load_shock_table()
    return [batch_instance(d, table) for d in batch_draws(count, seed)]


# ---------------------------------------------------------------------------------------
# learned closure: training draws and held-out cases
# ---------------------------------------------------------------------------------------
CLOSURE_MACH = (1.1, 1.8)          # a Q = 8 student carries shocks up to about Mach 1.8
CLOSURE_HELD_OUT = {"mach": (1.5,), "denseness": (0.25, 0.45), "band": 0.05}


def _held_out(value, centres, band):
    return any(abs(value - c) <= band for c in centres)


def closure_draws(count=64, seed=4, nx_range=(64, 512)):
    """Seeded sweep-style parameters of the teacher runs that train the closure: the first
    half sound waves, the second half standing shocks.  N_x ~ U{nx_range}, E_l ~
    U[0.05, 0.5], Kn ~ logU[0.01, 1], amplitude ~ logU[1e-4, 1e-2], Mach ~ U[1.1, 1.8];
    values within 0.05 of a held-out Mach number or denseness are drawn again."""
    rng = np.random.default_rng(seed)
    band = CLOSURE_HELD_OUT["band"]
    out = []
    for i in range(count):
        while True:
            El = float(rng.uniform(0.05, 0.5))
            if not _held_out(El, CLOSURE_HELD_OUT["denseness"], band):
                break
        while True:
            mach = float(rng.uniform(*CLOSURE_MACH))
            if not _held_out(mach, CLOSURE_HELD_OUT["mach"], band):
                break
        d = {"index": i, "kind": "sound" if i < count // 2 else "shock",
             "nx": int(rng.integers(nx_range[0], nx_range[1] + 1)), "denseness": El,
             "kn": float(10.0 ** rng.uniform(-2.0, 0.0)),
             "amplitude": float(10.0 ** rng.uniform(-4.0, -2.0)), "mach": mach,
             "seed": int(rng.integers(0, 2 ** 31))}
        out.append(d)
    return out


def closure_instance(d, q, table=None, key="closure"):
    """Workload of a closure draw with q nodes: a periodic sound wave on [0, 1), or a
    standing shock on [-1/2, 1/2) with end states from the shock-state table."""
    if d["kind"] == "sound":
        return sound_wave(nx=d["nx"], q=q, denseness=d["denseness"], kn=d["kn"],
                          amplitude=d["amplitude"], pr_mode="enskog", steps=0,
                          name=f"{key}{d['index']}_sound")
    table = load_shock_table() if table is None else table
    st = table[key][str(d["index"])]
    nx, length = d["nx"], 1.0
    w = _base(nx, q, length, -0.5, "equilibrium", d["denseness"], d["kn"], 1.0, "enskog", 0.0,
              0.5, 0, f"{key}{d['index']}_shock")
    rng = np.random.default_rng(d["seed"])
    dx = length / nx
    width = 2.0 * dx * (1.0 + 0.25 * rng.uniform(-1.0, 1.0))
    x = cell_centres(nx, length, -0.5)
    left = (st["n1"], st["u1"], st["T1"])
    right = (st["n2"], st["u2"], st["T2"])
    w["n"], w["u"], w["T"] = _tanh_profile(x, left, right, width)
    w["left"], w["right"] = left, right
    w["mach"] = d["mach"]
    return w


def closure_held_out():
    """Held-out cases: a Mach 1.5 standing shock at E_l = 0.25, Kn = 0.1 and a sound wave at
    E_l = 0.45, Kn = 0.05, amplitude 1e-2."""
    return [{"index": 0, "kind": "shock", "nx": 256, "denseness": 0.25, "kn": 0.1,
             "amplitude": 0.0, "mach": 1.5, "seed": 11},
            {"index": 1, "kind": "sound", "nx": 256, "denseness": 0.45, "kn": 0.05,
             "amplitude": 1e-2, "mach": 0.0, "seed": 12}]


def closure_tubes(nx=65536, q=96):
    """Shock tubes that train the closure of the large shock tube's Q = 12 student: the same
    grid and node count, other end states and physics (left (1.4, 0, 1.15) at E_l = 0.35,
    Kn = 0.04, and left (1.6, 0, 1.25) at E_l = 0.45, Kn = 0.06; right (1, 0, 1))."""
    return [shock_tube(nx=nx, q=q, denseness=0.35, kn=0.04, left=(1.4, 0.0, 1.15),
                       name=f"tube_a_nx{nx}_q{q}"),
            shock_tube(nx=nx, q=q, denseness=0.45, kn=0.06, left=(1.6, 0.0, 1.25),
                       name=f"tube_b_nx{nx}_q{q}")]
