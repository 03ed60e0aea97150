"""CPU checks of the C ABI: the library loads, exports every declared symbol, and its host
functions (quadrature, unit mapping, validation) behave; no GPU is touched."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2211_16933_amd as elb
from oracle import physics
import workloads

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "elb.h")


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z0-9_]+\s*\*?\s*(elb_[a-z_]+)\s*\(", txt,
                                 flags=re.M)))


def test_library_exports_every_declared_symbol():
    syms = declared_symbols()
    assert len(syms) >= 14
    L = ctypes.CDLL(elb.library_path())
    for s in syms:
        assert hasattr(L, s), s


def test_supported_q():
    assert elb.supported_q() == [8, 12, 16, 20, 24, 32, 40, 48, 64, 96, 200]


@pytest.mark.parametrize("q", [8, 12, 16, 40, 48, 96, 200])
def test_library_quadrature_matches_numpy(q):
    p, w = elb.quadrature(q)
    pn, wn = np.polynomial.hermite_e.hermegauss(q)
    wn = wn / math.sqrt(2 * math.pi)
    assert np.max(np.abs(p - pn)) < 1e-13 * max(1, pn.max())
    assert np.max(np.abs(w - wn) / wn) < 1e-11
    assert p[::-1].tolist() == (-p).tolist()


@pytest.mark.parametrize("El,kn,L", [(0.1, 0.1, 1.0), (0.3, 1.0, 1.0), (0.4, 0.05, 1.0),
                                      (0.0, 0.02, 2.0)])
def test_unit_mapping_agrees_with_oracle(El, kn, L):
    w = workloads.sound_wave(nx=64, q=16, denseness=El, kn=kn)
    w["kn_length"] = L
    d = elb.derived(elb.params_from_workload(w))
    u = physics.units(El, kn, L, 1.0)
    assert d["b"] == pytest.approx(u["b"], rel=1e-13, abs=1e-300)
    assert d["mu_ref"] == pytest.approx(u["mu_ref"], rel=1e-13)
    assert d["eta0"] == pytest.approx(u["eta0"], rel=1e-13, abs=1e-300)
    p, _ = np.polynomial.hermite_e.hermegauss(16)
    assert d["dt"] == pytest.approx(0.5 / 64 / p.max(), rel=1e-14)
    assert d["n_herm"] == 15


def _base():
    return elb.params_from_workload(workloads.sound_wave(nx=64, q=16))


@pytest.mark.parametrize("field,value,code", [
    ("nx", 4, elb.ELB_EINVAL), ("nx", (1 << 30) + 1, elb.ELB_EINVAL), ("q", 6, elb.ELB_EINVAL), ("q", 10, elb.ELB_EUNSUPPORTED),
    ("n_herm", 5, elb.ELB_EINVAL), ("n_herm", 16, elb.ELB_EINVAL), ("cfl", 1.5, elb.ELB_EINVAL),
    ("length", -1.0, elb.ELB_EINVAL), ("denseness", float("nan"), elb.ELB_EINVAL),
    ("kn", 0.0, elb.ELB_EINVAL), ("pr_mode", 7, elb.ELB_EINVAL), ("bc", 3, elb.ELB_EINVAL),
    ("precision", 9, elb.ELB_EINVAL), ("dt", 1.0, elb.ELB_EINVAL)])
def test_invalid_params_rejected_before_launch(field, value, code):
    P = _base()
    setattr(P, field, value)
    with pytest.raises(elb.ElbError) as e:
        elb.derived(P)
    assert e.value.code == code
    assert elb.workspace_bytes(P) < 0


def test_rejection_reason_is_reported():
    """A failed elb_derived or elb_workspace_bytes leaves its reason in elb_last_error(NULL),
    and the binding's Solver raises with it before touching a device."""
    P = _base()
    P.q = 10
    assert elb.workspace_bytes(P) < 0
    assert b"q not among" in elb.lib().elb_last_error(None)
    P.q, P.cfl = 16, 1.5
    with pytest.raises(elb.ElbError, match="cfl"):
        elb.derived(P)
    with pytest.raises(elb.ElbError, match="cfl"):
        elb.Solver(P, device="cpu")


def test_batch_rejection_reason_is_reported():
    """Batch set-up failures carry their reason: mixed precisions, and an invalid instance
    named by its index (with the instance's own status code)."""
    a, b = _base(), _base()
    b.precision = elb.FP32
    with pytest.raises(elb.ElbError, match="share the precision") as e:
        elb.BatchSolver([a, b], device="cpu")
    assert e.value.code == elb.ELB_EINVAL
    b = _base()
    b.chi_mode = elb.CHI_RETFM
    b.kn = 200.0 * (b.length / b.nx) / (b.denseness * b.kn_length)   # sigma = 200 dx
    assert elb.lib().elb_batch_workspace_bytes((elb.Params * 2)(a, b), 2) < 0
    assert elb.lib().elb_batch_last_error(None).startswith(b"instance 1: ")
    with pytest.raises(elb.ElbError, match="instance 1"):
        elb.BatchSolver([a, b], device="cpu")


def test_equilibrium_ghosts_validated():
    w = workloads.shock_tube(nx=64, q=16)
    P = elb.params_from_workload(w)
    P.ghost_left[2] = -1.0
    with pytest.raises(elb.ElbError):
        elb.derived(P)


def test_create_without_workspace_fails_cleanly():
    P = _base()
    ctx = ctypes.c_void_p()
    rc = elb.lib().elb_create(ctypes.byref(P), None, 0, None, ctypes.byref(ctx))
    assert rc == elb.ELB_ENOMEM and not ctx.value


def test_workspace_size_scales_with_problem():
    P = _base()
    a = elb.workspace_bytes(P)
    P.precision = elb.FP32
    b = elb.workspace_bytes(P)
    P.precision = elb.FP32_MIXED
    c = elb.workspace_bytes(P)
    assert a > b and c > b


def test_chi_mode_validation():
    """chi_RET-FM: a bad mode is EINVAL; sigma / dx above 128 and the learned closure are
    EUNSUPPORTED; a valid request reserves the ball-average buffers."""
    P = _base()
    P.chi_mode = 5
    with pytest.raises(elb.ElbError) as e:
        elb.derived(P)
    assert e.value.code == elb.ELB_EINVAL
    P = _base()
    base = elb.workspace_bytes(P)
    P.chi_mode = elb.CHI_RETFM
    elb.derived(P)
    assert elb.workspace_bytes(P) > base
    P.closure = 1
    with pytest.raises(elb.ElbError) as e:
        elb.derived(P)
    assert e.value.code == elb.ELB_EUNSUPPORTED
    P = _base()
    P.chi_mode = elb.CHI_RETFM
    P.kn = 200.0 * (P.length / P.nx) / (P.denseness * P.kn_length)   # sigma = 200 dx
    with pytest.raises(elb.ElbError) as e:
        elb.derived(P)
    assert e.value.code == elb.ELB_EUNSUPPORTED


def test_moment_fixup_validation():
    """The moment fix-up is an option of FP32 with FP64 bookkeeping only; batches refuse it."""
    P = _base()
    P.moment_fixup = 2
    with pytest.raises(elb.ElbError) as e:
        elb.derived(P)
    assert e.value.code == elb.ELB_EINVAL
    P.moment_fixup = 1
    for prec in (elb.FP64, elb.FP32):
        P.precision = prec
        with pytest.raises(elb.ElbError, match="FP32_MIXED") as e:
            elb.derived(P)
        assert e.value.code == elb.ELB_EINVAL
    P.precision = elb.FP32_MIXED
    elb.derived(P)
    Q = _base()
    Q.precision = elb.FP32_MIXED
    assert elb.workspace_bytes(P) == elb.workspace_bytes(Q)
    assert elb.lib().elb_batch_workspace_bytes((elb.Params * 2)(P, Q), 2) < 0
    assert b"fix-up" in elb.lib().elb_batch_last_error(None)


def test_workload_chi_key_reaches_the_params():
    w = workloads.sound_wave(nx=64, q=16)
    assert elb.params_from_workload(w).chi_mode == elb.CHI_SET
    w["chi"] = "ret"
    assert elb.params_from_workload(w).chi_mode == elb.CHI_RETFM


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with status 2 and says why,
    before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
