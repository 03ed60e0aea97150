"""Throughput of the FDLB step on one MI355X: cell-velocity updates per second.

Default workload: the large single shock tube (Nx = 65536 cells, Q = 96 Gauss-Hermite
nodes, E_l = 0.4, Kn = 0.05, left (1.5, 0, 1.2) / right (1, 0, 1)), FP32 bulk with FP64
moment sums and FP64 conserved bookkeeping.  One step is
one full SSP-RK3 step (three stage launches) over every (cell, node).  Inputs are resident
in HBM before the timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32_mixed|fp32|fp64]
                  [--nx 65536] [--q 96] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

REPO = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, REPO)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# MI355X FP32 vector rate: 256 CUs x 4 SIMDs x 32 lanes x 2 flop (FMA) x 2.4 GHz = 157.3
# TFLOP/s.  The library is compiled without packed FP32 instructions, but on this GPU a plain
# v_fma_f32 (VOP2 or VOP3) issues at close to two cycles per wave64 instruction, i.e. 32 lanes
# per clock per SIMD (measured with a throughput micro-benchmark: about 2.8 cycles including
# launch overhead, against 4.8-5.2 for FP64 FMA, whose vector peak is 78.6 TFLOP/s), so the
# unpacked rate is the vendor's figure
FP32_VECTOR_PEAK_TFLOPS = 157.3
TIMED_RUNS = 5  # the reported time is the median of this many timed runs of K steps
# rocprofv3 summary of the stage kernel on the default workload: FETCH_SIZE and WRITE_SIZE
# per launch, scaled by a plain device copy, stamped with the hash of the kernel source
TRAFFIC_PROFILE = os.path.join(REPO, "profiles", "k_stage_shock_tube_nx65536_q96_fp32_mixed.md")
KERNEL_SOURCE = os.path.join(REPO, "paper_2211_16933_amd", "csrc", "elb_kernels.h")

PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_mixed": 2}
DTYPES = {"fp64": "f64", "fp32": "f32", "fp32_mixed": "f32+f64"}


def stage_bytes_per_pair(elem, mixed_q=None):
    """Algorithmic HBM bytes per (cell, node) per stage launch, averaged over the three
    stages: stage 1 reads psi^n (2 values) and writes psi^(1) (2); stages 2 and 3 read
    psi^n and psi^(s) (4) and write 2.  (4 + 6 + 6) / 3 values of `elem` bytes.  The mixed
    mode adds per cell FP64 (n, nu, E): read 3 (stage 1) or 6 (stages 2, 3), write 3,
    spread over the Q nodes of the cell."""
    b = (4 + 6 + 6) / 3.0 * elem
    if mixed_q:
        b += (6 + 9 + 9) / 3.0 * 8.0 / mixed_q
    return b


def stage_flop_per_pair(q):
    """Operation count of the method per (cell, node) per stage launch: two WENO-5
    reconstructions (~70 flop each, 3 reciprocals counted as 1 flop), the Hermite projection
    (2Q: one multiply-add per coefficient), the Shakhov target and J1 (~40), the moments
    (~12) and the RK combination (~8)."""
    return 2 * 70 + 2 * q + 40 + 12 + 8


def kernel_source_hash():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic():
    """HBM bytes per stage launch from the committed counter summary, or None when it is
    missing or was taken on a different kernel source."""
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    h = re.search(r"kernel source sha256: `([0-9a-f]{64})`", text)
    b = re.search(r"HBM bytes per launch \(scaled\): `([0-9.eE+]+)`", text)
    if not h or not b or h.group(1) != kernel_source_hash():
        return None
    return float(b.group(1))


def cpu_baseline(w, seconds=10.0, threads=None):
    """Time the FP64 oracle (test infrastructure, untuned) on the host on a bounded sample
    of the same workload: whole steps of the full problem until `seconds` have passed."""
    import oracle
    from oracle.run import solver_from_workload
    threads = threads or min(16, os.cpu_count() or 1)
    oracle.set_threads(threads)
    s = solver_from_workload(w)
    steps, t0 = 0, time.perf_counter()
    while True:
        s.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 50:
            break
    rate = w["nx"] * w["q"] * steps / el
    return {"value": rate, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{steps} full RK3 step(s) of the same {w['nx']}x{w['q']} problem in FP64 "
                      f"({el:.1f} s on {threads} OpenMP threads)",
            "single_thread_table1": cpu_single_thread_table1()}


def cpu_model():
    """Model name of the host CPU, from /proc/cpuinfo."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_single_thread_table1(seconds=3.0):
    """The oracle on one thread on the first Table I run (sigma = 1e-3, Q = 8, Nx = 1600,
    chi_RET-FM, dt = 1e-3), the like-for-like of the paper's single-core t_LB = 62 s:
    steps for `seconds`, extrapolated to 9000 steps."""
    import oracle
    from oracle.run import solver_from_workload
    import workloads
    oracle.set_threads(1)
    El = 0.4825
    w = workloads.sod_tube(El, 1e-3 / El, nx=1600, q=8)
    w["chi"], w["dt"] = "ret", 1e-3
    s = solver_from_workload(w)
    steps, t0 = 0, time.perf_counter()
    while True:
        s.step(10)
        steps += 10
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"updates_per_s": 1600 * 8 * steps / el, "cores": 1,
            "extrapolated_9000_steps_s": el / steps * 9000, "paper_t_lb_s": 62.0,
            "sample": f"{steps} steps in {el:.1f} s"}


def copy_calibration(torch, nbytes=1 << 30, reps=5, quiet=False):
    """A plain device-to-device copy of `nbytes` (reads nbytes, writes nbytes): the reference
    for scaling the HBM read/write counters, and the bandwidth a plain copy reaches on this
    GPU (median over `reps` copies, beside the vendor's 8 TB/s)."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record()
        dst.copy_(src)
        end.record()
        end.synchronize()
        times.append(start.elapsed_time(end))
    ms = sorted(times)[len(times) // 2]
    out = {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "ms_per_copy": ms,
           "GBps_read_plus_write": 2 * nbytes / ms / 1e6}
    del src, dst
    torch.cuda.empty_cache()
    if not quiet:
        print(json.dumps(out), flush=True)
    return out


def time_single(elb, torch, w, precision, steps, warmup, moment_fixup=0, runs=TIMED_RUNS):
    """Milliseconds for `steps` RK3 steps of one context on workload `w`: the median of `runs`
    timed runs of `steps` steps each, after `warmup` untimed steps.  Every timed run is
    bracketed by a device synchronisation on both sides, and its events are recorded on the
    stream the library launches on."""
    solver = elb.Solver(elb.params_from_workload(w, precision=precision, moment_fixup=moment_fixup),
                        device="cuda:0")
    solver.set_state_moments(w["n"], w["u"], w["T"])
    stream = solver.stream
    solver.step(warmup)
    times = []
    for _ in range(runs):
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        solver.step(steps)
        end.record(stream)
        end.synchronize()
        torch.cuda.synchronize()
        times.append(start.elapsed_time(end))
    solver.moments()  # surfaces ELB_ENONFINITE if the run went bad
    return sorted(times)[len(times) // 2]


def bench_batched(elb, torch, steps=50, warmup=10):
    """The 512-instance sweep (sound waves and standing shocks of uneven N_x, Q, E_l, Kn),
    FP32 with FP64 bookkeeping: one batch (tuned tile shapes, captured graph) against the
    same instances stepped one context after another on one stream."""
    import workloads
    ws = workloads.config3()
    pairs = sum(w["nx"] * w["q"] for w in ws)
    params = [elb.params_from_workload(w, precision=PRECISIONS["fp32_mixed"]) for w in ws]
    b = elb.BatchSolver(params, device="cuda:0")
    for i, w in enumerate(ws):
        b.set_state_moments(i, w["n"], w["u"], w["T"])
    b.tune()
    b.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(b.stream)
    b.step(steps)
    end.record(b.stream)
    end.synchronize()
    ms_batch = start.elapsed_time(end)
    for i in range(len(ws)):
        b.moments(i)
    groups = b.groups()
    b.close()
    del b

    solvers = []
    for p, w in zip(params, ws):
        s = elb.Solver(p, device="cuda:0")
        s.set_state_moments(w["n"], w["u"], w["T"])
        solvers.append(s)
    for s in solvers:
        s.step(warmup)
    torch.cuda.synchronize()
    stream = solvers[0].stream
    start.record(stream)
    for s in solvers:
        s.step(steps)
    end.record(stream)
    end.synchronize()
    ms_plain = start.elapsed_time(end)
    solvers[0].moments()
    del solvers
    torch.cuda.synchronize()
    v_b = pairs * steps / (ms_batch / 1e3)
    v_p = pairs * steps / (ms_plain / 1e3)
    return {"workload": f"sweep_{len(ws)}_instances_sum_nxq_{pairs}", "steps": steps,
            "value": v_b, "unit": "updates/s", "ms_per_step": ms_batch / steps,
            "plain_loop_value": v_p, "plain_loop_ms_per_step": ms_plain / steps,
            "speedup_vs_plain_loop": v_b / v_p, "groups": groups}


def _timed(torch, stream, fn):
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end)


def _rel(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _fit(learned, X, Y):
    tr = learned.Trainer(X, Y, batch=4096, lr=1e-3, seed=0, margin=0.1)
    tr.train(1500)
    tr.lr = 3e-4
    losses = tr.train(1500)
    return tr.result(), losses


def bench_learned(elb, torch, w, q_student=12, plain_steps=10000):
    """The shock tube run to the same physical time by the plain Q = 96 solver and by a
    Q = 12 student with the learned closure, trained here, on the GPU, outside the timed
    regions, on two other shock tubes of the same resolution: first on the teacher's own
    states, then again with samples along the corrected student's own runs added (one
    round of dataset aggregation, including the student's first steps).  The corrected runs
    add learned.CORRECTION_WEIGHT times the correction.  FP32 with FP64 bookkeeping."""
    import numpy as np
    from paper_2211_16933_amd import learned
    import workloads
    mixed = PRECISIONS["fp32_mixed"]
    t0 = time.perf_counter()
    tubes = workloads.closure_tubes(w["nx"], w["q"])
    X, Y = learned.generate(tubes, w["q"], q_student, start=500, every=1000, count=10, active=1e-4)
    (p0, n0), _ = _fit(learned, X, Y)
    Xs, Ys = learned.generate_on_student(tubes, w["q"], q_student, p0, n0, start=150, every=300,
                                         count=10, relax=20, active=1e-4, seed=1)
    # the student's first steps, while the initial jump is still sharp (every 15 steps up to
    # 135 with the teacher relaxed 20 steps, and each of the first 8 steps with 3): without
    # them the corrected run leaves the training range near the membrane in its first steps
    Xe, Ye = learned.generate_on_student(tubes, w["q"], q_student, p0, n0, start=0, every=15,
                                         count=10, relax=20, active=1e-4, seed=2)
    Xf, Yf = learned.generate_on_student(tubes, w["q"], q_student, p0, n0, start=0, every=1,
                                         count=8, relax=3, active=1e-4, seed=3)
    (params, norm), losses = _fit(learned, np.concatenate([X, Xs, Xe, Xf]),
                                  np.concatenate([Y, Ys, Ye, Yf]))
    prep_s = time.perf_counter() - t0

    plain = elb.Solver(elb.params_from_workload(w, precision=mixed), device="cuda:0")
    plain.set_state_moments(w["n"], w["u"], w["T"])
    ms_plain = _timed(torch, plain.stream, lambda: plain.step(plain_steps))
    ref = plain.moments()
    t_end = plain_steps * plain.info["dt"]
    ws = dict(w, q=q_student)
    alone = elb.Solver(elb.params_from_workload(ws, precision=mixed), device="cuda:0")
    alone.set_state_moments(w["n"], w["u"], w["T"])
    ns = int(round(t_end / alone.info["dt"]))
    ms_alone = _timed(torch, alone.stream, lambda: alone.step(ns))
    m_alone = alone.moments()
    # the correction evaluated by two kernels before each stage (the reference form), timed
    # for comparison; then inside the stage kernel (the default), whose result is used
    sep = elb.Solver(elb.params_from_workload(ws, precision=mixed, closure=1), device="cuda:0")
    sep.set_state_moments(w["n"], w["u"], w["T"])
    sep.set_closure(params, learned.weighted_norm(norm), 2)
    ms_separate = _timed(torch, sep.stream, lambda: sep.step(ns))
    sep.close()
    stud = elb.Solver(elb.params_from_workload(ws, precision=mixed, closure=1), device="cuda:0")
    stud.set_state_moments(w["n"], w["u"], w["T"])
    stud.set_closure(params, learned.weighted_norm(norm), True)
    ms_learned = _timed(torch, stud.stream, lambda: stud.step(ns))
    try:
        outside = stud.closure_outside()
        m_learned = stud.moments()
    except elb.ElbError:     # the corrected run broke down: the fine solver's answer is used
        outside, m_learned = -1, None
    used = "learned" if outside == 0 else "fallback"
    cs = float(np.sqrt(np.mean(ref[2])))

    def errs(m):
        return {"n": _rel(m[0], ref[0]), "T": _rel(m[2], ref[2]),
                "u_over_cs": float(np.linalg.norm(m[1] - ref[1]) / (np.sqrt(ref[1].size) * cs))}

    ms_used = ms_learned if used == "learned" else ms_learned + ms_plain
    return {"workload": f"{w['name']} to t={t_end:.4e}: plain q{w['q']} vs student q{q_student}",
            "plain_ms": ms_plain, "plain_steps": plain_steps,
            "student_steps": ns, "student_alone_ms": ms_alone, "learned_ms": ms_learned,
            "learned_separate_kernels_ms": ms_separate,
            "learned_updates_per_s": w["nx"] * q_student * ns / (ms_learned / 1e3),
            "speedup_vs_plain": ms_plain / ms_used, "used": used, "cells_outside": outside,
            "errors_vs_plain": {"learned": errs(m_learned) if m_learned is not None else None,
                                "student_alone": errs(m_alone)},
            "training": {"samples_teacher_states": int(X.shape[0]),
                         "samples_student_states": int(Xs.shape[0] + Xe.shape[0] + Xf.shape[0]),
                         "final_loss": losses[-1],
                         "prep_seconds": prep_s}}


# Table I of the paper (Sod tube, eta_i = 0.05, L = 80, dt = 1e-3, chi_RET-FM): molecular
# diameter, velocity nodes, cells and the single-core time t_LB it reports (seconds; Xeon Gold
# 6330, end time not stated).
TABLE1 = [(1e-3, 8, 1600, 62.0), (1e-2, 8, 800, 32.0), (1e-1, 20, 640, 71.0), (1.0, 200, 160, 176.0)]


def bench_table1(elb, torch, steps=9000, precision="fp64"):
    """The Sod runs of Table I on the GPU, 9000 steps each (t = 9, the time the paper's
    profiles are labelled with), in FP64.  The paper's single-core times are context: its
    step count is not stated."""
    import workloads
    El = 0.4825  # the denseness the paper prints for eta_i = 0.05
    out = []
    for sigma, q, nx, t_lb in TABLE1:
        w = workloads.sod_tube(El, sigma / El, nx=nx, q=q)
        w["chi"], w["dt"] = "ret", 1e-3
        s = elb.Solver(elb.params_from_workload(w, precision=PRECISIONS[precision]), device="cuda:0")
        s.set_state_moments(w["n"], w["u"], w["T"])
        s.step(100)
        torch.cuda.synchronize()
        ms = _timed(torch, s.stream, lambda: s.step(steps))
        s.moments()
        out.append({"sigma": sigma, "q": q, "nx": nx, "steps": steps, "gpu_s": ms / 1e3,
                    "updates_per_s": nx * q * steps / (ms / 1e3), "paper_t_lb_s": t_lb})
    return {"workload": "sod_tube_eta0.05_L80_dt1e-3_chi_ret (Table I)", "dtype": DTYPES[precision],
            "runs": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32_mixed", choices=sorted(PRECISIONS))
    ap.add_argument("--nx", type=int, default=65536)
    ap.add_argument("--q", type=int, default=96)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the other precisions and the batched sweep")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for HBM counter scaling)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched sweep against the plain loop (for profiling)")
    ap.add_argument("--learned-only", action="store_true",
                    help="only the learned-closure comparison on the large tube (for profiling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    import paper_2211_16933_amd as elb
    import workloads

    w = workloads.shock_tube(nx=args.nx, q=args.q)
    if args.batched_only:
        print(json.dumps({"batched_sweep_fp32_mixed": bench_batched(elb, torch, steps=args.steps,
                                                                    warmup=args.warmup)}),
              flush=True)
        return
    if args.learned_only:
        print(json.dumps({"learned_closure_q12": bench_learned(elb, torch, w)}), flush=True)
        return
    copy = copy_calibration(torch, quiet=True)
    ms = time_single(elb, torch, w, PRECISIONS[args.precision], args.steps, args.warmup)

    pairs = w["nx"] * w["q"]
    value = pairs * args.steps / (ms / 1e3)
    elem = 8 if args.precision == "fp64" else 4
    per_pair = stage_bytes_per_pair(elem, w["q"] if args.precision == "fp32_mixed" else None)
    launch_s = ms / 1e3 / (3 * args.steps)
    achieved = pairs * per_pair / launch_s / 1e9
    traffic_bytes = measured_traffic() if (args.precision == "fp32_mixed" and args.nx == 65536
                                           and args.q == 96) else None
    traffic = traffic_bytes / launch_s / 1e9 if traffic_bytes else None
    out = {
        "metric": "cell-velocity updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic",
        "config": {"workload": f"shock_tube_nx{w['nx']}_q{w['q']}", "nx": w["nx"], "q": w["q"],
                   "denseness": w["denseness"], "kn": w["kn"], "precision": args.precision},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_stage", "bytes_per_pair_per_launch": per_pair,
                     "algorithmic_bytes_per_launch": pairs * per_pair,
                     "traffic_bytes_per_launch": traffic_bytes,
                     "avg_launch_us": launch_s * 1e6,
                     "timing": f"median of {TIMED_RUNS} timed runs of {args.steps} steps",
                     # a plain 1 GiB device copy on the same GPU, read + write bytes
                     "measured_copy_GBps": copy["GBps_read_plus_write"],
                     # the same launches against the vector ALU (operation count of the
                     # method, not instructions issued), at the FP32 vector rate
                     "alu_view": {"flop_per_pair_per_launch": stage_flop_per_pair(w["q"]),
                                  "achieved": pairs * stage_flop_per_pair(w["q"]) / launch_s / 1e12,
                                  "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": pairs * stage_flop_per_pair(w["q"]) / launch_s / 1e12
                                  / FP32_VECTOR_PEAK_TFLOPS}},
    }
    if not args.no_variants:
        variants = {}
        for name in sorted(PRECISIONS):
            if name == args.precision:
                continue
            vms = time_single(elb, torch, w, PRECISIONS[name], args.steps, args.warmup)
            variants[f"{out['config']['workload']}_{name}"] = {
                "value": pairs * args.steps / (vms / 1e3), "unit": "updates/s",
                "ms_per_step": vms / args.steps, "dtype": DTYPES[name]}
        # FP32 with bookkeeping and the moment fix-up of the FP32 rows in every stage
        vms = time_single(elb, torch, w, PRECISIONS["fp32_mixed"], args.steps, args.warmup,
                          moment_fixup=1)
        variants[f"{out['config']['workload']}_fp32_mixed_fixup"] = {
            "value": pairs * args.steps / (vms / 1e3), "unit": "updates/s",
            "ms_per_step": vms / args.steps, "dtype": DTYPES["fp32_mixed"]}
        variants["batched_sweep_fp32_mixed"] = bench_batched(elb, torch)
        # four times the cells (604 MB of FP32 state per level set, well past the 256 MB
        # last-level cache): the per-pair rate should not depend on cache residency
        wl = workloads.shock_tube(nx=4 * args.nx, q=args.q)
        lms = time_single(elb, torch, wl, PRECISIONS[args.precision], max(1, args.steps // 4),
                          max(1, args.warmup // 4))
        lsteps = max(1, args.steps // 4)
        l_launch_s = lms / 1e3 / lsteps / 3
        variants[f"shock_tube_nx{4 * args.nx}_q{args.q}_{args.precision}"] = {
            "value": 4 * pairs * lsteps / (lms / 1e3), "unit": "updates/s",
            "ms_per_step": lms / lsteps, "dtype": DTYPES[args.precision],
            "avg_launch_us": l_launch_s * 1e6,
            "hbm_frac": 4 * pairs * per_pair / l_launch_s / 1e9 / HBM_PEAK_GBS}
        variants["table1_sod_replay"] = bench_table1(elb, torch)
        if args.nx == 65536 and args.q == 96:
            variants["learned_closure_q12"] = bench_learned(elb, torch, w)
        out["variants"] = variants
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, seconds=args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
