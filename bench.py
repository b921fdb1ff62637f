"""Benchmark: fused J + gradient evaluations of a batch of KS connecting curves
on one MI355X.

A step is one evaluation of J^2 and its adjoint gradient for every curve of
the batch (the fused tile kernel plus the post kernel that finishes the tile
boundary rows and the FP64 per-curve cost).  Workload (default): 64 curves,
L = 66, N_x = 128 (43 kept modes), N_s = 1024, finite map T = 20, FP32 with
FP64 cost reduction; each curve is a stored KS trajectory piece (20 time
units) plus a seeded smooth perturbation.  --workload c1/c2/c3 selects the
single-curve and uneven-batch shapes, p22 the paper-shape batch (64 curves,
L = 22, N_x = 64, N_s = 552, rational map S = 55), --dtype f64 the FP64
finish, --space odd the inversion-symmetric subspace (the same curves' sine
coefficients b_k = Im u_hat_k), --ds spectral the rational-Chebyshev d/ds
(then the roofline is the FP64 matrix-core one of the D_t products).

Prints one JSON line.  value = curve-point evals/s = sum_c (N_s - 2) * steps / s
over K timed steps; the roofline block uses the fused kernel's own duration
from HIP events recorded by the library around each launch (a second window
of K steps).  Extra legs: the plain policy (one launch per curve), the fused
descent step, the captured-graph descent loop, autograd forward+backward, the
streaming roofline (the batch replicated past the 256 MB last-level cache),
the same curves in the inversion-symmetric subspace, the descent step with
the s-part implicit (banded solves), the paper-shape batch with the spectral
d/ds, and the FP64 oracle timed on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "curve-point gradient evals/s (J+∇J) & % HBM roofline, batched vs plain"
HBM_PEAK_GBS = 8000.0
# Vector ALU peak without packed FP32 (the kernels are built without it): one
# FP32 or FP64 FMA per lane per clock, 256 CUs x 4 SIMDs x 16 lanes x 2 flop
# x 2.4 GHz.
ALU_PEAK_TFLOPS = 78.6
# Dense FP64 matrix-core peak: the products along s run in FP64 for both dtypes.
MFMA_F64_PEAK_TFLOPS = 78.6


def flops_per_row(n_x: int) -> float:
    """Algorithmic flops of one J + gradient row evaluation: four real
    transforms of n_x points (2.5 n log2 n flops each, half of a complex FFT's
    5 n log2 n) plus the pointwise and per-mode work: n_x (10 log2 n_x + 12)."""
    import math
    return n_x * (10 * math.log2(n_x) + 12)


def flops_per_row_odd(n_x: int) -> float:
    """The same for a row of the inversion-symmetric subspace, m = n_x / 2:
    four real DFTs of m points (2.5 m log2 m each) inside the DST-I / DCT-I
    pairs, their pre/post-processing (about 5 m each) and the pointwise and
    per-mode work (about 15 m): m (10 log2 m + 35)."""
    import math
    m = n_x // 2
    return m * (10 * math.log2(m) + 35)


# Sources of the fused tile kernel (full space, inversion-symmetric subspace);
# a traffic summary under profiles/ applies only while their hash is the one
# recorded there.
KERNEL_SOURCES = {
    "full": ("ksc_tile.hpp", "ksc_fft.hpp", "ksc_lanes.hpp", "ksc_fused.hip", "ksc_launch.hpp"),
    "odd": ("ksc_tile.hpp", "ksc_fft.hpp", "ksc_sym.hpp", "ksc_odd.hpp", "ksc_odd.hip",
            "ksc_launch_odd.hpp"),
}
# Launch shapes chosen by the autotuner (ksc_tune) on an MI355X for the bench
# workloads, so that every run (and every profiler run) uses the same shape.
TUNE_CACHE = os.path.join(ROOT, "paper_2301_11704_amd", "tuning_gfx950.json")
STREAM_REPLICAS = {"c4": 48, "c2": 191, "c3": 20, "c1": 0}
DTAU = {"c4": 5e-4, "c2": 1e-4, "c3": 1e-3, "c1": 1e-3, "p22": 0.01}


def kernel_source_hash(space: str = "full") -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[space]:
        with open(os.path.join(ROOT, "paper_2301_11704_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload: str, dtype: str, space: str = "full"):
    """HBM bytes per launch of the fused J+gradient kernel from the committed
    rocprofv3 counter summary, or None if there is none or the kernel sources
    changed since it was taken."""
    kind = "fused_grad" if space == "full" else "odd_grad"
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}_{dtype}_traffic.md")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                kv[k.strip()] = v.strip().strip("`")
    if kv.get("kernel_source_sha256") != kernel_source_hash(space):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _specs_and_states(workload: str):
    import ksinputs
    if workload == "c4":
        specs, Us = ksinputs.config4_curves(64)
        return specs, Us, "finite"
    if workload == "p22":
        specs = ksinputs.paper_shape_specs(64)
        Us = [ksinputs.make_curve(s, (s.n_x - 1) // 3 + 1)[2] for s in specs]
        return specs, Us, "rational"
    cfg = {"c1": 1, "c2": 2, "c3": 3}[workload]
    specs = ksinputs.config_specs(cfg)
    Us = []
    for s in specs:
        K1 = (s.n_x - 1) // 3 + 1
        Us.append(ksinputs.make_curve(s, K1)[2])
    return specs, Us, specs[0].map


def _describe(workload, specs, space="full"):
    ns = [s.n_s for s in specs]
    nx = sorted(set(s.n_x for s in specs))
    return {
        "workload": {
            "c4": "64 KS curves, L=66, N_x=128, N_s=1024, finite map T=20 (batched autograd-path shape)",
            "c1": "1 KS curve, L=39, N_x=64, N_s=512",
            "c2": "1 KS curve, L=100, N_x=256, N_s=8192",
            "c3": "256 uneven KS curves, N_x in {32,64,128}, N_s in [128,2048]",
            "p22": "64 KS curves with the paper's E1->E2 discretization: L=22, N_x=64, "
                   "N_s=552 (M=550), rational map S=55",
        }[workload],
        "curves": len(specs),
        "n_x": nx if len(nx) > 1 else nx[0],
        "n_s_total": int(sum(ns)),
        "curve_points": int(sum(n - 2 for n in ns)),
        # FP32 state: K+1 complex values per row, or K reals in the odd subspace
        "state_MB": round(sum(n * ((s.n_x - 1) // 3 * 4 if space == "odd" else ((s.n_x - 1) // 3 + 1) * 8)
                              for n, s in zip(ns, specs)) / 1e6, 3),
    }


def odd_states(Us):
    """The sine coefficients b_k = Im u_hat_k, k = 1..K, of full-space curves
    (their projection onto the inversion-symmetric subspace)."""
    return [np.ascontiguousarray(U[:, 1:].imag) for U in Us]


def _time(torch, fn, steps, stream):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms


def _oracle_eval(args):
    """One curve's J2 + gradient with the FP64 oracle (a pool task)."""
    import oracle
    import ksinputs
    s, U = args
    c = oracle.Curve(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0)
    Ur = ksinputs.round_to(U, np.float32)
    oracle.J2(c, Ur)
    oracle.grad(c, Ur)
    return s.n_s - 2


def cpu_baseline(specs, Us, budget_s=12.0, single_s=6.0):
    """The FP64 oracle (as it stands) on the host, J2 + gradient per curve:
    a pool of worker processes over the host cores (one curve per task, curves
    taken in order, about budget_s of wall time), and one thread alone (about
    single_s).  NumPy's FFT is single-threaded, so each worker uses one core."""
    import concurrent.futures as cf
    import multiprocessing as mp
    # one thread alone
    t0 = time.perf_counter()
    pts = n = 0
    while True:
        pts += _oracle_eval((specs[n % len(specs)], Us[n % len(Us)]))
        n += 1
        el1 = time.perf_counter() - t0
        if el1 >= single_s:
            break
    single = {"value": pts / el1, "cores": 1,
              "sample": f"{n} curve evaluations in {el1:.1f} s"}
    # pool over the host cores (fresh interpreters: the parent holds a GPU context)
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    workers = max(1, min(16, ncpu))
    per_task_s = el1 / n
    n_tasks = max(workers, int(budget_s * workers / per_task_s))
    tasks = [(specs[i % len(specs)], Us[i % len(Us)]) for i in range(n_tasks)]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_oracle_eval, tasks[:workers]))  # start-up and imports, not timed
        t0 = time.perf_counter()
        # chunks of tasks per hand-off, so that inter-process traffic does not
        # dominate the few-millisecond tasks
        pts = sum(ex.map(_oracle_eval, tasks, chunksize=max(1, n_tasks // (8 * workers))))
        el = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": pts / el, "unit": "curve-point evals/s", "cores": workers, "kind": "oracle",
        "cpu_model": model,
        "sample": f"{n_tasks} curve evaluations (J2 + gradient, FP64 NumPy) by {workers} worker "
                  f"processes in {el:.1f} s",
        "single_thread": single,
    }


def spectral_gemm_flops(specs, n_products):
    """Flops of the dense D_t products along s: 2 N_s^2 2(K+1) per curve each."""
    return n_products * sum(2.0 * s.n_s * s.n_s * 2 * ((s.n_x - 1) // 3 + 1) for s in specs)


def spectral_leg(ksc, torch, tdt, esz, args, stream):
    """J + gradient with the paper's spectral d/ds (dense D_t on matrix cores)
    on the paper-shape batch: time per evaluation and the MFMA fraction of the
    two products over the whole evaluation window (per-kernel durations are in
    the kernel-trace profile)."""
    specs, Us, _ = _specs_and_states("p22")
    descs = [ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs]
    ps = ksc.Problem(descs, dtype=tdt, ds="spectral")
    Xs = ps.new_state()
    for c, U in enumerate(Us):
        ps.upload(Xs, c, U)
    Gs = torch.empty_like(Xs)
    ps.tune(None if args.retune else args.tune_cache)
    pol, w = ps.launch

    def f():
        ps.eval_grad(Xs, Gs)

    for _ in range(args.warmup):
        f()
    ms = _time(torch, f, args.steps, stream)
    ps.set_timing(True)
    _time(torch, f, args.steps, stream)
    fs, qs, ns = ps.read_timing()
    ps.set_timing(False)
    win = fs / ns
    gf = spectral_gemm_flops(specs, 2)
    peak = MFMA_F64_PEAK_TFLOPS
    pts = sum(s.n_s - 2 for s in specs)
    res = {
        "workload": _describe("p22", specs)["workload"], "ms_per_step": ms,
        "curve_points_per_s": pts / (ms * 1e-3), "window_ms": win, "post_kernel_ms": qs / ns,
        "launch": {"policy": pol, "waves_per_tile": w},
        "mfma": {"gemm_flops_per_eval": gf, "achieved_over_window": gf / (win * 1e-3) / 1e12,
                 "peak": peak, "unit": "TFLOP/s", "frac": gf / (win * 1e-3) / 1e12 / peak},
    }
    del Xs, Gs, ps
    return res


def _alg_per_launch(specs, esz, space):
    """Algorithmic bytes (read the state, write the gradient) and flops of one
    J + gradient launch over the batch."""
    if space == "odd":
        elems = sum(s.n_s * ((s.n_x - 1) // 3) for s in specs)  # K reals per row
        return 2.0 * esz * elems, sum(s.n_s * flops_per_row_odd(s.n_x) for s in specs)
    elems = sum(s.n_s * ((s.n_x - 1) // 3 + 1) for s in specs)  # K+1 complex per row
    return 2.0 * 2 * esz * elems, sum(s.n_s * flops_per_row(s.n_x) for s in specs)


def odd_leg(ksc, torch, descs, Us, tdt, esz, specs, args, stream, full_kernel_ms):
    """J + gradient of the same curves in the inversion-symmetric subspace:
    step time, the kernel's own duration and its rooflines."""
    po = ksc.Problem(descs, dtype=tdt, space="odd")
    Xo = po.new_state()
    for c, B in enumerate(odd_states(Us)):
        po.upload(Xo, c, B)
    Go = torch.empty_like(Xo)
    po.tune(None if args.retune else args.tune_cache)
    pol, w = po.launch

    def f():
        po.eval_grad(Xo, Go)

    for _ in range(args.warmup):
        f()
    ms = _time(torch, f, args.steps, stream)
    po.set_timing(True)
    _time(torch, f, args.steps, stream)
    fo, qo, no = po.read_timing()
    po.set_timing(False)
    k_ms = fo / no
    b, fl = _alg_per_launch(specs, esz, "odd")
    pts = sum(s.n_s - 2 for s in specs)
    res = {
        "ms_per_step": ms, "curve_points_per_s": pts / (ms * 1e-3), "kernel_ms": k_ms,
        "post_kernel_ms": qo / no, "launch": {"policy": pol, "waves_per_tile": w},
        "kernel_speedup_vs_full": full_kernel_ms / k_ms,
        "alu": {"achieved": fl / (k_ms * 1e-3) / 1e12, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": fl / (k_ms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS},
        "hbm": {"achieved": b / (k_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": b / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "traffic": recorded_traffic(args.workload, args.dtype, "odd"),
    }
    del Xo, Go, po
    return res


def implicit_s_leg(ksc, torch, descs, Us, tdt, esz, args, stream, ms_paper):
    """The implicit-in-s descent step (the whole linear part implicit, banded
    solves along s) on the same curves: ms per step in captured-graph descent
    against the paper's step, and the solve's share (the step minus the J +
    gradient evaluation it starts with)."""
    pi = ksc.Problem(descs, dtype=tdt, space=args.space)
    pi.set_scheme("implicit_s")
    Xi = pi.new_state()
    for c, U in enumerate(odd_states(Us) if args.space == "odd" else Us):
        pi.upload(Xi, c, U)
    Gi = torch.empty_like(Xi)
    Si = torch.empty_like(Xi)
    pi.tune(None if args.retune else args.tune_cache)
    dtau = DTAU[args.workload]
    pi.descend(Xi, 200, dtau, every=100, scratch=Si)
    nd = 100 * max(2, args.steps // 50)
    ms_i = _time(torch, lambda: pi.descend(Xi, nd, dtau, every=100, scratch=Si), 1, stream) / nd
    ms_g = _time(torch, lambda: pi.eval_grad(Xi, Gi), args.steps, stream)
    solve_ms = max(ms_i - ms_g, 0.0)
    state_b = Xi.numel() * esz
    res = {"ms_per_step": ms_i, "ms_per_step_paper_scheme": ms_paper,
           "cost_ratio_vs_paper_step": ms_i / ms_paper, "eval_grad_ms": ms_g,
           "solve_ms_est": solve_ms,
           # the solve reads the state and the gradient and writes the next state
           "solve_alg_GBs_est": 3 * state_b / (solve_ms * 1e-3) / 1e9 if solve_ms > 0 else None}
    del Xi, Gi, Si, pi
    return res


def streaming_leg(ksc, torch, tdt, esz, workload, args, stream):
    """J + gradient of another workload replicated past the 256 MB last-level
    cache (STREAM_REPLICAS copies of its batch, >= 1 GB per state array), with
    its tuned launch shape: the fused kernel's duration from the library's
    events and its HBM fraction (algorithmic bytes / kernel time / 8 TB/s)."""
    specs, Us, _ = _specs_and_states(workload)
    descs = [ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs]
    p1 = ksc.Problem(descs, dtype=tdt)
    p1.tune(None if args.retune else args.tune_cache)
    pol, w = p1.launch
    X1 = p1.new_state()
    for c, U in enumerate(Us):
        p1.upload(X1, c, U)
    reps = STREAM_REPLICAS[workload]
    pb = ksc.Problem([d for _ in range(reps) for d in descs], dtype=tdt)
    pb.set_launch(pol, w)
    Xb = X1.repeat(reps)
    Gb = torch.empty_like(Xb)
    del X1, p1
    for _ in range(3):
        pb.eval_grad(Xb, Gb, want_J2=False)
    nb = max(5, args.steps // 10)
    pb.set_timing(True)
    msb = _time(torch, lambda: pb.eval_grad(Xb, Gb), nb, stream)
    fb, _, nbe = pb.read_timing()
    pb.set_timing(False)
    kb = fb / nbe
    bb = _alg_per_launch(specs, esz, "full")[0] * reps
    res = {"workload": _describe(workload, specs)["workload"], "replicas": reps,
           "state_GB": Xb.numel() * esz / 1e9, "launch": {"policy": pol, "waves_per_tile": w},
           "ms_per_step": msb, "kernel_ms": kb, "achieved_GBs": bb / (kb * 1e-3) / 1e9,
           "frac_hbm": bb / (kb * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "curve_points_per_s": sum(s.n_s - 2 for s in specs) * reps / (msb * 1e-3)}
    del Xb, Gb, pb
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c4", choices=["c4", "c1", "c2", "c3", "p22"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the host oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip plain and streaming legs")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--space", default="full", choices=["full", "odd"],
                    help="state space of the timed problem (odd: inversion-symmetric subspace)")
    ap.add_argument("--ds", default="stencil", choices=["stencil", "spectral"],
                    help="d/ds of the timed problem (spectral: the paper's D_t; rational map)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE, metavar="PATH",
                    help="launch-shape cache read (or, for a shape it lacks, tuned and "
                         "appended) by the autotuner; default: the cache shipped with the package")
    ap.add_argument("--retune", action="store_true",
                    help="time the launch shapes now instead of reading the cache")
    ap.add_argument("--replicas", type=int, default=None,
                    help="streaming-leg replication factor (default per workload)")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="GB",
                    help="only run one plain device-to-device copy of this many GB (calibrates "
                         "the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the batched path "
              "is single-device by design", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.copy_probe > 0:
        n = int(args.copy_probe * 1e9) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n}))
        return

    import paper_2301_11704_amd as ksc
    stream = torch.cuda.current_stream()
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    esz = 8 if args.dtype == "f64" else 4
    specs, Us, _ = _specs_and_states(args.workload)
    descs = [ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs]
    prob = ksc.Problem(descs, dtype=tdt, space=args.space, ds=args.ds)
    X = prob.new_state()
    for c, U in enumerate(odd_states(Us) if args.space == "odd" else Us):
        prob.upload(X, c, U)
    G = torch.empty_like(X)
    prob.tune(None if args.retune else args.tune_cache)
    policy, waves = prob.launch

    def step():
        prob.eval_grad(X, G)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ms = _time(torch, step, args.steps, stream)
    # the same K evaluations again with HIP events around each kernel (on the
    # stream the library launches on): the dominant kernel's own duration
    prob.set_timing(True)
    ms_ev = _time(torch, step, args.steps, stream)
    fused_ms, post_ms, n_ev = prob.read_timing()
    prob.set_timing(False)
    kernel_ms = fused_ms / n_ev
    post_kernel_ms = post_ms / n_ev

    info = _describe(args.workload, specs, args.space)
    pts = info["curve_points"]
    value = pts / (ms * 1e-3)
    alg_bytes, alg_flops = _alg_per_launch(specs, esz, args.space)
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    tflops = alg_flops / (kernel_ms * 1e-3) / 1e12
    traffic = recorded_traffic(args.workload, args.dtype, args.space)

    if args.ds == "spectral":
        # the products along s dominate: MFMA roofline over the evaluation window
        gf = spectral_gemm_flops(specs, 2)
        peak = MFMA_F64_PEAK_TFLOPS
        roof = {"bound": "mfma", "achieved": gf / (kernel_ms * 1e-3) / 1e12, "peak": peak,
                "unit": "TFLOP/s", "frac": gf / (kernel_ms * 1e-3) / 1e12 / peak, "traffic": None,
                "kernel": "D_t products + row kernel (window)", "kernel_ms": kernel_ms,
                "alg_flops_per_launch": gf, "post_kernel_ms": post_kernel_ms,
                "ms_per_step_with_events": ms_ev}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "curve-point evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": dict(info, space=args.space, ds=args.ds,
                       launch={"policy": policy, "waves_per_tile": waves,
                               "tuned": "now" if args.retune else "cache"}),
        # The metric's roofline is HBM bandwidth: algorithmic bytes (read the
        # state, write the gradient) over the fused kernel's own duration,
        # against 8 TB/s.  The kernel also sits near the ridge of the
        # non-packed vector ALU (78.6 TFLOP/s / 8 TB/s = 9.8 flop/B against
        # ~15 flop/B of algorithmic work at n_x = 128), so its ALU fraction is
        # reported beside it; the streaming leg gives the HBM fraction with the
        # batch replicated past the last-level cache.
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "fused J+gradient tile kernel" + (" (odd subspace)" if args.space == "odd" else ""),
            "kernel_ms": kernel_ms,
            "alg_bytes_per_launch": alg_bytes, "alg_flops_per_launch": alg_flops,
            "alu": {"achieved": tflops, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tflops / ALU_PEAK_TFLOPS},
            "target_frac": 0.60,
            "post_kernel_ms": post_kernel_ms, "ms_per_step_with_events": ms_ev,
            "grid_point_evals_per_s": sum((s.n_s - 2) * s.n_x for s in specs) / (ms * 1e-3),
        },
    }
    if args.ds == "spectral":
        out["roofline"] = roof

    if not args.no_extras:
        # plain: one non-persistent launch per curve and step
        prob.set_launch(ksc.KSC_LAUNCH_PLAIN, waves)
        ms_plain = _time(torch, step, max(10, args.steps // 4), stream)
        prob.set_launch(policy, waves)
        out["plain"] = {"value": pts / (ms_plain * 1e-3), "ms_per_step": ms_plain,
                        "speedup_batched_vs_plain": ms_plain / ms}
        # the fused descent step (state -> scratch), eager launches
        Y = X.clone()
        dtau = DTAU[args.workload]
        ms_step = _time(torch, lambda: prob.step(X, Y, dtau), args.steps, stream)
        out["step"] = {"ms_per_step": ms_step, "curve_points_per_s": pts / (ms_step * 1e-3),
                       "alg_GBs": alg_bytes / (ms_step * 1e-3) / 1e9}
        # descent loop as captured HIP graphs (100 steps per graph)
        Z = X.clone()
        prob.descend(Z, 200, dtau, every=100, scratch=Y)
        nd = 100 * max(2, args.steps // 50)
        ms_d = _time(torch, lambda: prob.descend(Z, nd, dtau, every=100, scratch=Y), 1, stream)
        out["descend_graph"] = {"steps": nd, "ms_per_step": ms_d / nd,
                                "curve_points_per_s": pts * nd / (ms_d * 1e-3)}
        del Z
        # autograd forward (J only) + backward (recomputing adjoint)
        Xr = X.clone().requires_grad_(True)

        def fwd_bwd():
            Xr.grad = None
            ksc.curve_J2(Xr, prob).sum().backward()

        for _ in range(3):
            fwd_bwd()
        ms_ag = _time(torch, fwd_bwd, max(10, args.steps // 4), stream)
        out["autograd"] = {"ms_per_step": ms_ag, "curve_points_per_s": pts / (ms_ag * 1e-3),
                           "GBs_vs_method_minimum": alg_bytes / (ms_ag * 1e-3) / 1e9,
                           "GBs_vs_recompute_design": 1.5 * alg_bytes / (ms_ag * 1e-3) / 1e9}
        del Xr, Y
        if args.ds == "stencil":
            out["implicit_s"] = implicit_s_leg(ksc, torch, descs, Us, tdt, esz, args, stream,
                                               ms_d / nd)
        if args.ds == "stencil" and args.dtype == "f32":
            out["spectral_ds"] = spectral_leg(ksc, torch, tdt, esz, args, stream)
        if args.space == "full" and args.ds == "stencil" and \
                not (args.dtype == "f64" and max(s.n_x for s in specs) > 128):
            out["odd_space"] = odd_leg(ksc, torch, descs, Us, tdt, esz, specs, args, stream,
                                       kernel_ms)
        reps = STREAM_REPLICAS[args.workload] if args.replicas is None else args.replicas
        if reps > 1:
            # the batch replicated past the caches (MALL is 256 MB)
            big = [d for _ in range(reps) for d in descs]
            pb = ksc.Problem(big, dtype=tdt)
            Xb = X.repeat(reps)
            Gb = torch.empty_like(Xb)
            pb.set_launch(policy, waves)
            for _ in range(3):
                pb.eval_grad(Xb, Gb, want_J2=False)
            nb = max(5, args.steps // 10)
            pb.set_timing(True)
            msb = _time(torch, lambda: pb.eval_grad(Xb, Gb), nb, stream)
            fb, _, nbe = pb.read_timing()
            pb.set_timing(False)
            kb = fb / nbe
            bb = alg_bytes * reps
            out["streaming"] = {
                "replicas": reps, "state_GB": Xb.numel() * esz / 1e9, "ms_per_step": msb,
                "kernel_ms": kb, "achieved_GBs": bb / (kb * 1e-3) / 1e9,
                "frac_hbm": bb / (kb * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "frac_alu": alg_flops * reps / (kb * 1e-3) / 1e12 / ALU_PEAK_TFLOPS,
                "curve_points_per_s": pts * reps / (msb * 1e-3),
            }
            if args.ds == "stencil":
                out["roofline"]["streaming_frac"] = out["streaming"]["frac_hbm"]
            del Xb, Gb, pb

        # streaming legs of the other two roofline workloads (the batch
        # replicated past the caches), so that one default run records all
        # three HBM fractions
        if args.workload == "c4" and args.dtype == "f32" and args.space == "full" and \
                args.ds == "stencil" and args.replicas is None:
            out["streaming_other"] = {w: streaming_leg(ksc, torch, tdt, esz, w, args, stream)
                                      for w in ("c2", "c3")}

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(specs, Us)
        out["cpu_baseline"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
