#!/usr/bin/env python3
"""Throughput of the differentiable sparse solve's hot path on one MI355X.

Default workload (one "step" = one full solve): 3D 7-point cell-centred
diffusion on a 256^3 grid (n = 16,777,216, nnz = 117,047,296), log-normal
kappa = exp(g), g ~ N(0,1) per cell, harmonic-mean faces, Dirichlet ghosts,
b ~ N(0,1); Jacobi-preconditioned CG to ||r|| <= 1e-8 ||b|| from x0 = 0, FP64.
Inputs are generated on the host from fixed seeds and are resident in HBM
before the timed region starts.

Prints one JSON line on stdout (progress goes to stderr):
  value      solves/s (whole job, one GPU)
  roofline   the dominant kernel (SpMV fused with p.q) against HBM peak:
             achieved = algorithmic bytes per launch of the stored form the
             kernel streams / mean launch duration, durations from HIP events
             around every SpMV launch of profiled solves run right after the
             timed region (the timed solves replay graphs and carry no
             events); csr_unit prices the same launches at the CSR SpMV
             unit 12 nnz + 4(n+1) + 16n; traffic = FETCH_SIZE + WRITE_SIZE
             per launch from the committed rocprofv3 counter summary (null if
             the kernel source changed since the counters were taken)
  cpu_baseline  the CPU oracle timed on a bounded sample of the same system
             on all host cores (threaded mode) and on one thread: the
             difference of a short and a longer capped PCG run, scaled by the
             GPU solve's iteration count

Other modes:
  --summarize-rocprof DIR --label NAME   turn rocprofv3 output into a text
                                         summary under profiles/
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "solves/s to rtol 1e-8, learned-FSAI vs Jacobi PCG; SpMV/CG HBM GB/s vs peak"
HBM_PEAK_GBPS = 8000.0
DOMINANT = "k_cg_spmv_dot"
COUNTER_FILE = os.path.join(ROOT, "profiles", "k_cg_spmv_dot_diffusion3d_256_counters.json")
CSR_COUNTER_FILE = os.path.join(ROOT, "profiles", "k_cg_spmv_dot_csr_diffusion3d_256_counters.json")
KERNEL_SOURCES = ["paper_2601_13994_amd/csrc/krylov.hip", "paper_2601_13994_amd/csrc/common.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def matrix_bytes(n: int, nnz: int, form: str, nofs: int = 0) -> int:
    """Bytes of one pass over the operator in the SpMV form a solve used:
    CSR (values, column indices, row pointers: 12 nnz + 4(n+1)); row tiles
    with 16-bit row masks (8 nnz + 2n); the per-solve diagonal-major copy
    (8 nofs n, zeros where a row has no entry, + masks); its symmetric half
    form (main and upper diagonals only: 8 (nofs/2 + 1) n + masks), and
    that of Jacobi CG's scaled operator S A S, whose unit diagonal is not
    stored (8 (nofs/2) n + masks).  A "-paired" form (two adjacent rows per
    thread) reads no row masks."""
    base = form.removesuffix("-paired")
    b = {"csr": 12 * nnz + 4 * (n + 1), "mask-tiles": 8 * nnz + 2 * n, "diagonal": 8 * nofs * n + 2 * n,
         "diagonal-half": 8 * (nofs // 2 + 1) * n + 2 * n,
         "diagonal-half-unit": 8 * (nofs // 2) * n + 2 * n, "diagonal-unit": 8 * (nofs - 1) * n + 2 * n}[base]
    return b - 2 * n if form.endswith("-paired") else b


def spmv_bytes(n: int, nnz: int, form: str, nofs: int = 0) -> int:
    """Algorithmic HBM bytes of one q = A p (+ p.q) launch: the operator once,
    p gathered once with cache reuse (8n), q written once (8n)."""
    return matrix_bytes(n, nnz, form, nofs) + 16 * n


def form_of(info: dict, pat) -> str:
    """The SpMV form a solve reports (hsla_info.spmv_form, spmv_paired) as a
    byte-model key."""
    f = info["spmv_form"]
    if f in ("diagonal", "diagonal-half", "diagonal-half-unit", "diagonal-unit"):
        return f + "-paired" if info.get("spmv_paired") else f
    return "mask-tiles" if f == "tiles" and pat.stencil[0] else "csr"


FORM_TEXT = {"diagonal": "diagonal-major values + row masks, {} diagonals",
             "diagonal-half": "symmetric half diagonal-major values (main + upper) + row masks, {} diagonals",
             "diagonal-half-unit": "symmetric half diagonal-major values of S A S (upper only, unit diagonal) + "
                                   "row masks, {} diagonals",
             "diagonal-unit": "diagonal-major values of A D^-1 without its unit diagonal + row masks, {} diagonals",
             "mask-tiles": "row tiles with row masks, {} diagonals", "csr": "csr row tiles"}


def form_text(form: str, nofs: int) -> str:
    base = form.removesuffix("-paired")
    t = FORM_TEXT[base].format(nofs)
    return t.replace(" + row masks", "") + ", two adjacent rows per thread" if form.endswith("-paired") else t


def pcg_iteration_bytes(n: int, nnz: int, nofs: int) -> int:
    """Algorithmic bytes of one Jacobi-PCG iteration as scheduled here:
    SpMV+dot on the scaled operator S A S, update (reads r q and the FP32
    stop-test weights, writes r: 28n), direction with the iteration's x
    update (reads r p x, writes p x: 40n)."""
    return spmv_bytes(n, nnz, "diagonal" if nofs else "csr", nofs) + 68 * n


def cpu_info() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def load_traffic(n: int, nnz: int, path: str = COUNTER_FILE):
    """Per-launch HBM bytes of the dominant kernel from the committed
    counter summary, scaled by the copy-kernel calibration; None if absent
    or taken on different kernel source."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("n") != n or d.get("nnz") != nnz:
        return None
    return d.get("bytes_per_launch")


def host_threads() -> int:
    """Host threads the CPU oracle may use: the CPUs this process may run on,
    at most 16 (the host share of one GPU on the measurement machine)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_rate(run, k1: int, k2: int):
    """Seconds per iteration and set-up seconds of an oracle solver from the
    difference of a k1- and a k2-iteration capped run."""
    t0 = time.perf_counter()
    run(k1)
    t1 = time.perf_counter()
    run(k2)
    t2 = time.perf_counter()
    per_it = ((t2 - t1) - (t1 - t0)) / (k2 - k1)
    return per_it, max(0.0, (t1 - t0) - k1 * per_it)


def cpu_baseline(a, b, gpu_iters: int):
    """The oracle's Jacobi-PCG on the headline system: all host cores
    (value) and one thread, each from a capped-run difference scaled to the
    GPU solve's iteration count."""
    import oracle

    oracle.lib()
    cores = host_threads()

    def run(k):
        oracle.cg(a, b, precond="jacobi", rtol=1e-8, max_iter=k)

    with oracle.threads(cores):
        per_all, setup_all = _oracle_rate(run, 1, 61)
    with oracle.threads(1):
        per_one, setup_one = _oracle_rate(run, 1, 11)
    all_s = setup_all + gpu_iters * per_all
    one_s = setup_one + gpu_iters * per_one
    return {
        "value": 1.0 / all_s,
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"60 Jacobi-PCG iterations of the same 256^3 system on {cores} threads (difference of 61- and "
                   f"1-iteration runs: {per_all * 1e3:.1f} ms/iteration, {setup_all:.2f} s set-up), scaled to the "
                   f"GPU solve's {gpu_iters} iterations; FP64 C with OpenMP over rows and per-thread partial sums, "
                   f"{cpu_info()}"),
        "seconds_per_iteration": per_all,
        "one_thread": {"value": 1.0 / one_s, "unit": "solves/s", "cores": 1, "seconds_per_iteration": per_one,
                       "sample": "10 iterations (difference of 11- and 1-iteration runs), same scaling"},
        "host_cpus": os.cpu_count(),
    }


ALL_WORKLOADS = ("diffusion3d", "bicgstab", "poisson2d", "knn", "adjoint", "learned", "paper", "inverse",
                 "nonlinear", "eigen")

# The paper's own numbers for the same operator (context only: other hardware,
# its own residual definitions): Table tab:benchmark, Jacobi-CG with the
# PyTorch-native backend on one NVIDIA H200, and Table tab:adjoint_vs_naive_full,
# adjoint backward time by forced CG iterations on an RTX PRO 6000 Blackwell.
PAPER_POISSON_MS = {100: 20.0, 316: 43.0, 1000: 190.0, 1414: 418.0, 4000: 7300.0}
PAPER_ADJOINT_MS = {10: 35.0, 50: 9.0, 100: 13.0, 200: 25.0, 500: 60.0, 1000: 117.0, 2000: 230.0, 5000: 332.0}
# Sec. "End-to-End: Inverse Coefficient Learning": 1500 Adam steps in 48.6 s on
# one RTX PRO 6000 Blackwell; recovered kappa error 2.3e-3, solution misfit 3.0e-5.
PAPER_INVERSE = {"steps": 1500, "seconds": 48.6, "kappa_rel_error": 2.3e-3, "u_rel_error": 3.0e-5}


def generate(sel, args):
    """Host-side inputs of every selected workload.  Runs before the process
    touches the GPU, so the k-NN and shared-pattern generators may fork."""
    import numpy as np

    import workloads as W

    ctx = {}
    workers = max(1, min(16, os.cpu_count() or 1))
    t = time.time()
    if "diffusion3d" in sel or "bicgstab" in sel:
        log(f"[bench] generating 3D diffusion m={args.m} ...")
        ctx["d3"] = W.diffusion3d_workload(args.m)
        if "bicgstab" in sel:
            ctx["d3_conv_val"] = W.diffusion3d_values(args.m, W.diffusion3d_kappa(args.m), velocity=10.0)
    if "poisson2d" in sel:
        ctx["p2"] = W.poisson2d_workload(64)
        ctx["p2_bs"] = np.stack([W.rng(1, 1, s).standard_normal(64 * 64) for s in range(args.poisson_copies)])
    if "knn" in sel:
        log(f"[bench] generating {args.knn_systems} k-NN systems on {workers} processes ...")
        ctx["knn"] = W.knn_systems(args.knn_systems, workers=workers)
    if "adjoint" in sel:
        log(f"[bench] generating {args.adj_batch} shared-pattern systems m={args.adj_m} ...")
        ctx["adj"] = W.shared_pattern_batch(args.adj_m, args.adj_batch, workers=workers)
    if "paper" in sel:
        ctx["paper"] = {m: W.poisson2d(m) for m in list(PAPER_POISSON_MS) + [800]}
    if "inverse" in sel:
        ctx["inverse"] = W.inverse_truth(64)
    if "eigen" in sel:
        ctx["eigen"] = W.diffusion3d(64, W.diffusion3d_kappa(64))
    if "nonlinear" in sel:
        m = args.nonlinear_m
        a = W.diffusion3d(m, W.diffusion3d_kappa(m))
        ctx["nonlinear"] = (a.with_values(a.val * m * m), 1.0 + 0.5 * W.rng(2, 1, 7).standard_normal(a.n))
    if "learned" in sel:
        ctx["aniso_pat"] = W.aniso_pattern(args.aniso_m)
        ctx["aniso_train"] = np.stack([W.aniso_stencil(*W.aniso_params(s)) for s in range(args.train_systems)])
        ctx["aniso_eval"] = np.stack([W.aniso_stencil(*W.aniso_params(s, heldout=True))
                                      for s in range(args.eval_systems)])
        n = args.aniso_m ** 2
        bs = np.empty((args.eval_systems, n))
        for s in range(args.eval_systems):
            bs[s] = W.rng(5, 5, s).standard_normal(n)
        ctx["aniso_b"] = bs
    log(f"[bench] inputs generated in {time.time() - t:.1f}s")
    return ctx


def _sync():
    import torch

    torch.cuda.synchronize()


def _pattern(dev, a):
    import torch

    from paper_2601_13994_amd import _lib

    return _lib.Pattern(torch.as_tensor(a.row_ptr).to(dev), torch.as_tensor(a.col).to(dev))


def _profiled_spmv(pat, vals, bt, opts_kw, solves: int):
    """Mean duration of the SpMV(+dot) launches that did work, from HIP
    events the library records around each of them on its stream (profile
    mode: graphs off), over `solves` full solves."""
    from paper_2601_13994_amd import _lib

    opts = _lib.make_opts(profile=True, **opts_kw)
    ms, launches, info = 0.0, 0, None
    for _ in range(solves):
        _, infos, _ = _lib.solve(pat, vals, bt, opts)
        info = infos[0]
        ms += info["spmv_ms"]
        launches += info["spmv_launches"]
    return ms / max(launches, 1), launches, info


def csr_unit_spmv_bytes(n: int, nnz: int) -> int:
    """The scope table's SpMV unit: CSR values, int32 column indices and row
    pointers, p gathered once and q written once."""
    return 12 * nnz + 4 * (n + 1) + 16 * n


def run_diffusion(ctx, args, dev, pat, vals, bt):
    """Workload 2: Jacobi-PCG on the 256^3 log-normal diffusion system (the
    headline line: value, roofline, CPU baseline), plus the same solve on the
    plain CSR form."""
    from paper_2601_13994_amd import _lib

    a, b = ctx["d3"]
    n, nnz = a.n, a.nnz
    t0 = time.perf_counter()
    tuning = pat.autotune(B=1, effort=5) if args.autotune else None
    tune_ms = (time.perf_counter() - t0) * 1e3
    if tuning:
        log(f"[bench] autotune: {tuning}")
    kw = dict(method="cg", precond="jacobi", rtol=1e-8, max_iter=args.max_iter)
    opts = _lib.make_opts(**kw)  # the production path: graph-replayed iteration chunks
    for i in range(args.warmup):
        x, infos, st = _lib.solve(pat, vals, bt, opts)
        log(f"[bench] diffusion3d warmup {i}: status={st} iters={infos[0]['iters']} "
            f"true_res={infos[0]['true_residual']:.2e}")
    _sync()
    t0 = time.perf_counter()
    recs = []
    for i in range(args.steps):
        x, infos, st = _lib.solve(pat, vals, bt, opts)
        recs.append(infos[0])
        log(f"[bench] diffusion3d step {i}: status={st} iters={infos[0]['iters']}")
    _sync()
    elapsed = time.perf_counter() - t0
    iters = recs[-1]["iters"]
    ms_step = elapsed / args.steps * 1e3
    # the dominant kernel's launch time, from profiled solves of the same system
    avg_ms, launches, pinfo = _profiled_spmv(pat, vals, bt, kw, args.profile_solves)
    stencil, nofs = pat.stencil
    form = form_of(pinfo, pat)
    bytes_launch = spmv_bytes(n, nnz, form, nofs)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    unit_bytes = csr_unit_spmv_bytes(n, nnz)
    it_bytes = bytes_launch + 68 * n  # update 28n, direction 40n
    csr_it_bytes = pcg_iteration_bytes(n, nnz, 0)
    top = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"diffusion3d-{args.m}^3 log-normal kappa, Jacobi-PCG to rtol 1e-8, x0=0",
            "n": n, "nnz": nnz, "method": "cg", "precond": "jacobi", "rtol": 1e-8,
            "index_dtype": "int32", "value_dtype": "float64",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": DOMINANT,
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": load_traffic(n, nnz),
            "bytes_model": "stored form: " + form_text(form, nofs) + ", p gathered once, q written once",
            "algorithmic_bytes_per_launch": bytes_launch,
            "mean_launch_ms": avg_ms,
            "launches_timed": launches,
            "launch_timing": (f"HIP events around every SpMV launch of {args.profile_solves} profiled solve(s) of "
                              "the same system run after the timed region"),
            "csr_unit": {
                "bytes_per_launch": unit_bytes,
                "achieved_GBps": unit_bytes / (avg_ms * 1e-3) / 1e9,
                "frac": unit_bytes / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                "note": ("work-equivalent rate: the same launches priced at the CSR SpMV unit "
                         "12 nnz + 4(n+1) + 16n; above the peak because the stored form streams fewer bytes"),
            },
            "full_copy_equivalent_GBps": (spmv_bytes(n, nnz, "diagonal", nofs) / (avg_ms * 1e-3) / 1e9
                                          if stencil else None),
        },
        "detail": {
            "iterations": iters,
            "true_relative_residual": recs[-1]["true_residual"],
            "status": recs[-1]["status"],
            "ms_per_iteration": ms_step / max(iters, 1),
            "iteration_model_GBps": it_bytes * iters / (ms_step * 1e-3) / 1e9,
            "iteration_frac_of_peak": it_bytes * iters / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "GFLOPs": (2 * nnz + 13 * n) * iters / (ms_step * 1e-3) / 1e9,
            "algorithmic_bytes_per_iteration": it_bytes,
            "spmv_share_of_step": avg_ms * iters / ms_step,
            "spmv_form": recs[-1]["spmv_form"],
            "setup_excluded_ms": {"pattern": ctx.get("setup_ms"), "autotune": tune_ms if tuning else None},
            "autotune": tuning,
            "csr_unit_bytes_per_iteration": csr_it_bytes,
            "csr_unit_equivalent_iteration_GBps": csr_it_bytes * iters / (ms_step * 1e-3) / 1e9,
        },
    }
    if args.csr_line:
        top["csr_path"] = run_diffusion_csr(pat, vals, bt, kw, n, nnz, args)
    top["single_reduction"] = run_single_reduction(pat, vals, bt, kw, args, ms_step, iters)
    top["s_step"] = run_single_reduction(pat, vals, bt, kw, args, ms_step, iters, s_step=4)
    return top, iters


# kernel launches per iteration of the per-iteration path: CG runs SpMV+dot,
# alpha finalize, update, beta finalize, direction; the single-reduction
# recurrence runs SpMV with both dots, one finalize, one vector sweep;
# s-step CG runs 2s - 1 basis SpMVs, the Gram pass, one finalize and the
# recovery sweep per s steps
CG_LAUNCHES_PER_ITERATION, SR_LAUNCHES_PER_ITERATION = 5, 3


def run_single_reduction(pat, vals, bt, kw, args, ms_cg, iters_cg, B=1, s_step=0):
    """The same solve(s) with the single-reduction recurrence (CG_SR:
    Chronopoulos and Gear) or, with s_step, s-step CG (one Gram reduction
    per s steps), against the two-reduction schedule just timed."""
    from paper_2601_13994_amd import _lib

    if s_step:
        opts = _lib.make_opts(**dict(kw, method="cg_sstep", s_step=s_step, persistent=False))
    else:
        opts = _lib.make_opts(**dict(kw, method="cg_sr"))
    _lib.solve(pat, vals, bt, opts)
    _sync()
    t0 = time.perf_counter()
    reps = max(1, args.sub_steps)
    for _ in range(reps):
        _, infos, st = _lib.solve(pat, vals, bt, opts)
    _sync()
    dt = (time.perf_counter() - t0) / reps
    it = max(f["iters"] for f in infos)
    return {
        "method": infos[0]["method"], "status": st, "iterations_max": it,
        "iterations_two_reduction": iters_cg, "ms_per_solve": dt * 1e3,
        "ms_per_iteration": dt * 1e3 / max(it, 1),
        "two_reduction_ms_per_iteration": ms_cg / max(iters_cg, 1),
        "launches_per_iteration": (2 * s_step + 2) / s_step if s_step else SR_LAUNCHES_PER_ITERATION,
        "two_reduction_launches_per_iteration": CG_LAUNCHES_PER_ITERATION,
        "true_relative_residual_max": max(f["true_residual"] for f in infos), "systems": B, "reps": reps,
        **({"s": s_step} if s_step else {}),
    }


def run_diffusion_csr(pat, vals, bt, kw, n, nnz, args):
    """The same Jacobi-PCG solve with the pattern forced to plain CSR (row
    tiles with int32 column indices; S A S values scaled once into a CSR
    copy): the unstructured-SpMV path, whose SpMV moves exactly the scope
    table's unit."""
    from paper_2601_13994_amd import _lib

    pat.set_format("csr")
    try:
        opts = _lib.make_opts(**kw)
        _lib.solve(pat, vals, bt, opts)
        _sync()
        t0 = time.perf_counter()
        reps = max(1, args.sub_steps)
        for _ in range(reps):
            _, infos, st = _lib.solve(pat, vals, bt, opts)
        _sync()
        dt = (time.perf_counter() - t0) / reps
        avg_ms, launches, _ = _profiled_spmv(pat, vals, bt, kw, 1)
    finally:
        pat.set_format("auto")
    it = infos[0]["iters"]
    ub = csr_unit_spmv_bytes(n, nnz)
    it_bytes = ub + 68 * n
    return {
        "workload": "the headline system with the CSR form forced (k_cg_spmv_dot<0>)",
        "solves_per_s": 1.0 / dt, "ms_per_solve": dt * 1e3, "iterations": it, "status": st,
        "true_relative_residual": infos[0]["true_residual"], "spmv_form": infos[0]["spmv_form"],
        "spmv_mean_launch_ms": avg_ms, "spmv_launches_timed": launches, "spmv_bytes_per_launch": ub,
        "spmv_GBps": ub / (avg_ms * 1e-3) / 1e9, "spmv_frac_of_peak": ub / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        "ms_per_iteration": dt * 1e3 / max(it, 1),
        "iteration_model_GBps": it_bytes * it / dt / 1e9,
        "iteration_frac_of_peak": it_bytes * it / dt / 1e9 / HBM_PEAK_GBPS,
        "algorithmic_bytes_per_iteration": it_bytes, "reps": reps,
        "traffic": load_traffic(n, nnz, CSR_COUNTER_FILE),
    }


def run_bicgstab(ctx, args, dev, pat):
    """Workload 2b: Jacobi-BiCGStab on the same grid with upwind convection
    at cell Peclet 10 along (1,1,1)/sqrt(3)."""
    import torch

    from paper_2601_13994_amd import _lib

    a, b = ctx["d3"]
    n, nnz = a.n, a.nnz
    vals = torch.as_tensor(ctx["d3_conv_val"]).to(dev)
    bt = torch.as_tensor(b).to(dev)
    opts = _lib.make_opts(method="bicgstab", precond="jacobi", rtol=1e-8, max_iter=args.max_iter)
    for _ in range(2):
        x, infos, st = _lib.solve(pat, vals, bt, opts)
    log(f"[bench] bicgstab warmup: status={st} iters={infos[0]['iters']} true_res={infos[0]['true_residual']:.2e}")
    _sync()
    t0 = time.perf_counter()
    for i in range(args.sub_steps):
        x, infos, st = _lib.solve(pat, vals, bt, opts)
    _sync()
    dt = (time.perf_counter() - t0) / args.sub_steps
    it = infos[0]["iters"]
    # two SpMVs (p and s gathered, v and t written) + the vector sweeps on
    # A D^{-1}: direction 32n, r_hat in the first SpMV 8n, s 24n, update 56n
    it_bytes = 2 * spmv_bytes(n, nnz, form_of(infos[0], pat), pat.stencil[1]) + 120 * n
    return {
        "workload": f"diffusion3d-{args.m}^3 + upwind convection (cell Peclet 10), Jacobi-BiCGStab to rtol 1e-8",
        "solves_per_s": 1.0 / dt, "ms_per_solve": dt * 1e3, "iterations": it, "status": st,
        "true_relative_residual": infos[0]["true_residual"],
        "ms_per_iteration": dt * 1e3 / max(it, 1),
        "iteration_model_GBps": it_bytes * it / dt / 1e9,
        "iteration_frac_of_peak": it_bytes * it / dt / 1e9 / HBM_PEAK_GBPS,
        "GFLOPs": (4 * nnz + 26 * n) * it / dt / 1e9,
        "algorithmic_bytes_per_iteration": it_bytes, "spmv_form": infos[0]["spmv_form"], "reps": args.sub_steps,
        **(oracle_bicgstab(ctx, it) if not args.no_cpu_baseline else {}),
    }


def oracle_bicgstab(ctx, gpu_iters):
    """The oracle's Jacobi-BiCGStab on the same system, all host cores, from
    a capped-run difference scaled to the GPU's iteration count."""
    import oracle

    a, b = ctx["d3"]
    ac = a.with_values(ctx["d3_conv_val"])
    cores = host_threads()

    def run(k):
        oracle.bicgstab(ac, b, precond="jacobi", rtol=1e-8, max_iter=k)

    oracle.lib()
    with oracle.threads(cores):
        per, setup = _oracle_rate(run, 1, 21)
    return {"oracle_solves_per_s": 1.0 / (setup + gpu_iters * per), "oracle_cores": cores,
            "oracle_sample": (f"20 iterations on {cores} threads (difference of 21- and 1-iteration runs: "
                              f"{per * 1e3:.1f} ms/iteration), scaled to the GPU's {gpu_iters} iterations")}


def run_poisson(ctx, args, dev):
    """Workload 1: 2D Poisson 64^2, plain CG to rtol 1e-10 -- latency of one
    solve, and throughput of many independent right-hand sides on copies of
    the matrix solved as one shared-pattern batch."""
    import numpy as np
    import torch

    import oracle
    from paper_2601_13994_amd import _lib

    a, b = ctx["p2"]
    pat = _pattern(dev, a)
    vals = torch.as_tensor(a.val).to(dev)
    bt = torch.as_tensor(b).to(dev)
    opts = _lib.make_opts(method="cg", precond="none", rtol=1e-10)
    for _ in range(3):
        x, infos, st = _lib.solve(pat, vals, bt, opts)
    reps = 50
    _sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        x, infos, st = _lib.solve(pat, vals, bt, opts)
    _sync()
    lat = (time.perf_counter() - t0) / reps
    # the single-reduction recurrence (CG_SR) in the same kernel
    opts_sr = _lib.make_opts(method="cg_sr", precond="none", rtol=1e-10)
    for _ in range(3):
        _lib.solve(pat, vals, bt, opts_sr)
    _sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        xs, infos_sr, st_sr = _lib.solve(pat, vals, bt, opts_sr)
    _sync()
    lat_sr = (time.perf_counter() - t0) / reps
    B = args.poisson_copies
    vb = vals.repeat(B, 1).contiguous()
    bb = torch.as_tensor(ctx["p2_bs"]).to(dev)
    for _ in range(2):  # the second call's fresh output buffer costs a one-off device allocation
        xb, ib, stb = _lib.solve(pat, vb, bb, opts)
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.sub_steps):
        xb, ib, stb = _lib.solve(pat, vb, bb, opts)
    _sync()
    tb = (time.perf_counter() - t0) / args.sub_steps
    for _ in range(2):
        _lib.solve(pat, vb, bb, opts_sr)
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.sub_steps):
        _, ib_sr, stb_sr = _lib.solve(pat, vb, bb, opts_sr)
    _sync()
    tb_sr = (time.perf_counter() - t0) / args.sub_steps
    it = infos[0]["iters"]
    itb = np.array([f["iters"] for f in ib])
    it_bytes = spmv_bytes(a.n, a.nnz, "csr") + 72 * a.n  # the persistent kernel reads CSR
    res = {
        "workload": "poisson2d-64^2 (n=4096, nnz=20224), plain CG to rtol 1e-10, x0=0",
        "latency_us_per_solve": lat * 1e6, "iterations": it, "status": st,
        "true_relative_residual": infos[0]["true_residual"],
        "us_per_iteration": lat * 1e6 / max(it, 1),
        "batched_copies": B, "batched_solves_per_s": B / tb, "batched_status": stb,
        "batched_max_iterations": int(itb.max()),
        "batched_model_GBps": float(it_bytes * itb.sum() / tb / 1e9),
        "single_reduction": {"latency_us_per_solve": lat_sr * 1e6, "iterations": infos_sr[0]["iters"],
                             "status": st_sr, "true_relative_residual": infos_sr[0]["true_residual"],
                             "batched_solves_per_s": B / tb_sr, "batched_status": stb_sr},
    }
    if not args.no_cpu_baseline:
        oracle.lib()
        t0 = time.perf_counter()
        k = 20
        for _ in range(k):
            oracle.cg(a, b, precond="none", rtol=1e-10)
        res["oracle_ms_per_solve"] = (time.perf_counter() - t0) / k * 1e3
        res["oracle_cores"] = 1
    return res


def run_knn(ctx, args, dev):
    """Workload 3: ragged k-NN Laplacian systems with distinct patterns, all
    solved together (Jacobi-PCG to rtol 1e-8): this batch is large enough for
    the segmented per-iteration path over all systems at once."""
    import numpy as np
    import torch

    import oracle
    import paper_2601_13994_amd as hs

    systems = ctx["knn"]
    mats = [(torch.as_tensor(a.val).to(dev), torch.as_tensor(a.row_ptr).to(dev), torch.as_tensor(a.col).to(dev))
            for a, _ in systems]
    L = hs.SparseCSRList(mats)
    del mats
    bcat = torch.as_tensor(np.concatenate([b for _, b in systems])).to(dev)
    for _ in range(2):
        xs, infos, st = L.solve(bcat, rtol=1e-8)
    log(f"[bench] knn warmup: status={st}")
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.sub_steps):
        xs, infos, st = L.solve(bcat, rtol=1e-8)
    _sync()
    dt = (time.perf_counter() - t0) / args.sub_steps
    its = np.array([f["iters"] for f in infos])
    ns = np.array([a.n for a, _ in systems])
    nnzs = np.array([a.nnz for a, _ in systems])
    # the same batch in one persistent launch (workgroups take systems from a
    # longest-first queue): time and load balance from the device clock
    L.solve(bcat, rtol=1e-8, persistent="force")
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.sub_steps):
        _, pinfos, pst = L.solve(bcat, rtol=1e-8, persistent="force")
    _sync()
    dtp = (time.perf_counter() - t0) / args.sub_steps
    wg = pinfos[0]["workgroups"]
    busy = sum(f["t_end_ms"] - f["t_start_ms"] for f in pinfos)
    wall = max(f["t_end_ms"] for f in pinfos)
    pits = np.array([f["iters"] for f in pinfos])
    pwork = float(((12 * nnzs + 4 * (ns + 1) + 104 * ns) * pits).sum())
    persistent = {
        "solves_per_s": len(systems) / dtp, "ms_per_batch": dtp * 1e3, "status": pst, "workgroups": wg,
        "kernel_wall_ms": wall, "load_balance_efficiency": busy / (wg * wall) if wall > 0 else None,
        "load_balance_definition": ("sum over systems of (end - start) on the workgroup that ran it / "
                                    "(workgroups x kernel wall), device wall clock"),
        "model_GBps": pwork / dtp / 1e9, "model_frac_of_peak": pwork / dtp / 1e9 / HBM_PEAK_GBPS,
        "iterations_mean": float(pits.mean()),
        "true_relative_residual_max": max(f["true_residual"] for f in pinfos),
    }
    # per system per iteration: CSR once, p gathered and q written (16n), and
    # the vector updates: 88n in the persistent kernel, 80n in the
    # segmented path (x += alpha p folded into the direction sweep)
    vec = 104 if infos[0]["spmv_form"] == "persistent" else 96
    work = float(((12 * nnzs + 4 * (ns + 1) + vec * ns) * its).sum())
    res = {
        "workload": (f"{len(systems)} k-NN (k=8) Laplacians + 0.01 I, n ~ U[1000, 50000], distinct patterns, "
                     "one launch sequence for the whole batch, Jacobi-PCG to rtol 1e-8"),
        "solves_per_s": len(systems) / dt, "ms_per_batch": dt * 1e3, "status": st,
        "path": "persistent" if infos[0]["spmv_form"] == "persistent" else "segmented",
        "total_rows": int(ns.sum()), "total_nnz": int(nnzs.sum()),
        "iterations_mean": float(its.mean()), "iterations_max": int(its.max()),
        "true_relative_residual_max": max(f["true_residual"] for f in infos),
        "model_GBps": work / dt / 1e9, "model_frac_of_peak": work / dt / 1e9 / HBM_PEAK_GBPS,
        "reps": args.sub_steps, "persistent_launch": persistent,
    }
    if not args.no_cpu_baseline:
        import concurrent.futures as cf

        oracle.lib()
        cores = host_threads()
        order = sorted(range(len(systems)), key=lambda i: -systems[i][0].nnz)  # longest first
        with oracle.threads(1):
            t0 = time.perf_counter()
            with cf.ThreadPoolExecutor(max_workers=cores) as ex:
                list(ex.map(lambda i: oracle.cg(systems[i][0], systems[i][1], precond="jacobi", rtol=1e-8), order))
            dto = time.perf_counter() - t0
        res["oracle_solves_per_s"] = len(systems) / dto
        res["oracle_sample"] = (f"all {len(systems)} systems, one system per thread on {cores} threads, longest "
                                f"first ({dto:.2f} s)")
        res["oracle_cores"] = cores
    return res


def run_adjoint(ctx, args, dev):
    """Workload 4: shared-pattern batch, forward Jacobi-PCG plus adjoint
    backward (loss 1/2 ||x - x*||^2) giving dL/db and dL/dA on the pattern."""
    import numpy as np
    import torch

    from paper_2601_13994_amd import _lib

    a0, V, Bs, Xs = ctx["adj"]
    B, n, nnz = V.shape[0], a0.n, a0.nnz
    pat = _pattern(dev, a0)
    vals = torch.as_tensor(V).to(dev)
    bt = torch.as_tensor(Bs).to(dev)
    xst = torch.as_tensor(Xs).to(dev)
    tuning = pat.autotune(B=B, effort=3) if args.autotune else None
    opts = _lib.make_opts(method="cg", precond="jacobi", rtol=1e-8)

    def pair():
        x, fi, st = _lib.solve(pat, vals, bt, opts)
        gx = x - xst
        gA, gb, bi, st2 = _lib.adjoint(pat, vals, x, gx, opts)
        return x, gA, gb, fi, bi, st, st2

    pair()
    pair()
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.sub_steps):
        x, gA, gb, fi, bi, st, st2 = pair()
    _sync()
    dt = (time.perf_counter() - t0) / args.sub_steps
    itf = np.array([f["iters"] for f in fi])
    itb = np.array([f["iters"] for f in bi])
    # the forward solves alone, two-reduction CG against the single-reduction
    # recurrence (the batch runs until its slowest system stops)
    _lib.solve(pat, vals, bt, opts)
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.sub_steps):
        _lib.solve(pat, vals, bt, opts)
    _sync()
    t_fwd = (time.perf_counter() - t0) / args.sub_steps
    sr = run_single_reduction(pat, vals, bt, dict(method="cg", precond="jacobi", rtol=1e-8), args,
                              t_fwd * 1e3, int(itf.max()), B)
    sr["two_reduction_ms_per_solve"] = t_fwd * 1e3
    # per system per iteration: the operator's values in the form used (the
    # row masks or CSR indices, shared by the batch, amortised over B) + 84n
    # (p gathered, q written: 16n; update and direction: 68n)
    form = form_of(fi[0], pat)
    nofs = pat.stencil[1]
    base = form.removesuffix("-paired")
    per_it = {"diagonal-half-unit": 8 * (nofs // 2) * n, "diagonal-half": 8 * (nofs // 2 + 1) * n,
              "diagonal": 8 * nofs * n,
              "mask-tiles": 8 * nnz, "csr": 8 * nnz}[base] + 84 * n
    if not form.endswith("-paired"):
        per_it += (2 * n if form != "csr" else 4 * nnz + 4 * (n + 1)) / B
    work = float(per_it * (itf.sum() + itb.sum()) + B * (12 * nnz + 28 * n))
    return {
        "workload": (f"{B} systems on one 3D 7-point pattern, {args.adj_m}^3 (n={n}, nnz={nnz}), log-normal kappa "
                     "per sample; forward Jacobi-PCG + adjoint, rtol 1e-8, loss 1/2||x - x*||^2"),
        "pairs_per_s": B / dt, "ms_per_batch": dt * 1e3, "status_forward": st, "status_adjoint": st2,
        "autotune": tuning, "spmv_form": fi[0]["spmv_form"],
        "iterations_forward_mean": float(itf.mean()), "iterations_adjoint_mean": float(itb.mean()),
        "true_relative_residual_max": max(max(f["true_residual"] for f in fi), max(f["true_residual"] for f in bi)),
        "model_GBps": work / dt / 1e9, "model_frac_of_peak": work / dt / 1e9 / HBM_PEAK_GBPS,
        "reps": args.sub_steps, "forward_single_reduction": sr,
        **(oracle_adjoint(ctx, args.oracle_adj_systems) if not args.no_cpu_baseline else {}),
    }


def oracle_adjoint(ctx, k):
    """The oracle's forward Jacobi-PCG plus adjoint (gradients w.r.t. b and
    every stored value) on the first k systems of the batch, all host
    cores, one system after another."""
    import oracle

    a0, V, Bs, Xs = ctx["adj"]
    cores = host_threads()
    oracle.lib()
    with oracle.threads(cores):
        t0 = time.perf_counter()
        for s in range(k):
            a = a0.with_values(V[s])
            x = oracle.cg(a, Bs[s], precond="jacobi", rtol=1e-8).x
            oracle.adjoint(a, x, x - Xs[s], precond="jacobi", rtol=1e-8)
        dto = time.perf_counter() - t0
    return {"oracle_pairs_per_s": k / dto, "oracle_cores": cores,
            "oracle_sample": f"forward + adjoint of the first {k} systems, one after another on {cores} threads"}


def run_learned(ctx, args, dev):
    """Workload 5: train the preconditioner network on the GPU on generated
    anisotropic systems, then solve the held-out systems batched with
    learned-FSAI PCG and with Jacobi-PCG; wall-clock time to rtol 1e-8."""
    import numpy as np
    import torch

    from paper_2601_13994_amd import _lib, learned

    pa, slots = ctx["aniso_pat"]
    pat = _pattern(dev, pa)
    sl = torch.as_tensor(slots).to(dev)
    st_train = torch.as_tensor(ctx["aniso_train"]).to(dev)
    st_eval = torch.as_tensor(ctx["aniso_eval"]).to(dev)
    gen = np.random.default_rng(0)
    model = learned.LearnedFSAI(seed=0, device=dev)
    ntr = st_train.shape[0]
    # systems in a fresh random order each pass over the training set, each
    # drawn once per pass (the default steps make exactly one pass)
    order = []

    def sample(step):
        nonlocal order
        if len(order) < args.train_batch:
            order = list(gen.permutation(ntr)) + order
        idx = torch.as_tensor([order.pop() for _ in range(args.train_batch)]).to(dev)
        return learned.aniso_batch_values(sl, st_train[idx])

    _sync()
    t0 = time.perf_counter()
    hist_loss = model.train(pat, sample, steps=args.train_steps, probes=args.train_probes, lr=args.train_lr,
                            lr_final=args.train_lr / 10)
    _sync()
    t_train = time.perf_counter() - t0
    log(f"[bench] learned: trained {args.train_steps} steps in {t_train:.1f}s, loss {np.mean(hist_loss[:5]):.4f} -> "
        f"{np.mean(hist_loss[-20:]):.4f}")
    V = learned.aniso_batch_values(sl, st_eval)
    bt = torch.as_tensor(ctx["aniso_b"]).to(dev)
    E = V.shape[0]
    tuning = pat.autotune(B=E, effort=3) if args.autotune else None
    jopts = _lib.make_opts(method="cg", precond="jacobi", rtol=1e-8)
    # warm up both paths at the full batch (graphs, workspaces, output buffers)
    _lib.solve(pat, V, bt, jopts)
    model.solve(pat, V, bt, rtol=1e-8, factors=model.factors(pat, V))
    _sync()
    t0 = time.perf_counter()
    xj, ij, stj = _lib.solve(pat, V, bt, jopts)
    _sync()
    tj = time.perf_counter() - t0
    t0 = time.perf_counter()
    G, GT = model.factors(pat, V)
    _sync()
    tf = time.perf_counter() - t0
    xl, il, stl = model.solve(pat, V, bt, rtol=1e-8, factors=(G, GT))
    _sync()
    tl = time.perf_counter() - t0
    # independent FP64 residual check of every returned solution
    rl, bn = _lib.residual_norms(pat, V, bt, xl)
    rj, _ = _lib.residual_norms(pat, V, bt, xj)
    rel_l = max(r / max(c, 1e-300) for r, c in zip(rl, bn))
    rel_j = max(r / max(c, 1e-300) for r, c in zip(rj, bn))
    itj = np.array([f["iters"] for f in ij])
    itl = np.array([f["iters"] for f in il])
    fell = sum(f["status"] == _lib.FELL_BACK for f in il)
    edges = np.linspace(min(itl.min(), itj.min()), max(itl.max(), itj.max()) + 1, 13).round().astype(int)
    hist = {"bin_edges": edges.tolist(), "learned": np.histogram(itl, edges)[0].tolist(),
            "jacobi": np.histogram(itj, edges)[0].tolist()}
    # the network's forward alone (matrix-core GEMMs: three 128 -> 64 node
    # layers and the 132 -> 32 edge head) on the held-out batch
    params = model.params
    _lib.mpnn_forward(pat, V, params)
    _sync()
    t0 = time.perf_counter()
    _lib.mpnn_forward(pat, V, params)
    _sync()
    t_fwd = time.perf_counter() - t0
    mfma_flops = E * (3 * 2 * pa.n * 128 * 64 + 2 * pat.nnz_lower * 132 * 32)
    mfma = {"forward_seconds": t_fwd, "mfma_flops": mfma_flops, "TFLOPs": mfma_flops / t_fwd / 1e12,
            "peak_TFLOPs_bf16_dense": 2500.0, "frac_of_peak": mfma_flops / t_fwd / 1e12 / 2500.0,
            "note": ("dense-layer flops only; the forward also gathers neighbour activations and aggregates "
                     "them on the vector units, which bounds it")}
    return {
        "workload": (f"2D anisotropic diffusion {args.aniso_m}^2 9-point (n={pa.n}, nnz={pa.nnz}), ratio ~ "
                     f"logU[1,1000], angle ~ U[0,pi); network trained on {ntr} generated systems, evaluated on "
                     f"{E} held-out systems batched, PCG to rtol 1e-8"),
        "learned_solves_per_s": E / tl, "jacobi_solves_per_s": E / tj, "speedup_wall_clock": tj / tl,
        "learned_seconds": tl, "learned_factor_seconds": tf, "jacobi_seconds": tj,
        "iterations_mean_learned": float(itl.mean()), "iterations_mean_jacobi": float(itj.mean()),
        "iterations_max_learned": int(itl.max()), "iterations_max_jacobi": int(itj.max()),
        "iteration_ratio_mean": float((itl / np.maximum(itj, 1)).mean()),
        "fell_back": int(fell), "status_learned": stl, "status_jacobi": stj, "autotune": tuning,
        "true_relative_residual_max_learned": rel_l, "true_relative_residual_max_jacobi": rel_j,
        "train_seconds": t_train, "train_steps": args.train_steps, "train_batch": args.train_batch,
        "train_systems_seen": min(ntr, args.train_steps * args.train_batch),
        "train_probes": args.train_probes, "train_loss_first": float(np.mean(hist_loss[:5])),
        "train_loss_last": float(np.mean(hist_loss[-20:])), "iteration_histogram": hist, "mpnn_forward": mfma,
        **(oracle_learned(ctx, pa, args.oracle_aniso_systems) if not args.no_cpu_baseline else {}),
    }


def oracle_learned(ctx, pa, k):
    """The oracle on the first k held-out systems, one system per thread:
    Jacobi-PCG, and classical FSAI-PCG (the textbook factor on A's lower
    pattern) as a yardstick for the learned factor."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    pat_a, slots = ctx["aniso_pat"]
    cores = host_threads()
    oracle.lib()
    mats = [pat_a.with_values(ctx["aniso_eval"][s][slots]) for s in range(k)]
    bs = ctx["aniso_b"][:k]

    def jac(s):
        return oracle.cg(mats[s], bs[s], precond="jacobi", rtol=1e-8).iters

    def fsai(s):
        rpL, colL, g = oracle.fsai(mats[s])
        return oracle.fsai_pcg(mats[s], rpL, colL, g, bs[s], rtol=1e-8).iters

    out = {}
    with oracle.threads(1):
        for name, fn in (("jacobi", jac), ("classical_fsai", fsai)):
            t0 = time.perf_counter()
            with cf.ThreadPoolExecutor(max_workers=cores) as ex:
                its = list(ex.map(fn, range(k)))
            dt = time.perf_counter() - t0
            out[name] = {"solves_per_s": k / dt, "iterations_mean": float(np.mean(its))}
    return {"oracle": out, "oracle_cores": cores,
            "oracle_sample": f"first {k} held-out systems, one system per thread on {cores} threads"}


def run_paper(ctx, args, dev):
    """The paper's 2D Poisson shapes: Jacobi-PCG solve time at the sizes of
    Table tab:benchmark (rtol 1e-6), and the adjoint backward time by forced
    CG iterations on N = 640,000 as in Table tab:adjoint_vs_naive_full."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2601_13994_amd import _lib

    rows = []
    for m, paper_ms in PAPER_POISSON_MS.items():
        a = ctx["paper"][m]
        pat = _pattern(dev, a)
        vals = torch.as_tensor(a.val).to(dev)
        bt = torch.as_tensor(W.rng(1, 1, m).standard_normal(a.n)).to(dev)
        opts = _lib.make_opts(method="cg", precond="jacobi", rtol=1e-6)
        _lib.solve(pat, vals, bt, opts)
        _sync()
        t0 = time.perf_counter()
        x, infos, st = _lib.solve(pat, vals, bt, opts)
        _sync()
        dt = time.perf_counter() - t0
        rows.append({"dof": a.n, "iterations": infos[0]["iters"], "ms": dt * 1e3, "status": st,
                     "true_relative_residual": infos[0]["true_residual"], "paper_ms_h200": paper_ms})
        del pat, vals, bt, x
    a = ctx["paper"][800]
    pat = _pattern(dev, a)
    vals = torch.as_tensor(a.val).to(dev)
    gx = torch.as_tensor(W.rng(1, 2, 800).standard_normal(a.n)).to(dev)
    x = torch.as_tensor(W.rng(1, 3, 800).standard_normal(a.n)).to(dev)
    adj = []
    for k, paper_ms in PAPER_ADJOINT_MS.items():
        opts = _lib.make_opts(method="cg", precond="none", rtol=0.0, max_iter=k, persistent=False)
        _lib.adjoint(pat, vals, x, gx, opts)
        _sync()
        t0 = time.perf_counter()
        _lib.adjoint(pat, vals, x, gx, opts)
        _sync()
        adj.append({"k": k, "ms": (time.perf_counter() - t0) * 1e3, "paper_ms_rtx_pro_6000": paper_ms})
    return {"workload": "2D Poisson 5-point (the paper's benchmark operator), context only",
            "jacobi_pcg_rtol_1e-6": rows, "adjoint_backward_forced_k_n640000": adj}


def run_inverse(ctx, args, dev):
    """Sec. "End-to-End: Inverse Coefficient Learning": recover kappa on the
    64 x 64 grid with 1500 Adam steps (lr 5e-2) through the adjoint solve
    (CG with Jacobi to rtol 1e-10, forward and backward)."""
    import numpy as np

    from paper_2601_13994_amd import inverse

    kt, f = ctx["inverse"]
    prob = inverse.InverseProblem(kt, f, m=64, device=dev, rtol=1e-10)
    for _ in range(2):  # first-call set-up (graphs, workspace, allocator)
        prob.loss()[0].backward()
    prob.opt.zero_grad(set_to_none=True)
    _sync()
    steps = args.inverse_steps
    hist = []
    t0 = time.perf_counter()
    for _ in range(steps):
        hist.append(prob.step())
    _sync()
    dt = time.perf_counter() - t0
    ek, eu, kmin, kmax = prob.errors()
    res = {
        "workload": "inverse coefficient learning, 64x64 cells, kappa = softplus(theta), Adam lr 5e-2, "
                    "loss ||u - u_obs||^2 + 1e-3 ||grad_h kappa||^2 / N, CG+Jacobi rtol 1e-10 forward and adjoint",
        "steps": steps, "seconds": dt, "ms_per_step": dt / steps * 1e3,
        "kappa_rel_error": ek, "u_rel_error": eu, "kappa_min": kmin, "kappa_max": kmax,
        "loss_first": hist[0], "loss_last": hist[-1], "paper_rtx_pro_6000": PAPER_INVERSE,
    }
    if not args.no_cpu_baseline:
        import oracle
        from oracle import inverse as OI

        oracle.lib()
        u_obs = OI.observe(64, kt, f, rtol=1e-10)
        theta = np.full(64 * 64, np.log(np.e - 1.0))
        st = {"t": 0, "m": np.zeros_like(theta), "v": np.zeros_like(theta)}
        k = 3
        t0 = time.perf_counter()
        for _ in range(k):
            _, g, _ = OI.loss_and_grad(theta, 64, u_obs, f, rtol=1e-10)
            theta = OI.adam(theta, g, st)
        dto = (time.perf_counter() - t0) / k
        res["oracle_ms_per_step"] = dto * 1e3
        res["oracle_sample"] = f"first {k} steps of the same loop on the CPU oracle (numpy + sequential C), 1 core"
    return res


def run_nonlinear(ctx, args, dev):
    """Sec. "Adjoint Differentiation", nonlinear systems: F(u) = A u + u^2 - f
    (the paper's listing example) on the 3D log-normal diffusion operator
    scaled to unit-cube spacing, Newton from u = 0 (each step a Jacobi-PCG
    solve on A + 2 diag(u) to rtol 1e-10), then one adjoint solve for
    dL/dA and dL/df of L = 1/2 ||u||^2."""
    import torch

    import paper_2601_13994_amd as hs
    from paper_2601_13994_amd import nonlinear

    a, f = ctx["nonlinear"]
    rp, col = torch.as_tensor(a.row_ptr).to(dev), torch.as_tensor(a.col).to(dev)
    pat = _pattern(dev, a)
    ft0 = torch.as_tensor(f).to(dev)

    def run_once():
        vals = torch.as_tensor(a.val).to(dev).requires_grad_(True)
        ft = ft0.clone().requires_grad_(True)
        A = hs.SparseCSR(vals, rp, col, pattern=pat)
        info = {}
        _sync()
        t0 = time.perf_counter()
        u = nonlinear.newton_solve(A, ft, tol=1e-10, lin_rtol=1e-10, info=info)
        _sync()
        t1 = time.perf_counter()
        (0.5 * (u * u).sum()).backward()
        _sync()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, info["newton_steps"]

    run_once()
    fw, bw, steps = run_once()
    return {"workload": (f"A u + u^2 = f on the {args.nonlinear_m}^3 log-normal diffusion operator (h^-2 scaled, "
                         f"n={a.n}), Newton from 0 to ||F|| <= 1e-10 ||f||, Jacobi-PCG steps to rtol 1e-10"),
            "newton_steps": steps, "forward_ms": fw * 1e3, "backward_ms": bw * 1e3,
            "backward_over_forward": bw / fw}


def run_eigen(ctx, args, dev):
    """Sec. "Adjoint Differentiation", eigenvalue problems: the 6 smallest
    eigenpairs of the 64^3 log-normal diffusion operator by shift-invert
    Lanczos (library CG solves to rtol 1e-14 per step), then the
    Hellmann-Feynman gradient of their sum (one on-pattern outer product)."""
    import torch

    import paper_2601_13994_amd as hs
    from paper_2601_13994_amd import eigen

    a = ctx["eigen"]
    rp, col = torch.as_tensor(a.row_ptr).to(dev), torch.as_tensor(a.col).to(dev)
    pat = _pattern(dev, a)

    def run_once():
        vals = torch.as_tensor(a.val).to(dev).requires_grad_(True)
        A = hs.SparseCSR(vals, rp, col, pattern=pat)
        info = {}
        _sync()
        t0 = time.perf_counter()
        lam, _ = eigen.eigsh(A, k=6, which="SA", info=info)
        _sync()
        t1 = time.perf_counter()
        lam.sum().backward()
        _sync()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, info, lam.detach().cpu().tolist()

    run_once()
    fw, bw, info, lam = run_once()
    return {"workload": f"6 smallest eigenpairs of the 64^3 log-normal diffusion operator (n={a.n}), shift-invert "
                        "Lanczos with full reorthogonalisation, CG solves to rtol 1e-14",
            "eigenvalues": lam, "lanczos_steps": info["lanczos_steps"],
            "max_rel_residual": info["max_rel_residual"], "forward_ms": fw * 1e3, "backward_ms": bw * 1e3}


def run(args):
    sel = ALL_WORKLOADS if args.workloads == "all" else tuple(w.strip() for w in args.workloads.split(","))
    bad = [w for w in sel if w not in ALL_WORKLOADS]
    if bad:
        raise SystemExit(f"unknown workload(s) {bad}; choose from {ALL_WORKLOADS}")
    ctx = generate(sel, args)

    import torch

    from paper_2601_13994_amd import _lib

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    pat = None
    if "d3" in ctx:
        a, b = ctx["d3"]
        log(f"[bench] n={a.n} nnz={a.nnz}")
        vals = torch.as_tensor(a.val).to(dev)
        bt = torch.as_tensor(b).to(dev)
        _sync()
        t0 = time.perf_counter()
        pat = _pattern(dev, a)
        _sync()
        ctx["setup_ms"] = (time.perf_counter() - t0) * 1e3
        if args.format == "csr":
            pat.set_format("csr")
            args.csr_line = False
        log(f"[bench] pattern ready ({ctx['setup_ms']:.1f} ms)")
    if args.calibrate_copy:
        # plain copy kernel of known size for counter calibration (1 GiB read + 1 GiB write)
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        _sync()
        dst.copy_(src)
        _sync()
        del src, dst
        log("[bench] calibration copy done (1 GiB -> 1 GiB)")

    if "diffusion3d" in sel:
        out, iters = run_diffusion(ctx, args, dev, pat, vals, bt)
        del vals
    else:
        # a profiling run of other workloads only: no headline line
        out, iters = {"metric": METRIC, "value": None, "unit": "solves/s", "n_gpus": 1,
                      "note": "diffusion3d workload not selected"}, None
    sub = {}
    runners = {"bicgstab": lambda: run_bicgstab(ctx, args, dev, pat), "poisson2d": lambda: run_poisson(ctx, args, dev),
               "knn": lambda: run_knn(ctx, args, dev), "adjoint": lambda: run_adjoint(ctx, args, dev),
               "learned": lambda: run_learned(ctx, args, dev), "paper": lambda: run_paper(ctx, args, dev),
               "inverse": lambda: run_inverse(ctx, args, dev), "nonlinear": lambda: run_nonlinear(ctx, args, dev),
               "eigen": lambda: run_eigen(ctx, args, dev)}
    for name in sel:
        if name == "diffusion3d":
            continue
        log(f"[bench] workload {name} ...")
        t = time.time()
        sub[name] = runners[name]()
        torch.cuda.empty_cache()
        log(f"[bench] workload {name} done in {time.time() - t:.1f}s: "
            + json.dumps({k: v for k, v in sub[name].items() if k != "workload"})[:400])
    out["workloads"] = sub
    if not args.no_cpu_baseline and iters is not None:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(a, b, iters)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# rocprofv3 summaries
# ---------------------------------------------------------------------------

def _read_csv(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def summarize(args):
    d = args.summarize_rocprof
    lines = [f"# rocprofv3 summary: {args.label}", "", f"Command: `{args.command}`", ""]
    stats = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    result = {}
    if stats:
        rows = _read_csv(stats[0])
        lines += ["| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
        for r in rows[:25]:
            name = r.get("Name", "")
            short = name.split("(")[0][:90]
            calls = int(r.get("Calls", 0))
            tot = float(r.get("TotalDurationNs", 0)) / 1e6
            avg = float(r.get("AverageNs", 0)) / 1e3
            mn = float(r.get("MinNs", 0)) / 1e3
            mx = float(r.get("MaxNs", 0)) / 1e3
            pct = float(r.get("Percentage", 0))
            lines.append(f"| `{short}` | {calls} | {tot:.2f} | {avg:.1f} | {mn:.1f} | {mx:.1f} | {pct:.1f} |")
        lines.append("")
    counters = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if counters:
        rows = _read_csv(counters[0])
        agg = {}
        for r in rows:
            name = r.get("Kernel_Name", "")
            cn = r.get("Counter_Name", "")
            v = float(r.get("Counter_Value", 0))
            key = (name.split("(")[0], cn)
            agg.setdefault(key, []).append(v)
        lines += ["| kernel | counter | dispatches | mean per dispatch |", "|---|---|---|---|"]
        for (k, cn), vs in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
            lines.append(f"| `{k[:90]}` | {cn} | {len(vs)} | {sum(vs) / len(vs):.1f} |")
            result[f"{k}|{cn}"] = sum(vs) / len(vs)
        lines.append("")
    out = os.path.join(ROOT, "profiles", args.label + ".md")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    if result:
        with open(os.path.join(ROOT, "profiles", args.label + ".json"), "w") as f:
            json.dump({"command": args.command, "mean_per_dispatch": result,
                       "kernel_source_hash": kernel_source_hash()}, f, indent=1)
    print(out)


def counters(args):
    """Per-launch HBM traffic of the dominant kernel from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the
    same counter read for the 1 GiB calibration copy of that run."""
    fetch_dir, write_dir = args.counters_from
    out = {}
    for tag, d, cname in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        rows = [r for f in files for r in _read_csv(f) if r.get("Counter_Name") == cname]
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        calib = max(copies)  # the 1 GiB device-to-device copy is the largest one
        scale = (1 << 20) / calib  # true KiB per counted KiB
        vals = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"].split("(")[0].endswith(DOMINANT)
                or (DOMINANT + "<") in r["Kernel_Name"]]
        # launches of a graph chunk after the system stopped return at entry;
        # the per-launch figure is over the launches that did work
        worked = [v for v in vals if v > 0.1 * max(vals)]
        out[tag] = {"kib_per_dispatch": sum(worked) / len(worked), "dispatches": len(worked),
                    "dispatches_returned_at_entry": len(vals) - len(worked), "calibration_kib": calib,
                    "scale": scale, "bytes_per_dispatch": sum(worked) / len(worked) * 1024 * scale}
    total = out["fetch"]["bytes_per_dispatch"] + out["write"]["bytes_per_dispatch"]
    rec = {"kernel": DOMINANT, "kernel_source_hash": kernel_source_hash(), "n": args.n, "nnz": args.nnz,
           "bytes_per_launch": total, "fetch": out["fetch"], "write": out["write"], "command": args.command,
           "format": args.format}
    path = CSR_COUNTER_FILE if args.format == "csr" else COUNTER_FILE
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    md = path.replace(".json", ".md")
    what = "CSR form" if args.format == "csr" else "the solve's stored form"
    with open(md, "w") as f:
        f.write(f"# HBM traffic of {DOMINANT}, diffusion3d 256^3, {what} (rocprofv3 --pmc)\n\n")
        f.write(f"Commands: `{args.command}`\n\n")
        f.write("| counter | dispatches that did work (returned at entry) | KiB per dispatch | calibration copy KiB "
                "(1 GiB copied) | scale | bytes per dispatch |\n")
        f.write("|---|---|---|---|---|---|\n")
        for tag in ("fetch", "write"):
            o = out[tag]
            f.write(f"| {tag.upper()}_SIZE | {o['dispatches']} ({o['dispatches_returned_at_entry']}) | "
                    f"{o['kib_per_dispatch']:.1f} | {o['calibration_kib']:.1f} | {o['scale']:.3f} | "
                    f"{o['bytes_per_dispatch']:.4g} |\n")
        f.write(f"\nTotal HBM traffic per launch: {total:.4g} bytes (kernel source hash {rec['kernel_source_hash']}).\n")
    print(path)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=256, help="grid edge (256 is the benchmark size)")
    ap.add_argument("--max-iter", type=int, default=0, help="cap iterations (profiling runs only)")
    ap.add_argument("--profile-solves", type=int, default=1,
                    help="profiled solves after the timed region that give the SpMV launch time")
    ap.add_argument("--no-csr-line", dest="csr_line", action="store_false",
                    help="skip the headline system's solve on the forced CSR form")
    ap.add_argument("--format", default="auto", choices=["auto", "csr"],
                    help="SpMV form of the headline pattern (csr: profiling runs of the CSR kernel)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="skip the SpMV autotuner (set-up, not timed)")
    ap.add_argument("--workloads", default="all", help="comma list from " + ",".join(ALL_WORKLOADS))
    ap.add_argument("--sub-steps", type=int, default=2, help="timed repetitions of the other workloads")
    ap.add_argument("--poisson-copies", type=int, default=1024)
    ap.add_argument("--inverse-steps", type=int, default=1500)
    ap.add_argument("--nonlinear-m", type=int, default=128)
    ap.add_argument("--knn-systems", type=int, default=512)
    ap.add_argument("--adj-m", type=int, default=96)
    ap.add_argument("--adj-batch", type=int, default=128)
    ap.add_argument("--aniso-m", type=int, default=256)
    ap.add_argument("--train-systems", type=int, default=4096)
    ap.add_argument("--eval-systems", type=int, default=1024)
    ap.add_argument("--train-steps", type=int, default=256, help="4096 systems / 16 per step: one pass")
    ap.add_argument("--train-batch", type=int, default=16)
    ap.add_argument("--train-probes", type=int, default=4)
    ap.add_argument("--train-lr", type=float, default=3e-3)
    ap.add_argument("--oracle-adj-systems", type=int, default=2, help="systems of the oracle's adjoint timing")
    ap.add_argument("--oracle-aniso-systems", type=int, default=32, help="held-out systems the oracle solves")
    ap.add_argument("--calibrate-copy", action="store_true", help="also run a 1 GiB copy for counter calibration")
    ap.add_argument("--summarize-rocprof", metavar="DIR")
    ap.add_argument("--counters-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the dominant kernel's counter summary from two --pmc runs")
    ap.add_argument("--n", type=int, default=256 ** 3)
    ap.add_argument("--nnz", type=int, default=7 * 256 ** 3 - 6 * 256 ** 2)
    ap.add_argument("--label", default="summary")
    ap.add_argument("--command", default="")
    args = ap.parse_args()
    if args.summarize_rocprof:
        summarize(args)
        return
    if args.counters_from:
        counters(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}), flush=True)
        log("bench.py: only --gpus 1 is supported (the method is measured on one GPU)")
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
