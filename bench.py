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
             achieved = algorithmic bytes per launch / mean launch duration,
             durations from HIP events around every launch of the timed
             solves; traffic = FETCH_SIZE + WRITE_SIZE per launch from the
             committed rocprofv3 counter summary (null if the kernel source
             changed since the counters were taken)
  cpu_baseline  the CPU oracle (single thread) timed on a bounded sample of
             the same system: a few PCG iterations, scaled by the GPU solve's
             iteration count

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
KERNEL_SOURCES = ["paper_2601_13994_amd/csrc/krylov.hip", "paper_2601_13994_amd/csrc/common.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def spmv_bytes(n: int, nnz: int) -> int:
    """Algorithmic HBM bytes of one q = A p (+ p.q) launch: values and
    column indices once (12 nnz), row pointers once (4(n+1)), p gathered
    once with cache reuse (8n), q written once (8n)."""
    return 12 * nnz + 4 * (n + 1) + 16 * n


def pcg_iteration_bytes(n: int, nnz: int) -> int:
    """Algorithmic bytes of one Jacobi-PCG iteration as scheduled here:
    SpMV+dot (12nnz + 4(n+1) + 16n), update (reads x p r q D^-1, writes x r:
    56n), direction (reads D^-1 r p, writes p: 32n)."""
    return 12 * nnz + 4 * (n + 1) + 104 * n


def cpu_info() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def load_traffic(n: int, nnz: int):
    """Per-launch HBM bytes of the dominant kernel from the committed
    counter summary, scaled by the copy-kernel calibration; None if absent
    or taken on different kernel source."""
    if not os.path.exists(COUNTER_FILE):
        return None
    with open(COUNTER_FILE) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("n") != n or d.get("nnz") != nnz:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(a, b, gpu_iters: int, k1: int = 1, k2: int = 31):
    import oracle

    oracle.lib()
    t0 = time.perf_counter()
    oracle.cg(a, b, precond="jacobi", rtol=1e-8, max_iter=k1)
    t1 = time.perf_counter()
    oracle.cg(a, b, precond="jacobi", rtol=1e-8, max_iter=k2)
    t2 = time.perf_counter()
    per_it = ((t2 - t1) - (t1 - t0)) / (k2 - k1)
    setup = (t1 - t0) - k1 * per_it
    solve_s = setup + gpu_iters * per_it
    return {
        "value": 1.0 / solve_s,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{k2 - k1} Jacobi-PCG iterations of the same 256^3 system (difference of {k2}- and "
                   f"{k1}-iteration runs: {per_it:.3f} s/iteration, {setup:.2f} s set-up), scaled to the "
                   f"GPU solve's {gpu_iters} iterations; sequential FP64 C, {cpu_info()}"),
        "seconds_per_iteration": per_it,
        "host_cpus": os.cpu_count(),
    }


def run(args):
    import numpy as np
    import torch

    import workloads as W
    from paper_2601_13994_amd import _lib

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    m = args.m
    log(f"[bench] generating 3D diffusion m={m} ...")
    t = time.time()
    a, b = W.diffusion3d_workload(m)
    n, nnz = a.n, a.nnz
    log(f"[bench] n={n} nnz={nnz} generated in {time.time() - t:.1f}s")
    vals = torch.as_tensor(a.val).to(dev)
    bt = torch.as_tensor(b).to(dev)
    pat = _lib.Pattern(torch.as_tensor(a.row_ptr).to(dev), torch.as_tensor(a.col).to(dev))
    torch.cuda.synchronize()
    log("[bench] pattern ready")

    if args.calibrate_copy:
        # plain copy kernel of known size for counter calibration (1 GiB read + 1 GiB write)
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] calibration copy done (1 GiB -> 1 GiB)")

    opts_w = _lib.make_opts(method="cg", precond="jacobi", rtol=1e-8, max_iter=args.max_iter)
    for i in range(args.warmup):
        x, infos, st = _lib.solve(pat, vals, bt, opts_w)
        log(f"[bench] warmup {i}: status={st} iters={infos[0]['iters']} true_res={infos[0]['true_residual']:.2e}")

    opts = _lib.make_opts(method="cg", precond="jacobi", rtol=1e-8, max_iter=args.max_iter, profile=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for i in range(args.steps):
        x, infos, st = _lib.solve(pat, vals, bt, opts)
        recs.append(infos[0])
        log(f"[bench] step {i}: status={st} iters={infos[0]['iters']}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    iters = recs[-1]["iters"]
    spmv_ms = sum(r["spmv_ms"] for r in recs)
    launches = sum(r["spmv_launches"] for r in recs)
    avg_ms = spmv_ms / max(launches, 1)
    bytes_launch = spmv_bytes(n, nnz)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    traffic = load_traffic(n, nnz)
    ms_step = elapsed / args.steps * 1e3
    it_bytes = pcg_iteration_bytes(n, nnz)
    out = {
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
            "workload": f"diffusion3d-{m}^3 log-normal kappa, Jacobi-PCG to rtol 1e-8, x0=0",
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
            "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_launch,
            "mean_launch_ms": avg_ms,
            "launches_timed": launches,
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
            "spmv_share_of_step": spmv_ms / args.steps / ms_step,
        },
    }
    if not args.no_cpu_baseline:
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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=256, help="grid edge (256 is the benchmark size)")
    ap.add_argument("--max-iter", type=int, default=0, help="cap iterations (profiling runs only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true", help="also run a 1 GiB copy for counter calibration")
    ap.add_argument("--summarize-rocprof", metavar="DIR")
    ap.add_argument("--label", default="summary")
    ap.add_argument("--command", default="")
    args = ap.parse_args()
    if args.summarize_rocprof:
        summarize(args)
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
