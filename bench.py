#!/usr/bin/env python3
"""Throughput of the Toeplitz tridiagonal dichotomy solve on one MI355X.

Workload: the paper's single-system case, one Toeplitz tridiagonal system of
N = 2**26 unknowns, T = tridiag{-0.9, 2.5, -1.1} (dominance ratio 1.25),
F ~ N(0, 1) from seed 0, resident in HBM before the timed region.  A step is
one full solve T X = F (first pass over tiles, interface pass, final pass).
The headline path is float sweeps with double residual refinement
('f32_refine', data in and out in double); the all-double path ('f64') is
timed the same way beside it.

Prints one JSON line.  `roofline` is for the kernel with the longest average
duration in the headline path, from HIP events recorded on the solve stream
around each kernel during the timed steps; its `traffic` comes from the
committed rocprofv3 counter summary (profiles/) when it was taken on the
current kernel source, else null.  `cpu_baseline` is the CPU oracle (plain
Thomas, one thread: the single system is a sequential recurrence) timed on
this host on the same system; the same oracle output gives the error of both
GPU results.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "unknowns/s + HBM GB/s (% peak): FP32+refine vs FP64 solve at rel err ≤1e-12"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per unknown of each kernel group (double data)
BYTES_PER_UNKNOWN = {"first_pass": 8.0,    # read F
                     "final_pass": 16.0}   # read F, write X
KERNEL_NAMES = {"first_pass": "k_beta<double> (Green-row tile summaries, first pass)",
                "final_pass": "k_tile<double, float, REFINE, final> (solve, refine and store)"}
KERNEL_NAMES_F64 = {"first_pass": "k_beta<double> (Green-row tile summaries, first pass)",
                    "final_pass": "k_tile<double, double, final> (solve and store)"}


def kernel_source_hash() -> str:
    """Hash of the device code (comments and blank lines removed, so that a
    comment edit does not invalidate the committed counter summary)."""
    h = hashlib.sha256()
    for rel in ("paper_1002_2469_amd/csrc/tdt_kernels.hip", "paper_1002_2469_amd/csrc/tdt_internal.h"):
        with open(os.path.join(ROOT, rel)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        src = "\n".join(line.rstrip() for line in src.splitlines() if line.strip())
        h.update(src.encode())
    return h.hexdigest()[:16]


def committed_traffic(kernel_key: str, mode: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_single_large.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("kernel_source_sha") != kernel_source_hash():
            return None
        return rec["modes"][mode][kernel_key]["hbm_bytes_per_launch"]
    except Exception:
        return None


def run_mode(tdt, d, F, X, mode, steps, warmup, torch):
    plan = tdt.Plan(d["t_m1"], d["t_0"], d["t_1"], d["N"], mode)
    plan.reserve(1)
    for _ in range(warmup):
        plan.solve(F, X)
    torch.cuda.synchronize()
    plan.info()                     # clears the refinement counter
    plan.profile(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        plan.solve(F, X)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    prof = plan.profile_read()
    plan.profile(False)
    info = plan.info()
    n = prof["solves"]
    kern = {"first_pass": prof["first_pass_ms"] / n, "interface": prof["interface_ms"] / n,
            "final_pass": prof["final_ms"] / n}
    plan.close()
    return dict(ms=ms, kernels_ms=kern, refine_iters=info["refine_iters"], X=X.cpu().numpy())


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1 << 26, help="system order (default 2**26)")
    ap.add_argument("--modes", default="f32_refine,f64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain device copy of F (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU; --gpus {args.gpus} is not "
              "supported (one GPU's share of a sharded solve is what is measured here)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1002_2469_amd as tdt
    from paper_1002_2469_amd import workloads as W

    d = W.single_large(seed=0, n=args.n)
    F = torch.from_numpy(d["F"]).to("cuda:0")
    X = torch.empty_like(F)
    torch.cuda.synchronize()
    modes = [m for m in args.modes.split(",") if m]
    res = {}
    for mode in modes:
        res[mode] = run_mode(tdt, d, F, X, mode, args.steps, args.warmup, torch)
        print(f"[bench] {mode}: {res[mode]['ms']:.4f} ms/step  kernels(ms) "
              f"{json.dumps({k: round(v, 5) for k, v in res[mode]['kernels_ms'].items()})}",
              file=sys.stderr, flush=True)

    if args.copy_calib:
        Y = torch.empty_like(F)
        for _ in range(5):
            Y.copy_(F)
        torch.cuda.synchronize()
        del Y

    N = d["N"]
    head = modes[0]

    # CPU oracle leg: time it on this host and use its output for the errors
    cpu = None
    errs = {}
    if not args.no_cpu:
        import oracle
        threads = oracle.threads(1)
        times = []
        Xo = None
        t_budget = time.perf_counter()
        while len(times) < 25 and (time.perf_counter() - t_budget < 12.0 or len(times) < 3):
            t0 = time.perf_counter()
            Xo = oracle.solve(d["F"], d["t_m1"], d["t_0"], d["t_1"], nthreads=1)
            times.append(time.perf_counter() - t0)
        med = statistics.median(times)
        cpu = {"value": N / med, "unit": "unknowns/s", "cores": threads, "kind": "oracle",
               "sample": f"the whole workload (one system, N={N}), plain Thomas in double, "
                         f"1 thread, median of {len(times)} runs of {med:.3f} s"}
        for mode in modes:
            errs[mode] = oracle.rel_err(res[mode]["X"], Xo)

    def path_record(mode):
        r = res[mode]
        return {"value": N / (r["ms"] * 1e-3), "unit": "unknowns/s", "ms_per_step": r["ms"],
                "step_gbs_at_16B": 16.0 * N / (r["ms"] * 1e-3) / 1e9,
                "kernels_ms": {k: round(v, 6) for k, v in r["kernels_ms"].items()},
                "rel_err_vs_oracle": errs.get(mode), "refine_iters": r["refine_iters"]}

    hk = res[head]["kernels_ms"]
    dom = "final_pass" if hk["final_pass"] >= hk["first_pass"] else "first_pass"
    achieved = BYTES_PER_UNKNOWN[dom] * N / (hk[dom] * 1e-3) / 1e9
    traffic = committed_traffic(dom, head)
    names = KERNEL_NAMES if head == "f32_refine" else KERNEL_NAMES_F64
    line = {
        "metric": METRIC,
        "value": N / (res[head]["ms"] * 1e-3),
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res[head]["ms"],
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32 sweeps + f64 residual/update" if head == "f32_refine" else head,
        "data": "synthetic (seeded normal right-hand side; no dataset involved)",
        "config": {"workload": f"single_large: one Toeplitz tridiagonal system, N={N}, "
                               f"t=(-0.9, 2.5, -1.1), F~N(0,1) seed 0, double in/out",
                   "N": N, "M": 1, "path": head},
        "rel_err_vs_oracle": errs.get(head),
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "bytes_per_unknown": BYTES_PER_UNKNOWN[dom], "avg_ms": hk[dom]},
        "paths": {m: path_record(m) for m in modes},
        "cpu_baseline": cpu,
    }
    if "f64" in res and head != "f64":
        line["speedup_vs_f64"] = res["f64"]["ms"] / res[head]["ms"]
    line["kernel_source_sha"] = kernel_source_hash()
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
