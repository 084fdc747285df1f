#!/usr/bin/env python3
"""Throughput of the Toeplitz tridiagonal dichotomy solve on one MI355X.

Default workload (`single_large`): the paper's single-system case, one
Toeplitz tridiagonal system of N = 2**26 unknowns, T = tridiag{-0.9, 2.5, -1.1}
(dominance ratio 1.25), F ~ N(0, 1) from seed 0, resident in HBM before the
timed region.  A step is one full solve T X = F (first pass over tiles,
interface pass, final pass).  The headline path is float sweeps with double
residual refinement ('f32_refine', data in and out in double); the all-double
path ('f64') is timed the same way beside it.

Other workloads (`--workload`): `single_small` (one system of N = 65536,
T = tridiag{-1, 4, -1}: launch-bound), `series` (8192 right-hand sides of N = 8192
sharing T = tridiag{-1, 3, -1}), `sov` (2048 separation-of-variables systems,
N_k log-uniform in [256, 65536], each with its own t_0; one step is a replay
of the solve captured in a hipGraph), `sov_neumann` (the same batch with
Neumann ends: quasi-Toeplitz systems with psi = chi = 1) and `diff` (1024
systems of N = 16384 with their own T; a step is the forward solve plus the
adjoint backward pass) and `general` (64 right-hand sides of N = 2**20 sharing a
general tridiagonal matrix with per-row entries; paths f64 and f32) and
`poisson2d` (the 2D Poisson problem on 8191 x 8191 interior points, 2^13
intervals per side, solved end to end by separation of variables: sine
transforms, 8191 line systems of 8191 solved in place as a strided batch,
inverse transforms; path f64) and
`poisson3d` (the 3D problem of Sec. 3.5 on 511^3 interior points: sine
transform along x, Peaceman-Rachford ADI on every mode's (y, z) plane with
strided line solves, inverse transform; path f64).

Launch options: the library's autotuner picks them on the data, unless
`--shape`, `--whole` or `--wg` fix them (then nothing else is tried, so a
profiler trace of the run holds one configuration per kernel).  The plan
creation (the paper's Stage 1, the preliminary step) is timed beside the
solve (Stage 2).

Prints one JSON line.  `roofline` is for the kernel with the longest average
duration in the headline path, from HIP events recorded on the solve stream
around each kernel during the timed steps; its `traffic` comes from the
committed rocprofv3 counter summary (profiles/) when it was taken on the
current device code, else null.  `cpu_baseline` is the CPU oracle (plain
Thomas; one thread for a single system, all host threads for batches) timed
on this host on the same inputs; the same oracle output gives the error of
every GPU result.
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
WORKLOADS = ("single_large", "single_small", "series", "sov", "sov_neumann", "diff", "general",
             "poisson2d", "poisson3d")


# the device sources of each workload's kernels
# (with the host code that decides the launches: tiling, work lists, shapes)
SOURCES_TILES = ("paper_1002_2469_amd/csrc/tdt_kernels.hip", "paper_1002_2469_amd/csrc/tdt_internal.h",
                 "paper_1002_2469_amd/csrc/tdt_api.cpp")
SOURCES_POISSON = ("paper_1002_2469_amd/csrc/tdt_poisson.hip", "paper_1002_2469_amd/csrc/tdt_strided.hip",
                   "paper_1002_2469_amd/csrc/tdt_strided.h", "paper_1002_2469_amd/csrc/tdt_internal.h",
                   "paper_1002_2469_amd/csrc/tdt_api.cpp")


def kernel_source_hash(workload: str = "") -> str:
    """Hash of the device code of a workload's kernels (comments and blank
    lines removed, so that a comment edit does not invalidate the committed
    counter summary)."""
    h = hashlib.sha256()
    for rel in (SOURCES_POISSON if workload.startswith("poisson") else SOURCES_TILES):
        with open(os.path.join(ROOT, rel)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        src = "\n".join(line.rstrip() for line in src.splitlines() if line.strip())
        h.update(src.encode())
    return h.hexdigest()[:16]


def committed_traffic(workload: str, kernel_key: str, mode: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current device code."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("kernel_source_sha") != kernel_source_hash(workload):
            return None
        return rec["modes"][mode][kernel_key]["hbm_bytes_per_launch"]
    except Exception:
        return None


# --------------------------------------------------------------------------
# workloads: inputs, plans, per-kernel algorithmic bytes
# --------------------------------------------------------------------------

def load_workload(name: str, args):
    from paper_1002_2469_amd import workloads as W
    if name == "single_large":
        d = W.single_large(seed=0, n=args.n)
        d.update(kind="series", units=d["N"],
                 desc=f"single_large: one Toeplitz tridiagonal system, N={d['N']}, "
                      f"t=(-0.9, 2.5, -1.1), F~N(0,1) seed 0, double in/out")
    elif name == "single_small":
        d = W.single_small(seed=0)
        d.update(kind="series", units=d["N"],
                 desc=f"single_small: one Toeplitz tridiagonal system, N={d['N']}, "
                      f"t=(-1, 4, -1), F~U[-1,1] seed 0, double in/out (launch-bound)")
    elif name == "series":
        d = W.series(seed=0)
        d.update(kind="series", units=d["N"] * d["M"],
                 desc=f"series: M={d['M']} right-hand sides of N={d['N']} sharing "
                      f"t=(-1, 3, -1), F~U[-1,1] seed 0, [M][N] double in/out")
    elif name == "sov":
        d = W.sov_batch(seed=0)
        d.update(kind="varlen", units=int(d["offsets"][-1]), graph=True,
                 desc=f"sov: S={d['S']} separation-of-variables systems, N_k log-uniform "
                      f"in [256, 65536] (sum {int(d['offsets'][-1])}), t_+-1=1, own t_0, "
                      f"F~N(0,1) seed 0, packed, solve replayed from a hipGraph")
    elif name == "sov_neumann":
        d = W.sov_neumann_batch(seed=0)
        d.update(kind="varlen", units=int(d["offsets"][-1]), graph=True,
                 desc=f"sov_neumann: S={d['S']} separation-of-variables systems with Neumann "
                      f"ends (quasi-Toeplitz, psi=chi=1), N_k log-uniform in [256, 65536] "
                      f"(sum {int(d['offsets'][-1])}), t_+-1=1, own t_0, F~N(0,1) seed 0, "
                      f"packed, solve replayed from a hipGraph")
    elif name == "general":
        d = W.general_series(seed=0)
        d.update(kind="general", units=d["N"] * d["M"],
                 desc=f"general: M={d['M']} right-hand sides of N={d['N']} sharing a general "
                      f"tridiagonal matrix (variable-coefficient diffusion-reaction rows, "
                      f"dominance 1.1-1.6), F~N(0,1) seed 0, [M][N] double in/out")
    elif name == "poisson2d":
        d = W.poisson2d(seed=0)
        d.update(kind="poisson", units=d["nx"] * d["ny"],
                 desc=f"poisson2d: five-point Poisson problem on {d['nx']}x{d['ny']} interior "
                      f"points of the unit square, zero boundary, F~N(0,1) seed 0, [Ny][Nx] "
                      f"double in/out; sine transforms of the rows (fused: fold, FFT in LDS, "
                      f"prefix sum) + one Toeplitz line system per mode, solved in place down "
                      f"the columns of the transformed rows + inverse transforms")
    elif name == "poisson3d":
        d = W.poisson3d(seed=0)
        d.update(kind="poisson3d", units=d["nx"] * d["ny"] * d["nz"], eps=1e-13,
                 desc=f"poisson3d: seven-point Poisson problem on {d['nx']}x{d['ny']}x{d['nz']} "
                      f"interior points of the unit cube, zero boundary, F~N(0,1) seed 0, "
                      f"[Nz][Ny][Nx] double in/out; sine transform along x (fused row transform), "
                      f"Peaceman-Rachford ADI per mode plane (optimal parameters, eps 1e-13, "
                      f"strided line solves along y and z), inverse transform")
    elif name == "diff":
        d = W.diff_batch(seed=0)
        d.update(kind="varlen", units=int(d["offsets"][-1]), adjoint=True,
                 desc=f"diff: S={d['S']} systems of N={d['N']}, own t's, forward solve "
                      f"plus adjoint backward (gF, dL/dt), F,W~N(0,1) seed 0")
    else:
        raise ValueError(name)
    return d


def make_plan(tdt, d, mode):
    if d["kind"] == "general":
        return tdt.GeneralPlan(d["a"], d["b"], d["c"], mode)
    if d["kind"] == "series":
        return tdt.Plan(d["t_m1"], d["t_0"], d["t_1"], d["N"], mode)
    return tdt.VarlenPlan(d["offsets"], d["t_m1"], d["t_0"], d["t_1"], mode,
                          psi=d.get("psi"), chi=d.get("chi"))


def tile_counts(d, tile):
    """Unknowns that go through the first pass (systems of more than one
    tile of `tile` rows) and through the final pass (all)."""
    if d["kind"] in ("series", "general"):
        multi = d["N"] > tile
        return (d["N"] * d["M"] if multi else 0), d["N"] * d["M"]
    sizes = d["offsets"][1:] - d["offsets"][:-1]
    inner = sizes - (2 if "psi" in d else 0)     # quasi-Toeplitz: tiles cover the inner rows
    return int(sizes[inner > tile].sum()), int(sizes.sum())


def plan_create_ms(tdt, d, mode, reps=3):
    """The preliminary step (the paper's Stage 1): plan creation on the host
    in long double plus the blocking upload, median of `reps` creations."""
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        p = make_plan(tdt, d, mode)
        times.append((time.perf_counter() - t0) * 1e3)
        p.close()
    return statistics.median(times)


def run_mode(tdt, d, F, X, mode, steps, warmup, torch, opts=None):
    """opts None: the library's autotuner picks the work shape and launch
    options on this data (timed afresh, not from a cache file); otherwise
    the given options are set and nothing else is tried (one launch
    configuration, e.g. for a profiler trace)."""
    stage1_ms = plan_create_ms(tdt, d, mode)
    plan = make_plan(tdt, d, mode)
    if opts is None:
        plan.reserve(d.get("M", 1))
        tuned = plan.autotune(F, X, cache=False, adjoint=d.get("adjoint", False))
    else:
        for k, v in opts.items():
            # whole-system threshold: varlen plans only; a general plan has one work shape
            if (k != "whole_max_tiles" or d["kind"] == "varlen") and \
                    (k != "shape" or d["kind"] != "general"):
                plan.set_option(k, v)
        plan.reserve(d.get("M", 1))
        tuned = {k: plan.get_option(k) for k in ("shape", "whole_max_tiles", "wg_per_cu")}
        tuned["fixed"] = True
    support = plan.green_support()["forward"] if d["kind"] in ("series", "general") else (0, 0)
    adj = d.get("adjoint", False)
    gX = gF = gt = None
    if adj:
        gX = torch.from_numpy(d["W"].reshape(-1)).to(F.device)
        gF = torch.empty_like(gX)
        gt = torch.empty((d["S"], 3), dtype=torch.float64, device=F.device)

    def step():
        plan.solve(F, X)
        if adj:
            plan.backward(gX, X, gF, gt)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()

    # kernel-group times: eager solves with HIP events around each kernel
    plan.info()                     # clears the refinement counter
    kern = {}
    for direction in (("fwd", "bwd") if adj else ("fwd",)):
        plan.profile(True)
        for _ in range(steps):
            if direction == "fwd":
                plan.solve(F, X)
            else:
                plan.backward(gX, X, gF, gt)
        torch.cuda.synchronize()
        prof = plan.profile_read()
        plan.profile(False)
        n = max(prof["solves"], 1)
        pre = "" if direction == "fwd" else "bwd_"
        kern[pre + "first_pass"] = prof["first_pass_ms"] / n
        kern[pre + "interface"] = prof["interface_ms"] / n
        kern[pre + "final_pass"] = prof["final_ms"] / n
    info = plan.info()

    # step time: eager, or replays of a captured graph
    graph = None
    if d.get("graph"):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        for _ in range(warmup):
            graph.replay()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        if graph is not None:
            graph.replay()
        else:
            step()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    # steps run on this plan after tuning (warm-up, event loop, graph warm-up, timed)
    solves = warmup + 2 * steps + (1 + warmup if d.get("graph") else 0)
    out = dict(ms=ms, kernels_ms=kern, refine_iters=info["refine_iters"],
               X=X.cpu().numpy().reshape(-1), tuned=tuned, stage1_ms=stage1_ms,
               green_support=support, solves=solves)
    if adj:
        out["gF"] = gF.cpu().numpy().reshape(-1)
        out["gt"] = gt.cpu().numpy()
    del graph
    plan.close()
    return out


def run_poisson(tdt, d, F, mode, steps, warmup, torch):
    """A step is one whole 2D solve (transforms and line solves)."""
    t0 = time.perf_counter()
    solver = tdt.Poisson2D(d["nx"], d["ny"], d["hx"], d["hy"], mode)
    stage1_ms = (time.perf_counter() - t0) * 1e3
    U = torch.empty_like(F)
    for _ in range(warmup):
        solver.solve(F, U)
    torch.cuda.synchronize()
    solver.profile(True)
    for _ in range(steps):
        solver.solve(F, U)
    torch.cuda.synchronize()
    prof = solver.profile_read()
    solver.profile(False)
    n = max(prof["solves"], 1)
    kern = {"forward_transform": prof["forward_ms"] / n, "line_solve": prof["line_ms"] / n,
            "inverse_transform": prof["inverse_ms"] / n}
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        solver.solve(F, U)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    out = dict(ms=ms, kernels_ms=kern, refine_iters=0, X=U.cpu().numpy().reshape(-1), tuned=None,
               stage1_ms=stage1_ms, solves=warmup + 2 * steps)
    solver.close()
    return out


def run_poisson3d(tdt, d, F, steps, warmup, torch):
    """A step is one whole 3D solve (transforms and all ADI half-steps)."""
    t0 = time.perf_counter()
    solver = tdt.Poisson3D(d["nx"], d["ny"], d["nz"], d["hx"], d["hy"], d["hz"], d["eps"])
    stage1_ms = (time.perf_counter() - t0) * 1e3
    U = torch.empty_like(F)
    for _ in range(warmup):
        solver.solve(F, U)
    torch.cuda.synchronize()
    solver.profile(True)
    for _ in range(steps):
        solver.solve(F, U)
    torch.cuda.synchronize()
    prof = solver.profile_read()
    solver.profile(False)
    n = max(prof["solves"], 1)
    kern = {"forward_transform": prof["forward_ms"] / n, "adi": prof["adi_ms"] / n,
            "inverse_transform": prof["inverse_ms"] / n}
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        solver.solve(F, U)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    counts, _om = solver.schedule()
    out = dict(ms=ms, kernels_ms=kern, refine_iters=0, X=U.cpu().numpy().reshape(-1), tuned=None,
               counts=counts, stage1_ms=stage1_ms, solves=warmup + 2 * steps)
    solver.close()
    return out


def adi_bytes(d, counts):
    """Algorithmic HBM bytes of the ADI half-steps of one solve: per active
    mode and line unknown, a y-sweep reads its right-hand side and writes
    the next one (16 B), a z-sweep reads that and fhat and writes (24 B)."""
    import numpy as np
    counts = np.asarray(counts)
    plane = d["ny"] * d["nz"]
    total = 0
    for j in range(int(counts.max())):
        P = int(np.sum(counts > j))
        total += (16 + 24) * P * plane
    return float(total)


def cpu_leg_poisson3d(d, budget_s=12.0, n_sample=127):
    """The oracle (explicit sine transform, ADI per mode with Thomas per
    line) on a smaller cube; the ADI parameters (mpmath) are computed once
    outside the timed runs, as the GPU's are at plan creation."""
    import numpy as np
    import oracle
    from oracle import poisson3d as P3
    threads = oracle.threads(0)
    h = 1.0 / (n_sample + 1)
    modes = P3.plan(n_sample, n_sample, n_sample, h, h, h, d["eps"])
    F = np.random.default_rng(1).standard_normal((n_sample, n_sample, n_sample))
    times = []
    t_budget = time.perf_counter()
    while len(times) < 10 and (time.perf_counter() - t_budget < budget_s or len(times) < 2):
        t0 = time.perf_counter()
        P3.solve(F, h, h, h, eps=d["eps"], modes=modes)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    return {"value": n_sample ** 3 / med, "unit": "unknowns/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the same problem on a {n_sample}^3 grid (the oracle's explicit sine "
                      f"transform costs O(N^4): the full grid would take many minutes), numpy + "
                      f"the C Thomas oracle, {threads} thread(s), median of {len(times)} runs "
                      f"of {med:.3f} s, ADI parameters computed once outside the runs"}


def cpu_leg_poisson(d, budget_s=12.0, n_sample=2048):
    """The oracle (explicit sine transforms, Thomas per mode) on a smaller
    grid of the same problem: at the full size its O(N^3) transforms take
    minutes."""
    import numpy as np
    import oracle
    from oracle import poisson2d as P2
    threads = oracle.threads(0)
    h = 1.0 / (n_sample + 1)
    F = np.random.default_rng(1).standard_normal((n_sample, n_sample))
    times = []
    t_budget = time.perf_counter()
    while len(times) < 10 and (time.perf_counter() - t_budget < budget_s or len(times) < 2):
        t0 = time.perf_counter()
        P2.solve(F, h, h)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    return {"value": n_sample * n_sample / med, "unit": "unknowns/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the same problem on a {n_sample}x{n_sample} grid (the oracle's explicit "
                      f"sine transforms cost O(N^3): the full grid would take minutes), "
                      f"numpy + the C Thomas oracle, {threads} thread(s), median of "
                      f"{len(times)} runs of {med:.3f} s"}


def cpu_leg(d, budget_s=12.0):
    """Time the oracle on this host (same inputs) and return its outputs."""
    import numpy as np
    import oracle
    single = d["kind"] in ("series", "general") and d["M"] == 1
    nthreads = 1 if single else 0
    threads = oracle.threads(1 if single else 0)
    times, Xo, gFo, gto = [], None, None, None
    t_budget = time.perf_counter()
    while len(times) < 25 and (time.perf_counter() - t_budget < budget_s or len(times) < 3):
        t0 = time.perf_counter()
        if d["kind"] == "general":
            Xo = oracle.solve_general(d["F"], d["a"], d["b"], d["c"], nthreads=nthreads)
        elif d["kind"] == "series":
            Xo = oracle.solve(d["F"], d["t_m1"], d["t_0"], d["t_1"], nthreads=nthreads)
        else:
            Xo = oracle.solve_varlen(d["F"].reshape(-1), d["offsets"], d["t_m1"], d["t_0"],
                                     d["t_1"], nthreads=nthreads, psi=d.get("psi"),
                                     chi=d.get("chi"))
        if d.get("adjoint"):
            gFo, gto = oracle.adjoint_varlen(d["W"].reshape(-1), Xo, d["offsets"], d["t_m1"],
                                             d["t_0"], d["t_1"], nthreads=nthreads)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    what = "forward solve + adjoint" if d.get("adjoint") else "solve"
    cpu = {"value": d["units"] / med, "unit": "unknowns/s", "cores": threads, "kind": "oracle",
           "sample": f"the whole workload ({d['units']} unknowns, {what}), plain Thomas in "
                     f"double, {threads} thread(s), median of {len(times)} runs of {med:.3f} s"}
    return cpu, np.asarray(Xo).reshape(-1), gFo, gto


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="single_large", choices=WORKLOADS)
    ap.add_argument("--n", type=int, default=1 << 26, help="single_large: system order")
    ap.add_argument("--modes", default=None,
                    help="paths to time, first = headline (default f32_refine,f64; "
                         "f64,f32 for the general workload)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain device copy of F (counter calibration)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default launch options instead of the autotuner's choice")
    ap.add_argument("--shape", type=int, default=None,
                    help="fixed work shape (no autotuning; with --whole and --wg)")
    ap.add_argument("--whole", type=int, default=None,
                    help="fixed whole-system threshold of varlen plans (no autotuning)")
    ap.add_argument("--wg", type=int, default=None,
                    help="fixed cap of workgroups per CU (no autotuning)")
    ap.add_argument("--fixed", action="append", default=[], metavar="MODE:SHAPE,WHOLE,WG",
                    help="fixed launch options of one path (no autotuning for it), e.g. "
                         "f32_refine:2,0,0; repeatable, overrides --shape/--whole/--wg")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(one GPU's share of a sharded solve is what is measured here)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1002_2469_amd as tdt

    d = load_workload(args.workload, args)
    F = torch.from_numpy(np.ascontiguousarray(d["F"]).reshape(-1)).to("cuda:0")
    X = torch.empty_like(F)
    torch.cuda.synchronize()
    if args.modes is None:
        args.modes = {"general": "f64,f32", "poisson2d": "f64",
                      "poisson3d": "f64"}.get(args.workload, "f32_refine,f64")
    modes = [m for m in args.modes.split(",") if m]
    res = {}
    for mode in modes:
        Fm = F.float() if mode == "f32" else F      # plain float takes float data
        Xm = torch.empty_like(Fm) if mode == "f32" else X
        if d["kind"] == "poisson":
            res[mode] = run_poisson(tdt, d, F, mode, args.steps, args.warmup, torch)
        elif d["kind"] == "poisson3d":
            if mode != "f64":
                raise SystemExit("poisson3d runs the f64 path only")
            res[mode] = run_poisson3d(tdt, d, F, args.steps, args.warmup, torch)
        else:
            fixed = {k: v for k, v in (("shape", args.shape), ("whole_max_tiles", args.whole),
                                       ("wg_per_cu", args.wg)) if v is not None}
            for spec in args.fixed:
                m, _, vals = spec.partition(":")
                if m == mode:
                    fixed = dict(zip(("shape", "whole_max_tiles", "wg_per_cu"),
                                     (int(v) for v in vals.split(","))))
            opts = fixed if (fixed or args.no_autotune) else None
            res[mode] = run_mode(tdt, d, Fm, Xm, mode, args.steps, args.warmup, torch, opts=opts)
        print(f"[bench] {args.workload} {mode}: {res[mode]['ms']:.4f} ms/step  kernels(ms) "
              f"{json.dumps({k: round(v, 5) for k, v in res[mode]['kernels_ms'].items()})}",
              file=sys.stderr, flush=True)

    if args.copy_calib:
        Y = torch.empty_like(F)
        for _ in range(5):
            Y.copy_(F)
        torch.cuda.synchronize()
        del Y

    U = d["units"]
    head = modes[0]
    from paper_1002_2469_amd import _lib
    shape = (res[head]["tuned"] or {}).get("shape", 0)
    if d["kind"] in ("poisson", "poisson3d"):
        n_first, n_final = 0, U
    else:
        n_first, n_final = tile_counts(d, _lib.SHAPES[shape][0] * _lib.SHAPES[shape][1])
    # algorithmic HBM bytes per launch of each kernel group (double data);
    # the transforms read and write every unknown once (16 B), the 2D line
    # solve in tiles (columns of more than 1024 rows) reads them twice and
    # writes them once (24 B), in one column 16 B
    line_bytes = (24.0 if d.get("ny", 0) > 1024 else 16.0) * U
    # a series plan whose Green rows decay reads only their supports per tile
    # in the first pass (tdt_plan_green_support)
    kf, kl = res[head].get("green_support", (0, 0))
    if kf + kl > 0 and n_first > 0:
        tile = _lib.SHAPES[shape][0] * _lib.SHAPES[shape][1]
        n_first = (n_first // tile) * (kf + kl)
    per_launch = {"first_pass": 8.0 * n_first, "final_pass": 16.0 * n_final,
                  "bwd_first_pass": 8.0 * n_first, "bwd_final_pass": 24.0 * n_final,
                  "line_solve": line_bytes if d["kind"] == "poisson" else 0.0,
                  "forward_transform": 16.0 * U if d["kind"] in ("poisson", "poisson3d") else 0.0,
                  "inverse_transform": 16.0 * U if d["kind"] in ("poisson", "poisson3d") else 0.0,
                  "adi": adi_bytes(d, res[head]["counts"]) if d["kind"] == "poisson3d" else 0.0}
    # plans whose multi-tile systems have at most 64 tiles and no corner rows
    # run the interface pass inside the final pass (no launch of its own)
    inline_itf = False
    if d["kind"] in ("series", "varlen") and "psi" not in d:
        tile = _lib.SHAPES[shape][0] * _lib.SHAPES[shape][1]
        o = [int(x) for x in d["offsets"]] if d["kind"] == "varlen" else []
        nmax = d["N"] if d["kind"] == "series" else max(b - a for a, b in zip(o, o[1:]))
        inline_itf = tile < nmax <= 64 * tile
    itf = ", interface pass inline" if inline_itf else ""
    # a small series of whole tiles with short supports is solved by the
    # final pass alone (at most 256 tiles in all and four per wavefront of a
    # workgroup): the summaries' rows are read there
    if d["kind"] == "series" and 0 < kf + kl <= 256 and n_first > 0:
        tile = _lib.SHAPES[shape][0] * _lib.SHAPES[shape][1]
        tiles = d["N"] // tile
        if (d["N"] % tile == 0 and tiles <= 4 * (_lib.SHAPES[shape][1] // 64)
                and d["M"] * tiles <= 256):
            per_launch["final_pass"] += per_launch["first_pass"]
            per_launch["first_pass"] = 0.0
            itf = ", tile summaries and interface pass inline: one launch"
    names = {"first_pass": (f"k_beta_ends<double> (tile summaries from the Green rows' "
                            f"supports, {kf} + {kl} rows per tile)" if kf + kl > 0 else
                            "k_beta<double> (Green-row tile summaries, first pass)"
                            if d["kind"] == "series" else
                            "k_gtile<double, SUMMARY> (general matrix, tile summaries)"
                            if d["kind"] == "general" else
                            "k_tile<double, *, SUMMARY> (tile summaries, first pass)"),
             "final_pass": ("k_gtile<double, final> (general matrix: solve and store)"
                            if d["kind"] == "general" else
                            f"k_tile<double, float, REFINE, final> (solve, refine and store{itf})"
                            if head == "f32_refine" else
                            f"k_tile<double, double, final> (solve and store{itf})"),
             "forward_transform": "k_dst_rows<N2> (the sine transform of every row: fold, "
                                  "complex FFT in LDS, real split, prefix sum)",
             "inverse_transform": "k_dst_rows<N2> (the inverse sine transform of every row)",
             "line_solve": "k_strided in tiles (the mode line systems in place down the "
                           "columns: end-value pass, interface, re-solve; summed)",
             "adi": "k_strided<double> with the ADI epilogue (all 2 J_1 half-steps of one "
                    "solve: bytes and time summed over them)",
             "bwd_first_pass": "k_tile<double, *, SUMMARY> on T^T (adjoint first pass)",
             "bwd_final_pass": f"k_tile<..., BWD> (adjoint solve, store gF, dL/dt partial sums{itf})"}

    cpu = None
    errs = {}
    if not args.no_cpu and d["kind"] == "poisson":
        from oracle import poisson2d as P2
        cpu = cpu_leg_poisson(d)
        for mode in modes:
            Um = res[mode]["X"].reshape(d["ny"], d["nx"])
            r = P2.laplacian(Um, d["hx"], d["hy"]) - d["F"]
            errs[mode] = {"residual": float(np.max(np.abs(r)) / np.max(np.abs(d["F"])))}
    elif not args.no_cpu and d["kind"] == "poisson3d":
        from oracle import poisson3d as P3
        cpu = cpu_leg_poisson3d(d)
        for mode in modes:
            Um = res[mode]["X"].reshape(d["nz"], d["ny"], d["nx"])
            r = P3.laplacian(Um, d["hx"], d["hy"], d["hz"]) - d["F"]
            errs[mode] = {"residual": float(np.max(np.abs(r)) / np.max(np.abs(d["F"]))),
                          "residual_2norm": float(np.linalg.norm(r) / np.linalg.norm(d["F"]))}
            del r, Um
    elif not args.no_cpu:
        cpu, Xo, gFo, gto = cpu_leg(d)
        import oracle
        for mode in modes:
            if d["kind"] in ("series", "general"):
                e = float(np.max(oracle.rel_err_rows(res[mode]["X"].reshape(d["M"], d["N"]),
                                                     Xo.reshape(d["M"], d["N"]))))
            else:
                e = float(np.max(oracle.rel_err_rows(res[mode]["X"], Xo, d["offsets"])))
            errs[mode] = {"X": e}
            if gFo is not None:
                errs[mode]["gF"] = float(np.max(oracle.rel_err_rows(res[mode]["gF"], gFo,
                                                                    d["offsets"])))
                errs[mode]["gt"] = float(np.max(np.abs(res[mode]["gt"] - gto))
                                         / np.max(np.abs(gto)))

    def err_of(mode):
        e = errs.get(mode)
        if e is None:
            return None
        return e["X"] if len(e) == 1 and "X" in e else e

    def path_record(mode):
        r = res[mode]
        return {"value": U / (r["ms"] * 1e-3), "unit": "unknowns/s", "ms_per_step": r["ms"],
                "stage1_ms": r.get("stage1_ms"),
                "kernels_ms": {k: round(v, 6) for k, v in r["kernels_ms"].items()},
                "rel_err_vs_oracle": err_of(mode), "refine_iters": r["refine_iters"],
                "tuned": r["tuned"], "steps_run": r["solves"]}

    hk = res[head]["kernels_ms"]
    dom = max((k for k in per_launch if hk.get(k, 0) > 0 and per_launch[k] > 0),
              key=lambda k: hk[k])
    achieved = per_launch[dom] / (hk[dom] * 1e-3) / 1e9
    traffic = committed_traffic(args.workload, dom, head)
    line = {
        "metric": METRIC,
        "value": U / (res[head]["ms"] * 1e-3),
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res[head]["ms"],
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32 sweeps + f64 residual/update" if head == "f32_refine" else head,
        "data": "synthetic (seeded right-hand sides; no dataset involved)",
        "config": {"workload": d["desc"], "unknowns": U, "path": head},
        "rel_err_vs_oracle": err_of(head),
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": per_launch[dom], "avg_ms": hk[dom]},
        "paths": {m: path_record(m) for m in modes},
        "cpu_baseline": cpu,
    }
    if cpu is not None:
        cpu["host_cores"] = len(os.sched_getaffinity(0))
    # the paper's Stage 1 (preliminary step) beside Stage 2 (the solve)
    line["stage1_ms"] = res[head].get("stage1_ms")
    line["first_pass_bytes_per_launch"] = per_launch["first_pass"]
    if "f64" in res and head != "f64":
        line["speedup_vs_f64"] = res["f64"]["ms"] / res[head]["ms"]
    if d["kind"] == "poisson3d":
        c = np.asarray(res[head]["counts"])
        line["adi_schedule"] = {"iterations_mode_1": int(c[0]), "iterations_last_mode": int(c[-1]),
                                "mean_iterations": float(c.mean()),
                                "half_step_launches": 2 * int(c.max())}
    line["kernel_source_sha"] = kernel_source_hash(args.workload)
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
