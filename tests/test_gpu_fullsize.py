"""Full-size parity of the two batched workloads in the form they are timed:

* the separation-of-variables batch (2048 systems, sizes log-uniform in
  [256, 65536], each with its own t_0 from the sin^2 mode shift of Sec. 3.2),
  float sweeps with double refinement, solved by a launch sequence captured
  once in a hipGraph and replayed on new right-hand sides, every system
  checked against the double oracle and the long double oracle;
* the differentiable batch (1024 systems of 16384 with their own t's): the
  float-plus-refinement forward solve and the adjoint (gF and the three
  t-gradients of every system) against the oracle's adjoint, and the
  t-gradients of two systems against central finite differences (absolute
  step 1e-6) of the loss sum(W X) computed by the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host, tol_f64
from paper_1002_2469_amd import workloads as W

pytestmark = pytest.mark.gpu


def _tdt():
    import paper_1002_2469_amd as tdt
    return tdt


@pytest.mark.parametrize("dtype", ["f32_refine", "f64"])
def test_sov_batch_graph_replay_full_size(dtype):
    import torch
    tdt = _tdt()
    d = W.sov_batch(0)
    off = d["offsets"]
    sizes = np.diff(off)
    S = d["S"]
    print(f"[case] sov batch graph replay dtype={dtype} S={S} sum N={int(off[-1])}", flush=True)
    plan = tdt.VarlenPlan(off, d["t_m1"], d["t_0"], d["t_1"], dtype)
    plan.reserve(1)
    Fd = to_dev(d["F"])
    Xd = torch.empty_like(Fd)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.solve(Fd, Xd)                         # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.solve(Fd, Xd)
    tols = np.array([tol_f64(1.0, d["t_0"][k], 1.0, int(sizes[k])) for k in range(S)])
    rng = np.random.default_rng(100)
    for rep in range(3):
        Fh = d["F"] if rep == 0 else rng.standard_normal(int(off[-1]))
        Fd.copy_(torch.from_numpy(Fh))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        X = to_host(Xd)
        for prec in ("f64", "ld"):
            ref = oracle.solve_varlen(Fh, off, d["t_m1"], d["t_0"], d["t_1"], precision=prec)
            errs = oracle.rel_err_rows(X, ref, off)
            bad = np.nonzero(errs > tols)[0]
            assert bad.size == 0, (rep, prec, [(int(k), int(sizes[k]), errs[k], tols[k])
                                               for k in bad[:5]])
        _ = (Xd * 2).sum().item()                  # eager work between replays
    del g
    plan.close()


@pytest.mark.parametrize("dtype", ["f32_refine", "f64"])
def test_diff_batch_adjoint_full_size(dtype):
    tdt = _tdt()
    d = W.diff_batch(0)                            # 1024 systems of 16384
    off = d["offsets"]
    F, Wt = d["F"].reshape(-1), d["W"].reshape(-1)
    print(f"[case] diff batch adjoint dtype={dtype} S={d['S']}", flush=True)
    plan = tdt.VarlenPlan(off, d["t_m1"], d["t_0"], d["t_1"], dtype)
    Xd = plan.solve(to_dev(F))
    gF, gt = plan.backward(to_dev(Wt), Xd)
    X = oracle.solve_varlen(F, off, d["t_m1"], d["t_0"], d["t_1"])
    gFr, gtr = oracle.adjoint_varlen(Wt, X, off, d["t_m1"], d["t_0"], d["t_1"])
    assert oracle.rel_err_rows(to_host(Xd), X, off).max() <= 1e-12
    assert oracle.rel_err_rows(to_host(gF), gFr, off).max() <= 1e-12
    gt = to_host(gt)
    assert np.max(np.abs(gt - gtr) / np.maximum(1.0, np.abs(gtr))) <= 1e-11
    # central differences of L_s(t) = W_s . T(t)^{-1} F_s for two systems
    N, h = d["N"], 1e-6
    for s in (0, 777):
        Fs, Ws = d["F"][s], d["W"][s]
        t = np.array([d["t_m1"][s], d["t_0"][s], d["t_1"][s]])

        def loss(tt):
            return float(Ws @ oracle.solve(Fs, tt[0], tt[1], tt[2]))

        fd = np.empty(3)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd[k] = (loss(t + e) - loss(t - e)) / (2 * h)
        assert np.max(np.abs(gt[s] - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd))), (s, gt[s], fd)
    assert N == 16384
    plan.close()
