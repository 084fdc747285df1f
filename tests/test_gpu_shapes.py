"""GPU parity of every compiled work shape (rows per lane x lanes per
workgroup, TDT_OPT_SHAPE) against the CPU oracle: sizes around each shape's
block and tile boundaries, batches on both varlen paths, the adjoint, and the
single large system whose tile count selects each interface-pass variant."""
import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host, tol_f32, tol_f64
from paper_1002_2469_amd import _lib
from paper_1002_2469_amd import workloads as W

pytestmark = pytest.mark.gpu
SHAPES = list(range(len(_lib.SHAPES)))


def _tdt():
    import paper_1002_2469_amd as tdt
    return tdt


def _sizes(shape):
    B, NT = _lib.SHAPES[shape]
    L = B * NT
    return [1, B - 1, B, B + 1, 64 * B + 3, L - 1, L, L + 1, 3 * L + 5, 33 * L + 17]


@pytest.mark.parametrize("dtype", ["f64", "f32_refine", "f32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_shape_sizes(shape, dtype):
    tdt = _tdt()
    rng = np.random.default_rng(100 + shape)
    for n in _sizes(shape):
        M = 2
        a, b, c = W.random_system(rng, 1.25 if dtype == "f32" else 1.0, 3.0)
        F = rng.standard_normal((M, n))
        print(f"[case] shape={shape} n={n} dtype={dtype}", flush=True)
        plan = tdt.Plan(a, b, c, n, dtype)
        plan.set_option("shape", shape)
        assert plan.get_option("shape") == shape
        X = to_host(plan.solve(to_dev(F, dtype)))
        Fr = F.astype(np.float32).astype(np.float64) if dtype == "f32" else F
        ref = oracle.solve(Fr, a, b, c)
        err = oracle.rel_err_rows(X, ref).max()
        tol = tol_f32(a, b, c, n) if dtype == "f32" else tol_f64(a, b, c, n)
        assert err <= tol, (shape, n, dtype, err)


@pytest.mark.parametrize("whole", [0, 16])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
@pytest.mark.parametrize("shape", SHAPES)
def test_shape_varlen(shape, dtype, whole):
    tdt = _tdt()
    print(f"[case] shape={shape} varlen dtype={dtype} whole={whole}", flush=True)
    rng = np.random.default_rng(7)
    sizes = np.array([1, 2, 3, 33, 4096, 4097, 8192, 8193, 65, 20000, 5, 16384, 100000])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    ts = [W.random_system(rng, 1.0, 3.0) for _ in sizes]
    tm1, t0, t1 = (np.array([t[k] for t in ts]) for k in range(3))
    F = rng.standard_normal(int(off[-1]))
    plan = tdt.VarlenPlan(off, tm1, t0, t1, dtype)
    plan.reserve(1)
    plan.set_option("whole_max_tiles", whole)
    plan.set_option("shape", shape)
    assert plan.get_option("whole_max_tiles") == whole     # options survive the rebuild
    X = to_host(plan.solve(to_dev(F)))
    ref = oracle.solve_varlen(F, off, tm1, t0, t1)
    errs = oracle.rel_err_rows(X, ref, off)
    tols = np.array([tol_f64(tm1[s], t0[s], t1[s], int(sizes[s])) for s in range(len(sizes))])
    assert np.all(errs <= tols), errs
    # adjoint on the same plan
    G = rng.standard_normal(int(off[-1]))
    gF, gt = plan.backward(to_dev(G), to_dev(X))
    gFr, gtr = oracle.adjoint_varlen(G, ref, off, tm1, t0, t1)
    assert oracle.rel_err_rows(to_host(gF), gFr, off).max() <= 1e-11
    assert np.max(np.abs(to_host(gt) - gtr) / np.maximum(1.0, np.abs(gtr))) <= 1e-10


@pytest.mark.parametrize("shape", [1, 2])
def test_shape_single_large(shape):
    """N = 2^26 with tiles of 4096 rows: 16384 tiles, the largest the
    chunked interface pass of a series plan takes (256 chunks of 64 tiles)."""
    tdt = _tdt()
    d = W.single_large(0)
    print(f"[case] shape={shape} single_large", flush=True)
    plan = tdt.Plan(d["t_m1"], d["t_0"], d["t_1"], d["N"], "f32_refine")
    plan.set_option("shape", shape)
    X = to_host(plan.solve(to_dev(d["F"])))
    ref = oracle.solve(d["F"], d["t_m1"], d["t_0"], d["t_1"])
    assert oracle.rel_err(X, ref) <= 1e-12


def test_shape_beyond_affine_interface():
    """More than 16384 tiles (tiles of 4096 rows) uses the segment-merge
    interface kernel."""
    tdt = _tdt()
    n = 16385 * 4096 + 7
    rng = np.random.default_rng(77)
    a, b, c = W.random_system(rng, 1.05, 2.0)
    F = rng.standard_normal(n)
    print(f"[case] shape=1 n={n} segment-merge interface", flush=True)
    plan = tdt.Plan(a, b, c, n, "f64")
    plan.set_option("shape", 1)
    X = to_host(plan.solve(to_dev(F)))
    assert oracle.rel_err(X, oracle.solve(F, a, b, c)) <= tol_f64(a, b, c, n)


def test_shape_graph_capture_after_rebuild():
    """A reserved plan stays allocation-free across a change of shape."""
    import torch
    tdt = _tdt()
    rng = np.random.default_rng(12)
    sizes = np.array([300, 9000, 17, 20000])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    t0 = rng.uniform(2.5, 4.0, 4)
    plan = tdt.VarlenPlan(off, -1.0, t0, -0.9, "f32_refine")
    plan.reserve(1)
    plan.set_option("whole_max_tiles", 0)
    plan.set_option("shape", 2)
    Fd = to_dev(rng.standard_normal(int(off[-1])))
    Xd = torch.empty_like(Fd)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.solve(Fd, Xd)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.solve(Fd, Xd)
    for k in range(3):
        Fh = rng.standard_normal(int(off[-1]))
        Fd.copy_(torch.from_numpy(Fh))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = oracle.solve_varlen(Fh, off, -1.0, t0, -0.9)
        assert oracle.rel_err_rows(to_host(Xd), ref, off).max() <= 1e-12, k
        _ = (Xd * 2).sum().item()
