"""GPU parity of general (per-row) tridiagonal matrices against the CPU
oracle, through the C ABI: series of right-hand sides over sizes from one row
to many tiles (tiles of 4096 rows; every variant of the interface pass
across tiles), float and double, constant rows against the Toeplitz plan,
and the adjoint with the per-entry gradients.

Inputs: rows with dominance ratio |b_i| / (|a_i| + |c_i|) in [1.2, 3]
(in [1.25, 3] for plain float), entries of both signs, and the
variable-coefficient diffusion-reaction rows of the benchmark workload."""
import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host
from oracle_pins import random_rows
from paper_1002_2469_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}
L = 4096   # rows per tile of a general plan


def _tdt():
    import paper_1002_2469_amd as tdt
    return tdt


def _f32_round(F, dtype):
    return F.astype(np.float32).astype(np.float64) if dtype == "f32" else F


SIZES = [1, 2, 7, 8, 9, 63, 64, 65, 4095, 4096, 4097, 3 * L + 5, 20 * L + 3]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_general_sizes(n, dtype):
    tdt = _tdt()
    rng = np.random.default_rng(2000 + n)
    for M in (1, 3):
        a, b, c = random_rows(rng, n, 1.25 if dtype == "f32" else 1.2, 3.0)
        F = rng.standard_normal((M, n))
        print(f"[case] general n={n} M={M} dtype={dtype}", flush=True)
        plan = tdt.GeneralPlan(a, b, c, dtype)
        X = to_host(plan.solve(to_dev(F, dtype)))
        ref = oracle.solve_general(_f32_round(F, dtype), a, b, c)
        err = oracle.rel_err_rows(X, ref).max()
        assert err <= TOL[dtype], (n, M, dtype, err)


@pytest.mark.parametrize("tiles,extra", [(257, 0), (2049, 9), (8193, 1)])
def test_general_many_tiles(tiles, extra):
    """The interface variants up to 256, 2048, 8192 and 16384 tiles."""
    tdt = _tdt()
    n = (tiles - 1) * L + (extra if extra else L)
    rng = np.random.default_rng(tiles)
    a, b, c = W.general_rows(rng, n)
    F = rng.standard_normal(n)
    print(f"[case] general tiles={tiles} n={n}", flush=True)
    X = to_host(tdt.GeneralPlan(a, b, c, "f64").solve(to_dev(F)))
    assert oracle.rel_err(X, oracle.solve_general(F, a, b, c)) <= 1e-12


@pytest.mark.parametrize("M", [1, 5])
def test_general_truncated_first_pass(M):
    """Whole tiles of dominant rows: the first pass reads only the supports
    of the tiles' own Green rows (multiples of 64 rows from each end,
    together under a quarter of the tile), forward and adjoint; the solve and
    the adjoint against the oracle, and a float plan's solve.  Rows of weak dominance
    (ratio 1.0002: the rows decay over thousands of entries) keep whole
    tiles, and so does a size with a ragged last tile."""
    tdt = _tdt()
    rng = np.random.default_rng(77 + M)
    n = 6 * L
    a, b, c = random_rows(rng, n, 1.2, 3.0)
    F = rng.standard_normal((M, n))
    G = rng.standard_normal((M, n))
    print(f"[case] general truncated first pass M={M}", flush=True)
    plan = tdt.GeneralPlan(a, b, c, "f64")
    sup = plan.green_support()
    for kf, kl in (sup["forward"], sup["adjoint"]):
        assert kf > 0 and kl > 0 and kf % 64 == 0 and kl % 64 == 0 and 4 * (kf + kl) <= L, sup
    X = plan.solve(to_dev(F))
    Xr = oracle.solve_general(F, a, b, c)
    assert oracle.rel_err_rows(to_host(X), Xr).max() <= 1e-12
    gF, g = plan.backward(to_dev(G), X)
    gFr, (ga, gb, gc) = oracle.adjoint_general(G, Xr, a, b, c)
    assert oracle.rel_err_rows(to_host(gF), gFr).max() <= 1e-12
    ref = np.stack([ga, gb, gc])
    assert np.max(np.abs(to_host(g) - ref)) <= 1e-11 * np.max(np.abs(ref))
    plan.close()
    # a float plan reads the same supports (its rows are computed in double)
    plan = tdt.GeneralPlan(a, b, c, "f32")
    assert plan.green_support() == sup
    X = to_host(plan.solve(to_dev(F, "f32")))
    assert oracle.rel_err_rows(X, oracle.solve_general(_f32_round(F, "f32"), a, b, c)).max() <= TOL["f32"]
    plan.close()
    assert tdt.GeneralPlan(a[:n - 5], b[:n - 5], c[:n - 5], "f64").green_support() == \
        dict(forward=(0, 0), adjoint=(0, 0))
    a, b, c = W.general_rows(rng, n, 1.0002, 1.0002)
    assert tdt.GeneralPlan(a, b, c, "f64").green_support() == dict(forward=(0, 0), adjoint=(0, 0))


@pytest.mark.slow
def test_general_segment_merge_interface():
    """More than 16384 tiles: the segment-merge interface pass."""
    tdt = _tdt()
    n = 16384 * L + 77
    rng = np.random.default_rng(16385)
    a, b, c = W.general_rows(rng, n)
    F = rng.standard_normal(n)
    print(f"[case] general segment-merge n={n}", flush=True)
    X = to_host(tdt.GeneralPlan(a, b, c, "f64").solve(to_dev(F)))
    assert oracle.rel_err(X, oracle.solve_general(F, a, b, c)) <= 1e-12


def test_general_constant_rows_match_toeplitz():
    tdt = _tdt()
    rng = np.random.default_rng(4)
    n = 5 * L + 100
    a, b, c = W.random_system(rng, 1.2, 3.0)
    F = rng.standard_normal((2, n))
    print(f"[case] general constant rows n={n}", flush=True)
    Xg = to_host(tdt.GeneralPlan(np.full(n, a), np.full(n, b), np.full(n, c)).solve(to_dev(F)))
    Xt = to_host(tdt.Plan(a, b, c, n, "f64").solve(to_dev(F)))
    ref = oracle.solve(F, a, b, c)
    assert oracle.rel_err(Xg, ref) <= 1e-12
    assert oracle.rel_err(Xg, Xt) <= 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_general_series_config(dtype):
    """The benchmark workload: 64 right-hand sides of N = 2^20 (256 tiles)."""
    tdt = _tdt()
    d = W.general_series(0)
    print(f"[case] general series config dtype={dtype}", flush=True)
    plan = tdt.GeneralPlan(d["a"], d["b"], d["c"], dtype)
    X = to_host(plan.solve(to_dev(d["F"], dtype)))
    ref = oracle.solve_general(_f32_round(d["F"], dtype), d["a"], d["b"], d["c"])
    err = oracle.rel_err_rows(X, ref).max()
    assert err <= (1e-4 if dtype == "f32" else 1e-12), err


@pytest.mark.parametrize("n", [1, 9, 3 * L + 5])
def test_general_adjoint(n):
    tdt = _tdt()
    rng = np.random.default_rng(31 + n)
    a, b, c = random_rows(rng, n, 1.2, 3.0)
    F = rng.standard_normal((3, n))
    G = rng.standard_normal((3, n))
    print(f"[case] general adjoint n={n}", flush=True)
    plan = tdt.GeneralPlan(a, b, c, "f64")
    X = plan.solve(to_dev(F))
    gF, g = plan.backward(to_dev(G), X)
    Xr = oracle.solve_general(F, a, b, c)
    gFr, (ga, gb, gc) = oracle.adjoint_general(G, Xr, a, b, c)
    assert oracle.rel_err(to_host(gF), gFr) <= 1e-12
    gh = to_host(g)
    ref = np.stack([ga, gb, gc])
    assert np.max(np.abs(gh - ref)) <= 1e-11 * np.max(np.abs(ref)), np.max(np.abs(gh - ref))


def test_general_options_and_autotune(tmp_path, monkeypatch):
    tdt = _tdt()
    from paper_1002_2469_amd import _lib
    monkeypatch.setenv("TDT_TUNE_CACHE", str(tmp_path / "tune.json"))
    rng = np.random.default_rng(8)
    n = 7 * L + 11
    a, b, c = random_rows(rng, n, 1.2, 3.0)
    F = to_dev(rng.standard_normal((2, n)))
    print("[case] general options", flush=True)
    plan = tdt.GeneralPlan(a, b, c, "f64")
    assert plan.get_option("shape") == 1
    with pytest.raises(_lib.TDTError):
        plan.set_option("shape", 0)
    with pytest.raises(_lib.TDTError):
        plan.set_option("whole_max_tiles", 4)
    choice = plan.autotune(F, cache=False)
    assert choice["shape"] == 1
    X = to_host(plan.solve(F))
    assert oracle.rel_err(X, oracle.solve_general(to_host(F), a, b, c)) <= 1e-12
    info = plan.info()
    assert info["dominance"] >= 1.2 - 1e-12
    with pytest.raises(ValueError):
        tdt.GeneralPlan(a, b, c, "f32_refine")


def test_general_repeatable_and_graph():
    """Bitwise repeatable solves, and a captured solve replayed from a
    hipGraph (after tdt_plan_reserve) matches the eager one on every replay."""
    import torch
    tdt = _tdt()
    rng = np.random.default_rng(9)
    n = 4 * L + 3
    a, b, c = random_rows(rng, n, 1.2, 3.0)
    F = to_dev(rng.standard_normal((3, n)))
    print("[case] general repeatable/graph", flush=True)
    plan = tdt.GeneralPlan(a, b, c, "f64")
    plan.reserve(3)
    X1 = to_host(plan.solve(F))
    X2 = to_host(plan.solve(F))
    assert np.array_equal(X1, X2)
    X = torch.empty_like(F)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.solve(F, X)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.solve(F, X)
    for _ in range(3):
        X.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(X), X1)
