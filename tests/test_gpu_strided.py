"""GPU parity of the strided batch solve (systems along a slow axis: unknown
i of system s of batch b at b*ldb + i*ld + s) against the CPU oracle,
through the C ABI: orders 1 to 1024 (every block count, full and ragged last
blocks), one to hundreds of adjacent systems with their own matrices, both
batch layouts, padded rows, in place (orders up to 1024 are one column per
workgroup, 33 to 64 blocks in the widest kernel); longer systems in tiles
of 512 rows (a last tile of 1 to 512 rows, up to 8191 rows, weakly dominant
classes); plus errors, bitwise repeatability and hipGraph replay, with and
without a reservation.

Inputs: F ~ N(0, 1); classes with t_0 ~ U[2.5, 4], t_+-1 ~ U[-1, -0.5]
independently (dominance >= 1.25), and the weakly dominant line operators
of an ADI half-step, tridiag{-1, 2 + s, -1} with s down to 1e-5."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import U64, kappa2, to_dev, to_host

pytestmark = pytest.mark.gpu


def _tdt():
    import paper_1002_2469_amd as tdt
    return tdt


def classes(rng, P, kind="dominant"):
    if kind == "dominant":
        return (rng.uniform(-1.0, -0.5, P), rng.uniform(2.5, 4.0, P), rng.uniform(-1.0, -0.5, P))
    # ADI-like: -1, 2 + s, -1 with s log-uniform in [1e-5, 4]
    s = np.exp(rng.uniform(math.log(1e-5), math.log(4.0), P))
    return -np.ones(P), 2.0 + s, -np.ones(P)


def oracle_strided(F, N, M, ld, nb, ldb, tm1, t0, t1):
    """Gather every (b, s) system, solve it with the oracle, scatter back."""
    flat = F.reshape(-1)
    idx = (np.arange(nb)[:, None, None] * ldb + np.arange(N)[None, :, None] * ld +
           np.arange(M)[None, None, :])                      # [nb][N][M]
    sysF = np.ascontiguousarray(flat[idx].transpose(0, 2, 1)).reshape(-1)   # [nb][M][N]
    off = np.arange(nb * M + 1, dtype=np.int64) * N
    X = oracle.solve_varlen(sysF, off, np.tile(tm1[:M], nb), np.tile(t0[:M], nb),
                            np.tile(t1[:M], nb))
    out = np.full_like(flat, np.nan)
    out[idx] = X.reshape(nb, M, N).transpose(0, 2, 1)
    return out, idx


def check(X, ref, idx, N, M, nb, tm1, t0, t1):
    """Per-system normwise relative error against the oracle, each system to
    max(1e-12, 8 u cond2)."""
    Xs = X.reshape(-1)[idx].transpose(0, 2, 1).reshape(nb * M, N)
    Rs = ref[idx].transpose(0, 2, 1).reshape(nb * M, N)
    err = np.max(np.abs(Xs - Rs), axis=1) / np.maximum(np.max(np.abs(Rs), axis=1), 1e-300)
    tol = np.array([max(1e-12, 8 * U64 * kappa2(tm1[s], t0[s], t1[s], N)) for s in range(M)])
    tol = np.tile(tol, nb)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (bad[:5], err[bad[:5]], tol[bad[:5]])


NS = [1, 2, 15, 16, 17, 31, 33, 100, 255, 256, 257, 511, 512, 513, 777, 1023, 1024]


@pytest.mark.parametrize("n", NS)
def test_strided_orders(n):
    tdt = _tdt()
    rng = np.random.default_rng(100 + n)
    P = 37
    tm1, t0, t1 = classes(rng, P)
    F = rng.standard_normal((n, P))
    print(f"[case] strided N={n} P={P}", flush=True)
    plan = tdt.StridedPlan(n, tm1, t0, t1)
    X = to_host(plan.solve(to_dev(F)))
    ref, idx = oracle_strided(F, n, P, P, 1, 0, tm1, t0, t1)
    check(X, ref, idx, n, P, 1, tm1, t0, t1)


@pytest.mark.parametrize("n,M,kind", [(64, 1, "dominant"), (64, 16, "adi"), (200, 17, "adi"),
                                      (511, 300, "adi"), (1023, 70, "adi"),
                                      (1024, 129, "dominant"), (9, 1000, "dominant")])
def test_strided_system_counts(n, M, kind):
    """M adjacent systems (groups of 16 to 256 per workgroup, ragged last
    group), M below the plan's class count, padded rows (ld > M)."""
    tdt = _tdt()
    rng = np.random.default_rng(n * 7 + M)
    P = M + 5
    tm1, t0, t1 = classes(rng, P, kind)
    ld = M + 3
    F = rng.standard_normal((n, ld))
    print(f"[case] strided N={n} M={M} {kind}", flush=True)
    plan = tdt.StridedPlan(n, tm1, t0, t1)
    Fd = to_dev(F)
    Xd = to_dev(np.full_like(F, 7.0))
    plan.solve(Fd, Xd, M=M, ld=ld, nb=1, ldb=0)
    X = to_host(Xd)
    ref, idx = oracle_strided(F, n, M, ld, 1, 0, tm1, t0, t1)
    check(X, ref, idx, n, M, 1, tm1, t0, t1)
    assert np.all(X[:, M:] == 7.0)          # padding untouched


@pytest.mark.parametrize("layout", ["outer", "inner"])
def test_strided_batches(layout):
    """nb batches one after another ([nb][N][M]) or interleaved in each row
    ([N][nb][M], the lines along z of a [Nz][Ny][Nx] array)."""
    tdt = _tdt()
    rng = np.random.default_rng(11 if layout == "outer" else 12)
    n, M, nb = 130, 45, 19
    tm1, t0, t1 = classes(rng, M, "adi")
    plan = tdt.StridedPlan(n, tm1, t0, t1)
    if layout == "outer":
        F = rng.standard_normal((nb, n, M))
        ld, ldb = M, n * M
    else:
        F = rng.standard_normal((n, nb, M))
        ld, ldb = nb * M, M
    print(f"[case] strided batches {layout}", flush=True)
    Xd = plan.solve(to_dev(F), M=M, ld=ld, nb=nb, ldb=ldb)
    ref, idx = oracle_strided(F, n, M, ld, nb, ldb, tm1, t0, t1)
    check(to_host(Xd), ref, idx, n, M, nb, tm1, t0, t1)


def test_strided_in_place_and_repeatable():
    tdt = _tdt()
    rng = np.random.default_rng(5)
    n, M = 700, 250
    tm1, t0, t1 = classes(rng, M, "adi")
    plan = tdt.StridedPlan(n, tm1, t0, t1)
    F = to_dev(rng.standard_normal((n, M)))
    print("[case] strided in place", flush=True)
    X1 = to_host(plan.solve(F))
    X2 = to_host(plan.solve(F))
    G = F.clone()
    plan.solve(G, G)
    assert np.array_equal(X1, X2)
    assert np.array_equal(X1, to_host(G))


TILED = [(1025, "dominant"), (1040, "adi"), (2048, "dominant"), (2049, "adi"),
         (3000, "adi"), (4097, "dominant"), (8191, "adi")]


@pytest.mark.parametrize("n,kind", TILED)
def test_strided_tiled_orders(n, kind):
    """Systems longer than one column: full tiles of 512 rows and a last
    tile of 1, 16, 512, 1, 440, 1 and 511 rows."""
    tdt = _tdt()
    rng = np.random.default_rng(300 + n)
    P = 37
    tm1, t0, t1 = classes(rng, P, kind)
    F = rng.standard_normal((n, P))
    print(f"[case] strided tiled N={n} P={P} {kind}", flush=True)
    plan = tdt.StridedPlan(n, tm1, t0, t1)
    X = to_host(plan.solve(to_dev(F)))
    ref, idx = oracle_strided(F, n, P, P, 1, 0, tm1, t0, t1)
    check(X, ref, idx, n, P, 1, tm1, t0, t1)


@pytest.mark.parametrize("layout", ["outer", "inner"])
def test_strided_tiled_layouts(layout):
    """Tiles with M below P, padded rows and nb batches in both layouts."""
    tdt = _tdt()
    rng = np.random.default_rng(21 if layout == "outer" else 22)
    n, M, nb = 2500, 45, 3
    P = M + 4
    tm1, t0, t1 = classes(rng, P, "adi")
    plan = tdt.StridedPlan(n, tm1, t0, t1)
    if layout == "outer":
        ld = M + 3
        F = rng.standard_normal((nb, n, ld))
        ldb = n * ld
    else:
        F = rng.standard_normal((n, nb, M + 2))
        ld, ldb = nb * (M + 2), M + 2
    print(f"[case] strided tiled {layout}", flush=True)
    Xd = to_dev(np.full_like(F, 7.0))
    plan.solve(to_dev(F), Xd, M=M, ld=ld, nb=nb, ldb=ldb)
    X = to_host(Xd)
    ref, idx = oracle_strided(F, n, M, ld, nb, ldb, tm1, t0, t1)
    check(X, ref, idx, n, M, nb, tm1, t0, t1)
    mask = np.ones(X.size, dtype=bool)
    mask[idx.reshape(-1)] = False
    assert np.all(X.reshape(-1)[mask] == 7.0)   # what no system owns is untouched


def test_strided_tiled_in_place_repeatable_graph():
    """In place equals out of place bit for bit, twice; a captured solve
    (workspace reserved first) replays to the eager result."""
    import torch
    tdt = _tdt()
    rng = np.random.default_rng(23)
    n, M = 5000, 100
    tm1, t0, t1 = classes(rng, M, "adi")
    plan = tdt.StridedPlan(n, tm1, t0, t1)
    plan.reserve(M)
    F = to_dev(rng.standard_normal((n, M)))
    print("[case] strided tiled in place / graph", flush=True)
    X1 = to_host(plan.solve(F))
    X2 = to_host(plan.solve(F))
    G = F.clone()
    plan.solve(G, G)
    assert np.array_equal(X1, X2)
    assert np.array_equal(X1, to_host(G))
    X = torch.empty_like(F)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.solve(F, X, stream=s)
    for r in range(3):
        X.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(X), X1), r
        plan.solve(F)


def test_strided_errors():
    tdt = _tdt()
    from paper_1002_2469_amd import _lib
    import ctypes
    import torch
    L = _lib.lib()
    rng = np.random.default_rng(6)
    tm1, t0, t1 = classes(rng, 8)
    plan = tdt.StridedPlan(40, tm1, t0, t1)
    F = to_dev(rng.standard_normal((40, 8)))
    X = torch.empty_like(F)
    fp, xp = ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(X.data_ptr())
    bad = [(9, 8, 1, 0),      # M > P
           (8, 7, 1, 0),      # ld < M
           (8, 8, 2, 100),    # batches overlapping
           (0, 8, 1, 0)]
    for M, ld, nb, ldb in bad:
        assert L.tdt_solve_strided(plan._h, fp, xp, M, ld, nb, ldb, None) == \
            _lib.TDT_ERR_INVALID_ARG, (M, ld, nb, ldb)
    # partial overlap of F and X
    xo = ctypes.c_void_p(F.data_ptr() + 8)
    assert L.tdt_solve_strided(plan._h, fp, xo, 8, 8, 1, 0, None) == _lib.TDT_ERR_INVALID_ARG
    # a strided plan is refused by the other solves, and vice versa
    assert L.tdt_solve(plan._h, fp, xp, 1, None) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_solve_varlen(plan._h, fp, xp, None) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_plan_set_option(plan._h, 0, 1) == _lib.TDT_ERR_INVALID_ARG
    series = tdt.Plan(-1.0, 4.0, -1.0, 40)
    assert L.tdt_solve_strided(series._h, fp, xp, 8, 8, 1, 0, None) == _lib.TDT_ERR_INVALID_ARG
    # not dominant: a warning, and the solve still runs
    w = tdt.StridedPlan(20, [-1.0], [1.5], [-1.0])
    assert w.status == _lib.TDT_WARN_NOT_DOMINANT


def test_strided_graph_replay():
    """Captured once, replayed four times with eager work in between; every
    replay equals the eager solve bit for bit."""
    import torch
    tdt = _tdt()
    rng = np.random.default_rng(8)
    n, M = 300, 64
    tm1, t0, t1 = classes(rng, M, "adi")
    plan = tdt.StridedPlan(n, tm1, t0, t1)
    F = to_dev(rng.standard_normal((n, M)))
    X = torch.empty_like(F)
    print("[case] strided graph", flush=True)
    ref = to_host(plan.solve(F))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.solve(F, X, stream=s)
    for r in range(4):
        X.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(X), ref), r
        plan.solve(F)


@pytest.mark.parametrize("n", [1000, 1024])
def test_strided_one_column_captures_without_reserve(n):
    """Orders up to 1024 run as one column per workgroup with no workspace, so
    a hipGraph capture needs no tdt_plan_reserve; replays equal the eager
    solve bit for bit, and the result matches the oracle."""
    import torch
    tdt = _tdt()
    rng = np.random.default_rng(40 + n)
    M = 40
    tm1, t0, t1 = classes(rng, M, "adi")
    plan = tdt.StridedPlan(n, tm1, t0, t1)
    Fh = rng.standard_normal((n, M))
    F = to_dev(Fh)
    X = torch.empty_like(F)
    print(f"[case] strided capture without reserve N={n}", flush=True)
    ref = to_host(plan.solve(F))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.solve(F, X, stream=s)
    for r in range(3):
        X.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(X), ref), r
    o, idx = oracle_strided(Fh, n, M, M, 1, 0, tm1, t0, t1)
    check(ref, o, idx, n, M, 1, tm1, t0, t1)
