"""GPU parity of the forward solve against the CPU oracle (through the C ABI).

Sizes span one lane, one wavefront, one tile and several tiles, with ragged
last blocks and tiles; matrices are nonsymmetric with off-diagonals of both
signs and dominance ratios in [1, 3]."""
import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host, tol_f32, tol_f64
from paper_1002_2469_amd import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 31, 32, 33, 63, 64, 65, 2047, 2048, 2049, 8191, 8192, 8193, 16383, 16385,
         3 * 8192 + 5, 10 * 8192 + 31]


def _tdt():
    import paper_1002_2469_amd as tdt
    return tdt


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dtype", ["f64", "f32_refine", "f32"])
def test_sweep_sizes(n, dtype):
    tdt = _tdt()
    rng = np.random.default_rng(n)
    for rep, M in enumerate((1, 3)):
        a, b, c = W.random_system(rng, 1.25 if dtype == "f32" else 1.0, 3.0)
        F = rng.standard_normal((M, n))
        print(f"[case] n={n} M={M} dtype={dtype} t=({a:.3f},{b:.3f},{c:.3f})", flush=True)
        plan = tdt.Plan(a, b, c, n, dtype)
        X = to_host(plan.solve(to_dev(F, dtype)))
        Fr = F.astype(np.float32).astype(np.float64) if dtype == "f32" else F
        ref = oracle.solve(Fr, a, b, c)
        err = oracle.rel_err_rows(X, ref).max()
        tol = tol_f32(a, b, c, n) if dtype == "f32" else tol_f64(a, b, c, n)
        assert err <= tol, (n, M, dtype, (a, b, c), err)


@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_single_small_config_and_manufactured(dtype):
    tdt = _tdt()
    d = W.single_small(0)
    plan = tdt.Plan(d["t_m1"], d["t_0"], d["t_1"], d["N"], dtype)
    X = to_host(plan.solve(to_dev(d["F"])))
    ref = oracle.solve(d["F"], d["t_m1"], d["t_0"], d["t_1"])
    assert oracle.rel_err(X, ref) <= 1e-12
    m = W.single_small(0, manufactured=True)
    from oracle_pins import stencil
    F = stencil(m["X_true"].copy(), m["t_m1"], m["t_0"], m["t_1"])
    X = to_host(plan.solve(to_dev(F)))
    assert oracle.rel_err(X, oracle.solve(F, m["t_m1"], m["t_0"], m["t_1"])) <= 1e-12
    assert oracle.rel_err(X, m["X_true"]) <= 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32_refine", "f32"])
def test_series_config(dtype):
    tdt = _tdt()
    d = W.series(0)
    plan = tdt.Plan(d["t_m1"], d["t_0"], d["t_1"], d["N"], dtype)
    X = to_host(plan.solve(to_dev(d["F"], dtype)))
    Fr = d["F"].astype(np.float32).astype(np.float64) if dtype == "f32" else d["F"]
    ref = oracle.solve(Fr, d["t_m1"], d["t_0"], d["t_1"])
    err = oracle.rel_err_rows(X, ref).max()
    assert err <= (2e-5 if dtype == "f32" else 1e-12), err


@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_single_large_config(dtype):
    tdt = _tdt()
    d = W.single_large(0)
    plan = tdt.Plan(d["t_m1"], d["t_0"], d["t_1"], d["N"], dtype)
    X = to_host(plan.solve(to_dev(d["F"])))
    ref = oracle.solve(d["F"], d["t_m1"], d["t_0"], d["t_1"])
    assert oracle.rel_err(X, ref) <= 1e-12


def _varlen_check(d, dtype, tol_of, whole=None):
    tdt = _tdt()
    plan = tdt.VarlenPlan(d["offsets"], d["t_m1"], d["t_0"], d["t_1"], dtype)
    if whole is not None:
        plan.set_option("whole_max_tiles", whole)
        assert plan.get_option("whole_max_tiles") == whole
    X = to_host(plan.solve(to_dev(d["F"], dtype)))
    F = d["F"].astype(np.float32).astype(np.float64) if dtype == "f32" else d["F"]
    ref = oracle.solve_varlen(F, d["offsets"], d["t_m1"], d["t_0"], d["t_1"])
    errs = oracle.rel_err_rows(X, ref, d["offsets"])
    sizes = np.diff(d["offsets"])
    tols = np.array([tol_of(d["t_m1"][s], d["t_0"][s], d["t_1"][s], int(sizes[s]))
                     for s in range(len(sizes))])
    bad = np.nonzero(errs > tols)[0]
    assert bad.size == 0, [(int(s), int(sizes[s]), errs[s], tols[s]) for s in bad[:5]]
    return plan


@pytest.mark.parametrize("whole", [0, 1, 2, 8, 16])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine", "f32"])
def test_varlen_ragged(dtype, whole):
    """Systems of 1 to 13 tiles, solved whole by one workgroup each up to
    `whole` tiles and by the three-kernel path beyond."""
    print(f"[case] varlen ragged dtype={dtype} whole_max_tiles={whole}", flush=True)
    rng = np.random.default_rng(7)
    sizes = np.array([1, 2, 3, 33, 8192, 8193, 65, 20000, 5, 16384, 31, 64, 100000])
    S = len(sizes)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    ts = [W.random_system(rng, 1.25 if dtype == "f32" else 1.0, 3.0) for _ in range(S)]
    d = dict(offsets=off, t_m1=np.array([t[0] for t in ts]), t_0=np.array([t[1] for t in ts]),
             t_1=np.array([t[2] for t in ts]), F=rng.standard_normal(int(off[-1])))
    _varlen_check(d, dtype, tol_f32 if dtype == "f32" else tol_f64, whole)


@pytest.mark.parametrize("whole", [0, 8])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_sov_batch_config(dtype, whole):
    print(f"[case] sov batch dtype={dtype} whole_max_tiles={whole}", flush=True)
    d = W.sov_batch(0)
    plan = _varlen_check(d, dtype, tol_f64, whole)
    # against the long double truth too (the ill-conditioned low modes)
    X = to_host(plan.solve(to_dev(d["F"])))
    truth = oracle.solve_varlen(d["F"], d["offsets"], d["t_m1"], d["t_0"], d["t_1"],
                                precision="ld")
    errs = oracle.rel_err_rows(X, truth, d["offsets"])
    sizes = np.diff(d["offsets"])
    tols = np.array([tol_f64(1.0, d["t_0"][s], 1.0, int(sizes[s])) for s in range(len(sizes))])
    assert np.all(errs <= tols)


@pytest.mark.parametrize("whole", [0, 8])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_diff_batch_config_forward(dtype, whole):
    print(f"[case] diff batch forward dtype={dtype} whole_max_tiles={whole}", flush=True)
    d = W.diff_batch(0)
    _varlen_check(dict(offsets=d["offsets"], t_m1=d["t_m1"], t_0=d["t_0"], t_1=d["t_1"],
                       F=d["F"].reshape(-1)), dtype, tol_f64, whole)


def test_repeatable_bitwise():
    tdt = _tdt()
    rng = np.random.default_rng(3)
    n = 3 * 8192 + 77
    F = to_dev(rng.standard_normal((2, n)))
    for dtype in ("f64", "f32_refine"):
        plan = tdt.Plan(-0.9, 2.5, -1.1, n, dtype)
        X1 = to_host(plan.solve(F))
        X2 = to_host(plan.solve(F))
        assert np.array_equal(X1, X2)
    # varlen, both paths, and a different workgroup count (the persistent
    # grid must not change any result)
    sizes = np.array([40000, 9000, 300, 8192, 17])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    Fv = to_dev(rng.standard_normal(int(off[-1])))
    for whole in (0, 8):
        plan = tdt.VarlenPlan(off, -1.0, 3.2, -0.7, "f32_refine")
        plan.set_option("whole_max_tiles", whole)
        X1 = to_host(plan.solve(Fv))
        plan.set_option("wg_per_cu", 1)
        X2 = to_host(plan.solve(Fv))
        assert np.array_equal(X1, X2), whole


@pytest.mark.parametrize("tiles,extra", [(64, 0), (64, 5), (65, 0), (257, 0), (2048, 17),
                                         (2049, 3), (8193, 100)])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_many_tiles(tiles, extra, dtype):
    """Every variant of the interface pass across tiles: up to 64 tiles (one
    wavefront), up to 256, up to 2048, up to 8192 (the single-system
    workload) and the general one beyond."""
    tdt = _tdt()
    n = (tiles - 1) * 8192 + (extra if extra else 8192)   # last tile partial if extra
    rng = np.random.default_rng(tiles)
    a, b, c = W.random_system(rng, 1.05, 2.0)
    F = rng.standard_normal(n)
    print(f"[case] tiles n={n} dtype={dtype}", flush=True)
    plan = tdt.Plan(a, b, c, n, dtype)
    X = to_host(plan.solve(to_dev(F)))
    ref = oracle.solve(F, a, b, c)
    assert oracle.rel_err(X, ref) <= tol_f64(a, b, c, n)


@pytest.mark.parametrize("tiles,M,dom,sym", [(2, 1, 2.0, False), (64, 2, 2.0, False),
                                             (64, 3, 2.0, False), (17, 2, 1.02, True)])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_interface_inside_final_pass(tiles, M, dom, sym, dtype):
    """A series of at most 64 tiles per right-hand side runs the interface
    pass inside the final pass (every wavefront scans its system's tiles, one
    per lane) instead of in a launch of its own: two solves in a row with
    other data, the adjoint after them, and a weakly dominant matrix whose
    supports are long enough to split every tile end into its own
    first-pass wavefront."""
    tdt = _tdt()
    n = tiles * 8192
    rng = np.random.default_rng(tiles * 10 + M)
    a, b, c = W.random_system(rng, dom, dom, symmetric=sym)
    print(f"[case] first pass with interface n={n} M={M} dtype={dtype}", flush=True)
    plan = tdt.Plan(a, b, c, n, dtype)
    plan.set_option("shape", 0)
    assert plan.green_support()["forward"][0] > 0
    for rep in range(2):
        F = rng.standard_normal((M, n))
        Xd = plan.solve(to_dev(F))
        ref = oracle.solve(F, a, b, c)
        assert oracle.rel_err_rows(to_host(Xd), ref).max() <= tol_f64(a, b, c, n), rep
    G = rng.standard_normal((M, n))
    gF, gt = plan.backward(to_dev(G), Xd)
    gFr, gtr = oracle.adjoint(G, ref, a, b, c)
    assert oracle.rel_err_rows(to_host(gF), gFr).max() <= tol_f64(c, b, a, n)
    gt = to_host(gt)
    assert np.max(np.abs(gt - gtr)) <= 1e-10 * max(1.0, np.max(np.abs(gtr)))
    plan.close()


@pytest.mark.parametrize("shape,M", [(2, 1), (2, 3), (0, 2), (1, 5)])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine", "f32"])
def test_small_series_in_one_launch(shape, M, dtype):
    """A small series of whole tiles with short supports (at most 256 tiles
    in all, at most four per wavefront of a workgroup) is solved by the
    final pass alone: each workgroup computes its system's tile summaries
    from the supports, runs the interface pass and solves its tile.  The
    65536-row system at every work shape, several right-hand sides, two
    solves in a row with other data (the second with persistent workgroups
    that loop over tiles and recompute the summaries per tile)."""
    tdt = _tdt()
    n = 65536
    rng = np.random.default_rng(31 + shape + M)
    a, b, c = -1.0, 4.0, -1.0
    print(f"[case] small series in one launch shape={shape} M={M} dtype={dtype}", flush=True)
    plan = tdt.Plan(a, b, c, n, dtype)
    plan.set_option("shape", shape)
    assert plan.green_support()["forward"][0] > 0
    for rep in range(2):
        plan.set_option("wg_per_cu", 0 if rep == 0 else 1)
        F = rng.uniform(-1.0, 1.0, (M, n))
        X = to_host(plan.solve(to_dev(F, dtype)))
        Fr = F.astype(np.float32).astype(np.float64) if dtype == "f32" else F
        ref = oracle.solve(Fr, a, b, c)
        tol = tol_f32(a, b, c, n) if dtype == "f32" else tol_f64(a, b, c, n)
        assert oracle.rel_err_rows(X, ref).max() <= tol, (rep, dtype)
    plan.close()


@pytest.mark.parametrize("extra,dom,sym", [(5, (1.05, 2.0), False), (0, (1.05, 2.0), False),
                                           (0, (1.02, 1.02), True)])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_chunked_interface_series(dtype, extra, dom, sym):
    """Series of 2049 to 16384 tiles take the interface pass in chunks of 64
    tiles (chunk composites, then every chunk's tiles): several right-hand
    sides (the chunks of all of them in one launch), a ragged last chunk,
    a partial or a whole last tile, and long supports of a weakly dominant
    matrix (every tile end a first-pass wavefront of its own); forward and
    adjoint against the oracle."""
    tdt = _tdt()
    n = 2100 * 8192 + extra      # 2100 or 2101 tiles: 33 chunks, the last one of 52 or 53
    M = 3
    rng = np.random.default_rng(2101)
    a, b, c = W.random_system(rng, dom[0], dom[1], symmetric=sym, signs=not sym)
    F = rng.standard_normal((M, n))
    print(f"[case] chunked interface n={n} M={M} dtype={dtype} sym={sym}", flush=True)
    plan = tdt.Plan(a, b, c, n, dtype)
    plan.set_option("shape", 0)
    Xd = plan.solve(to_dev(F))
    ref = oracle.solve(F, a, b, c)
    assert oracle.rel_err_rows(to_host(Xd), ref).max() <= tol_f64(a, b, c, n)
    if dtype == "f64":
        G = rng.standard_normal((M, n))
        gF, gt = plan.backward(to_dev(G), Xd)
        gFr, gtr = oracle.adjoint(G, ref, a, b, c)
        assert oracle.rel_err_rows(to_host(gF), gFr).max() <= tol_f64(c, b, a, n)
        gt = to_host(gt)
        assert np.max(np.abs(gt - gtr)) <= 1e-11 * max(1.0, np.max(np.abs(gtr)))
    plan.close()
