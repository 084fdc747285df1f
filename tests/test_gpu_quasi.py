"""GPU parity of quasi-Toeplitz systems (eq. (21): t_0 + psi in the first
diagonal entry, t_0 + chi in the last) against the CPU oracle, through the C
ABI: the forward solve over sizes from 3 rows to many tiles (every variant of
the interface pass across tiles, ragged and exact last tiles), series of
right-hand sides, varlen batches on both paths, the other work shapes, and
the adjoint with dL/dpsi and dL/dchi.

Inputs: nonsymmetric t's with dominance ratio in [1.2, 3] (in [1.25, 3] for
plain float) and corner terms drawn so that the corner rows are dominant by
a ratio in the same range, with either sign of psi and chi."""
import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host
from paper_1002_2469_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32_refine": 1e-12, "f32": 2e-5}


def _tdt():
    import paper_1002_2469_amd as tdt
    return tdt


def quasi_system(rng, lo=1.2, hi=3.0):
    """(t_-1, t_0, t_1, psi, chi) with every row dominant by a ratio in [lo, hi]."""
    a, b, c = W.random_system(rng, lo, hi)
    d0 = np.sign(b) * abs(c) * rng.uniform(lo, hi)     # t_0 + psi against |t_1|
    d1 = np.sign(b) * abs(a) * rng.uniform(lo, hi)     # t_0 + chi against |t_-1|
    return a, b, c, float(d0 - b), float(d1 - b)


def _f32_round(F, dtype):
    return F.astype(np.float32).astype(np.float64) if dtype == "f32" else F


SIZES = [3, 4, 5, 17, 66, 8193, 8194, 8195, 8209, 16386, 16387, 3 * 8192 + 7, 10 * 8192 + 2]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dtype", ["f64", "f32_refine", "f32"])
def test_quasi_sizes(n, dtype):
    """N - 2 inner rows: one row, one block, one tile exactly (8194), one tile
    plus a one-row tile (8195), several tiles with ragged and exact ends."""
    tdt = _tdt()
    rng = np.random.default_rng(1000 + n)
    for M in (1, 3):
        a, b, c, psi, chi = quasi_system(rng, 1.25 if dtype == "f32" else 1.2)
        F = rng.standard_normal((M, n))
        print(f"[case] quasi n={n} M={M} dtype={dtype} t=({a:.3f},{b:.3f},{c:.3f}) "
              f"psi={psi:.3f} chi={chi:.3f}", flush=True)
        plan = tdt.Plan(a, b, c, n, dtype, psi=psi, chi=chi)
        X = to_host(plan.solve(to_dev(F, dtype)))
        ref = oracle.solve(_f32_round(F, dtype), a, b, c, psi=psi, chi=chi)
        err = oracle.rel_err_rows(X, ref).max()
        assert err <= TOL[dtype], (n, M, dtype, err)


def test_quasi_zero_corners_is_the_toeplitz_solve():
    """psi = chi = 0 takes the quasi-Toeplitz path (corner rows as interface
    segments) and must give the Toeplitz solution."""
    tdt = _tdt()
    rng = np.random.default_rng(5)
    n = 2 * 8192 + 300
    a, b, c = W.random_system(rng, 1.2, 3.0)
    F = rng.standard_normal((2, n))
    print(f"[case] quasi zero corners n={n}", flush=True)
    Xq = to_host(tdt.Plan(a, b, c, n, "f64", psi=0.0, chi=0.0).solve(to_dev(F)))
    Xt = to_host(tdt.Plan(a, b, c, n, "f64").solve(to_dev(F)))
    ref = oracle.solve(F, a, b, c)
    assert oracle.rel_err(Xq, ref) <= 1e-12
    assert oracle.rel_err(Xq, Xt) <= 1e-12


@pytest.mark.parametrize("tiles,extra", [(1, 0), (2, 1), (257, 0), (2048, 17), (2049, 3),
                                         (8193, 100)])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_quasi_many_tiles(tiles, extra, dtype):
    """Each variant of the interface pass across tiles with the corner rows
    at both ends of it (inner rows = tiles of 8192, the last one `extra` rows
    long when extra > 0)."""
    tdt = _tdt()
    inner = (tiles - 1) * 8192 + (extra if extra else 8192)
    n = inner + 2
    rng = np.random.default_rng(tiles * 7 + extra)
    a, b, c, psi, chi = quasi_system(rng, 1.1, 2.0)
    F = rng.standard_normal(n)
    print(f"[case] quasi tiles={tiles} n={n} dtype={dtype}", flush=True)
    plan = tdt.Plan(a, b, c, n, dtype, psi=psi, chi=chi)
    X = to_host(plan.solve(to_dev(F)))
    ref = oracle.solve(F, a, b, c, psi=psi, chi=chi)
    assert oracle.rel_err(X, ref) <= 1e-12


def _ragged_quasi(rng, sizes, lo=1.2):
    S = len(sizes)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    qs = [quasi_system(rng, lo) for _ in range(S)]
    cols = [np.array([q[k] for q in qs]) for k in range(5)]
    return off, cols, rng.standard_normal(int(off[-1]))


@pytest.mark.parametrize("whole", [0, 1, 2, 8, 16])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine", "f32"])
def test_quasi_varlen_ragged(dtype, whole):
    """Quasi-Toeplitz systems of 3 rows to 13 tiles, solved whole by one
    workgroup each up to `whole` tiles (of inner rows) and tile-parallel
    beyond (f64 and f32: the final pass closes the chain of tiles with the
    corner rows itself and stores them; f32_refine: the interface launch)."""
    tdt = _tdt()
    rng = np.random.default_rng(77)
    sizes = np.array([3, 4, 35, 8194, 8195, 67, 20000, 7, 16386, 33, 66, 100002])
    off, (a, b, c, psi, chi), F = _ragged_quasi(rng, sizes, 1.25 if dtype == "f32" else 1.2)
    print(f"[case] quasi varlen dtype={dtype} whole_max_tiles={whole}", flush=True)
    plan = tdt.VarlenPlan(off, a, b, c, dtype, psi=psi, chi=chi)
    plan.set_option("whole_max_tiles", whole)
    X = to_host(plan.solve(to_dev(F, dtype)))
    ref = oracle.solve_varlen(_f32_round(F, dtype), off, a, b, c, psi=psi, chi=chi)
    errs = oracle.rel_err_rows(X, ref, off)
    bad = np.nonzero(errs > TOL[dtype])[0]
    assert bad.size == 0, [(int(s), int(sizes[s]), errs[s]) for s in bad[:5]]


@pytest.mark.parametrize("shape", [1, 2])
def test_quasi_shapes(shape):
    """The other work shapes (tiles of 4096 rows), series and varlen."""
    tdt = _tdt()
    rng = np.random.default_rng(shape)
    n = 5 * 4096 + 33
    a, b, c, psi, chi = quasi_system(rng)
    F = rng.standard_normal((2, n))
    print(f"[case] quasi shape={shape} n={n}", flush=True)
    plan = tdt.Plan(a, b, c, n, "f32_refine", psi=psi, chi=chi)
    plan.set_option("shape", shape)
    X = to_host(plan.solve(to_dev(F)))
    assert oracle.rel_err(X, oracle.solve(F, a, b, c, psi=psi, chi=chi)) <= 1e-12
    sizes = np.array([3, 4096, 4097, 4098, 9000, 5])
    off, (va, vb, vc, vpsi, vchi), Fv = _ragged_quasi(rng, sizes)
    for whole in (0, 4):
        vp = tdt.VarlenPlan(off, va, vb, vc, "f64", psi=vpsi, chi=vchi)
        vp.set_option("shape", shape)
        vp.set_option("whole_max_tiles", whole)
        Xv = to_host(vp.solve(to_dev(Fv)))
        ref = oracle.solve_varlen(Fv, off, va, vb, vc, psi=vpsi, chi=vchi)
        assert oracle.rel_err_rows(Xv, ref, off).max() <= 1e-12, whole


@pytest.mark.slow
def test_quasi_segment_merge_interface():
    """More than 16384 tiles of inner rows (tiles of 4096) selects the
    segment-merge interface pass; in a varlen plan it then serves every
    multi-tile system, including small ones whose threads past the last tile
    hold empty runs that the corner value must pass through."""
    tdt = _tdt()
    rng = np.random.default_rng(16385)
    sizes = np.array([16385 * 4096 + 11, 5, 3, 9000, 70000])
    off, (a, b, c, psi, chi), F = _ragged_quasi(rng, sizes, 1.1)
    print(f"[case] quasi segment-merge interface total={int(off[-1])}", flush=True)
    plan = tdt.VarlenPlan(off, a, b, c, "f64", psi=psi, chi=chi)
    plan.set_option("shape", 1)
    plan.set_option("whole_max_tiles", 0)
    X = to_host(plan.solve(to_dev(F)))
    ref = oracle.solve_varlen(F, off, a, b, c, psi=psi, chi=chi)
    assert oracle.rel_err_rows(X, ref, off).max() <= 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_quasi_adjoint_series(dtype):
    """gF = T^{-T} gX and the five t-gradients summed over the right-hand
    sides, against the oracle's adjoint (itself pinned to finite differences)."""
    tdt = _tdt()
    rng = np.random.default_rng(21)
    for n in (3, 70, 3 * 8192 + 9, 2 * 8192 + 2):
        a, b, c, psi, chi = quasi_system(rng)
        F = rng.standard_normal((2, n))
        G = rng.standard_normal((2, n))
        print(f"[case] quasi adjoint series n={n} dtype={dtype}", flush=True)
        plan = tdt.Plan(a, b, c, n, dtype, psi=psi, chi=chi)
        X = plan.solve(to_dev(F))
        gF, gt = plan.backward(to_dev(G), X)
        Xr = oracle.solve(F, a, b, c, psi=psi, chi=chi)
        gFr, gtr = oracle.adjoint(G, Xr, a, b, c, psi=psi, chi=chi, corners=True)
        assert oracle.rel_err(to_host(gF), gFr) <= 1e-12
        gth = to_host(gt)
        assert gth.shape == (5,)
        assert np.max(np.abs(gth - gtr)) <= 1e-11 * np.max(np.abs(gtr)), (n, gth, gtr)


@pytest.mark.parametrize("whole", [0, 8])
def test_quasi_adjoint_varlen(whole):
    tdt = _tdt()
    rng = np.random.default_rng(31)
    sizes = np.array([3, 8195, 100002, 66, 16386, 4])
    off, (a, b, c, psi, chi), F = _ragged_quasi(rng, sizes)
    G = rng.standard_normal(int(off[-1]))
    print(f"[case] quasi adjoint varlen whole_max_tiles={whole}", flush=True)
    plan = tdt.VarlenPlan(off, a, b, c, "f64", psi=psi, chi=chi)
    plan.set_option("whole_max_tiles", whole)
    X = plan.solve(to_dev(F))
    gF, gt = plan.backward(to_dev(G), X)
    Xr = oracle.solve_varlen(F, off, a, b, c, psi=psi, chi=chi)
    gFr, gtr = oracle.adjoint_varlen(G, Xr, off, a, b, c, psi=psi, chi=chi, corners=True)
    assert oracle.rel_err_rows(to_host(gF), gFr, off).max() <= 1e-12
    gth = to_host(gt)
    assert gth.shape == (len(sizes), 5)
    scale = np.max(np.abs(gtr), axis=1, keepdims=True)
    assert np.all(np.abs(gth - gtr) <= 1e-11 * scale), (gth, gtr)


def test_quasi_autograd_function():
    """TridiagToeplitzSolve with t of 5 values differentiates psi and chi."""
    import torch
    tdt = _tdt()
    rng = np.random.default_rng(41)
    n = 9000
    a, b, c, psi, chi = quasi_system(rng)
    F = torch.tensor(rng.standard_normal(n), device="cuda", requires_grad=True)
    t = torch.tensor([a, b, c, psi, chi], dtype=torch.float64, requires_grad=True)
    G = rng.standard_normal(n)
    print("[case] quasi autograd", flush=True)
    X = tdt.TridiagToeplitzSolve.apply(F, t)
    (X * torch.tensor(G, device="cuda")).sum().backward()
    Xr = oracle.solve(F.detach().cpu().numpy(), a, b, c, psi=psi, chi=chi)
    gFr, gtr = oracle.adjoint(G, Xr, a, b, c, psi=psi, chi=chi, corners=True)
    assert oracle.rel_err(F.grad.cpu().numpy(), gFr) <= 1e-12
    assert np.max(np.abs(t.grad.numpy() - gtr)) <= 1e-11 * np.max(np.abs(gtr))


def test_quasi_info_and_singular_corner():
    tdt = _tdt()
    n = 1000
    plan = tdt.Plan(-1.0, 4.0, -1.0, n, "f64", psi=-2.5, chi=1.0)
    info = plan.info()
    assert abs(info["dominance"] - 1.5) < 1e-15     # first row: |4 - 2.5| / |t_1|
    # the bound is at least the true 2-norm condition number
    from oracle_pins import dense_T
    T = dense_T(n, -1.0, 4.0, -1.0, -2.5, 1.0)
    assert info["kappa2"] >= np.linalg.cond(T) * (1 - 1e-12)
    from paper_1002_2469_amd import _lib
    with pytest.raises(_lib.TDTError):
        tdt.Plan(-1.0, 4.0, -1.0, n, "f64", psi=-4.0, chi=0.0)   # t_0 + psi = 0


def _kappa_bound(a, b, c, psi, chi):
    """sqrt(kappa_1 kappa_inf) from strict row and column dominance."""
    A, C, d, d0, d1 = abs(a), abs(c), abs(b), abs(b + psi), abs(b + chi)
    rex = min(d0 - C, d - A - C, d1 - A)
    cex = min(d0 - A, d - A - C, d1 - C)
    rn = max(d0 + C, d + A + C, d1 + A)
    cn = max(d0 + A, d + A + C, d1 + C)
    return float(np.sqrt((rn / rex) * (cn / cex)))


@pytest.mark.parametrize("whole", [0, 8])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_sov_neumann_config(dtype, whole):
    """The separation-of-variables batch with Neumann ends (psi = chi = 1) at
    full size, against the long double oracle; the low modes are nearly
    singular (kappa up to ~1e7), hence the per-system 4 u kappa tolerance."""
    tdt = _tdt()
    d = W.sov_neumann_batch(0)
    print(f"[case] sov_neumann dtype={dtype} whole_max_tiles={whole}", flush=True)
    plan = tdt.VarlenPlan(d["offsets"], d["t_m1"], d["t_0"], d["t_1"], dtype,
                          psi=d["psi"], chi=d["chi"])
    plan.set_option("whole_max_tiles", whole)
    X = to_host(plan.solve(to_dev(d["F"])))
    truth = oracle.solve_varlen(d["F"], d["offsets"], d["t_m1"], d["t_0"], d["t_1"],
                                precision="ld", psi=d["psi"], chi=d["chi"])
    errs = oracle.rel_err_rows(X, truth, d["offsets"])
    tols = np.array([max(1e-12, 4 * 2.0 ** -53 * _kappa_bound(1.0, d["t_0"][s], 1.0, 1.0, 1.0))
                     for s in range(d["S"])])
    bad = np.nonzero(errs > tols)[0]
    assert bad.size == 0, [(int(s), errs[s], tols[s]) for s in bad[:5]]
