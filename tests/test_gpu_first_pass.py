"""GPU parity of the first pass of series plans, which forms each tile's
summary (eq. (13)) as dot products of the tile's right-hand side with the
first and last Green rows of the tile.  Under diagonal dominance (Sec. 3.4)
those rows decay geometrically, and the pass then reads only the rows of a
tile the plan found to carry all but 2^-60 of each row's mass; for weakly
dominant matrices the supports cover the tile and the pass reads it whole.
Both forms are compared with the oracle, forward and adjoint."""
import numpy as np
import pytest

import oracle
from gpu_util import kappa2, to_dev, to_host, tol_f32, tol_f64
from paper_1002_2469_amd import workloads as W

pytestmark = pytest.mark.gpu


def _tdt():
    import paper_1002_2469_amd as tdt
    return tdt


def test_plan_supports():
    """The supports a plan's first pass uses, rounded up to 64-row runs, for
    the forward matrix and for T^T (the adjoint's first pass)."""
    tdt = _tdt()
    n = 4 * 8192
    assert tdt.Plan(-0.9, 2.5, -1.1, n).green_support() == {"forward": (128, 64),
                                                             "adjoint": (64, 128)}
    assert tdt.Plan(-1.0, 2.01, -1.0, n).green_support()["forward"] == (448, 448)
    assert tdt.Plan(1.0, -2.0000006, 1.0, n).green_support()["forward"] == (0, 0)
    assert tdt.Plan(-1.0, 4.0, -1.0, 8192).green_support()["forward"] == (0, 0)   # one tile


# (matrix, what the pass reads): short supports, supports of several 64-row
# runs, whole tiles (dominance ratio 1 + 3e-7), nonsymmetric of both signs
CASES = [((-0.9, 2.5, -1.1), "ends"), ((-1.0, 2.01, -1.0), "ends, 7 runs"),
         ((1.0, -2.0000006, 1.0), "whole tiles"), ((0.3, -1.0, 0.45), "ends"),
         ((-1.0, 2.0, -1.0), "whole tiles")]


@pytest.mark.parametrize("t,what", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32_refine", "f32"])
@pytest.mark.parametrize("n", [5 * 8192 + 37, 3 * 8192])
def test_first_pass_parity(t, what, dtype, n):
    tdt = _tdt()
    a, b, c = t
    if dtype == "f32" and abs(b) < 1.25 * (abs(a) + abs(c)):
        pytest.skip("plain float is specified at dominance ratio >= 1.25")
    if dtype == "f32_refine" and kappa2(a, b, c, n) * 2.0 ** -24 > 0.5:
        pytest.skip("float sweeps cannot contract a refinement at this condition number")
    rng = np.random.default_rng(n + int(1000 * abs(b)))
    M = 2
    F = rng.standard_normal((M, n))
    print(f"[case] first pass t={t} ({what}) dtype={dtype} n={n}", flush=True)
    plan = tdt.Plan(a, b, c, n, dtype)
    X = to_host(plan.solve(to_dev(F, dtype)))
    Fr = F.astype(np.float32).astype(np.float64) if dtype == "f32" else F
    ref = oracle.solve(Fr, a, b, c)
    err = oracle.rel_err_rows(X, ref).max()
    tol = tol_f32(a, b, c, n) if dtype == "f32" else tol_f64(a, b, c, n)
    assert err <= tol, (t, dtype, n, err, tol)
    if dtype == "f64":
        # the adjoint's first pass runs on T^T, whose supports are swapped
        G = rng.standard_normal((M, n))
        gF, gt = plan.backward(to_dev(G), to_dev(X))
        gFr, gtr = oracle.adjoint(G, ref, a, b, c)
        assert oracle.rel_err_rows(to_host(gF), gFr).max() <= tol_f64(c, b, a, n)
        gt = to_host(gt)
        assert np.max(np.abs(gt - gtr)) <= max(1e-11, 4 * tol_f64(a, b, c, n)) * \
            max(1.0, np.max(np.abs(gtr)))


def test_headline_first_pass_support_and_parity():
    """The single-system workload (N = 2^26, 8192 tiles): the pass reads 192
    of every 8192 rows, and both paths stay within 1e-12 of the oracle."""
    tdt = _tdt()
    d = W.single_large(0)
    Fd = to_dev(d["F"])
    ref = oracle.solve(d["F"], d["t_m1"], d["t_0"], d["t_1"])
    for dtype in ("f64", "f32_refine"):
        print(f"[case] headline first pass dtype={dtype}", flush=True)
        plan = tdt.Plan(d["t_m1"], d["t_0"], d["t_1"], d["N"], dtype)
        assert plan.green_support()["forward"] == (128, 64)
        X = to_host(plan.solve(Fd))
        assert oracle.rel_err(X, ref) <= 1e-12
        plan.close()


# last-tile lengths on both sides of where the shorter tile can take the
# full tile's support entries (supports of 64 to 448 rows, pivots settling
# within tens to a few hundred rows), and full tiles
TAILS = [0, 1, 17, 63, 64, 65, 100, 129, 200, 257, 450, 511, 700, 1000, 3000, 8191]


@pytest.mark.parametrize("quasi", [False, True])
@pytest.mark.parametrize("whole", [0, 16])
@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_varlen_first_pass_last_tiles(whole, dtype, quasi):
    """Varlen plans: each multi-tile system's full tiles are summarised from
    its supports, and so is its shorter last tile where that tile is long
    enough, otherwise swept; through the tile kernels (whole 0) and the
    whole-system kernel (whole 16).  Quasi-Toeplitz plans (corner terms
    psi, chi) also summarise a system of one shorter tile that way.  Solve
    and adjoint against the oracle, system by system, for strongly,
    moderately and weakly dominant matrices of both signs."""
    tdt = _tdt()
    mats = [(-0.9, 2.5, -1.1), (-1.0, 2.01, -1.0), (0.3, -1.0, 0.45), (1.0, -2.3, 1.0),
            (-1.0, 2.0001, -1.0)]
    sizes, tm1, t0, t1 = [], [], [], []
    for i, r in enumerate(TAILS):
        for k in ((0, 1, 2, 3) if quasi else (1, 2, 3)):
            if k == 0 and r == 0:
                continue
            a, b, c = mats[(i + k) % len(mats)]
            sizes.append(k * 8192 + r + (2 if quasi else 0))   # quasi: tiles over the inner rows
            tm1.append(a)
            t0.append(b)
            t1.append(c)
    sizes += [5, 8192]            # one-tile systems in the same plan
    tm1 += [-1.0, -1.0]
    t0 += [3.0, 3.0]
    t1 += [-1.0, -1.0]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    tm1, t0, t1 = np.array(tm1), np.array(t0), np.array(t1)
    # corner terms that keep the corner rows dominant
    psi = 0.25 * np.sign(t0) if quasi else None
    chi = 0.15 * np.sign(t0) if quasi else None
    rng = np.random.default_rng(4242 + whole)
    F = rng.standard_normal(int(off[-1]))
    G = rng.standard_normal(int(off[-1]))
    print(f"[case] varlen first pass last tiles whole={whole} dtype={dtype} quasi={quasi} "
          f"S={len(sizes)} sum N={int(off[-1])}", flush=True)
    plan = tdt.VarlenPlan(off, tm1, t0, t1, dtype, psi=psi, chi=chi)
    plan.set_option("shape", 0)
    plan.set_option("whole_max_tiles", whole)
    Xd = plan.solve(to_dev(F))
    ref = oracle.solve_varlen(F, off, tm1, t0, t1, psi=psi, chi=chi)
    tols = np.array([tol_f64(tm1[s], t0[s], t1[s], sizes[s]) for s in range(len(sizes))])
    errs = oracle.rel_err_rows(to_host(Xd), ref, off)
    bad = np.nonzero(errs > tols)[0]
    assert bad.size == 0, [(int(s), sizes[s], errs[s], tols[s]) for s in bad[:5]]
    if dtype == "f64":
        gF, gt = plan.backward(to_dev(G), Xd)
        gFr, gtr = oracle.adjoint_varlen(G, ref, off, tm1, t0, t1, psi=psi, chi=chi,
                                         corners=quasi)
        tolT = np.array([tol_f64(t1[s], t0[s], tm1[s], sizes[s]) for s in range(len(sizes))])
        errs = oracle.rel_err_rows(to_host(gF), gFr, off)
        bad = np.nonzero(errs > tolT)[0]
        assert bad.size == 0, [(int(s), sizes[s], errs[s], tolT[s]) for s in bad[:5]]
        gt = to_host(gt)
        assert gt.shape == gtr.shape
        scale = np.maximum(1.0, np.max(np.abs(gtr), axis=1))
        rel = np.max(np.abs(gt - gtr), axis=1) / scale
        lim = np.maximum(1e-11, 4 * tols)
        assert np.all(rel <= lim), [(int(s), rel[s], lim[s]) for s in np.nonzero(rel > lim)[0][:5]]
    plan.close()
