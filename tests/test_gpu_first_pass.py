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
