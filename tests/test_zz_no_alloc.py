"""The allocation-free solve (tdt_solve_noalloc: the workspace is the
library's static device array) against tdt_solve through the C ABI: two
calls in a row, the second with a smaller input, each equal to tdt_solve bit
for bit and within the f64 tolerance of the oracle; the size limit."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host, tol_f64

pytestmark = pytest.mark.gpu


def _call(lib, plan, F, X, M):
    import torch
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib.tdt_solve_noalloc(plan._h, ctypes.c_void_p(F.data_ptr()),
                                 ctypes.c_void_p(X.data_ptr()), int(M), s)


@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_noalloc_matches_tdt_solve(dtype):
    import torch
    import paper_1002_2469_amd as tdt
    from paper_1002_2469_amd import _lib
    lib = _lib.lib()
    rng = np.random.default_rng(77)
    a, b, c = -0.9, 2.5, -1.1
    # two calls in a row on one plan, the second with fewer right-hand sides,
    # then a smaller plan (fewer tiles, a ragged last tile)
    cases = [(5 * 8192 + 37, 3), (5 * 8192 + 37, 1), (20000, 2)]
    plans = {}
    for n, M in cases:
        print(f"[case] noalloc dtype={dtype} n={n} M={M}", flush=True)
        if n not in plans:
            plans[n] = tdt.Plan(a, b, c, n, dtype)
        plan = plans[n]
        Fh = rng.standard_normal((M, n))
        F = to_dev(Fh)
        X = torch.full_like(F, float("nan"))
        assert _call(lib, plan, F, X, M) == _lib.TDT_OK
        Xn = to_host(X)
        Xr = to_host(plan.solve(F))
        assert np.array_equal(Xn, Xr)
        assert oracle.rel_err_rows(Xn, oracle.solve(Fh, a, b, c)).max() <= tol_f64(a, b, c, n)
    for p in plans.values():
        p.close()


def test_noalloc_quasi_and_general_plans():
    import torch
    import paper_1002_2469_amd as tdt
    from paper_1002_2469_amd import _lib
    lib = _lib.lib()
    rng = np.random.default_rng(78)
    n, M = 3 * 8192 + 11, 2
    Fh = rng.standard_normal((M, n))
    F = to_dev(Fh)
    print("[case] noalloc quasi", flush=True)
    q = tdt.Plan(-1.0, 3.0, -0.8, n, "f64", psi=0.5, chi=-0.3)
    X = torch.empty_like(F)
    assert _call(lib, q, F, X, M) == _lib.TDT_OK
    assert np.array_equal(to_host(X), to_host(q.solve(F)))
    print("[case] noalloc general", flush=True)
    ga = rng.uniform(-1.0, -0.5, n)
    gc = rng.uniform(-1.0, -0.5, n)
    gb = 2.5 + rng.uniform(0.0, 1.0, n)
    g = tdt.GeneralPlan(ga, gb, gc, "f64")
    X = torch.empty_like(F)
    assert _call(lib, g, F, X, M) == _lib.TDT_OK
    assert np.array_equal(to_host(X), to_host(g.solve(F)))
    q.close()
    g.close()


def test_noalloc_refuses_beyond_its_scratch_and_bad_arguments():
    """2^26 rows (8192 tiles) times 17 right-hand sides need 139264 tile
    slots, more than the 131072 the static array holds: refused before any
    launch.  Varlen plans, M < 1 and overlapping buffers are refused as by
    tdt_solve."""
    import torch
    import paper_1002_2469_amd as tdt
    from paper_1002_2469_amd import _lib
    lib = _lib.lib()
    n = 1 << 26
    plan = tdt.Plan(-0.9, 2.5, -1.1, n, "f64")
    F = torch.empty(17 * n, dtype=torch.float64, device="cuda:0")
    X = torch.empty_like(F)
    assert _call(lib, plan, F, X, 17) == _lib.TDT_ERR_INVALID_ARG
    assert _call(lib, plan, F, X, 0) == _lib.TDT_ERR_INVALID_ARG
    assert _call(lib, plan, F, F, 1) == _lib.TDT_ERR_INVALID_ARG
    del F, X
    plan.close()
    vp = tdt.VarlenPlan(np.array([0, 10, 30], dtype=np.int64), -1.0, 3.0, -1.0, "f64")
    Fv = to_dev(np.ones(30))
    Xv = torch.empty_like(Fv)
    assert _call(lib, vp, Fv, Xv, 1) == _lib.TDT_ERR_INVALID_ARG
    vp.close()
