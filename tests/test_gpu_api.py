"""Error paths, warnings, info and hipGraph capture through the C ABI."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host
from paper_1002_2469_amd import _lib

pytestmark = pytest.mark.gpu


def _tdt():
    import paper_1002_2469_amd as tdt
    return tdt


def test_error_paths():
    import torch
    tdt = _tdt()
    L = _lib.lib()
    plan = tdt.Plan(-1.0, 4.0, -1.0, 100)
    F = to_dev(np.ones(300))
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    assert L.tdt_solve(plan._h, p(F), p(F), 3, None) == _lib.TDT_ERR_INVALID_ARG   # X aliases F
    X = torch.empty_like(F)
    assert L.tdt_solve(plan._h, p(F), p(X), 0, None) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_solve(plan._h, None, p(X), 1, None) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_solve_varlen(plan._h, p(F), p(X), None) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_solve_backward(plan._h, p(F), p(X), p(F), None, 3, None) == \
        _lib.TDT_ERR_INVALID_ARG                                                  # gF aliases gX
    assert L.tdt_plan_reserve(plan._h, 0) == _lib.TDT_ERR_INVALID_ARG
    with pytest.raises(tdt.TDTError) as e:
        tdt.Plan(1.0, 0.0, 1.0, 10)                         # zero pivot in the block
    assert e.value.status == _lib.TDT_ERR_SINGULAR
    vp = tdt.VarlenPlan([0, 5, 9], [-1, -1], [3, 3], [-1, -1])
    assert L.tdt_solve(vp._h, p(F), p(X), 1, None) == _lib.TDT_ERR_INVALID_ARG


def test_not_dominant_warns_and_solves():
    tdt = _tdt()
    a, b, c = 0.5, 0.9, 0.7          # ratio 0.75
    n = 40
    plan = tdt.Plan(a, b, c, n)
    assert plan.status == _lib.TDT_WARN_NOT_DOMINANT and not plan.dominant
    rng = np.random.default_rng(1)
    F = rng.standard_normal(n)
    X = to_host(plan.solve(to_dev(F)))
    from oracle_pins import dense_T
    kap = np.linalg.cond(dense_T(n, a, b, c))
    assert oracle.rel_err(X, oracle.solve(F, a, b, c)) <= 1e-12 * max(1.0, kap)


def test_nan_propagates_without_crash():
    tdt = _tdt()
    F = np.ones(5000)
    F[1234] = np.nan
    X = to_host(tdt.Plan(-1.0, 4.0, -1.0, 5000).solve(to_dev(F)))
    assert np.isnan(X).any()


def test_info():
    tdt = _tdt()
    plan = tdt.Plan(-0.9, 2.5, -1.1, 10000, "f32_refine")
    plan.solve(to_dev(np.random.default_rng(0).standard_normal(10000)))
    info = plan.info()
    assert 1 <= info["refine_iters"] <= 40
    assert info["dominance"] == pytest.approx(1.25)
    assert 1 < info["kappa2"] < 20
    assert info["converged"] and 0 <= info["last_rel_update"] <= 1e-12
    assert plan.info()["refine_iters"] == 0            # the record was cleared


def test_not_converged_is_reported():
    """A cap of one float solve leaves no refinement update: the plan reports
    it through tdt_last_info (the solution is the float one)."""
    tdt = _tdt()
    n = 10000
    F = np.random.default_rng(1).standard_normal(n)
    plan = tdt.Plan(-0.9, 2.5, -1.1, n, "f32_refine")
    plan.set_option("max_refine", 1)
    X = to_host(plan.solve(to_dev(F)))
    info = plan.info()
    assert info["refine_iters"] == 1 and not info["converged"]
    assert info["last_rel_update"] == 1.0
    assert oracle.rel_err(X, oracle.solve(F, -0.9, 2.5, -1.1)) <= 1e-5
    plan.set_option("max_refine", 40)
    X = to_host(plan.solve(to_dev(F)))
    assert plan.info()["converged"]
    assert oracle.rel_err(X, oracle.solve(F, -0.9, 2.5, -1.1)) <= 1e-12


def test_solve_varlen_function():
    tdt = _tdt()
    rng = np.random.default_rng(8)
    off = np.array([0, 5, 9000, 9001, 30000], dtype=np.int64)
    t0 = rng.uniform(2.5, 4.0, 4)
    F = rng.standard_normal(int(off[-1]))
    X = to_host(tdt.solve_varlen(to_dev(F), off, -1.0, t0, -0.8, "f32_refine"))
    ref = oracle.solve_varlen(F, off, -1.0, t0, -0.8)
    assert oracle.rel_err_rows(X, ref, off).max() <= 1e-12


@pytest.mark.parametrize("varlen", [False, True])
def test_hipgraph_capture_replay(varlen):
    import torch
    tdt = _tdt()
    rng = np.random.default_rng(11)
    if varlen:
        sizes = np.array([300, 9000, 17, 20000])
        off = np.concatenate([[0], np.cumsum(sizes)])
        t0 = rng.uniform(2.5, 4.0, 4)
        plan = tdt.VarlenPlan(off, -1.0, t0, -0.9, "f32_refine")
        n_total = int(off[-1])
        ref_fn = lambda F: oracle.solve_varlen(F, off, -1.0, t0, -0.9)
        solve = plan.solve
    else:
        n_total = 3 * 20000
        plan = tdt.Plan(-1.0, 3.0, -0.8, 20000, "f64")
        ref_fn = lambda F: oracle.solve(F.reshape(3, -1), -1.0, 3.0, -0.8).reshape(-1)
        solve = plan.solve
    plan.reserve(3)
    Fd = to_dev(rng.standard_normal(n_total))
    Xd = torch.empty_like(Fd)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        solve(Fd, Xd)                                   # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        solve(Fd, Xd)
    for k in range(4):
        Fh = rng.standard_normal(n_total)
        Fd.copy_(torch.from_numpy(Fh))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert oracle.rel_err(to_host(Xd), ref_fn(Fh)) <= 1e-12, k
        _ = (Xd * 2).sum().item()                       # eager work between replays


def test_capture_without_reserve_is_refused():
    import torch
    tdt = _tdt()
    plan = tdt.Plan(-1.0, 3.0, -1.0, 50000)              # multi-tile: needs workspace
    Fd = to_dev(np.ones(50000))
    Xd = torch.empty_like(Fd)
    g = torch.cuda.CUDAGraph()
    with pytest.raises(tdt.TDTError) as e:
        with torch.cuda.graph(g):
            plan.solve(Fd, Xd)
    assert e.value.status == _lib.TDT_ERR_CAPTURE


def test_options_validation():
    tdt = _tdt()
    plan = tdt.Plan(-1.0, 3.0, -1.0, 1000)
    with pytest.raises(tdt.TDTError):
        plan.set_option("whole_max_tiles", 4)           # series plan: no such choice
    off = np.array([0, 100, 20000], dtype=np.int64)
    vp = tdt.VarlenPlan(off, -1.0, 3.0, -1.0)
    for name, bad in (("whole_max_tiles", -1), ("whole_max_tiles", 17), ("wg_per_cu", -1),
                      ("max_refine", 0), ("max_refine", 101), ("shape", -1),
                      ("shape", len(_lib.SHAPES))):
        with pytest.raises(tdt.TDTError) as e:
            vp.set_option(name, bad)
        assert e.value.status == _lib.TDT_ERR_INVALID_ARG
    assert vp.get_option("whole_max_tiles") == 8
    assert vp.get_option("wg_per_cu") == 0
    assert vp.get_option("max_refine") == 40
    assert vp.get_option("shape") == 0


def test_autotune_choice_cache_and_result(tmp_path, monkeypatch):
    """The autotuner times the launch shapes, keeps one, writes its cache
    file, reuses the entry without timing, and every shape gives the same
    solution (checked against the oracle)."""
    import json
    tdt = _tdt()
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("TDT_TUNE_CACHE", str(cache))
    rng = np.random.default_rng(5)
    sizes = np.array([30000, 700, 9000, 17, 20000, 65536])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    t0 = rng.uniform(2.5, 4.0, len(sizes))
    F = rng.standard_normal(int(off[-1]))
    ref = oracle.solve_varlen(F, off, -1.0, t0, -0.9)
    plan = tdt.VarlenPlan(off, -1.0, t0, -0.9, "f32_refine")
    Fd = to_dev(F)
    res = plan.autotune(Fd)
    assert res["ms"] > 0 and res["whole_max_tiles"] in (0, 1, 2, 4, 8, 16)
    assert res["wg_per_cu"] in (0, 1, 2) and res["shape"] in range(len(_lib.SHAPES))
    X = to_host(plan.solve(Fd))
    assert oracle.rel_err_rows(X, ref, off).max() <= 1e-12
    doc = json.loads(cache.read_text())
    assert doc["format"] == "tdt-autotune-1" and len(doc["entries"]) == 1
    (key, entry), = doc["entries"].items()
    assert "varlen|f32_refine" in key and entry["whole_max_tiles"] == res["whole_max_tiles"]
    assert entry["shape"] == res["shape"]
    plan2 = tdt.VarlenPlan(off, -1.0, t0, -0.9, "f32_refine")
    res2 = plan2.autotune(Fd)                     # from the cache: no timing
    assert res2["ms"] == 0.0 and res2["whole_max_tiles"] == res["whole_max_tiles"]
    assert res2["shape"] == res["shape"]
    X2 = to_host(plan2.solve(Fd))
    assert oracle.rel_err_rows(X2, ref, off).max() <= 1e-12
    # a series plan gets its own entry
    sp = tdt.Plan(-1.0, 3.0, -1.0, 20000, "f64")
    Fs = to_dev(rng.standard_normal((2, 20000)))
    r3 = sp.autotune(Fs, force=True)
    assert r3["ms"] > 0
    assert len(json.loads(cache.read_text())["entries"]) == 2


def test_autotune_with_adjoint(tmp_path, monkeypatch):
    """TDT_TUNE_ADJOINT times each trial as a solve plus its adjoint, keeps
    its own cache entry, and leaves the plan at parity in both directions."""
    import json
    tdt = _tdt()
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("TDT_TUNE_CACHE", str(cache))
    rng = np.random.default_rng(6)
    sizes = np.array([16384, 16384, 700, 40000])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    tm1, t0, t1 = rng.uniform(-1, -0.5, 4), rng.uniform(2.5, 4.0, 4), rng.uniform(-1, -0.5, 4)
    F = rng.standard_normal(int(off[-1]))
    G = rng.standard_normal(int(off[-1]))
    plan = tdt.VarlenPlan(off, tm1, t0, t1, "f64")
    Fd = to_dev(F)
    res = plan.autotune(Fd, adjoint=True)
    assert res["ms"] > 0
    (key, _), = json.loads(cache.read_text())["entries"].items()
    assert key.endswith("|adj")
    X = plan.solve(Fd)
    gF, gt = plan.backward(to_dev(G), X)
    Xr = oracle.solve_varlen(F, off, tm1, t0, t1)
    gFr, gtr = oracle.adjoint_varlen(G, Xr, off, tm1, t0, t1)
    assert oracle.rel_err_rows(to_host(X), Xr, off).max() <= 1e-12
    assert oracle.rel_err_rows(to_host(gF), gFr, off).max() <= 1e-12
    assert np.max(np.abs(to_host(gt) - gtr) / np.maximum(1.0, np.abs(gtr))) <= 1e-11
