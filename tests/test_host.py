"""Host-side checks of the C ABI library (no GPU): exported symbols, the
preliminary-step constants against dense inverses, the interface merge against
dense solves, and argument validation that happens before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle_pins import dense_T

import paper_1002_2469_amd as tdt
from paper_1002_2469_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "tdt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tdt_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    declared = _header_symbols()
    assert declared == sorted(_lib.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("t", [(-1.0, 4.0, -1.0), (-0.9, 2.5, -1.1), (0.7, -1.9, 0.45),
                               (1.0, -2.0000003, 1.0)])
@pytest.mark.parametrize("B", [1, 2, 5, 32])
def test_block_constants_match_dense_inverse(t, B):
    a, b, c = t
    k = tdt.block_constants(a, b, c, B)
    T = dense_T(B, a, b, c)
    Ti = np.linalg.inv(T)
    e0 = np.zeros(B); e0[0] = -a
    eB = np.zeros(B); eB[-1] = -c
    phi, chi = Ti @ e0, Ti @ eB
    scale = np.max(np.abs(Ti))
    assert np.allclose(k["phi"], phi, rtol=0, atol=1e-14 * max(1, scale))
    assert np.allclose(k["chi"], chi, rtol=0, atol=1e-14 * max(1, scale))
    # pivots u_k = det(T_k) / det(T_{k-1})
    dets = [1.0] + [np.linalg.det(T[:j, :j]) for j in range(1, B + 1)]
    piv = np.array([dets[j + 1] / dets[j] for j in range(B)])
    assert np.allclose(1.0 / k["inv_pivot"], piv, rtol=1e-12)
    assert np.allclose(k["cp"], c / piv, rtol=1e-12)
    assert np.allclose(k["ends"], [phi[0], phi[-1], chi[0], chi[-1]], rtol=0,
                       atol=1e-14 * max(1, scale))


def _dense_summary(f, a, b, c):
    n = len(f)
    T = dense_T(n, a, b, c)
    y = np.linalg.solve(T, f)
    e0 = np.zeros(n); e0[0] = -a
    en = np.zeros(n); en[-1] = -c
    phi, chi = np.linalg.solve(T, e0), np.linalg.solve(T, en)
    return np.array([y[0], y[-1], phi[0], phi[-1], chi[0], chi[-1]])


@pytest.mark.parametrize("t", [(-1.0, 4.0, -1.0), (-0.9, 2.5, -1.1), (0.5, 0.9, 0.7)])
@pytest.mark.parametrize("n1,n2", [(1, 1), (1, 7), (13, 2), (32, 32), (40, 23)])
def test_segment_merge_is_the_union_summary(t, n1, n2):
    a, b, c = t
    rng = np.random.default_rng(n1 * 100 + n2)
    f = rng.standard_normal(n1 + n2)
    left = _dense_summary(f[:n1], a, b, c)
    right = _dense_summary(f[n1:], a, b, c)
    merged = tdt.segment_merge(left, right)
    whole = _dense_summary(f, a, b, c)
    assert np.allclose(merged, whole, rtol=1e-11, atol=1e-12)


def test_empty_segment_is_the_merge_identity():
    """The segment of no rows (first row = the value right of it, last row =
    the value left of it: (0, 0, 0, 1, 1, 0)) leaves any segment unchanged on
    either side; the interface pass gives it to threads with no tiles, so that
    outside values pass through them."""
    rng = np.random.default_rng(11)
    E = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 0.0])
    for _ in range(20):
        s = rng.standard_normal(6) * 0.5
        assert np.array_equal(tdt.segment_merge(s, E), s)
        assert np.array_equal(tdt.segment_merge(E, s), s)
    assert np.array_equal(tdt.segment_merge(E, E), E)


def test_merge_associativity():
    a, b, c = -0.9, 2.5, -1.1
    rng = np.random.default_rng(5)
    f = rng.standard_normal(30)
    s = [_dense_summary(f[i:i + 10], a, b, c) for i in (0, 10, 20)]
    x = tdt.segment_merge(tdt.segment_merge(s[0], s[1]), s[2])
    y = tdt.segment_merge(s[0], tdt.segment_merge(s[1], s[2]))
    assert np.allclose(x, y, rtol=1e-13, atol=1e-15)


def test_argument_validation_without_device():
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.tdt_plan_create(-1.0, 4.0, -1.0, 0, 0, ctypes.byref(h)) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_plan_create(float("nan"), 4.0, -1.0, 10, 0, ctypes.byref(h)) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_plan_create(-1.0, 4.0, -1.0, 10, 7, ctypes.byref(h)) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_plan_create(-1.0, 4.0, -1.0, 10, 0, None) == _lib.TDT_ERR_INVALID_ARG
    off = np.array([0, 5, 5], dtype=np.int64)      # an empty system
    t3 = np.ones(2)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert L.tdt_plan_varlen_create(2, p(off), p(t3), p(t3), p(t3), 0, ctypes.byref(h)) == \
        _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_solve(None, None, None, 1, None) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_solve_varlen(None, None, None, None) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_solve_backward(None, None, None, None, None, 1, None) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_plan_reserve(None, 1) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_plan_destroy(None) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_last_info(None, None, None, None, None) == _lib.TDT_ERR_INVALID_ARG
    # quasi-Toeplitz plans: N >= 3, finite corner terms, both corner arrays
    assert L.tdt_plan_quasi_create(-1.0, 4.0, -1.0, 0.5, 0.5, 2, 0, ctypes.byref(h)) == \
        _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_plan_quasi_create(-1.0, 4.0, -1.0, float("inf"), 0.5, 10, 0,
                                   ctypes.byref(h)) == _lib.TDT_ERR_INVALID_ARG
    assert L.tdt_plan_quasi_create(-1.0, 4.0, -1.0, 0.5, float("nan"), 10, 0,
                                   ctypes.byref(h)) == _lib.TDT_ERR_INVALID_ARG
    offq = np.array([0, 5, 7], dtype=np.int64)     # a system of 2 rows
    assert L.tdt_plan_varlen_quasi_create(2, p(offq), p(t3), p(t3), p(t3), p(t3), p(t3), 0,
                                          ctypes.byref(h)) == _lib.TDT_ERR_INVALID_ARG
    offq = np.array([0, 5, 8], dtype=np.int64)
    assert L.tdt_plan_varlen_quasi_create(2, p(offq), p(t3), p(t3), p(t3), None, p(t3), 0,
                                          ctypes.byref(h)) == _lib.TDT_ERR_INVALID_ARG
    # strided plans: 1 <= N <= 2^24, P >= 1, finite entries, f64 only; a zero
    # block pivot is found on the host
    tm, t0s, tp = -np.ones(3), np.full(3, 4.0), -np.ones(3)
    for n, P_, dt in ((0, 3, 0), (2**24 + 1, 3, 0), (10, 0, 0), (10, 3, 1), (10, 3, 2)):
        assert L.tdt_plan_strided_create(n, P_, p(tm), p(t0s), p(tp), dt, ctypes.byref(h)) == \
            _lib.TDT_ERR_INVALID_ARG, (n, P_, dt)
    bad = np.array([4.0, float("nan"), 4.0])
    assert L.tdt_plan_strided_create(10, 3, p(tm), p(bad), p(tp), 0, ctypes.byref(h)) == \
        _lib.TDT_ERR_INVALID_ARG
    sing = np.array([4.0, 0.0, 4.0])
    assert L.tdt_plan_strided_create(10, 3, p(tm), p(sing), p(tp), 0, ctypes.byref(h)) == \
        _lib.TDT_ERR_SINGULAR
    assert L.tdt_solve_strided(None, None, None, 1, 1, 1, 0, None) == _lib.TDT_ERR_INVALID_ARG
    out = np.empty(4 * 3 + 4)
    assert L.tdt_block_constants(1.0, 0.0, 1.0, 3, p(out)) == _lib.TDT_ERR_SINGULAR
    assert L.tdt_block_constants(1.0, 2.0, 1.0, 65, p(out)) == _lib.TDT_ERR_INVALID_ARG


def test_status_strings():
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert _lib.status_string(code) not in ("", "unknown status")
    assert _lib.status_string(42) == "unknown status"


def test_product_path_has_no_oracle_or_fallback():
    """The package never imports the oracle, and raises if the library is missing."""
    pkg = os.path.join(ROOT, "paper_1002_2469_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn
    saved, _lib._lib = _lib._lib, None
    real = _lib.LIB_PATH
    try:
        _lib.LIB_PATH = real + ".missing"
        with pytest.raises(RuntimeError):
            _lib.lib()
    finally:
        _lib.LIB_PATH = real
        _lib._lib = saved


@pytest.mark.parametrize("t", [(-1.0, 4.0, -1.0), (-0.9, 2.5, -1.1), (0.7, -1.9, 0.45)])
@pytest.mark.parametrize("L", [1, 2, 7, 64])
def test_green_rows_match_dense_inverse(t, L):
    a, b, c = t
    first, last = tdt.green_rows(a, b, c, L)
    Ti = np.linalg.inv(dense_T(L, a, b, c))
    assert np.allclose(first, Ti[0], rtol=1e-13, atol=1e-15)
    assert np.allclose(last, Ti[-1], rtol=1e-13, atol=1e-15)


def test_adi_parameters_match_the_oracle():
    """The 3D solve's ADI parameters (long double AGM for K and dn, host
    side) against the oracle's (mpmath elliptic functions), and their bound;
    b/a up to 1e6 covers grids of up to 1024 points per side."""
    import paper_1002_2469_amd as tdt
    from oracle import poisson3d as P3
    for a, b in ((1.0, 1.0), (1.0, 3.0), (2.5, 1e3), (14.8, 1.05e6)):
        for J in (1, 2, 7, 16, 41):
            om, d = tdt.adi_parameters(a, b, J)
            ref = P3.adi_parameters(a, b, J)
            assert np.allclose(om, ref, rtol=2e-14, atol=0), (a, b, J)
            dref = abs(P3.adi_factor(ref, a))
            # d = prod_j |w_j - a| / (w_j + a): a relative change e in w_j moves
            # it by e w_j (1/|w_j - a| + 1/(w_j + a)); the reference parameters
            # carry double rounding (e <= u), amplified most where w_j nears a
            amp = float(np.sum(ref / np.abs(ref - a) + ref / (ref + a))) if a != b else 0.0
            tol = 16 * 2.0 ** -53 * max(amp, 1.0) * dref
            assert abs(d - dref) <= tol or (a == b and d == 0.0), (a, b, J, d, dref, tol)
    L = _lib.lib()
    out = np.zeros(4)
    p = out.ctypes.data_as(ctypes.c_void_p)
    for a, b, J in ((0.0, 1.0, 2), (2.0, 1.0, 2), (1.0, 2.0, 0), (1.0, 2.0, 401)):
        assert L.tdt_adi_parameters(a, b, J, p, None) == _lib.TDT_ERR_INVALID_ARG


@pytest.mark.parametrize("t", [(-0.9, 2.5, -1.1), (-1.1, 2.5, -0.9), (-1.0, 4.0, -1.0),
                               (-1.0, 2.01, -1.0), (0.3, -1.0, 0.45), (1.0, -2.0000006, 1.0)])
@pytest.mark.parametrize("L", [8192, 4096, 1000, 3])
def test_green_support_against_oracle_rows(t, L):
    """The supports of the first and last Green rows (Sec. 3.4's decay of the
    inverse's entries): the dropped entries' 1-norm is at most 2^-60 of the
    row's, and one entry fewer would drop more.  The rows come from the
    oracle's long double solves of T^T r = e_0 and T^T r = e_{L-1}."""
    import oracle
    a, b, c = t
    kf, kl = tdt.green_support(a, b, c, L)
    assert 1 <= kf <= L and 1 <= kl <= L
    E = np.zeros((2, L))
    E[0, 0] = 1.0
    E[1, -1] = 1.0
    R = np.abs(oracle.solve(E, c, b, a, precision="ld"))   # T^T = tridiag{c, b, a}
    r1, r2 = R[0], R[1][::-1]          # both now decay away from index 0
    drop = 2.0 ** -60
    for k, r in ((kf, r1), (kl, r2)):
        tail = np.concatenate([np.cumsum(r[::-1])[::-1], [0.0]])   # tail[j] = sum_{i >= j}
        n1 = tail[0]
        assert tail[k] <= drop * n1 * (1 + 1e-6), (k, tail[k] / n1)
        if k > 1:
            assert tail[k - 1] > drop * n1 * (1 - 1e-6), (k, tail[k - 1] / n1)


def test_green_support_headline_matrix():
    """For the matrix of the single-system workload the first Green row falls
    by 0.548 per entry and the last by 0.448 (1/q_1 and q_2 for the roots
    q_1 = 1.824, q_2 = 0.448 of t_1 q^2 + t_0 q + t_-1 = 0): 2^-60 of the
    mass is left after 70 and 52 entries."""
    assert tdt.green_support(-0.9, 2.5, -1.1, 8192) == (70, 52)
    assert tdt.green_support(-1.1, 2.5, -0.9, 8192) == (52, 70)
    assert tdt.green_support(1.0, -2.0, 1.0, 8192) == (8192, 8192)   # singular in the limit


def test_poisson2d_refinement_refused_before_any_device_call():
    """The 2D Poisson handle refuses float sweeps with refinement where the
    lowest mode's cond_2 (closed form, 1.4e7 at 8191 x 8191) is above the
    contraction limit; the check runs on the host before any allocation."""
    L = _lib.lib()
    h = ctypes.c_void_p()
    st = L.tdt_poisson2d_create(8191, 8191, 1.0 / 8192, 1.0 / 8192, _lib.DTYPES["f32_refine"],
                                ctypes.byref(h))
    assert st == _lib.TDT_ERR_NOT_CONVERGED and not h.value


@pytest.mark.parametrize("t", [(-0.9, 2.5, -1.1), (-1.0, 2.01, -1.0), (0.3, -1.0, 0.45),
                               (-0.5, -3.2, 0.7), (1.0, -18.0, 1.0), (1.0, -2.0000006, 1.0)])
@pytest.mark.parametrize("L", [8192, 4096])
def test_green_support_bound_against_oracle_rows(t, L):
    """The supports a varlen plan derives from the pivots' decay, without
    forming the rows: at least the minimal ones, dropping at most 2^-60 of
    each row's 1-norm (rows from the oracle's long double solves); none for
    the nearly singular matrix, whose rows do not decay within the tile."""
    import oracle
    a, b, c = t
    (kf, kl), (bf, bl) = tdt.green_support(a, b, c, L, bound=True)
    if b == -2.0000006:
        assert (bf, bl) == (0, 0)
        return
    assert bf >= kf and bl >= kl
    E = np.zeros((2, L))
    E[0, 0] = 1.0
    E[1, -1] = 1.0
    R = np.abs(oracle.solve(E, c, b, a, precision="ld"))
    for k, r in ((bf, R[0]), (bl, R[1][::-1])):
        assert r[k:].sum() <= 2.0 ** -60 * r.sum() * (1 + 1e-6), (k, r[k:].sum() / r.sum())


@pytest.mark.parametrize("t", [(-0.9, 2.5, -1.1), (-1.0, 2.01, -1.0), (0.3, -1.0, 0.45),
                               (-0.5, -3.2, 0.7)])
def test_green_support_entries_of_shorter_tiles(t):
    """A varlen plan's last tile, shorter than a tile, is summarised with the
    full tile's support entries when it is long enough that the entries
    under the supports involve only settled pivots: the first rows of T_n
    and T_L (and the last rows) agree there once n exceeds the supports by
    the pivots' settling length (a few hundred rows at most for these
    matrices).  Rows from the oracle's long double solves."""
    import oracle
    a, b, c = t
    L = 8192
    _, (bf, bl) = tdt.green_support(a, b, c, L, bound=True)
    rf, rl = -(-bf // 64) * 64, -(-bl // 64) * 64

    def rows(n):
        E = np.zeros((2, n))
        E[0, 0] = 1.0
        E[1, -1] = 1.0
        R = oracle.solve(E, c, b, a, precision="ld")   # T^T = tridiag{c, b, a}
        return R[0], R[1]

    f_L, l_L = rows(L)
    for n in (max(rf, rl) + 300, 2500, L - 1):
        f, l = rows(n)
        assert np.max(np.abs(f[:rf] - f_L[:rf])) <= 1e-15 * np.max(np.abs(f_L)), (t, n)
        assert np.max(np.abs(l[-rl:] - l_L[-rl:])) <= 1e-15 * np.max(np.abs(l_L)), (t, n)
