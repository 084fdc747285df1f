"""Pins of the CPU oracle to facts outside itself.

Each ``pin_*`` function takes an oracle binding (``oracle`` itself, or a copy
compiled from a deliberately broken source) and raises AssertionError when the
oracle disagrees with what the paper or the mathematics fixes:

  * pin_dense_ge       brute force: dense Gaussian elimination with partial
                       pivoting (LAPACK via numpy) on N <= 64, nonsymmetric t's;
  * pin_eigenpairs     closed form: T v_j = lambda_j v_j with
                       v_j(i) = (t-1/t1)^(i/2) sin(i j pi/(N+1)),
                       lambda_j = t0 + 2 sgn(t1) sqrt(t1 t-1) cos(j pi/(N+1));
  * pin_theorem1       Theorem 1 (Sec. 3.1) evaluated in 40-digit arithmetic,
                       with the sign reading recorded in the design notes
                       (as printed the formula yields -T^{-1} f);
  * pin_chebyshev      the Chebyshev form of Sec. 3.2 for tridiag{-1, 2x, -1};
  * pin_manufactured   draw X*, form F = T X* with a three-point stencil;
  * pin_special        t_{+-1} = 0 gives F / t0 exactly, N = 1, N = 2 by the
                       explicit 2x2 inverse, equal right-hand sides give equal
                       solutions, varlen equals one-by-one solves;
  * pin_long_double    the long double variant on a nearly singular system,
                       against the eigen-pair closed form;
  * pin_adjoint        gF against a dense solve with T^T, dL/dt against central
                       finite differences (step 1e-6) and the closed form at
                       t_{+-1} = 0;
  * pin_quasi          the quasi-Toeplitz matrices of eq. (21) (t0+psi, t0+chi
                       in the corners): dense elimination, the closed-form
                       eigenpairs of the Neumann (psi = chi = -1, cosine
                       vectors) and half-point Dirichlet (psi = chi = +1, sine
                       vectors) matrices, N = 1 and 2, manufactured solutions,
                       varlen, and the adjoint with dL/dpsi, dL/dchi against a
                       dense transposed solve and central differences.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np


def dense_T(n, a, b, c, psi=0.0, chi=0.0):
    """Dense Toeplitz tridiagonal matrix: a below, b on, c above the diagonal;
    psi and chi added to the first and last diagonal entry (eq. (21))."""
    T = np.diag(np.full(n, float(b)))
    if n > 1:
        T += np.diag(np.full(n - 1, float(c)), 1) + np.diag(np.full(n - 1, float(a)), -1)
    T[0, 0] += psi
    T[-1, -1] += chi
    return T


def stencil(x, a, b, c):
    """F = T x for T = tridiag{a, b, c} (x: [..., N])."""
    f = b * x
    f[..., 1:] += a * x[..., :-1]
    f[..., :-1] += c * x[..., 1:]
    return f


def _rand_t(rng, ratio_lo, ratio_hi):
    a = rng.uniform(0.2, 1.0) * rng.choice([-1, 1])
    c = rng.uniform(0.2, 1.0) * rng.choice([-1, 1])
    b = rng.uniform(ratio_lo, ratio_hi) * (abs(a) + abs(c)) * rng.choice([-1, 1])
    return a, b, c


def _relerr(x, y):
    return float(np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300))


def pin_dense_ge(orc, seed=1):
    rng = np.random.default_rng(seed)
    for n in (1, 2, 3, 5, 8, 13, 32, 64):
        for _ in range(6):
            a, b, c = _rand_t(rng, 1.0, 3.0)
            F = rng.standard_normal((3, n))
            X = orc.solve(F, a, b, c)
            ref = np.linalg.solve(dense_T(n, a, b, c), F.T).T
            assert _relerr(X, ref) < 1e-13, (n, a, b, c, _relerr(X, ref))
    # weaker dominance and non-dominant systems: tolerance scaled by cond
    for n in (4, 17, 40):
        for _ in range(4):
            a, b, c = _rand_t(rng, 0.6, 1.0)
            T = dense_T(n, a, b, c)
            kappa = np.linalg.cond(T, np.inf)
            if kappa > 1e6:
                continue
            F = rng.standard_normal((2, n))
            X = orc.solve(F, a, b, c)
            ref = np.linalg.solve(T, F.T).T
            assert _relerr(X, ref) < 200 * kappa * 2.2e-16, (n, a, b, c)


def pin_eigenpairs(orc, seed=2):
    rng = np.random.default_rng(seed)
    for n in (7, 50, 200):
        for sgn in (1.0, -1.0):
            a = sgn * rng.uniform(0.3, 1.0)
            c = sgn * rng.uniform(0.3, 1.0)
            b = rng.uniform(1.2, 2.5) * (abs(a) + abs(c)) * rng.choice([-1, 1])
            r = math.sqrt(a / c)
            i = np.arange(1, n + 1)
            for j in (1, 2, n // 2 + 1, n):
                th = j * math.pi / (n + 1)
                v = r ** i * np.sin(i * th)
                lam = b + 2.0 * math.copysign(1.0, c) * math.sqrt(a * c) * math.cos(th)
                x = orc.solve(v, a, b, c)
                assert _relerr(x, v / lam) < 1e-12, (n, a, b, c, j)


def theorem1_solution(f, t_m1, t_0, t_1, dps=40):
    """Theorem 1 of Sec. 3.1 in mpmath with the sign reading applied: the
    printed weights multiply f_k / t_1; the solution of T y = f is obtained
    with -f_k / t_1 (checked at N = 1: the printed form gives -f_1 / t_0)."""
    with mpmath.workdps(dps):
        n_ = len(f)
        a, b, c = mpmath.mpf(t_m1), mpmath.mpf(t_0), mpmath.mpf(t_1)
        disc = mpmath.sqrt(mpmath.mpc(b * b - 4 * a * c))
        q1 = (-b + disc) / (2 * c)
        q2 = (-b - disc) / (2 * c)
        N = n_
        den = (q2 - q1) * (q2 ** (N + 1) - q1 ** (N + 1))
        y = []
        for n in range(1, N + 1):
            s = mpmath.mpc(0)
            for k in range(1, n):
                w = (q1 * q2) ** (n - k) * (q2 ** (N + 1 - n) - q1 ** (N + 1 - n)) * (q2 ** k - q1 ** k)
                s += w / den * (-mpmath.mpf(f[k - 1]) / c)
            for k in range(n, N + 1):
                w = (q2 ** (N + 1 - k) - q1 ** (N + 1 - k)) * (q2 ** n - q1 ** n)
                s += w / den * (-mpmath.mpf(f[k - 1]) / c)
            y.append(s)
        return np.array([float(mpmath.re(v)) for v in y]), np.array([float(mpmath.im(v)) for v in y])


def pin_theorem1(orc, seed=3):
    rng = np.random.default_rng(seed)
    cases = []
    for n in (1, 2, 3, 7, 12):
        cases.append((n,) + _rand_t(rng, 1.05, 2.5))      # real distinct roots
    cases.append((9, 0.8, 1.0, 0.9))                       # complex roots (b^2 < 4ac)
    cases.append((6, -0.5, 1.1, 0.7))                      # a c < 0
    for n, a, b, c in cases:
        f = rng.standard_normal(n)
        y_re, y_im = theorem1_solution(f, a, b, c)
        x = orc.solve(f, a, b, c)
        kappa = np.linalg.cond(dense_T(n, a, b, c), np.inf)
        assert np.max(np.abs(y_im)) < 1e-25 * max(1.0, np.max(np.abs(y_re))) + 1e-20
        assert _relerr(x, y_re) < 50 * kappa * 2.2e-16, (n, a, b, c, _relerr(x, y_re))


def chebyshev_solution(g, x, dps=40):
    """Sec. 3.2: for tridiag{-1, 2x, -1} y = g (N - 1 unknowns, zero ends),
    y_n = U_{N-n-1}/U_{N-1} sum_{k<n} U_{k-1} g_k + U_{n-1}/U_{N-1} sum_{k>=n} U_{N-k-1} g_k."""
    with mpmath.workdps(dps):
        N = len(g) + 1
        xx = mpmath.mpf(x)
        U = lambda m: mpmath.chebyu(m, xx)
        UN1 = U(N - 1)
        y = []
        for n in range(1, N):
            s1 = mpmath.fsum(U(k - 1) * mpmath.mpf(g[k - 1]) for k in range(1, n))
            s2 = mpmath.fsum(U(N - k - 1) * mpmath.mpf(g[k - 1]) for k in range(n, N))
            y.append(U(N - n - 1) / UN1 * s1 + U(n - 1) / UN1 * s2)
        return np.array([float(v) for v in y])


def pin_chebyshev(orc, seed=4):
    rng = np.random.default_rng(seed)
    for n_unknowns, x in ((5, 1.5), (20, 1.02), (31, 3.0), (12, 0.9)):
        g = rng.standard_normal(n_unknowns)
        ref = chebyshev_solution(g, x)
        y = orc.solve(g, -1.0, 2.0 * x, -1.0)
        kappa = np.linalg.cond(dense_T(n_unknowns, -1.0, 2.0 * x, -1.0), np.inf)
        assert _relerr(y, ref) < 50 * kappa * 2.2e-16, (n_unknowns, x)


def pin_manufactured(orc, seed=5):
    rng = np.random.default_rng(seed)
    for n, (a, b, c) in ((1000, (-1.0, 4.0, -1.0)), (777, (-0.9, 2.5, -1.1)),
                         (513, (0.7, -1.9, 0.45))):
        X_true = rng.uniform(-1.0, 1.0, size=(2, n))
        F = stencil(X_true, a, b, c)
        X = orc.solve(F, a, b, c)
        assert _relerr(X, X_true) < 1e-14, (n, a, b, c, _relerr(X, X_true))


def pin_special(orc, seed=6):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((2, 33))
    assert np.array_equal(orc.solve(F, 0.0, 2.5, 0.0), F / 2.5)
    f1 = rng.standard_normal(1)
    assert np.array_equal(orc.solve(f1, 0.3, -1.7, 0.2), f1 / -1.7)
    a, b, c = 0.4, 1.3, -0.6
    f2 = rng.standard_normal(2)
    det = b * b - a * c
    ref = np.array([b * f2[0] - c * f2[1], -a * f2[0] + b * f2[1]]) / det
    assert _relerr(orc.solve(f2, a, b, c), ref) < 1e-15
    row = rng.standard_normal(50)
    X = orc.solve(np.stack([row, row, row]), -0.3, 1.1, 0.5)
    assert np.array_equal(X[0], X[1]) and np.array_equal(X[1], X[2])
    sizes = np.array([5, 1, 64, 2, 17])
    off = np.concatenate([[0], np.cumsum(sizes)])
    tm1 = rng.uniform(-1, -0.2, 5)
    t1 = rng.uniform(0.2, 1, 5)
    t0 = 2.2 * np.ones(5)
    Fp = rng.standard_normal(int(off[-1]))
    Xp = orc.solve_varlen(Fp, off, tm1, t0, t1)
    for s in range(5):
        xs = orc.solve(Fp[off[s]:off[s + 1]], tm1[s], t0[s], t1[s])
        assert np.array_equal(Xp[off[s]:off[s + 1]], xs)


def chebyshev_solution_fast(g, x, dps=60):
    """The same Chebyshev form as ``chebyshev_solution`` with the U_k taken
    from their defining three-term recurrence and the two sums as running
    sums (O(N) instead of O(N^2) high-precision operations)."""
    with mpmath.workdps(dps):
        N = len(g) + 1
        xx = mpmath.mpf(x)
        U = [mpmath.mpf(1), 2 * xx]
        for _ in range(2, N + 1):
            U.append(2 * xx * U[-1] - U[-2])
        gm = [mpmath.mpf(v) for v in g]
        s1 = [mpmath.mpf(0)] * (N + 1)      # s1[n] = sum_{k<n} U_{k-1} g_k
        for k in range(1, N):
            s1[k + 1] = s1[k] + U[k - 1] * gm[k - 1]
        s2 = [mpmath.mpf(0)] * (N + 1)      # s2[n] = sum_{k>=n} U_{N-k-1} g_k
        for k in range(N - 1, 0, -1):
            s2[k] = s2[k + 1] + U[N - k - 1] * gm[k - 1]
        return np.array([float((U[N - n - 1] * s1[n] + U[n - 1] * s2[n]) / U[N - 1])
                         for n in range(1, N)])


def pin_long_double(orc):
    # nearly singular symmetric system T = tridiag{1, b, 1}, lambda_min ~ 1e-7
    # (cond ~ 4e7): against the Chebyshev closed form of Sec. 3.2 in 60 digits
    # (T = -tridiag{-1, -b, -1}, so x = -y(x = -b/2)).  The long double result
    # must reach ~1e-15; the double one is limited by cond * 2^-53.
    n = 400
    with mpmath.workdps(40):
        b = float(-2 * mpmath.cos(mpmath.pi / (n + 1)) - mpmath.mpf("1e-7"))
    g = np.random.default_rng(9).standard_normal(n)
    ref = -chebyshev_solution_fast(g, -b / 2.0)
    e_ld = _relerr(orc.solve(g, 1.0, b, 1.0, precision="ld"), ref)
    e_64 = _relerr(orc.solve(g, 1.0, b, 1.0), ref)
    assert e_ld < 1e-13 and e_ld < e_64 / 100.0, (e_ld, e_64)
    # an independent well-conditioned case: both precisions agree to rounding
    rng = np.random.default_rng(7)
    F = rng.standard_normal((2, 300))
    assert _relerr(orc.solve(F, -1.0, 3.0, -0.5, precision="ld"),
                   orc.solve(F, -1.0, 3.0, -0.5)) < 1e-15


def pin_adjoint(orc, seed=8):
    rng = np.random.default_rng(seed)
    n, m = 40, 3
    a, b, c = -0.7, 2.3, -0.9
    F = rng.standard_normal((m, n))
    W = rng.standard_normal((m, n))
    X = orc.solve(F, a, b, c)
    gF, gt = orc.adjoint(W, X, a, b, c)
    ref_gF = np.linalg.solve(dense_T(n, a, b, c).T, W.T).T
    assert _relerr(gF, ref_gF) < 1e-13
    h = 1e-6

    def loss(a_, b_, c_):
        return float(np.sum(W * np.linalg.solve(dense_T(n, a_, b_, c_), F.T).T))

    fd = np.array([(loss(a + h, b, c) - loss(a - h, b, c)) / (2 * h),
                   (loss(a, b + h, c) - loss(a, b - h, c)) / (2 * h),
                   (loss(a, b, c + h) - loss(a, b, c - h)) / (2 * h)])
    assert np.max(np.abs(gt - fd)) < 1e-6 * max(1.0, np.max(np.abs(fd))), (gt, fd)
    # closed form with t_{+-1} = 0: X = F / t0
    t0 = 1.7
    X0 = orc.solve(F, 0.0, t0, 0.0)
    gF0, gt0 = orc.adjoint(W, X0, 0.0, t0, 0.0)
    assert np.allclose(gF0, W / t0, rtol=1e-15, atol=0)
    ref_t0 = -np.sum(W * F) / t0 ** 2
    ref_t1 = -np.sum(W[:, :-1] * F[:, 1:]) / t0 ** 2
    ref_tm1 = -np.sum(W[:, 1:] * F[:, :-1]) / t0 ** 2
    assert abs(gt0[1] - ref_t0) < 1e-12 * max(1, abs(ref_t0))
    assert abs(gt0[2] - ref_t1) < 1e-12 * max(1, abs(ref_t1))
    assert abs(gt0[0] - ref_tm1) < 1e-12 * max(1, abs(ref_tm1))
    # varlen adjoint: one triple per system equals the single-system adjoint
    sizes = np.array([12, 30, 7])
    off = np.concatenate([[0], np.cumsum(sizes)])
    tm1 = np.array([-0.7, 0.4, -0.2])
    tt0 = np.array([2.3, -1.9, 1.1])
    tt1 = np.array([-0.9, 0.6, 0.5])
    Fp = rng.standard_normal(int(off[-1]))
    Wp = rng.standard_normal(int(off[-1]))
    Xp = orc.solve_varlen(Fp, off, tm1, tt0, tt1)
    gFp, gtp = orc.adjoint_varlen(Wp, Xp, off, tm1, tt0, tt1)
    for s in range(3):
        sl = slice(off[s], off[s + 1])
        g1, t1s = orc.adjoint(Wp[sl], Xp[sl], tm1[s], tt0[s], tt1[s])
        assert np.allclose(gFp[sl], g1, rtol=1e-15, atol=0)
        assert np.allclose(gtp[s], t1s, rtol=1e-14, atol=0)
        ref = np.linalg.solve(dense_T(sizes[s], tm1[s], tt0[s], tt1[s]).T, Wp[sl])
        assert _relerr(gFp[sl], ref) < 1e-13


def pin_quasi(orc, seed=10):
    rng = np.random.default_rng(seed)
    # dense elimination, both corners, including N = 1 (one entry t0+psi+chi)
    for n in (1, 2, 3, 5, 13, 40):
        for _ in range(4):
            a, b, c = _rand_t(rng, 1.2, 3.0)
            psi, chi = rng.uniform(-0.5, 0.5, 2) * abs(b)
            F = rng.standard_normal((2, n))
            X = orc.solve(F, a, b, c, psi=psi, chi=chi)
            ref = np.linalg.solve(dense_T(n, a, b, c, psi, chi), F.T).T
            assert _relerr(X, ref) < 1e-13, (n, psi, chi, _relerr(X, ref))
    # N = 2: the explicit inverse of [[b+psi, c], [a, b+chi]]
    a, b, c, psi, chi = -0.6, 2.1, 0.8, 0.3, -0.45
    f = np.array([0.7, -1.3])
    d = (b + psi) * (b + chi) - a * c
    x2 = np.array([(b + chi) * f[0] - c * f[1], -a * f[0] + (b + psi) * f[1]]) / d
    assert _relerr(orc.solve(f, a, b, c, psi=psi, chi=chi), x2) < 1e-15
    # closed-form eigenpairs (t0 = 2 + eps, t_{+-1} = -1)
    n, eps = 37, 0.05
    i = np.arange(n)
    for psi, trig, ks in ((-1.0, np.cos, range(0, n)), (1.0, np.sin, range(1, n + 1))):
        for k in ks:
            v = trig(np.pi * k * (i + 0.5) / n)
            lam = eps + 4.0 * math.sin(math.pi * k / (2 * n)) ** 2
            x = orc.solve(v, -1.0, 2.0 + eps, -1.0, psi=psi, chi=psi)
            assert _relerr(x, v / lam) < 1e-12, (psi, k, _relerr(x, v / lam))
    # manufactured solution
    a, b, c, psi, chi = -0.8, 2.6, -1.1, 0.9, -0.7
    Xs = rng.uniform(-1, 1, (3, 500))
    F = stencil(Xs.copy(), a, b, c)
    F[:, 0] += psi * Xs[:, 0]
    F[:, -1] += chi * Xs[:, -1]
    assert _relerr(orc.solve(F, a, b, c, psi=psi, chi=chi), Xs) < 1e-13
    # varlen with per-system corners equals one-by-one solves and dense ones
    sizes = np.array([3, 17, 1, 40])
    off = np.concatenate([[0], np.cumsum(sizes)])
    ts = [_rand_t(rng, 1.2, 3.0) for _ in sizes]
    tm1, t0, t1 = (np.array([t[k] for t in ts]) for k in range(3))
    ps = rng.uniform(-0.4, 0.4, len(sizes))
    ch = rng.uniform(-0.4, 0.4, len(sizes))
    Fp = rng.standard_normal(int(off[-1]))
    Xp = orc.solve_varlen(Fp, off, tm1, t0, t1, psi=ps, chi=ch)
    for s in range(len(sizes)):
        sl = slice(off[s], off[s + 1])
        ref = np.linalg.solve(dense_T(sizes[s], tm1[s], t0[s], t1[s], ps[s], ch[s]), Fp[sl])
        assert _relerr(Xp[sl], ref) < 1e-13, s
    # adjoint: gF = A^{-T} gX and (dL/dt-1, dL/dt0, dL/dt1, dL/dpsi, dL/dchi)
    n, m = 30, 2
    a, b, c, psi, chi = -0.7, 2.3, -0.9, 0.6, -0.4
    F = rng.standard_normal((m, n))
    W = rng.standard_normal((m, n))
    X = orc.solve(F, a, b, c, psi=psi, chi=chi)
    gF, gt = orc.adjoint(W, X, a, b, c, psi=psi, chi=chi, corners=True)
    assert gt.shape == (5,)
    ref_gF = np.linalg.solve(dense_T(n, a, b, c, psi, chi).T, W.T).T
    assert _relerr(gF, ref_gF) < 1e-13
    h = 1e-6

    def loss(a_, b_, c_, p_, q_):
        return float(np.sum(W * np.linalg.solve(dense_T(n, a_, b_, c_, p_, q_), F.T).T))

    base = np.array([a, b, c, psi, chi])
    fd = []
    for k in range(5):
        e = np.zeros(5)
        e[k] = h
        fd.append((loss(*(base + e)) - loss(*(base - e))) / (2 * h))
    fd = np.array(fd)
    assert np.max(np.abs(gt - fd)) < 1e-6 * max(1.0, np.max(np.abs(fd))), (gt, fd)
    gFp, gtp = orc.adjoint_varlen(Fp, Xp, off, tm1, t0, t1, psi=ps, chi=ch, corners=True)
    for s in range(len(sizes)):
        sl = slice(off[s], off[s + 1])
        g1, t1s = orc.adjoint(Fp[sl], Xp[sl], tm1[s], t0[s], t1[s], psi=ps[s], chi=ch[s],
                              corners=True)
        assert np.allclose(gFp[sl], g1, rtol=1e-15, atol=0) and np.allclose(gtp[s], t1s)


def dense_general(a, b, c):
    """Dense tridiagonal matrix with rows (a_i, b_i, c_i); a_0, c_{N-1} unused."""
    n = len(b)
    A = np.diag(np.asarray(b, dtype=float))
    if n > 1:
        A += np.diag(np.asarray(a[1:], dtype=float), -1) + np.diag(np.asarray(c[:-1], dtype=float), 1)
    return A


def random_rows(rng, n, ratio_lo=1.0, ratio_hi=3.0):
    """Rows whose |b_i| / (|a_i| + |c_i|) lies in [ratio_lo, ratio_hi], entries
    of both signs."""
    a = rng.uniform(0.2, 1.0, n) * rng.choice([-1.0, 1.0], n)
    c = rng.uniform(0.2, 1.0, n) * rng.choice([-1.0, 1.0], n)
    b = rng.uniform(ratio_lo, ratio_hi, n) * (np.abs(a) + np.abs(c)) * rng.choice([-1.0, 1.0], n)
    return a, b, c


def pin_general(orc, seed=11):
    """General tridiagonal matrices (per-row entries): dense elimination,
    N = 1 and 2 in closed form, a manufactured solution, zero off-diagonals,
    constant rows against the Toeplitz solve, a nearly singular case against
    mpmath for the long double variant, and the adjoint against the dense
    transposed solve and central differences of every entry class."""
    rng = np.random.default_rng(seed)
    for n in (1, 2, 3, 7, 16, 40, 64):
        for _ in range(4):
            a, b, c = random_rows(rng, n)
            F = rng.standard_normal((3, n))
            X = orc.solve_general(F, a, b, c)
            ref = np.linalg.solve(dense_general(a, b, c), F.T).T
            assert _relerr(X, ref) < 1e-13, (n, _relerr(X, ref))
    # N = 1, N = 2
    assert orc.solve_general(np.array([0.7]), [0.3], [-2.0], [0.9])[0] == 0.7 / -2.0
    a, b, c = [0.0, -0.6], [2.1, 1.7], [0.8, 0.0]
    f = np.array([0.7, -1.3])
    d = b[0] * b[1] - c[0] * a[1]
    x2 = np.array([b[1] * f[0] - c[0] * f[1], -a[1] * f[0] + b[0] * f[1]]) / d
    assert _relerr(orc.solve_general(f, a, b, c), x2) < 1e-15
    # manufactured solution
    a, b, c = random_rows(rng, 500, 1.2, 2.5)
    Xs = rng.uniform(-1, 1, (2, 500))
    F = (dense_general(a, b, c) @ Xs.T).T
    assert _relerr(orc.solve_general(F, a, b, c), Xs) < 1e-13
    # zero off-diagonals: x = f / b exactly
    b = rng.uniform(0.5, 2.0, 50) * rng.choice([-1.0, 1.0], 50)
    F = rng.standard_normal(50)
    assert np.array_equal(orc.solve_general(F, np.zeros(50), b, np.zeros(50)), F / b)
    # constant rows: the Toeplitz solve (same recurrence, bit for bit)
    F = rng.standard_normal((2, 300))
    assert np.array_equal(orc.solve_general(F, np.full(300, -0.8), np.full(300, 2.6),
                                            np.full(300, 1.1)),
                          orc.solve(F, -0.8, 2.6, 1.1))
    # long double: a nearly singular nonsymmetric matrix against mpmath
    n = 24
    a, b, c = random_rows(rng, n, 1.0, 1.5)
    A = dense_general(a, b, c)
    lam = np.linalg.eigvals(A)
    b = b - lam[np.argmin(np.abs(lam))].real + 1e-7     # shift next to an eigenvalue
    A = dense_general(a, b, c)
    g = rng.standard_normal(n)
    with mpmath.workdps(50):
        ref = np.array([float(v) for v in mpmath.lu_solve(mpmath.matrix(A.tolist()),
                                                          mpmath.matrix(g.tolist()))])
    e_ld = _relerr(orc.solve_general(g, a, b, c, precision="ld"), ref)
    e_64 = _relerr(orc.solve_general(g, a, b, c), ref)
    assert e_ld < 1e-11 and e_ld < e_64 / 100.0, (e_ld, e_64)
    # adjoint
    n, m = 30, 2
    a, b, c = random_rows(rng, n, 1.2, 2.5)
    F = rng.standard_normal((m, n))
    W = rng.standard_normal((m, n))
    X = orc.solve_general(F, a, b, c)
    gF, (ga, gb, gc) = orc.adjoint_general(W, X, a, b, c)
    A = dense_general(a, b, c)
    assert _relerr(gF, np.linalg.solve(A.T, W.T).T) < 1e-13
    assert ga[0] == 0.0 and gc[-1] == 0.0
    h = 1e-6

    def loss(a_, b_, c_):
        return float(np.sum(W * np.linalg.solve(dense_general(a_, b_, c_), F.T).T))

    for i in (1, 7, n - 1):
        ap, am = a.copy(), a.copy()
        ap[i] += h
        am[i] -= h
        fd = (loss(ap, b, c) - loss(am, b, c)) / (2 * h)
        assert abs(fd - ga[i]) <= 1e-6 * max(1.0, abs(fd)), ("a", i, fd, ga[i])
    for i in (0, 11, n - 1):
        bp, bm = b.copy(), b.copy()
        bp[i] += h
        bm[i] -= h
        fd = (loss(a, bp, c) - loss(a, bm, c)) / (2 * h)
        assert abs(fd - gb[i]) <= 1e-6 * max(1.0, abs(fd)), ("b", i, fd, gb[i])
    for i in (0, 13, n - 2):
        cp, cm = c.copy(), c.copy()
        cp[i] += h
        cm[i] -= h
        fd = (loss(a, b, cp) - loss(a, b, cm)) / (2 * h)
        assert abs(fd - gc[i]) <= 1e-6 * max(1.0, abs(fd)), ("c", i, fd, gc[i])


ALL_PINS = [pin_dense_ge, pin_eigenpairs, pin_theorem1, pin_chebyshev, pin_manufactured,
            pin_special, pin_long_double, pin_adjoint, pin_quasi, pin_general]
