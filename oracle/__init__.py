"""CPU oracle for the Toeplitz tridiagonal solve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or executes anything here, and this
package imports nothing from the product.

What it computes (the plain definition, see ``tdt_oracle.c``):
  * ``solve``         X = T^{-1} F, T = tridiag{t_-1, t_0, t_1} (paper, eq. (1)),
                      one or many right-hand sides sharing T (eq. (2), the
                      series case), by the Thomas algorithm in double or in
                      long double (rounded to double at the end);
  * ``solve_varlen``  many systems of different sizes, each with its own T;
  * ``adjoint``       gF = T^{-T} gX and dL/dt for L = <W, X> (the transposed
                      solve is the (A^T)^{-1} = (A^{-1})^T remark of Sec. 2.3).

Error measure used across the project (not in the paper): the normwise
relative error max_i |x_i - x*_i| / max_i |x*_i| per right-hand side or system,
maximised over them (``rel_err``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tdt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain C, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
            "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _bind(path: str):
    lib = ctypes.CDLL(path)
    d, i64, i32, p = ctypes.c_double, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    lib.oracle_solve.argtypes = [d, d, d, d, d, i64, i64, p, p, i32, i32]
    lib.oracle_solve_varlen.argtypes = [i64, p, p, p, p, p, p, p, p, i32, i32]
    lib.oracle_adjoint.argtypes = [d, d, d, d, d, i64, i64, p, p, p, p, i32]
    lib.oracle_adjoint_varlen.argtypes = [i64, p, p, p, p, p, p, p, p, p, p, i32]
    lib.oracle_threads.argtypes = [i32]
    lib.oracle_solve_general.argtypes = [p, p, p, i64, i64, p, p, i32, i32]
    lib.oracle_adjoint_general.argtypes = [p, p, p, i64, i64, p, p, p, p, p, p, i32]
    for f in (lib.oracle_solve, lib.oracle_solve_varlen, lib.oracle_adjoint,
              lib.oracle_adjoint_varlen, lib.oracle_threads, lib.oracle_solve_general,
              lib.oracle_adjoint_general):
        f.restype = i32
    return lib


def _load():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB_PATH)
                or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build(force=True)
        _lib = _bind(_LIB_PATH)
    return _lib


class OracleSingular(RuntimeError):
    """A zero pivot appeared in the elimination."""


def _check(st: int):
    if st == 1:
        raise OracleSingular("zero pivot in Thomas elimination")
    if st:
        raise RuntimeError(f"oracle failed with status {st}")


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """Bindings of one compiled oracle library (the default one, or a test's
    deliberately broken copy)."""

    def __init__(self, lib=None):
        self._given = lib

    @property
    def lib(self):
        return self._given if self._given is not None else _load()

    def threads(self, nthreads: int = 0) -> int:
        """OpenMP threads the oracle uses (after setting ``nthreads`` if > 0)."""
        return self.lib.oracle_threads(int(nthreads))

    def solve(self, F, t_m1: float, t_0: float, t_1: float, precision: str = "f64",
              nthreads: int = 0, psi: float = 0.0, chi: float = 0.0) -> np.ndarray:
        """X = T^{-1} F.  F is [N] or [M, N] (one right-hand side per row).
        psi, chi: corner terms of the quasi-Toeplitz matrix of eq. (21)."""
        F = _f64(F)
        squeeze = F.ndim == 1
        F2 = F.reshape(1, -1) if squeeze else F
        M, N = F2.shape
        X = np.empty_like(F2)
        prec = {"f64": 0, "ld": 1}[precision]
        _check(self.lib.oracle_solve(float(t_m1), float(t_0), float(t_1), float(psi),
                                     float(chi), N, M, _ptr(F2), _ptr(X), prec, int(nthreads)))
        return X.reshape(-1) if squeeze else X

    def solve_varlen(self, F, offsets, t_m1, t_0, t_1, precision: str = "f64",
                     nthreads: int = 0, psi=None, chi=None) -> np.ndarray:
        """Packed systems: system s is F[offsets[s]:offsets[s+1]] with its own t's
        (and corner terms psi[s], chi[s] when given)."""
        F = _f64(F)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        S = off.size - 1
        tm1, t0, t1 = (_f64(np.broadcast_to(t, (S,))) for t in (t_m1, t_0, t_1))
        ps = None if psi is None else _f64(np.broadcast_to(psi, (S,)))
        ch = None if chi is None else _f64(np.broadcast_to(chi, (S,)))
        X = np.empty_like(F)
        prec = {"f64": 0, "ld": 1}[precision]
        _check(self.lib.oracle_solve_varlen(S, _ptr(off), _ptr(tm1), _ptr(t0), _ptr(t1),
                                            None if ps is None else _ptr(ps),
                                            None if ch is None else _ptr(ch),
                                            _ptr(F), _ptr(X), prec, int(nthreads)))
        return X

    def adjoint(self, gX, X, t_m1: float, t_0: float, t_1: float, nthreads: int = 0,
                psi: float = 0.0, chi: float = 0.0, corners: bool = False):
        """Returns (gF, gt) with gt = (dL/dt_-1, dL/dt_0, dL/dt_1) summed over RHS,
        followed by (dL/dpsi, dL/dchi) when ``corners``."""
        gX, X = _f64(gX), _f64(X)
        squeeze = gX.ndim == 1
        g2 = gX.reshape(1, -1) if squeeze else gX
        x2 = X.reshape(1, -1) if squeeze else X
        M, N = g2.shape
        gF = np.empty_like(g2)
        gt = np.empty(5)
        _check(self.lib.oracle_adjoint(float(t_m1), float(t_0), float(t_1), float(psi),
                                       float(chi), N, M, _ptr(g2), _ptr(x2), _ptr(gF),
                                       _ptr(gt), int(nthreads)))
        return (gF.reshape(-1) if squeeze else gF), (gt if corners else gt[:3])

    def adjoint_varlen(self, gX, X, offsets, t_m1, t_0, t_1, nthreads: int = 0,
                       psi=None, chi=None, corners: bool = False):
        """Returns (gF packed, gt [S, 3]), or gt [S, 5] with (dL/dpsi, dL/dchi)
        appended when ``corners``."""
        gX, X = _f64(gX), _f64(X)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        S = off.size - 1
        tm1, t0, t1 = (_f64(np.broadcast_to(t, (S,))) for t in (t_m1, t_0, t_1))
        ps = None if psi is None else _f64(np.broadcast_to(psi, (S,)))
        ch = None if chi is None else _f64(np.broadcast_to(chi, (S,)))
        gF = np.empty_like(gX)
        gt = np.empty((S, 5))
        _check(self.lib.oracle_adjoint_varlen(S, _ptr(off), _ptr(tm1), _ptr(t0), _ptr(t1),
                                              None if ps is None else _ptr(ps),
                                              None if ch is None else _ptr(ch),
                                              _ptr(gX), _ptr(X), _ptr(gF), _ptr(gt),
                                              int(nthreads)))
        return gF, (gt if corners else gt[:, :3])


    def solve_general(self, F, a, b, c, precision: str = "f64", nthreads: int = 0):
        """X = A^{-1} F for the general tridiagonal A with rows (a_i, b_i, c_i)
        (a_0 and c_{N-1} unused).  F is [N] or [M, N]."""
        F = _f64(F)
        squeeze = F.ndim == 1
        F2 = F.reshape(1, -1) if squeeze else F
        M, N = F2.shape
        av, bv, cv = (_f64(np.broadcast_to(v, (N,))) for v in (a, b, c))
        X = np.empty_like(F2)
        prec = {"f64": 0, "ld": 1}[precision]
        _check(self.lib.oracle_solve_general(_ptr(av), _ptr(bv), _ptr(cv), N, M, _ptr(F2),
                                             _ptr(X), prec, int(nthreads)))
        return X.reshape(-1) if squeeze else X

    def adjoint_general(self, gX, X, a, b, c, nthreads: int = 0):
        """Returns (gF, (dL/da, dL/db, dL/dc)) for the general matrix, the
        entry gradients summed over the right-hand sides."""
        gX, X = _f64(gX), _f64(X)
        squeeze = gX.ndim == 1
        g2 = gX.reshape(1, -1) if squeeze else gX
        x2 = X.reshape(1, -1) if squeeze else X
        M, N = g2.shape
        av, bv, cv = (_f64(np.broadcast_to(v, (N,))) for v in (a, b, c))
        gF = np.empty_like(g2)
        ga, gb, gc = np.empty(N), np.empty(N), np.empty(N)
        _check(self.lib.oracle_adjoint_general(_ptr(av), _ptr(bv), _ptr(cv), N, M, _ptr(g2),
                                               _ptr(x2), _ptr(gF), _ptr(ga), _ptr(gb),
                                               _ptr(gc), int(nthreads)))
        return (gF.reshape(-1) if squeeze else gF), (ga, gb, gc)


def load_library(path: str) -> Oracle:
    """Bind a separately compiled copy of the oracle source (used by the tests
    that plant a mistake in the oracle to show that the pins catch it)."""
    return Oracle(_bind(path))


_default = Oracle()
threads = _default.threads
solve = _default.solve
solve_varlen = _default.solve_varlen
adjoint = _default.adjoint
adjoint_varlen = _default.adjoint_varlen
solve_general = _default.solve_general
adjoint_general = _default.adjoint_general


def rel_err(x, ref) -> float:
    """Normwise relative error max|x - ref| / max|ref| (over the whole array)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref)) if ref.size else 0.0
    num = np.max(np.abs(x - ref)) if ref.size else 0.0
    return float(num / den) if den > 0 else float(num)


def rel_err_rows(x, ref, offsets=None) -> np.ndarray:
    """Per right-hand side (rows of [M, N]) or per packed system relative error."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if offsets is None:
        x2, r2 = x.reshape(-1, x.shape[-1]), ref.reshape(-1, ref.shape[-1])
        num = np.max(np.abs(x2 - r2), axis=1)
        den = np.max(np.abs(r2), axis=1)
    else:
        off = np.asarray(offsets, dtype=np.int64)
        num = np.maximum.reduceat(np.abs(x - ref), off[:-1])
        den = np.maximum.reduceat(np.abs(ref), off[:-1])
    den = np.where(den > 0, den, 1.0)
    return num / den
