"""Toeplitz tridiagonal solves T X = F on one MI355X by the partitioned
dichotomy method, T = tridiag{t_-1, t_0, t_1} (t_1 above the diagonal).

Thin Python layer over the C ABI of ``include/tdt.h``: it marshals torch
device pointers, sizes and the current stream; every arithmetic step runs in
the HIP kernels of ``libtdt.so``.  PyTorch is used for device memory and
streams only.

    plan = Plan(t_m1, t_0, t_1, N, dtype="f64")      # preliminary step, once per T
    X = plan.solve(F)                                # F: cuda [N] or [M, N]
    gF, gt = plan.backward(gX, X)                    # adjoint: T^T gF = gX, dL/dt
    vp = VarlenPlan(offsets, t_m1s, t_0s, t_1s)      # many systems, own sizes and T
    X = vp.solve(F_packed)
    X = TridiagToeplitzSolve.apply(F, t)             # autograd, t = (t_-1, t_0, t_1)
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import DTYPES, TDTError, build

__all__ = ["Plan", "VarlenPlan", "GeneralPlan", "StridedPlan", "Poisson2D", "Poisson3D", "solve", "solve_varlen", "TridiagToeplitzSolve", "block_constants",
           "green_rows", "green_support", "segment_merge", "build_info", "build", "TDTError"]


def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _data_dtype(dtype: str):
    torch = _torch()
    return torch.float32 if dtype == "f32" else torch.float64


def _check_tensor(t, dtype, numel, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


class _PlanBase:
    def __init__(self):
        self._h = ctypes.c_void_p()
        self.status = 0

    def reserve(self, m_max: int = 1):
        """Allocate the workspace now (required before capturing a hipGraph)."""
        _lib.check(_lib.lib().tdt_plan_reserve(self._h, int(m_max)), "tdt_plan_reserve")

    def info(self) -> dict:
        """Refinement record since the last call (synchronises), dominance
        ratio and condition number; converged is False when a refinement
        stopped above float resolution."""
        it = ctypes.c_int(0)
        upd, dom, kap = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = _lib.lib().tdt_last_info(self._h, ctypes.byref(it), ctypes.byref(upd),
                                      ctypes.byref(dom), ctypes.byref(kap))
        if st != _lib.TDT_ERR_NOT_CONVERGED:
            _lib.check(st, "tdt_last_info")
        return dict(refine_iters=it.value, last_rel_update=upd.value, dominance=dom.value,
                    kappa2=kap.value, converged=st != _lib.TDT_ERR_NOT_CONVERGED)

    def profile(self, enable: bool = True):
        """Record HIP events around the kernels of every later solve."""
        _lib.check(_lib.lib().tdt_plan_profile(self._h, int(bool(enable))), "tdt_plan_profile")

    def profile_read(self) -> dict:
        """Summed ms of (first pass, interface pass, final pass) since the last read."""
        ms = np.zeros(3)
        n = ctypes.c_int64(0)
        _lib.check(_lib.lib().tdt_plan_profile_read(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                                    ctypes.byref(n)), "tdt_plan_profile_read")
        return dict(first_pass_ms=ms[0], interface_ms=ms[1], final_ms=ms[2], solves=n.value)

    def green_support(self) -> dict:
        """Rows per full tile the first pass reads from the head and the tail
        of each tile ((0, 0): whole tiles, or no such pass), for the forward
        solve and the adjoint."""
        rows = np.zeros(4, dtype=np.int64)
        _lib.check(_lib.lib().tdt_plan_green_support(self._h, rows.ctypes.data_as(ctypes.c_void_p)),
                   "tdt_plan_green_support")
        return dict(forward=(int(rows[0]), int(rows[1])), adjoint=(int(rows[2]), int(rows[3])))

    def set_option(self, name: str, value: int):
        """Option of tdt_option_t: 'whole_max_tiles', 'wg_per_cu',
        'max_refine' or 'shape' (index into _lib.SHAPES)."""
        _lib.check(_lib.lib().tdt_plan_set_option(self._h, _lib.OPTIONS[name], int(value)),
                   "tdt_plan_set_option")

    def get_option(self, name: str) -> int:
        v = ctypes.c_int64(0)
        _lib.check(_lib.lib().tdt_plan_get_option(self._h, _lib.OPTIONS[name], ctypes.byref(v)),
                   "tdt_plan_get_option")
        return v.value

    def _autotune(self, F, X, M, cache=True, force=False, stream=None, adjoint=False) -> dict:
        flags = ((0 if cache else _lib.TUNE_NO_CACHE) | (_lib.TUNE_FORCE if force else 0) |
                 (_lib.TUNE_ADJOINT if adjoint else 0))
        ms = ctypes.c_double(0.0)
        _lib.check(_lib.lib().tdt_plan_autotune(self._h, ctypes.c_void_p(F.data_ptr()),
                                                ctypes.c_void_p(X.data_ptr()), int(M),
                                                _stream_handle(stream), flags, ctypes.byref(ms)),
                   "tdt_plan_autotune")
        out = {k: self.get_option(k) for k in ("shape", "whole_max_tiles", "wg_per_cu")}
        out["ms"] = ms.value
        return out

    def close(self):
        if self._h:
            _lib.lib().tdt_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan(_PlanBase):
    """Plan of one Toeplitz matrix of order N (data dtype: 'f64', 'f32' or
    'f32_refine'; the last takes and returns float64).  With psi and chi the
    matrix is quasi-Toeplitz (eq. (21): t_0 + psi in the first diagonal
    entry, t_0 + chi in the last; N >= 3) and backward returns 5 t-gradients
    (dL/dt_-1, dL/dt_0, dL/dt_1, dL/dpsi, dL/dchi)."""

    def __init__(self, t_m1: float, t_0: float, t_1: float, N: int, dtype: str = "f64",
                 psi=None, chi=None):
        super().__init__()
        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {list(DTYPES)}")
        if (psi is None) != (chi is None):
            raise ValueError("give both psi and chi, or neither")
        self.t = (float(t_m1), float(t_0), float(t_1))
        self.N = int(N)
        self.dtype = dtype
        self.quasi = psi is not None
        self.ngt = 5 if self.quasi else 3
        if self.quasi:
            self.corners = (float(psi), float(chi))
            self.status = _lib.check(_lib.lib().tdt_plan_quasi_create(
                self.t[0], self.t[1], self.t[2], self.corners[0], self.corners[1], self.N,
                DTYPES[dtype], ctypes.byref(self._h)), "tdt_plan_quasi_create")
        else:
            self.status = _lib.check(_lib.lib().tdt_plan_create(
                self.t[0], self.t[1], self.t[2], self.N, DTYPES[dtype], ctypes.byref(self._h)),
                "tdt_plan_create")

    @property
    def dominant(self) -> bool:
        return self.status != _lib.TDT_WARN_NOT_DOMINANT

    def solve(self, F, X=None, stream=None):
        torch = _torch()
        dt = _data_dtype(self.dtype)
        M = F.numel() // self.N if F.numel() else 0
        if F.numel() != M * self.N or M < 1:
            raise ValueError("F must hold M whole right-hand sides of length N")
        _check_tensor(F, dt, M * self.N, "F")
        if X is None:
            X = torch.empty_like(F)
        _check_tensor(X, dt, M * self.N, "X")
        _lib.check(_lib.lib().tdt_solve(self._h, ctypes.c_void_p(F.data_ptr()),
                                        ctypes.c_void_p(X.data_ptr()), M,
                                        _stream_handle(stream)), "tdt_solve")
        return X

    def autotune(self, F, X=None, cache=True, force=False, stream=None,
                 adjoint=False) -> dict:
        """Time the launch shapes on F (X is overwritten with the solution)
        and keep the fastest; cached per device and problem size.  adjoint:
        time each trial as a solve plus its adjoint."""
        torch = _torch()
        M = F.numel() // self.N
        if X is None:
            X = torch.empty_like(F)
        _check_tensor(F, _data_dtype(self.dtype), M * self.N, "F")
        _check_tensor(X, _data_dtype(self.dtype), M * self.N, "X")
        return self._autotune(F, X, M, cache, force, stream, adjoint)

    def backward(self, gX, X, gF=None, gt=None, stream=None):
        """gF = T^{-T} gX and gt = (dL/dt_-1, dL/dt_0, dL/dt_1[, dL/dpsi,
        dL/dchi]) summed over RHS."""
        torch = _torch()
        dt = _data_dtype(self.dtype)
        M = gX.numel() // self.N
        _check_tensor(gX, dt, M * self.N, "gX")
        _check_tensor(X, dt, M * self.N, "X")
        if gF is None:
            gF = torch.empty_like(gX)
        if gt is None:
            gt = torch.empty(self.ngt, dtype=torch.float64, device=gX.device)
        _check_tensor(gF, dt, M * self.N, "gF")
        _check_tensor(gt, torch.float64, self.ngt, "gt")
        _lib.check(_lib.lib().tdt_solve_backward(
            self._h, ctypes.c_void_p(gX.data_ptr()), ctypes.c_void_p(X.data_ptr()),
            ctypes.c_void_p(gF.data_ptr()), ctypes.c_void_p(gt.data_ptr()), M,
            _stream_handle(stream)), "tdt_solve_backward")
        return gF, gt


class VarlenPlan(_PlanBase):
    """S systems of sizes offsets[s+1]-offsets[s], each with its own t's,
    packed back to back.  With psi and chi (scalars or S values) every system
    is quasi-Toeplitz (eq. (21), sizes >= 3) and backward returns 5
    t-gradients per system."""

    def __init__(self, offsets, t_m1, t_0, t_1, dtype: str = "f64", psi=None, chi=None):
        super().__init__()
        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {list(DTYPES)}")
        if (psi is None) != (chi is None):
            raise ValueError("give both psi and chi, or neither")
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.S = self.offsets.size - 1

        def per_system(t):
            return np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64),
                                                        (self.S,)))

        ts = [per_system(t) for t in (t_m1, t_0, t_1)]
        self.t = ts
        self.total = int(self.offsets[-1])
        self.dtype = dtype
        self.quasi = psi is not None
        self.ngt = 5 if self.quasi else 3
        vp = [x.ctypes.data_as(ctypes.c_void_p) for x in ts]
        if self.quasi:
            self.corners = [per_system(psi), per_system(chi)]
            cp = [x.ctypes.data_as(ctypes.c_void_p) for x in self.corners]
            self.status = _lib.check(_lib.lib().tdt_plan_varlen_quasi_create(
                self.S, self.offsets.ctypes.data_as(ctypes.c_void_p), vp[0], vp[1], vp[2],
                cp[0], cp[1], DTYPES[dtype], ctypes.byref(self._h)),
                "tdt_plan_varlen_quasi_create")
        else:
            self.status = _lib.check(_lib.lib().tdt_plan_varlen_create(
                self.S, self.offsets.ctypes.data_as(ctypes.c_void_p), vp[0], vp[1], vp[2],
                DTYPES[dtype], ctypes.byref(self._h)), "tdt_plan_varlen_create")

    def solve(self, F, X=None, stream=None):
        torch = _torch()
        dt = _data_dtype(self.dtype)
        _check_tensor(F, dt, self.total, "F")
        if X is None:
            X = torch.empty_like(F)
        _check_tensor(X, dt, self.total, "X")
        _lib.check(_lib.lib().tdt_solve_varlen(self._h, ctypes.c_void_p(F.data_ptr()),
                                               ctypes.c_void_p(X.data_ptr()),
                                               _stream_handle(stream)), "tdt_solve_varlen")
        return X

    def autotune(self, F, X=None, cache=True, force=False, stream=None,
                 adjoint=False) -> dict:
        """Time the launch shapes (whole-system threshold, workgroups per CU)
        on F (X is overwritten with the solution) and keep the fastest;
        adjoint: time each trial as a solve plus its adjoint."""
        torch = _torch()
        if X is None:
            X = torch.empty_like(F)
        _check_tensor(F, _data_dtype(self.dtype), self.total, "F")
        _check_tensor(X, _data_dtype(self.dtype), self.total, "X")
        return self._autotune(F, X, 1, cache, force, stream, adjoint)

    def backward(self, gX, X, gF=None, gt=None, stream=None):
        """gF = T_s^{-T} gX per system and gt[s] = (dL/dt_-1, dL/dt_0,
        dL/dt_1[, dL/dpsi, dL/dchi])."""
        torch = _torch()
        dt = _data_dtype(self.dtype)
        _check_tensor(gX, dt, self.total, "gX")
        _check_tensor(X, dt, self.total, "X")
        if gF is None:
            gF = torch.empty_like(gX)
        if gt is None:
            gt = torch.empty((self.S, self.ngt), dtype=torch.float64, device=gX.device)
        _check_tensor(gF, dt, self.total, "gF")
        _check_tensor(gt, torch.float64, self.ngt * self.S, "gt")
        _lib.check(_lib.lib().tdt_solve_backward(
            self._h, ctypes.c_void_p(gX.data_ptr()), ctypes.c_void_p(X.data_ptr()),
            ctypes.c_void_p(gF.data_ptr()), ctypes.c_void_p(gt.data_ptr()), 1,
            _stream_handle(stream)), "tdt_solve_backward")
        return gF, gt


class GeneralPlan(_PlanBase):
    """Plan of a general tridiagonal matrix of order N (row i: a_i x_{i-1} +
    b_i x_i + c_i x_{i+1} = f_i; a_0 and c_{N-1} unused) for series of
    right-hand sides sharing it.  dtype: 'f64' or 'f32'."""

    def __init__(self, a, b, c, dtype: str = "f64"):
        super().__init__()
        if dtype not in ("f64", "f32"):
            raise ValueError("dtype must be 'f64' or 'f32' for a general matrix")
        self.b = np.ascontiguousarray(b, dtype=np.float64)
        self.N = int(self.b.size)
        self.a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64),
                                                      (self.N,)))
        self.c = np.ascontiguousarray(np.broadcast_to(np.asarray(c, dtype=np.float64),
                                                      (self.N,)))
        self.dtype = dtype
        self.status = _lib.check(_lib.lib().tdt_plan_general_create(
            self.N, self.a.ctypes.data_as(ctypes.c_void_p),
            self.b.ctypes.data_as(ctypes.c_void_p), self.c.ctypes.data_as(ctypes.c_void_p),
            DTYPES[dtype], ctypes.byref(self._h)), "tdt_plan_general_create")

    def solve(self, F, X=None, stream=None):
        return Plan.solve(self, F, X, stream)

    def autotune(self, F, X=None, cache=True, force=False, stream=None,
                 adjoint=False) -> dict:
        return Plan.autotune(self, F, X, cache, force, stream, adjoint)

    def backward(self, gX, X, gF=None, g=None, stream=None):
        """gF = A^{-T} gX and g = [3][N]: (dL/da, dL/db, dL/dc) summed over
        the right-hand sides."""
        torch = _torch()
        dt = _data_dtype(self.dtype)
        M = gX.numel() // self.N
        _check_tensor(gX, dt, M * self.N, "gX")
        _check_tensor(X, dt, M * self.N, "X")
        if gF is None:
            gF = torch.empty_like(gX)
        if g is None:
            g = torch.empty((3, self.N), dtype=torch.float64, device=gX.device)
        _check_tensor(gF, dt, M * self.N, "gF")
        _check_tensor(g, torch.float64, 3 * self.N, "g")
        _lib.check(_lib.lib().tdt_solve_backward(
            self._h, ctypes.c_void_p(gX.data_ptr()), ctypes.c_void_p(X.data_ptr()),
            ctypes.c_void_p(gF.data_ptr()), ctypes.c_void_p(g.data_ptr()), M,
            _stream_handle(stream)), "tdt_solve_backward")
        return gF, g


class StridedPlan(_PlanBase):
    """Plan of P classes of Toeplitz matrices of order N <= 2^24 (class k:
    tridiag{t_m1[k], t_0[k], t_1[k]}) for systems along a slow axis: unknown
    i of system s of batch b at element b*ldb + i*ld + s, system s using
    class s.  float64 only.  Scalars broadcast over the P classes.  Systems
    of more than 1024 rows are solved in tiles and need workspace: call
    reserve(nb * M) before capturing a solve in a hipGraph."""

    def __init__(self, N: int, t_m1, t_0, t_1):
        super().__init__()
        t0 = np.ascontiguousarray(np.asarray(t_0, dtype=np.float64).reshape(-1))
        self.N, self.P = int(N), int(t0.size)
        self.t_0 = t0
        self.t_m1 = np.ascontiguousarray(np.broadcast_to(np.asarray(t_m1, dtype=np.float64),
                                                         (self.P,)))
        self.t_1 = np.ascontiguousarray(np.broadcast_to(np.asarray(t_1, dtype=np.float64),
                                                        (self.P,)))
        self.dtype = "f64"
        self.status = _lib.check(_lib.lib().tdt_plan_strided_create(
            self.N, self.P, self.t_m1.ctypes.data_as(ctypes.c_void_p),
            self.t_0.ctypes.data_as(ctypes.c_void_p), self.t_1.ctypes.data_as(ctypes.c_void_p),
            DTYPES["f64"], ctypes.byref(self._h)), "tdt_plan_strided_create")

    def solve(self, F, X=None, M=None, ld=None, nb=None, ldb=None, stream=None):
        """F: float64 CUDA tensor.  Without layout arguments F is read as
        [N][M] (ld = M) or [nb][N][M] (ldb = N*M).  X may be F (in place)."""
        torch = _torch()
        if not isinstance(F, torch.Tensor) or not F.is_cuda or F.dtype != torch.float64:
            raise TypeError("F must be a float64 CUDA (HIP) tensor")
        if not F.is_contiguous():
            raise ValueError("F must be contiguous")
        if M is None:
            if F.dim() == 2:
                nb, M, ld, ldb = 1, F.shape[1], F.shape[1], 0
            elif F.dim() == 3:
                nb, M, ld, ldb = F.shape[0], F.shape[2], F.shape[2], F.shape[1] * F.shape[2]
            else:
                raise ValueError("give the layout (M, ld, nb, ldb) for this shape")
            if (F.shape[-2] != self.N):
                raise ValueError(f"F has {F.shape[-2]} rows, the plan {self.N}")
        nb = 1 if nb is None else int(nb)
        ld = int(M) if ld is None else int(ld)
        ldb = 0 if ldb is None else int(ldb)
        extent = (nb - 1) * ldb + (self.N - 1) * ld + int(M)
        if F.numel() < extent:
            raise ValueError(f"F has {F.numel()} elements, the layout reaches {extent}")
        if X is None:
            X = torch.empty_like(F)
        if X.shape != F.shape or X.dtype != F.dtype or not X.is_cuda or not X.is_contiguous():
            raise ValueError("X must be a contiguous float64 CUDA tensor shaped like F")
        _lib.check(_lib.lib().tdt_solve_strided(self._h, ctypes.c_void_p(F.data_ptr()),
                                                ctypes.c_void_p(X.data_ptr()), int(M), ld, nb,
                                                ldb, _stream_handle(stream)),
                   "tdt_solve_strided")
        return X


class Poisson2D:
    """2D Poisson solve by separation of variables (Sec. 3.2): the five-point
    system on Nx x Ny interior points with zero boundary values, F and U
    [Ny][Nx] float64 on the device.  Sine transforms along x (one fused
    kernel when Nx + 1 is a power of two from 128 to 8192, hipFFT
    otherwise), one Toeplitz line system per mode along y (in float64 with
    the fused transform, a strided plan solving the modes in place in the
    transformed rows; otherwise a varlen plan of dtype 'f64' or
    'f32_refine' after a transpose), inverse transform."""

    def __init__(self, nx: int, ny: int, hx: float, hy: float, dtype: str = "f64"):
        if dtype not in ("f64", "f32_refine"):
            raise ValueError("dtype must be 'f64' or 'f32_refine'")
        self._h = ctypes.c_void_p()
        self.nx, self.ny, self.hx, self.hy, self.dtype = int(nx), int(ny), float(hx), float(hy), dtype
        _lib.check(_lib.lib().tdt_poisson2d_create(self.nx, self.ny, self.hx, self.hy,
                                                   DTYPES[dtype], ctypes.byref(self._h)),
                   "tdt_poisson2d_create")

    def solve(self, F, U=None, stream=None):
        torch = _torch()
        _check_tensor(F, torch.float64, self.nx * self.ny, "F")
        if U is None:
            U = torch.empty_like(F)
        _check_tensor(U, torch.float64, self.nx * self.ny, "U")
        _lib.check(_lib.lib().tdt_poisson2d_solve(self._h, ctypes.c_void_p(F.data_ptr()),
                                                  ctypes.c_void_p(U.data_ptr()),
                                                  _stream_handle(stream)), "tdt_poisson2d_solve")
        return U

    def profile(self, enable: bool = True):
        """Record HIP events around the forward transform, the line solve
        and the inverse transform of every later solve."""
        _lib.check(_lib.lib().tdt_poisson2d_profile(self._h, 1 if enable else 0),
                   "tdt_poisson2d_profile")

    def profile_read(self) -> dict:
        ms = np.zeros(3)
        n = ctypes.c_int64(0)
        _lib.check(_lib.lib().tdt_poisson2d_profile_read(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                                         ctypes.byref(n)),
                   "tdt_poisson2d_profile_read")
        return dict(forward_ms=ms[0], line_ms=ms[1], inverse_ms=ms[2], solves=n.value)

    def _line(self):
        line = ctypes.c_void_p()
        _lib.check(_lib.lib().tdt_poisson2d_line_plan(self._h, ctypes.byref(line)),
                   "tdt_poisson2d_line_plan")
        return line

    def line_profile(self, enable: bool = True):
        """Record HIP events around the line plan's kernel groups."""
        _lib.check(_lib.lib().tdt_plan_profile(self._line(), 1 if enable else 0),
                   "tdt_plan_profile")

    def line_profile_read(self) -> dict:
        ms = np.zeros(3)
        n = ctypes.c_int64(0)
        _lib.check(_lib.lib().tdt_plan_profile_read(self._line(),
                                                    ms.ctypes.data_as(ctypes.c_void_p),
                                                    ctypes.byref(n)), "tdt_plan_profile_read")
        return dict(first_pass_ms=ms[0], interface_ms=ms[1], final_ms=ms[2], solves=n.value)

    def set_line_option(self, name: str, value: int):
        """A launch option of the line plan (see Plan.set_option)."""
        _lib.check(_lib.lib().tdt_plan_set_option(self._line(), _lib.OPTIONS[name], int(value)),
                   "tdt_plan_set_option")

    def close(self):
        if self._h:
            _lib.lib().tdt_poisson2d_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Poisson3D:
    """3D Poisson solve of Sec. 3.5: the seven-point system on Nx x Ny x Nz
    interior points with zero boundary values, F and U [Nz][Ny][Nx] float64
    on the device.  Sine transform along x (hipFFT), Peaceman-Rachford ADI
    on every mode's (y, z) plane with the optimal parameters (strided line
    solves along y and z), inverse transform.  eps bounds the ADI error
    relative to the exact discrete solution (2-norm)."""

    def __init__(self, nx: int, ny: int, nz: int, hx: float, hy: float, hz: float,
                 eps: float = 1e-13):
        self._h = ctypes.c_void_p()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.hx, self.hy, self.hz, self.eps = float(hx), float(hy), float(hz), float(eps)
        _lib.check(_lib.lib().tdt_poisson3d_create(self.nx, self.ny, self.nz, self.hx, self.hy,
                                                   self.hz, self.eps, ctypes.byref(self._h)),
                   "tdt_poisson3d_create")

    def solve(self, F, U=None, stream=None):
        torch = _torch()
        n = self.nx * self.ny * self.nz
        _check_tensor(F, torch.float64, n, "F")
        if U is None:
            U = torch.empty_like(F)
        _check_tensor(U, torch.float64, n, "U")
        _lib.check(_lib.lib().tdt_poisson3d_solve(self._h, ctypes.c_void_p(F.data_ptr()),
                                                  ctypes.c_void_p(U.data_ptr()),
                                                  _stream_handle(stream)), "tdt_poisson3d_solve")
        return U

    def schedule(self):
        """(counts J_k [Nx], parameters [Nx][jmax] with zeros past J_k)."""
        jm = ctypes.c_int(0)
        _lib.check(_lib.lib().tdt_poisson3d_schedule(self._h, None, None, 0, ctypes.byref(jm)),
                   "tdt_poisson3d_schedule")
        counts = np.zeros(self.nx, dtype=np.int32)
        om = np.zeros((self.nx, jm.value))
        _lib.check(_lib.lib().tdt_poisson3d_schedule(
            self._h, counts.ctypes.data_as(ctypes.c_void_p), om.ctypes.data_as(ctypes.c_void_p),
            om.size, ctypes.byref(jm)), "tdt_poisson3d_schedule")
        return counts, om

    def profile(self, enable: bool = True):
        _lib.check(_lib.lib().tdt_poisson3d_profile(self._h, 1 if enable else 0),
                   "tdt_poisson3d_profile")

    def profile_read(self) -> dict:
        ms = np.zeros(3)
        n = ctypes.c_int64(0)
        _lib.check(_lib.lib().tdt_poisson3d_profile_read(self._h,
                                                         ms.ctypes.data_as(ctypes.c_void_p),
                                                         ctypes.byref(n)),
                   "tdt_poisson3d_profile_read")
        return dict(forward_ms=ms[0], adi_ms=ms[1], inverse_ms=ms[2], solves=n.value)

    def close(self):
        if self._h:
            _lib.lib().tdt_poisson3d_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_plan_cache: dict = {}


def _cached_plan(t_m1, t_0, t_1, N, dtype, psi=None, chi=None) -> Plan:
    corners = None if psi is None else (float(psi), float(chi))
    key = (float(t_m1), float(t_0), float(t_1), int(N), dtype, corners)
    p = _plan_cache.get(key)
    if p is None:
        if len(_plan_cache) > 64:
            _plan_cache.clear()
        p = Plan(*key[:5], psi=psi, chi=chi)
        _plan_cache[key] = p
    return p


def solve(F, t_m1: float, t_0: float, t_1: float, dtype: str = "f64", psi=None, chi=None):
    """X = T^{-1} F along the last dimension of F (cached plan per T and N);
    psi/chi: quasi-Toeplitz corner terms."""
    return _cached_plan(t_m1, t_0, t_1, F.shape[-1], dtype, psi, chi).solve(F.contiguous())


def solve_varlen(F, offsets, t_m1, t_0, t_1, dtype: str = "f64", psi=None, chi=None):
    """X_s = T_s^{-1} F_s for packed systems s (F[offsets[s]:offsets[s+1]]),
    each with its own t's (scalars broadcast; psi/chi: quasi-Toeplitz corner
    terms).  Builds a plan per call: keep a VarlenPlan to solve the same
    systems again."""
    plan = VarlenPlan(offsets, t_m1, t_0, t_1, dtype, psi=psi, chi=chi)
    try:
        return plan.solve(F.contiguous())
    finally:
        plan.close()


class TridiagToeplitzSolve:
    """Differentiable X = T^{-1} F; t = (t_-1, t_0, t_1) as a tensor of 3, or
    (t_-1, t_0, t_1, psi, chi) as a tensor of 5 for the quasi-Toeplitz
    matrix of eq. (21).

    Backward is the hand-written adjoint kernel: gF = T^{-T} gX through the
    same dichotomy machinery, and the t-gradients reduced on the device."""

    _fn = None

    @classmethod
    def _function(cls):
        if cls._fn is None:
            torch = _torch()

            class _Fn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, F, t, dtype="f64"):
                    tv = [float(v) for v in t.detach().cpu().tolist()]
                    if len(tv) not in (3, 5):
                        raise ValueError("t must hold 3 (Toeplitz) or 5 (quasi-Toeplitz) values")
                    plan = _cached_plan(*tv[:3], F.shape[-1], dtype, *tv[3:])
                    X = plan.solve(F.contiguous())
                    ctx.plan = plan
                    ctx.t_device, ctx.t_dtype = t.device, t.dtype
                    ctx.save_for_backward(X)
                    return X

                @staticmethod
                def backward(ctx, gX):
                    (X,) = ctx.saved_tensors
                    gF, gt = ctx.plan.backward(gX.contiguous(), X)
                    return gF, gt.to(device=ctx.t_device, dtype=ctx.t_dtype), None

            cls._fn = _Fn
        return cls._fn

    @classmethod
    def apply(cls, F, t, dtype: str = "f64"):
        return cls._function().apply(F, t, dtype)


def block_constants(t_m1: float, t_0: float, t_1: float, B: int) -> dict:
    """Host-only: the per-T block constants the plan uploads (no GPU needed)."""
    out = np.empty(4 * B + 4)
    _lib.check(_lib.lib().tdt_block_constants(float(t_m1), float(t_0), float(t_1), int(B),
                                              out.ctypes.data_as(ctypes.c_void_p)),
               "tdt_block_constants")
    return dict(inv_pivot=out[:B], cp=out[B:2 * B], phi=out[2 * B:3 * B],
                chi=out[3 * B:4 * B], ends=out[4 * B:])


def green_rows(t_m1: float, t_0: float, t_1: float, L: int):
    """Host-only: first and last row of the inverse of the L x L Toeplitz matrix."""
    first, last = np.empty(int(L)), np.empty(int(L))
    _lib.check(_lib.lib().tdt_green_rows(float(t_m1), float(t_0), float(t_1), int(L),
                                         first.ctypes.data_as(ctypes.c_void_p),
                                         last.ctypes.data_as(ctypes.c_void_p)),
               "tdt_green_rows")
    return first, last


def green_support(t_m1: float, t_0: float, t_1: float, L: int, bound: bool = False):
    """Host-only: (kf, kl), the fewest leading entries of the first Green row
    and trailing entries of the last that hold all but 2^-60 of each row's
    1-norm (the supports a series plan's first pass reads); with bound=True
    also the supports a varlen plan derives from the pivots' decay (0, 0:
    no truncation), as ((kf, kl), (bkf, bkl))."""
    kf, kl = ctypes.c_int64(0), ctypes.c_int64(0)
    b2 = np.zeros(2, dtype=np.int64)
    _lib.check(_lib.lib().tdt_green_support(float(t_m1), float(t_0), float(t_1), int(L),
                                            ctypes.byref(kf), ctypes.byref(kl),
                                            b2.ctypes.data_as(ctypes.c_void_p)),
               "tdt_green_support")
    if bound:
        return (kf.value, kl.value), (int(b2[0]), int(b2[1]))
    return kf.value, kl.value


def segment_merge(left, right) -> np.ndarray:
    """Host-only: the kernels' interface merge of two segment summaries."""
    l = np.ascontiguousarray(left, dtype=np.float64)
    r = np.ascontiguousarray(right, dtype=np.float64)
    out = np.empty(6)
    _lib.check(_lib.lib().tdt_segment_merge(l.ctypes.data_as(ctypes.c_void_p),
                                            r.ctypes.data_as(ctypes.c_void_p),
                                            out.ctypes.data_as(ctypes.c_void_p)),
               "tdt_segment_merge")
    return out


def adi_parameters(a: float, b: float, J: int):
    """Host hook: the 3D solve's J optimal ADI parameters for [a, b] and
    their error bound d_J."""
    out = np.zeros(int(J))
    bound = ctypes.c_double(0.0)
    _lib.check(_lib.lib().tdt_adi_parameters(float(a), float(b), int(J),
                                             out.ctypes.data_as(ctypes.c_void_p),
                                             ctypes.byref(bound)), "tdt_adi_parameters")
    return out, bound.value


def build_info() -> dict:
    b64, b32, nt = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    tile = ctypes.c_int64()
    _lib.lib().tdt_build_info(ctypes.byref(b64), ctypes.byref(b32), ctypes.byref(nt),
                              ctypes.byref(tile))
    return dict(block_f64=b64.value, block_f32=b32.value, wg_threads=nt.value,
                tile=tile.value)
