"""TEST INFRASTRUCTURE ONLY: plain CPU reference of the 2D Poisson solve by
separation of variables (paper, Sec. 3.2; the application its timings use).

Problem: -(u_xx + u_yy) = f on a rectangle with u = 0 on the boundary,
discretised by the five-point scheme on the Nx x Ny interior points
(spacings hx, hy):

    (2 u_ij - u_{i-1,j} - u_{i+1,j}) / hx^2 + (2 u_ij - u_{i,j-1} - u_{i,j+1}) / hy^2 = f_ij,

with F and U stored [Ny][Nx] (x contiguous).  Separation of variables writes
u_ij = sum_k v_kj sin(pi k i / (Nx + 1)): the sine vectors are the
eigenvectors of the x operator, with eigenvalues mu_k = (4 / hx^2)
sin^2(pi k / (2 (Nx + 1))), so every mode k leaves one tridiagonal Toeplitz
system along y,

    -v_{k,j-1} + (2 + hy^2 mu_k) v_kj - v_{k,j+1} = hy^2 fhat_kj,
    fhat_kj = (2 / (Nx + 1)) sum_i f_ij sin(pi k i / (Nx + 1)),

solved here by the pinned Thomas oracle.  The sine transforms are explicit
matrix products (no FFT), so each step can be read off the formulas above.
Only tests/ and bench.py's CPU leg use this module; the product never does.
"""
import math

import numpy as np


def sine_matrix(n: int) -> np.ndarray:
    """S[i-1, k-1] = sin(pi i k / (n + 1)), i, k = 1..n (symmetric)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.sin(np.pi * np.outer(i, i) / (n + 1))


def mode_eigenvalues(nx: int, hx: float) -> np.ndarray:
    """mu_k = (4 / hx^2) sin^2(pi k / (2 (nx + 1))), k = 1..nx."""
    k = np.arange(1, nx + 1, dtype=np.float64)
    return (4.0 / (hx * hx)) * np.sin(np.pi * k / (2.0 * (nx + 1))) ** 2


def laplacian(U: np.ndarray, hx: float, hy: float) -> np.ndarray:
    """The five-point operator applied to U ([Ny][Nx], zero boundary)."""
    P = np.pad(np.asarray(U, dtype=np.float64), 1)
    return ((2.0 * P[1:-1, 1:-1] - P[1:-1, :-2] - P[1:-1, 2:]) / (hx * hx) +
            (2.0 * P[1:-1, 1:-1] - P[:-2, 1:-1] - P[2:, 1:-1]) / (hy * hy))


def solve(F: np.ndarray, hx: float, hy: float, orc=None) -> np.ndarray:
    """U with laplacian(U) = F, by the three steps of separation of variables."""
    if orc is None:
        import oracle as orc
    F = np.asarray(F, dtype=np.float64)
    ny, nx = F.shape
    S = sine_matrix(nx)
    fhat = (2.0 / (nx + 1)) * (F @ S)              # [Ny][Nx]: row j, mode k
    # one Toeplitz system per mode, packed mode-major (mode k: its Ny values)
    rhs = np.ascontiguousarray((hy * hy) * fhat.T).reshape(-1)
    off = np.arange(nx + 1, dtype=np.int64) * ny
    t0 = 2.0 + hy * hy * mode_eigenvalues(nx, hx)
    v = orc.solve_varlen(rhs, off, -1.0, t0, -1.0).reshape(nx, ny)
    return v.T @ S                                  # u_ij = sum_k v_kj sin(pi k i / (Nx+1))


def eigen_solution(nx: int, ny: int, p: int, q: int, hx: float, hy: float):
    """F = sin(pi p i / (Nx+1)) sin(pi q j / (Ny+1)) and its exact discrete
    solution F / lambda_pq, lambda_pq = mu_p(hx) + mu_q(hy)."""
    i = np.arange(1, nx + 1)
    j = np.arange(1, ny + 1)
    F = np.outer(np.sin(math.pi * q * j / (ny + 1)), np.sin(math.pi * p * i / (nx + 1)))
    lam = (4.0 / hx ** 2) * math.sin(math.pi * p / (2 * (nx + 1))) ** 2 + \
          (4.0 / hy ** 2) * math.sin(math.pi * q / (2 * (ny + 1))) ** 2
    return F, F / lam
