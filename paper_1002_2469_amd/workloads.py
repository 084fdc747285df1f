"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This module holds no arithmetic of the solver: it only draws matrices
(t_-1, t_0, t_1), system sizes and right-hand sides.  Every draw uses
``numpy.random.default_rng(seed)`` (PCG64) in float64, so the oracle and the
GPU path always see identical inputs.

The five workloads follow the problem classes of the paper:
  * ``single_small``  one system, N = 65536, T = tridiag{-1, 4, -1};
  * ``single_large``  the single-system case of the title, N = 2**26,
                      nonsymmetric T = tridiag{-0.9, 2.5, -1.1}
                      (dominance ratio |t0| / (|t1| + |t-1|) = 1.25);
  * ``series``        a series with a constant matrix (eq. (2)): M = 8192
                      right-hand sides of N = 8192, T = tridiag{-1, 3, -1};
  * ``sov_batch``     the per-mode systems of a separation-of-variables Poisson
                      solve (Sec. 3.2, Sec. 4): 2048 systems, sizes log-uniform
                      in [256, 65536], t_{+-1} = 1 and
                      t_0,k = -(2 + 4 r_k^2 sin^2(k pi / (2 (K + 1)))),
                      r_k = hy/hx ~ U[0.5, 2];
  * ``diff_batch``    1024 systems of N = 16384 with t_0 ~ U[2.5, 4] and
                      independent t_-1, t_1 ~ U[-1, -0.5], plus the loss weights W.
The paper does not state the right-hand sides of its experiments; the
distributions below are this project's choice.
"""
from __future__ import annotations

import math

import numpy as np


def single_small(seed: int = 0, n: int = 65536, manufactured: bool = False) -> dict:
    rng = np.random.default_rng(seed)
    d = dict(name="single_small", t_m1=-1.0, t_0=4.0, t_1=-1.0, N=n, M=1)
    if manufactured:
        d["X_true"] = rng.uniform(-1.0, 1.0, size=n)
    else:
        d["F"] = rng.uniform(-1.0, 1.0, size=n)
    return d


def single_large(seed: int = 0, n: int = 1 << 26) -> dict:
    rng = np.random.default_rng(seed)
    return dict(name="single_large", t_m1=-0.9, t_0=2.5, t_1=-1.1, N=n, M=1,
                F=rng.standard_normal(n))


def series(seed: int = 0, n: int = 8192, m: int = 8192) -> dict:
    rng = np.random.default_rng(seed)
    return dict(name="series", t_m1=-1.0, t_0=3.0, t_1=-1.0, N=n, M=m,
                F=rng.uniform(-1.0, 1.0, size=(m, n)))


def sov_sizes(seed: int = 0, s: int = 2048, n_min: int = 256, n_max: int = 65536):
    rng = np.random.default_rng(seed)
    n = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=s)))
    return n.astype(np.int64), rng


def sov_batch(seed: int = 0, s: int = 2048, n_min: int = 256, n_max: int = 65536,
              k_modes: int | None = None) -> dict:
    """Mode k = 1..S uses the sin^2 shift of a K = ``k_modes`` (default S) sine
    transform; r_k = hy/hx is drawn per system."""
    sizes, rng = sov_sizes(seed, s, n_min, n_max)
    K = s if k_modes is None else k_modes
    r = rng.uniform(0.5, 2.0, size=s)
    k = np.arange(1, s + 1, dtype=np.float64)
    t0 = -(2.0 + 4.0 * r * r * np.sin(k * math.pi / (2.0 * (K + 1))) ** 2)
    offsets = np.zeros(s + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    F = rng.standard_normal(int(offsets[-1]))
    return dict(name="sov_batch", S=s, offsets=offsets, sizes=sizes,
                t_m1=np.ones(s), t_0=t0, t_1=np.ones(s), F=F)


def sov_neumann_batch(seed: int = 0, s: int = 2048, n_min: int = 256,
                      n_max: int = 65536) -> dict:
    """The separation-of-variables batch with Neumann ends in the solved
    direction: the mirrored ghost value adds t_-1 = 1 to the first and t_1 = 1
    to the last diagonal entry, a quasi-Toeplitz matrix with psi = chi = 1."""
    d = sov_batch(seed, s, n_min, n_max)
    d.update(name="sov_neumann_batch", psi=np.ones(s), chi=np.ones(s))
    return d


def general_rows(rng: np.random.Generator, n: int, ratio_lo: float = 1.1,
                 ratio_hi: float = 1.6) -> tuple:
    """Rows of a variable-coefficient diffusion-reaction operator with a
    skewed (nonsymmetric) stencil: kappa(x) = exp(0.5 sin(2 pi x) + 0.3 xi),
    a_i = -kappa_{i-1/2} (1 + e_i), c_i = -kappa_{i+1/2} (1 - e_i) with
    e_i ~ U[-0.3, 0.3], and b_i = r_i (|a_i| + |c_i|) with the dominance ratio
    r_i ~ U[ratio_lo, ratio_hi] (the reaction term)."""
    x = (np.arange(n + 1) + 0.5) / (n + 1)
    kap = np.exp(0.5 * np.sin(2.0 * math.pi * x) + 0.3 * rng.uniform(-1.0, 1.0, n + 1))
    e = rng.uniform(-0.3, 0.3, n)
    a = -kap[:-1] * (1.0 + e)
    c = -kap[1:] * (1.0 - e)
    b = rng.uniform(ratio_lo, ratio_hi, n) * (np.abs(a) + np.abs(c))
    return a, b, c


def general_series(seed: int = 0, n: int = 1 << 20, m: int = 64) -> dict:
    """M right-hand sides [M][N] sharing one general tridiagonal matrix."""
    rng = np.random.default_rng(seed)
    a, b, c = general_rows(rng, n)
    F = rng.standard_normal((m, n))
    return dict(name="general_series", N=n, M=m, a=a, b=b, c=c, F=F)


def poisson2d(seed: int = 0, n: int = 8191) -> dict:
    """The 2D Poisson problem of the separation-of-variables application on
    the unit square cut into n + 1 = 2^13 intervals per side (n x n interior
    points, h = 1 / (n + 1)), F ~ N(0, 1) [Ny][Nx].  A power-of-two interval
    count keeps the sine transforms' FFT length 2 (n + 1) a power of two."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (n + 1)
    return dict(name="poisson2d", nx=n, ny=n, hx=h, hy=h, F=rng.standard_normal((n, n)))


def poisson3d(seed: int = 0, n: int = 511) -> dict:
    """The 3D Poisson problem of Sec. 3.5 on the unit cube cut into
    n + 1 = 2^9 intervals per side (n^3 interior points, h = 1 / (n + 1)),
    F ~ N(0, 1) [Nz][Ny][Nx]; the sine transform along x has FFT length
    n + 1, a power of two."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (n + 1)
    return dict(name="poisson3d", nx=n, ny=n, nz=n, hx=h, hy=h, hz=h,
                F=rng.standard_normal((n, n, n)))


def diff_batch(seed: int = 0, s: int = 1024, n: int = 16384) -> dict:
    rng = np.random.default_rng(seed)
    t0 = rng.uniform(2.5, 4.0, size=s)
    tm1 = rng.uniform(-1.0, -0.5, size=s)
    t1 = rng.uniform(-1.0, -0.5, size=s)
    F = rng.standard_normal((s, n))
    W = rng.standard_normal((s, n))
    offsets = np.arange(s + 1, dtype=np.int64) * n
    return dict(name="diff_batch", S=s, N=n, offsets=offsets,
                t_m1=tm1, t_0=t0, t_1=t1, F=F, W=W)


def random_system(rng: np.random.Generator, ratio_lo: float = 1.0, ratio_hi: float = 3.0,
                  symmetric: bool = False, signs: bool = True):
    """A random (t_-1, t_0, t_1) whose dominance ratio |t0|/(|t1|+|t-1|) lies
    in [ratio_lo, ratio_hi]; off-diagonals of either sign when ``signs``."""
    a = rng.uniform(0.2, 1.0)
    c = a if symmetric else rng.uniform(0.2, 1.0)
    if signs:
        a *= rng.choice([-1.0, 1.0])
        c *= rng.choice([-1.0, 1.0])
    ratio = rng.uniform(ratio_lo, ratio_hi)
    b = ratio * (abs(a) + abs(c)) * rng.choice([-1.0, 1.0])
    return float(a), float(b), float(c)
