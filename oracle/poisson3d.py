"""TEST INFRASTRUCTURE ONLY: plain CPU reference of the 3D Poisson solve of
Sec. 3.5: a sine transform along one axis turns the 3D problem into
independent 2D problems, and each of those is solved by the alternating
direction implicit (ADI) method, whose half-steps are series of tridiagonal
Toeplitz solves.

Problem: -(u_xx + u_yy + u_zz) = f on a box with u = 0 on the boundary, the
seven-point scheme on Nx x Ny x Nz interior points (spacings hx, hy, hz), F
and U stored [Nz][Ny][Nx] (x contiguous).  The transformed axis is x here
(the paper transforms its third index; the operator is symmetric in the
three axes, so the choice is one of data layout).

1. Sine transform along x: fhat_k = (2 / (Nx+1)) sum_i f_i sin(pi k i / (Nx+1)).
   Mode k leaves the 2D problem (A_y + A_z + mu_k) v_k = fhat_k on the
   (y, z) plane, mu_k = (4 / hx^2) sin^2(pi k / (2 (Nx+1))), where A_y, A_z
   are the second-difference operators (2 v_j - v_{j-1} - v_{j+1}) / h^2.
2. Peaceman-Rachford ADI on that plane with the shift split evenly,
   A1 = A_y + mu_k / 2 and A2 = A_z + mu_k / 2, starting from v = 0:
       (w_j + A1) v'  = (w_j - A2) v  + fhat,
       (w_j + A2) v'' = (w_j - A1) v' + fhat,     j = 1 .. J_k.
   Each half-step is one Toeplitz system per line, solved by the pinned
   Thomas oracle: (1/h^2) tridiag{-1, 2 + h^2 (w_j + mu_k / 2), -1}.
3. Inverse sine transform along x: u_i = sum_k v_k sin(pi k i / (Nx+1)).

The paper does not fix the ADI parameters.  Here they are the optimal
(Jordan, Wachspress) set for the interval [a, b] that holds the spectra of
both A1 and A2: w_j = b dn((2j - 1) K / (2J), m), m = 1 - (a/b)^2, K = K(m)
(Jacobi elliptic dn and the complete elliptic integral, from mpmath).
Because A1 and A2 commute, the error of eigenmode (p, q) after the cycle is
v_exact times prod_j r_j(lambda_p) r_j(lambda_q), r_j(l) = (w_j - l)/(w_j + l);
J_k is the smallest J whose bound d_J^2 <= eps, where d_J = max over [a, b] of
|prod_j r_j| is attained at the end point a for this set (the tests check it
on a dense grid).  As mu_k grows, b/a shrinks and so does J_k (the decrease
of the iteration count with the mode index that Sec. 3.5 describes).
Only tests/ and bench.py's CPU leg use this module; the product never does.
"""
import math

import mpmath as mp
import numpy as np

from oracle.poisson2d import mode_eigenvalues, sine_matrix

J_CAP = 400


def adi_parameters(a: float, b: float, J: int) -> np.ndarray:
    """The J optimal Peaceman-Rachford parameters for spectra in [a, b]."""
    if not (0.0 < a <= b):
        raise ValueError("need 0 < a <= b")
    with mp.workdps(40):
        A, B = mp.mpf(a), mp.mpf(b)
        m = 1 - (A / B) ** 2
        K = mp.ellipk(m)
        return np.array([float(B * mp.ellipfun("dn", (2 * j - 1) * K / (2 * J), m=m))
                         for j in range(1, J + 1)])


def adi_factor(om, lam) -> np.ndarray:
    """prod_j (w_j - lam) / (w_j + lam) (the ADI error factor of one direction)."""
    lam = np.asarray(lam, dtype=np.float64)
    out = np.ones_like(lam)
    for w in om:
        out = out * (w - lam) / (w + lam)
    return out


def adi_bound(a: float, b: float, J: int) -> float:
    """d_J: the largest |factor| over [a, b] for the optimal set (at lam = a)."""
    return float(abs(adi_factor(adi_parameters(a, b, J), a)))


def adi_count(a: float, b: float, eps: float) -> int:
    """Smallest J with d_J^2 <= eps."""
    for J in range(1, J_CAP + 1):
        if adi_bound(a, b, J) ** 2 <= eps:
            return J
    raise RuntimeError("ADI parameter count above the cap")


def line_eigenvalues(n: int, h: float) -> np.ndarray:
    """Spectrum of the second-difference operator of n interior points."""
    return mode_eigenvalues(n, h)


def mode_interval(mu: float, ny: int, nz: int, hy: float, hz: float):
    """[a, b] holding the spectra of A1 = A_y + mu/2 and A2 = A_z + mu/2."""
    ly, lz = line_eigenvalues(ny, hy), line_eigenvalues(nz, hz)
    return mu / 2 + min(ly[0], lz[0]), mu / 2 + max(ly[-1], lz[-1])


def plan(nx, ny, nz, hx, hy, hz, eps):
    """Per mode k: (mu_k, a_k, b_k, J_k, parameters)."""
    mus = mode_eigenvalues(nx, hx)
    out = []
    for mu in mus:
        a, b = mode_interval(mu, ny, nz, hy, hz)
        J = adi_count(a, b, eps)
        out.append((mu, a, b, J, adi_parameters(a, b, J)))
    return out


def second_difference(V: np.ndarray, axis: int, h: float) -> np.ndarray:
    """(2 v_j - v_{j-1} - v_{j+1}) / h^2 along one axis, zero outside."""
    P = np.pad(V, [(1, 1) if d == axis else (0, 0) for d in range(V.ndim)])
    sl = lambda lo, hi: tuple(slice(lo, hi) if d == axis else slice(None)
                              for d in range(V.ndim))
    n = V.shape[axis]
    return (2.0 * V - P[sl(0, n)] - P[sl(2, n + 2)]) / (h * h)


def adi_mode(G, mu, hy, hz, om, orc):
    """The Peaceman-Rachford cycle for one mode: G and the result are
    [Nz][Ny] (y along axis 1, z along axis 0)."""
    V = np.zeros_like(G)
    for w in om:
        # (w + A1) V' = (w - A2) V + G, one system along y per z
        R = w * V - (second_difference(V, 0, hz) + 0.5 * mu * V) + G
        V1 = orc.solve(hy * hy * R, -1.0, 2.0 + hy * hy * (w + 0.5 * mu), -1.0)
        # (w + A2) V'' = (w - A1) V' + G, one system along z per y
        R = w * V1 - (second_difference(V1, 1, hy) + 0.5 * mu * V1) + G
        V = orc.solve(np.ascontiguousarray((hz * hz * R).T), -1.0,
                      2.0 + hz * hz * (w + 0.5 * mu), -1.0).T
    return np.ascontiguousarray(V)


def solve(F, hx, hy, hz, eps=1e-13, orc=None, modes=None):
    """U for the seven-point problem by the three steps above.  ``modes``
    (from ``plan``) may be passed to reuse the parameters."""
    if orc is None:
        import oracle as orc
    F = np.asarray(F, dtype=np.float64)
    nz, ny, nx = F.shape
    S = sine_matrix(nx)
    fhat = (2.0 / (nx + 1)) * (F @ S)              # [Nz][Ny][k]
    if modes is None:
        modes = plan(nx, ny, nz, hx, hy, hz, eps)
    V = np.empty_like(fhat)
    for k, (mu, _a, _b, _J, om) in enumerate(modes):
        V[:, :, k] = adi_mode(np.ascontiguousarray(fhat[:, :, k]), mu, hy, hz, om, orc)
    return V @ S


def laplacian(U, hx, hy, hz):
    """The seven-point operator applied to U ([Nz][Ny][Nx], zero boundary)."""
    U = np.asarray(U, dtype=np.float64)
    return (second_difference(U, 2, hx) + second_difference(U, 1, hy) +
            second_difference(U, 0, hz))


def eigen_case(nx, ny, nz, p, q, r, hx, hy, hz, eps=1e-13):
    """F = sin(pi p i/(Nx+1)) sin(pi q j/(Ny+1)) sin(pi r l/(Nz+1)), the exact
    discrete solution F / lambda, and the ADI result in closed form,
    (F / lambda) (1 - prod_j r_j(lam_y + mu/2) r_j(lam_z + mu/2))."""
    i, j, l = np.arange(1, nx + 1), np.arange(1, ny + 1), np.arange(1, nz + 1)
    F = (np.sin(math.pi * r * l / (nz + 1))[:, None, None] *
         np.sin(math.pi * q * j / (ny + 1))[None, :, None] *
         np.sin(math.pi * p * i / (nx + 1))[None, None, :])
    mu = mode_eigenvalues(nx, hx)[p - 1]
    ly = line_eigenvalues(ny, hy)[q - 1]
    lz = line_eigenvalues(nz, hz)[r - 1]
    lam = mu + ly + lz
    a, b = mode_interval(mu, ny, nz, hy, hz)
    om = adi_parameters(a, b, adi_count(a, b, eps))
    rho = float(adi_factor(om, ly + mu / 2) * adi_factor(om, lz + mu / 2))
    return F, F / lam, F / lam * (1.0 - rho)
