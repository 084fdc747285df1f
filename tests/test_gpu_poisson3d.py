"""GPU parity of the 3D Poisson solve of Sec. 3.5 (sine transform along x,
Peaceman-Rachford ADI on every mode's (y, z) plane through the strided line
solves, inverse transform) against the CPU oracle, through the C ABI: the
ADI schedule (iteration counts and parameters), the solution on grids up to
63 x 64 x 65 and on grids whose lines along y or z are longer than 1024 (the
tiled line solves), element by element against the oracle's ADI iterates
(the same parameters), and at the benchmark size (511^3, 2^9 intervals per
side) the closed-form eigenmode results and the seven-point residual.

Inputs: F ~ N(0, 1); spacings drawn in [0.005, 0.1] (unequal hx, hy, hz)."""
import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host
from oracle import poisson3d as P3

pytestmark = pytest.mark.gpu


def _tdt():
    import paper_1002_2469_amd as tdt
    return tdt


def _rel2(x, y):
    """Relative 2-norm: used only against the exact discrete solution, whose
    ADI bound eps is a 2-norm bound."""
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def _kappa(nx, ny, nz, hx, hy, hz):
    """2-norm condition number of the seven-point operator (closed-form
    spectrum: the largest over the smallest eigenvalue)."""
    mu = P3.mode_eigenvalues(nx, hx)
    ly, lz = P3.line_eigenvalues(ny, hy), P3.line_eigenvalues(nz, hz)
    return float((mu[-1] + ly[-1] + lz[-1]) / (mu[0] + ly[0] + lz[0]))


def _tol(J, kappa):
    """Bound on the rounding difference of two evaluations of the same ADI
    iterates: 2 J line solves, each backward stable with a backward error of
    a few units of rounding, carried to the result by at most the operator's
    condition number: 8 J u kappa (u = 2^-53), at least 1e-13."""
    return max(1e-13, 8 * J * 2.0 ** -53 * kappa)


def _check_elementwise(U, ref, tol, what):
    """Every element against the array's max-norm (normwise inf), and, for
    lines of 16 points or more along x, every line against its own
    max-norm."""
    e = oracle.rel_err(U, ref)
    assert e <= tol, (what, "inf-norm", e, tol)
    if U.shape[-1] >= 16:
        rows = oracle.rel_err_rows(U.reshape(-1, U.shape[-1]), ref.reshape(-1, ref.shape[-1]))
        assert rows.max() <= tol, (what, "worst line", int(rows.argmax()), rows.max(), tol)
    print(f"[err] {what}: inf-norm {e:.2e} (tol {tol:.1e})", flush=True)


# Nx = 127, 255, 1023 take the fused row transform, the others hipFFT's;
# lines of more than 1024 points run in tiles of 512 (along y, along z, both)
GRIDS = [(1, 1, 1), (3, 4, 5), (7, 9, 4), (16, 17, 15), (31, 20, 17), (12, 1, 40),
         (20, 33, 1), (63, 64, 65), (127, 20, 30), (255, 17, 9), (1023, 3, 4),
         (5, 1100, 20), (127, 1030, 3), (7, 20, 1300), (2, 1030, 1029)]


@pytest.mark.parametrize("nx,ny,nz", GRIDS)
def test_poisson3d_grids(nx, ny, nz):
    tdt = _tdt()
    rng = np.random.default_rng(nx * 10000 + ny * 100 + nz)
    hx, hy, hz = rng.uniform(0.005, 0.1, 3)
    eps = 1e-13
    F = rng.standard_normal((nz, ny, nx))
    print(f"[case] poisson3d {nx}x{ny}x{nz}", flush=True)
    solver = tdt.Poisson3D(nx, ny, nz, hx, hy, hz, eps)
    modes = P3.plan(nx, ny, nz, hx, hy, hz, eps)
    counts, om = solver.schedule()
    assert list(counts) == [m[3] for m in modes]
    for k, m in enumerate(modes):
        assert np.allclose(om[k, :m[3]], m[4], rtol=1e-13, atol=0)
    U = to_host(solver.solve(to_dev(F)))
    ref = P3.solve(F, hx, hy, hz, eps=eps, modes=modes)
    _check_elementwise(U, ref, _tol(max(counts), _kappa(nx, ny, nz, hx, hy, hz)),
                       f"{nx}x{ny}x{nz}")


def test_poisson3d_eps_levels():
    """A loose eps: the result follows the oracle's ADI iterates (same
    parameters), not the exact solution, and stays within eps of it."""
    tdt = _tdt()
    rng = np.random.default_rng(3)
    nx, ny, nz, hx, hy, hz = 24, 30, 28, 0.04, 0.03, 0.035
    F = rng.standard_normal((nz, ny, nx))
    for eps in (1e-4, 1e-8):
        print(f"[case] poisson3d eps={eps}", flush=True)
        solver = tdt.Poisson3D(nx, ny, nz, hx, hy, hz, eps)
        U = to_host(solver.solve(to_dev(F)))
        ref = P3.solve(F, hx, hy, hz, eps=eps)
        counts, _ = solver.schedule()
        _check_elementwise(U, ref, _tol(max(counts), _kappa(nx, ny, nz, hx, hy, hz)),
                           f"eps={eps}")
        exact = P3.solve(F, hx, hy, hz, eps=1e-15)
        assert _rel2(U, exact) <= eps * 1.001 + 1e-12


def test_poisson3d_eigenmodes_medium():
    tdt = _tdt()
    nx, ny, nz, hx, hy, hz = 127, 100, 90, 1 / 128, 0.9 / 101, 1.1 / 91
    eps = 1e-6
    solver = tdt.Poisson3D(nx, ny, nz, hx, hy, hz, eps)
    for p, q, r in ((1, 1, 1), (64, 3, 80), (127, 100, 90), (5, 50, 2)):
        print(f"[case] poisson3d eigen ({p},{q},{r})", flush=True)
        F, Uex, Uadi = P3.eigen_case(nx, ny, nz, p, q, r, hx, hy, hz, eps=eps)
        U = to_host(solver.solve(to_dev(F)))
        e = oracle.rel_err(U, Uadi)
        assert e < 1e-12, (p, q, r, e)


def test_poisson3d_benchmark_size():
    """511^3 (the benchmark): closed-form eigenmodes and the seven-point
    residual of a random right-hand side (relative 2-norm)."""
    tdt = _tdt()
    n, h, eps = 511, 1.0 / 512, 1e-13
    solver = tdt.Poisson3D(n, n, n, h, h, h, eps)
    for p, q, r in ((1, 1, 1), (2, 300, 7), (511, 511, 511)):
        print(f"[case] poisson3d 511^3 eigen ({p},{q},{r})", flush=True)
        F, Uex, Uadi = P3.eigen_case(n, n, n, p, q, r, h, h, h, eps=eps)
        U = to_host(solver.solve(to_dev(F)))
        e = oracle.rel_err(U, Uadi)
        assert e < 1e-11, (p, q, r, e)
        del F, Uex, Uadi, U
    print("[case] poisson3d 511^3 residual", flush=True)
    F = np.random.default_rng(0).standard_normal((n, n, n))
    U = to_host(solver.solve(to_dev(F)))
    R = P3.laplacian(U, h, h, h)
    assert _rel2(R, F) < 1e-9
    assert oracle.rel_err(R, F) < 1e-9


def test_poisson3d_errors_and_repeatable():
    tdt = _tdt()
    from paper_1002_2469_amd import _lib
    for args in ((0, 5, 5, 0.1, 0.1, 0.1, 1e-10), (5, 2**24 + 1, 5, 0.1, 0.1, 0.1, 1e-10),
                 (5, 5, 5, -0.1, 0.1, 0.1, 1e-10), (5, 5, 5, 0.1, 0.1, 0.1, 0.0),
                 (5, 5, 5, 0.1, 0.1, 0.1, 1.0), (4000, 1000, 5, 0.1, 0.1, 0.1, 1e-10)):
        with pytest.raises(_lib.TDTError):
            tdt.Poisson3D(*args)
    rng = np.random.default_rng(2)
    F = to_dev(rng.standard_normal((20, 30, 40)))
    print("[case] poisson3d repeatable", flush=True)
    solver = tdt.Poisson3D(40, 30, 20, 0.01, 0.02, 0.015)
    assert np.array_equal(to_host(solver.solve(F)), to_host(solver.solve(F)))
    with pytest.raises(_lib.TDTError):
        solver.solve(F, F)
