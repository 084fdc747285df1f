"""GPU parity of the 2D Poisson solve by separation of variables (Sec. 3.2)
against the CPU oracle (explicit sine transforms and Thomas per mode, itself
pinned to the dense Kronecker-sum solve), through the C ABI; at the
benchmark size (8191 x 8191) against the closed-form discrete eigenfunctions
and the five-point residual, which hold at any size.

Inputs: F ~ N(0, 1), spacings drawn in [0.002, 0.2] (unequal hx, hy)."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host
from oracle import poisson2d as P2

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


def _tdt():
    import paper_1002_2469_amd as tdt
    return tdt


def kappa(nx, ny, hx, hy):
    """Condition number of the five-point operator (closed-form spectrum)."""
    lo = P2.mode_eigenvalues(nx, hx)[0] + P2.mode_eigenvalues(ny, hy)[0]
    hi = P2.mode_eigenvalues(nx, hx)[-1] + P2.mode_eigenvalues(ny, hy)[-1]
    return hi / lo


def tol(nx, ny, hx, hy):
    return max(1e-12, 8 * U64 * kappa(nx, ny, hx, hy))


# Nx + 1 = 2 N2 with N2 a power of two in [64, 4096] takes the fused row
# transform (127 .. 8191), the other sizes hipFFT's
# (in f64 these solve the mode systems in place as a strided batch: one
# column per system up to Ny = 1024, tiles of 512 rows above, e.g. 255 x 3001
# with a last tile of 441 rows and 511 x 1537 with one of 1 row)
GRIDS = [(1, 1), (1, 9), (7, 1), (31, 17), (64, 64), (100, 257), (513, 700), (16, 20000),
         (127, 3), (255, 130), (1023, 41), (2047, 5), (4095, 19), (255, 3001), (511, 1537)]


@pytest.mark.parametrize("nx,ny", GRIDS)
@pytest.mark.parametrize("dtype", ["f64", "f32_refine"])
def test_poisson_grids(nx, ny, dtype):
    tdt = _tdt()
    rng = np.random.default_rng(nx * 1000 + ny)
    hx, hy = rng.uniform(0.002, 0.2), rng.uniform(0.002, 0.2)
    F = rng.standard_normal((ny, nx))
    print(f"[case] poisson nx={nx} ny={ny} dtype={dtype}", flush=True)
    solver = tdt.Poisson2D(nx, ny, hx, hy, dtype)
    U = to_host(solver.solve(to_dev(F)))
    ref = P2.solve(F, hx, hy)
    err = oracle.rel_err(U, ref)
    assert err <= tol(nx, ny, hx, hy), (nx, ny, dtype, err, tol(nx, ny, hx, hy))


@pytest.mark.parametrize("whole", [0, 8])
def test_poisson_line_paths(whole):
    """Mode systems of 3 tiles, solved whole by one workgroup each or by the
    three-kernel path of the line plan."""
    tdt = _tdt()
    rng = np.random.default_rng(5)
    nx, ny, hx, hy = 40, 3 * 8192 + 11, 0.01, 0.003
    F = rng.standard_normal((ny, nx))
    print(f"[case] poisson line path whole={whole}", flush=True)
    solver = tdt.Poisson2D(nx, ny, hx, hy)
    solver.set_line_option("whole_max_tiles", whole)
    U = to_host(solver.solve(to_dev(F)))
    assert oracle.rel_err(U, P2.solve(F, hx, hy)) <= tol(nx, ny, hx, hy)


@pytest.mark.parametrize("n,dtype", [(8191, "f64"), (2047, "f32_refine")])
def test_poisson_benchmark_size(n, dtype):
    """8191 x 8191 (the benchmark, 2^13 intervals per side): closed-form
    eigenfunctions (U = F / lambda_pq) and the five-point residual of a random
    right-hand side.  The refinement path is checked at 2047 x 2047: at 8191
    the lowest modes' line systems have cond ~ 1e7, where float sweeps no
    longer contract."""
    tdt = _tdt()
    h = 1.0 / (n + 1)
    solver = tdt.Poisson2D(n, n, h, h, dtype)
    t = tol(n, n, h, h)
    for p, q in ((1, 1), (3, n // 2), (n, 17)):
        print(f"[case] poisson {n}^2 dtype={dtype} eigen ({p},{q})", flush=True)
        F, Uex = P2.eigen_solution(n, n, p, q, h, h)
        U = to_host(solver.solve(to_dev(F)))
        assert oracle.rel_err(U, Uex) <= t, (p, q, oracle.rel_err(U, Uex), t)
    print(f"[case] poisson {n}^2 dtype={dtype} residual", flush=True)
    F = np.random.default_rng(0).standard_normal((n, n))
    U = to_host(solver.solve(to_dev(F)))
    assert oracle.rel_err(P2.laplacian(U, h, h), F) <= t


def test_poisson_refinement_refused_where_it_cannot_converge():
    """At 8191 x 8191 the lowest mode's line system has cond_2 = 1.4e7, above
    the limit where float sweeps still contract a refinement to double
    accuracy: the f32_refine handle is refused with TDT_ERR_NOT_CONVERGED
    (the f64 one is made); at 2047 x 2047 (cond_2 = 8.5e5) it is made."""
    tdt = _tdt()
    from paper_1002_2469_amd import _lib
    h = 1.0 / 8192
    with pytest.raises(_lib.TDTError) as e:
        tdt.Poisson2D(8191, 8191, h, h, "f32_refine")
    assert e.value.status == _lib.TDT_ERR_NOT_CONVERGED
    tdt.Poisson2D(8191, 8191, h, h, "f64").close()
    tdt.Poisson2D(2047, 2047, 1.0 / 2048, 1.0 / 2048, "f32_refine").close()


def test_poisson_errors_and_repeatable():
    tdt = _tdt()
    from paper_1002_2469_amd import _lib
    with pytest.raises(_lib.TDTError):
        tdt.Poisson2D(0, 5, 0.1, 0.1)
    with pytest.raises(_lib.TDTError):
        tdt.Poisson2D(5, 5, -0.1, 0.1)
    with pytest.raises(ValueError):
        tdt.Poisson2D(5, 5, 0.1, 0.1, "f32")
    rng = np.random.default_rng(2)
    F = to_dev(rng.standard_normal((300, 200)))
    print("[case] poisson repeatable", flush=True)
    solver = tdt.Poisson2D(200, 300, 0.01, 0.02)
    assert np.array_equal(to_host(solver.solve(F)), to_host(solver.solve(F)))


@pytest.mark.parametrize("nx,ny,dtype", [(255, 2000, "f64"), (255, 40, "f32_refine"),
                                         (100, 30, "f64")])
def test_poisson_profile(nx, ny, dtype):
    """The handle's events: three positive durations per recorded solve (the
    in-place strided path, the transposing path, the hipFFT path), cleared
    by the read; the solve is unchanged by recording."""
    tdt = _tdt()
    rng = np.random.default_rng(nx + ny)
    F = to_dev(rng.standard_normal((ny, nx)))
    print(f"[case] poisson profile nx={nx} ny={ny} {dtype}", flush=True)
    solver = tdt.Poisson2D(nx, ny, 0.01, 0.02, dtype)
    ref = to_host(solver.solve(F))
    solver.profile(True)
    U1 = to_host(solver.solve(F))
    solver.solve(F)
    prof = solver.profile_read()
    assert prof["solves"] == 2
    assert prof["forward_ms"] > 0 and prof["line_ms"] > 0 and prof["inverse_ms"] > 0
    assert solver.profile_read()["solves"] == 0
    solver.profile(False)
    solver.solve(F)
    assert solver.profile_read()["solves"] == 0
    assert np.array_equal(U1, ref)
