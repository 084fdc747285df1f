"""Pins of the 3D Poisson oracle (sine transform along x, then
Peaceman-Rachford ADI on each mode's (y, z) plane; Sec. 3.5) on the CPU:

* the dense Kronecker-sum seven-point solve on small grids, within the ADI
  error bound;
* the closed-form discrete eigenfunctions, whose ADI result is known exactly
  (each eigenmode is multiplied by prod_j r_j(lambda_y) r_j(lambda_z));
* the optimality certificate of the ADI parameters: for the rational minimax
  problem on [a, b] the optimal set is the one whose error function
  equioscillates at J + 1 points (end points included), and it is symmetric
  under lambda -> ab / lambda; the single optimal parameter is sqrt(ab);
* the iteration count is minimal, measured on a dense grid, and falls with
  the mode index;

plus planted mistakes in a copy of the module that the pins must catch."""
import importlib.util
import math

import numpy as np
import pytest

import oracle
from oracle import poisson3d as P3


def _d1(n, h):
    return (np.diag(np.full(n, 2.0)) - np.diag(np.ones(n - 1), 1) -
            np.diag(np.ones(n - 1), -1)) / (h * h)


def _dense(nx, ny, nz, hx, hy, hz):
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(Iz, np.kron(Iy, _d1(nx, hx))) + np.kron(Iz, np.kron(_d1(ny, hy), Ix)) +
            np.kron(_d1(nz, hz), np.kron(Iy, Ix)))


def _rel2(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def _grid_max(om, a, b, n=40001):
    """max |prod_j r_j| over a dense log-spaced grid of [a, b] plus the
    parameters themselves' neighbourhoods (where the factor vanishes)."""
    lam = np.geomspace(a, b, n)
    return float(np.max(np.abs(P3.adi_factor(om, lam))))


def pin_dense(mod, seed=0):
    rng = np.random.default_rng(seed)
    for (nx, ny, nz), eps in (((1, 1, 1), 1e-13), ((3, 4, 5), 1e-13), ((6, 5, 7), 1e-6),
                              ((9, 8, 3), 1e-13), ((4, 1, 6), 1e-8), ((5, 7, 1), 1e-8)):
        hx, hy, hz = rng.uniform(0.03, 0.3, 3)
        F = rng.standard_normal((nz, ny, nx))
        U = mod.solve(F, hx, hy, hz, eps=eps, orc=oracle)
        ref = np.linalg.solve(_dense(nx, ny, nz, hx, hy, hz), F.reshape(-1)).reshape(nz, ny, nx)
        err = _rel2(U, ref)
        assert err <= eps + 1e-13, (nx, ny, nz, eps, err)


def pin_eigen(mod):
    nx, ny, nz, hx, hy, hz = 15, 12, 9, 1 / 16, 0.7 / 13, 1.3 / 10
    for p, q, r in ((1, 1, 1), (4, 11, 2), (15, 1, 9), (8, 6, 5)):
        F, Uex, Uadi = mod.eigen_case(nx, ny, nz, p, q, r, hx, hy, hz, eps=1e-5)
        U = mod.solve(F, hx, hy, hz, eps=1e-5, orc=oracle)
        assert _rel2(U, Uadi) < 1e-12, (p, q, r, _rel2(U, Uadi))
        # the closed form itself is within the bound of the exact solution
        assert _rel2(Uadi, Uex) <= 1e-5 * (1 + 1e-9)


def pin_parameters(mod):
    for a, b in ((1.0, 1.0), (1.0, 3.0), (2.5, 1e3), (14.8, 1.05e6)):
        om1 = mod.adi_parameters(a, b, 1)
        assert abs(om1[0] - math.sqrt(a * b)) <= 1e-13 * math.sqrt(a * b)
        for J in (2, 5, 12):
            om = mod.adi_parameters(a, b, J)
            assert np.all(np.diff(om) <= 0) and om[-1] >= a * (1 - 1e-14) and om[0] <= b
            assert np.allclose(om * om[::-1], a * b, rtol=1e-12)
            dJ = abs(P3.adi_factor(om, a))
            assert abs(abs(P3.adi_factor(om, b)) - dJ) <= 1e-12 * max(dJ, 1e-300)
            if a == b:
                continue
            gmax = _grid_max(om, a, b)
            assert gmax <= dJ * (1 + 1e-9), (a, b, J, gmax, dJ)
            # equioscillation: the factor reaches +-d_J at J + 1 points with
            # alternating signs (the end points and J - 1 interior extrema)
            lam = np.geomspace(a, b, 200001)
            f = P3.adi_factor(om, lam)
            ext = [0] + [i for i in range(1, lam.size - 1)
                         if (abs(f[i]) >= abs(f[i - 1]) and abs(f[i]) >= abs(f[i + 1]))] + \
                  [lam.size - 1]
            peaks = [f[i] for i in ext if abs(f[i]) >= dJ * (1 - 1e-5)]
            assert len(peaks) == J + 1, (a, b, J, len(peaks))
            assert all(peaks[i] * peaks[i + 1] < 0 for i in range(J))


def pin_count(mod):
    eps = 1e-10
    for a, b in ((1.0, 3.0), (3.0, 7e2), (14.8, 1.05e6)):
        J = mod.adi_count(a, b, eps)
        assert _grid_max(P3.adi_parameters(a, b, J), a, b) ** 2 <= eps * (1 + 1e-9)
        if J > 1:
            assert _grid_max(P3.adi_parameters(a, b, J - 1), a, b) ** 2 > eps
    modes = mod.plan(63, 40, 50, 1 / 64, 1 / 41, 1 / 51, 1e-13)
    counts = [m[3] for m in modes]
    assert all(counts[i] >= counts[i + 1] for i in range(len(counts) - 1))
    assert counts[0] > counts[-1]


PINS = [pin_dense, pin_eigen, pin_parameters, pin_count]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(P3)


def test_laplacian_is_the_seven_point_stencil():
    rng = np.random.default_rng(3)
    nx, ny, nz, hx, hy, hz = 5, 4, 3, 0.3, 0.2, 0.45
    U = rng.standard_normal((nz, ny, nx))
    assert np.allclose(P3.laplacian(U, hx, hy, hz).reshape(-1),
                       _dense(nx, ny, nz, hx, hy, hz) @ U.reshape(-1), rtol=0, atol=1e-11)


def test_residual_at_a_larger_grid():
    """31 x 20 x 17 with unequal spacings: the seven-point residual of the
    result is at the ADI bound times the operator's norm."""
    rng = np.random.default_rng(7)
    nx, ny, nz, hx, hy, hz = 31, 20, 17, 1 / 32, 0.9 / 21, 1.2 / 18
    F = rng.standard_normal((nz, ny, nx))
    U = P3.solve(F, hx, hy, hz, eps=1e-13)
    assert _rel2(P3.laplacian(U, hx, hy, hz), F) < 1e-11


MUTANTS = {
    "even_split": ("R = w * V - (second_difference(V, 0, hz) + 0.5 * mu * V) + G",
                   "R = w * V - (second_difference(V, 0, hz) + mu * V) + G"),
    "rhs_sign": ("R = w * V1 - (second_difference(V1, 1, hy) + 0.5 * mu * V1) + G",
                 "R = w * V1 + (second_difference(V1, 1, hy) + 0.5 * mu * V1) + G"),
    "axis_swap": ("R = w * V - (second_difference(V, 0, hz)",
                  "R = w * V - (second_difference(V, 1, hz)"),
    "spacing_swap": ("2.0 + hz * hz * (w + 0.5 * mu), -1.0).T",
                     "2.0 + hy * hy * (w + 0.5 * mu), -1.0).T"),
    "dn_argument": ("(2 * j - 1) * K / (2 * J)", "j * K / J"),
    "modulus": ("m = 1 - (A / B) ** 2", "m = 1 - (A / B)"),
    "transform_scale": ("fhat = (2.0 / (nx + 1)) * (F @ S)", "fhat = (1.0 / (nx + 1)) * (F @ S)"),
    "count_rule": ("if adi_bound(a, b, J) ** 2 <= eps:", "if adi_bound(a, b, J) <= eps:"),
    "interval": ("return mu / 2 + min(ly[0], lz[0]), mu / 2 + max(ly[-1], lz[-1])",
                 "return mu / 2 + max(ly[0], lz[0]), mu / 2 + max(ly[-1], lz[-1])"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    find, repl = MUTANTS[name]
    src = open(P3.__file__).read()
    assert find in src, name
    path = tmp_path / f"p3_{name}.py"
    path.write_text(src.replace(find, repl, 1))
    spec = importlib.util.spec_from_file_location(f"p3_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    caught = []
    for pin in PINS:
        try:
            pin(mod)
        except (AssertionError, ValueError, RuntimeError, np.linalg.LinAlgError):
            caught.append(pin.__name__)
    assert caught, f"no pin caught {name}"
