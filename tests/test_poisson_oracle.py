"""Pins of the 2D Poisson oracle (separation of variables, Sec. 3.2) on the
CPU: the dense Kronecker-sum solve of the five-point system on small grids,
the five-point residual of the solution at a larger grid, the closed-form
discrete eigenfunctions, and the orthogonality of the sine vectors; plus
planted mistakes in a copy of the module that the pins must catch."""
import importlib.util
import math
import os

import numpy as np
import pytest

import oracle
from oracle import poisson2d as P2


def _dense(nx, ny, hx, hy):
    def d1(n, h):
        return (np.diag(np.full(n, 2.0)) - np.diag(np.ones(n - 1), 1) -
                np.diag(np.ones(n - 1), -1)) / (h * h)
    # U flattened row-major [Ny][Nx]: index j * Nx + i
    return np.kron(np.eye(ny), d1(nx, hx)) + np.kron(d1(ny, hy), np.eye(nx))


def _rel(x, y):
    return float(np.max(np.abs(x - y)) / np.max(np.abs(y)))


def pin_dense(mod, seed=0):
    rng = np.random.default_rng(seed)
    for nx, ny in ((1, 1), (1, 5), (4, 1), (7, 9), (16, 11), (20, 20)):
        hx, hy = rng.uniform(0.01, 0.2), rng.uniform(0.01, 0.2)
        F = rng.standard_normal((ny, nx))
        U = mod.solve(F, hx, hy, oracle)
        ref = np.linalg.solve(_dense(nx, ny, hx, hy), F.reshape(-1)).reshape(ny, nx)
        assert _rel(U, ref) < 1e-12, (nx, ny, _rel(U, ref))


def pin_residual(mod, seed=1):
    rng = np.random.default_rng(seed)
    nx, ny, hx, hy = 300, 257, 1.0 / 301, 0.7 / 258
    F = rng.standard_normal((ny, nx))
    U = mod.solve(F, hx, hy, oracle)
    assert _rel(mod.laplacian(U, hx, hy), F) < 1e-11


def pin_eigen(mod):
    nx, ny, hx, hy = 63, 40, 1.0 / 64, 2.0 / 41
    for p, q in ((1, 1), (5, 7), (63, 40), (31, 2)):
        F, Uex = mod.eigen_solution(nx, ny, p, q, hx, hy)
        assert _rel(mod.solve(F, hx, hy, oracle), Uex) < 1e-12, (p, q)


def pin_sine_orthogonality(mod):
    for n in (1, 2, 5, 64):
        S = mod.sine_matrix(n)
        assert np.allclose(S @ S, (n + 1) / 2.0 * np.eye(n), atol=1e-12 * n)


PINS = [pin_dense, pin_residual, pin_eigen, pin_sine_orthogonality]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(P2)


def test_laplacian_is_the_five_point_stencil():
    """The residual pin's operator against the dense matrix."""
    rng = np.random.default_rng(3)
    nx, ny, hx, hy = 6, 4, 0.3, 0.2
    U = rng.standard_normal((ny, nx))
    assert np.allclose(P2.laplacian(U, hx, hy).reshape(-1),
                       _dense(nx, ny, hx, hy) @ U.reshape(-1), rtol=0, atol=1e-12)


MUTANTS = {
    "normalisation": ("fhat = (2.0 / (nx + 1)) * (F @ S)", "fhat = (1.0 / (nx + 1)) * (F @ S)"),
    "eigenvalue_spacing": ("t0 = 2.0 + hy * hy * mode_eigenvalues(nx, hx)",
                           "t0 = 2.0 + hy * hy * mode_eigenvalues(nx, hy)"),
    "eigenvalue_angle": ("np.sin(np.pi * k / (2.0 * (nx + 1))) ** 2",
                         "np.sin(np.pi * k / (2.0 * nx)) ** 2"),
    "sine_index": ("np.sin(np.pi * np.outer(i, i) / (n + 1))",
                   "np.sin(np.pi * np.outer(i - 1, i) / (n + 1))"),
    "rhs_scale_dropped": ("rhs = np.ascontiguousarray((hy * hy) * fhat.T).reshape(-1)",
                          "rhs = np.ascontiguousarray(fhat.T).reshape(-1)"),
    "untransposed_modes": ("return v.T @ S", "return v.reshape(ny, nx) @ S"),
    "offdiagonal_sign": ("v = orc.solve_varlen(rhs, off, -1.0, t0, -1.0)",
                         "v = orc.solve_varlen(rhs, off, 1.0, t0, -1.0)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    find, repl = MUTANTS[name]
    src = open(P2.__file__).read()
    assert find in src, name
    path = tmp_path / f"p2_{name}.py"
    path.write_text(src.replace(find, repl, 1))
    spec = importlib.util.spec_from_file_location(f"p2_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    caught = []
    for pin in PINS:
        try:
            pin(mod)
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            caught.append(pin.__name__)
    assert caught, f"no pin caught {name}"
