"""The CPU oracle against its pins (no GPU)."""
import numpy as np
import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_theorem1_as_printed_is_negated(orc):
    """The printed Theorem 1 weights times +f_k/t_1 give -T^{-1} f (the reading
    recorded in the design notes); this pins the sign convention of the pin."""
    rng = np.random.default_rng(11)
    for n in (1, 4, 9):
        a, b, c = -0.8, 2.6, -1.1
        f = rng.standard_normal(n)
        y_re, _ = P.theorem1_solution(-f, a, b, c)   # feeding -f undoes the reading
        x = orc.solve(f, a, b, c)
        assert np.max(np.abs(y_re + x)) < 1e-14 * max(1, np.max(np.abs(x)))


def test_golden_laplacian_inverse(orc):
    """tests/golden/laplacian_inverse_n7.txt: the textbook inverse of
    tridiag{-1, 2, -1} of order 7, (T^-1)_{ij} = min(i,j)(8 - max(i,j))/8."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "laplacian_inverse_n7.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    inv = np.array([[float(eval(v, {"__builtins__": {}})) for v in r] for r in rows])
    X = orc.solve(np.eye(7), -1.0, 2.0, -1.0)
    assert np.max(np.abs(X - inv.T)) < 1e-15


def test_rel_err_helpers(orc):
    x = np.array([1.0, 2.0, -4.0])
    assert orc.rel_err(x, x) == 0.0
    assert orc.rel_err(x + 0.04, x) == pytest.approx(0.01)
    off = np.array([0, 1, 3])
    r = orc.rel_err_rows(np.array([1.0, 2.0, -4.4]), x, off)
    assert r[0] == 0 and r[1] == pytest.approx(0.1)
