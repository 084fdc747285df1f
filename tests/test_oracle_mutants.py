"""Plant plausible mistakes in copies of the oracle source and check that the
pins catch every one of them (CPU only; the real oracle source is untouched).

Each mutant is a (find, replace) edit applied to the first occurrence in
``oracle/tdt_oracle.c``: a dropped term, a wrong sign, a wrong index or a
transposed operand, in the forward sweep, the back substitution, the long
double variant, the varlen driver and the adjoint."""
import os
import subprocess

import pytest

import oracle
import oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "tdt_oracle.c")

MUTANTS = {
    "forward_sign": ("x[i] = (f[i] - tm1 * x[i - 1]) / u;", "x[i] = (f[i] + tm1 * x[i - 1]) / u;"),
    "transposed_cp": ("cp[i] = t1 / u;", "cp[i] = tm1 / u;"),
    "constant_pivot": ("u = diag_f64(t0, psi, chi, i, n) - tm1 * cp[i - 1];",
                       "u = diag_f64(t0, psi, chi, i, n) - tm1 * cp[0];"),
    "first_row_dropped_pivot": ("x[0] = f[0] / u;", "x[0] = f[0];"),
    "dropped_backsub": ("x[i] = x[i] - cp[i] * x[i + 1];", "x[i] = x[i];"),
    "backsub_index": ("x[i] = x[i] - cp[i] * x[i + 1];", "x[i] = x[i] - cp[i + 1] * x[i + 1];"),
    "ld_forward_sign": ("x[i] = (f[i] - tm1 * x[i - 1]) / u;\n    }\n    for (int64_t i = n - 2; i >= 0; --i)\n        x[i] = x[i] - cp[i] * x[i + 1];\n    return 0;\n}\n\n/* Long",
                        "x[i] = (f[i] + tm1 * x[i - 1]) / u;\n    }\n    for (int64_t i = n - 2; i >= 0; --i)\n        x[i] = x[i] - cp[i] * x[i + 1];\n    return 0;\n}\n\n/* Long"),
    "ld_rounded_early": ("for (int64_t i = 0; i < n; ++i) fl[i] = (long double)f[i];",
                         "for (int64_t i = 0; i < n; ++i) fl[i] = (long double)(float)f[i];"),
    "varlen_param_index": ("thomas_f64(tm1[s], t0[s], t1[s], ps, ch, n, F + o, X + o, cp)",
                           "thomas_f64(tm1[i], t0[i], t1[i], ps, ch, n, F + o, X + o, cp)"),
    "adjoint_not_transposed": (
        "int st = oracle_solve(t1, t0, tm1, psi, chi, N, M, gX, gF, 0, nthreads);",
        "int st = oracle_solve(tm1, t0, t1, psi, chi, N, M, gX, gF, 0, nthreads);"),
    "adjoint_t1_index": ("s_p1 += (long double)g[i] * x[i + 1];",
                         "s_p1 += (long double)g[i + 1] * x[i];"),
    "adjoint_sign": ("gt[1] = (double)(-s_0);", "gt[1] = (double)(s_0);"),
    "varlen_adjoint_not_transposed": (
        "int st = oracle_solve_varlen(S, offsets, t1, t0, tm1, psi, chi, gX, gF, 0, nthreads);",
        "int st = oracle_solve_varlen(S, offsets, tm1, t0, t1, psi, chi, gX, gF, 0, nthreads);"),
    # quasi-Toeplitz corner terms (eq. (21))
    "corner_psi_dropped": ("if (i == 0) d += psi;", "if (i == 0) d += 0.0;"),
    "corner_chi_wrong_row": ("if (i == n - 1) d += chi;", "if (i == n - 2) d += chi;"),
    "corner_psi_sign": ("if (i == 0) d += psi;", "if (i == 0) d -= psi;"),
    "varlen_corners_swapped": (
        "const double ps = psi ? psi[s] : 0.0, ch = chi ? chi[s] : 0.0;",
        "const double ps = chi ? chi[s] : 0.0, ch = psi ? psi[s] : 0.0;"),
    "adjoint_gpsi_index": ("s_ps += (long double)g[0] * x[0];",
                           "s_ps += (long double)g[0] * x[1];"),
    "adjoint_gchi_sign": ("gt[4] = (double)(-s_ch);", "gt[4] = (double)(s_ch);"),
    # general tridiagonal matrices
    "gen_forward_sign": ("x[i] = (f[i] - a[i] * x[i - 1]) / u;",
                         "x[i] = (f[i] + a[i] * x[i - 1]) / u;"),
    "gen_pivot_row": ("u = b[i] - a[i] * cp[i - 1];", "u = b[i] - a[i - 1] * cp[i - 1];"),
    "gen_cp_transposed": ("cp[i] = c[i] / u;", "cp[i] = a[i] / u;"),
    "gen_backsub_dropped": ("x[i] = x[i] - cp[i] * x[i + 1];\n    return 0;\n}\n\n/* the same in long",
                            "x[i] = x[i];\n    return 0;\n}\n\n/* the same in long"),
    "gen_ld_pivot_rounded": (
        "u = (long double)b[i] - (long double)a[i] * cp[i - 1];",
        "u = (double)((long double)b[i] - (long double)a[i] * cp[i - 1]);"),
    "gen_adjoint_not_transposed": ("at[i] = i > 0 ? c[i - 1] : 0.0;",
                                   "at[i] = i > 0 ? a[i] : 0.0;"),
    "gen_adjoint_ga_index": ("if (i > 0) sa += (long double)g[i] * x[i - 1];",
                             "if (i > 0) sa += (long double)g[i - 1] * x[i];"),
    "gen_adjoint_gc_sign": ("gc[i] = (double)(-sc);", "gc[i] = (double)(sc);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    find, repl = MUTANTS[name]
    src = open(SRC).read()
    assert find in src, f"mutation site for {name} not found"
    mutated = src.replace(find, repl, 1)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"lib{name}.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                           "-shared", "-o", str(so), str(c)])
    mut = oracle.load_library(str(so))
    caught = []
    for pin in P.ALL_PINS:
        try:
            pin(mut)
        except (AssertionError, oracle.OracleSingular, FloatingPointError, ValueError,
                RuntimeError):
            caught.append(pin.__name__)
    assert caught, f"no pin caught mutant {name}"
