"""Plant plausible mistakes in a copy of the oracle and check that the pins in
test_oracle.py catch each one.  Runs on the CPU only: every mutant is built
from a patched copy of oracle/jacobi_oracle.c in a temporary directory."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "jacobi_oracle.c")

# (name, original text, mutated text, pins expected to catch it)
MUTANTS = [
    ("tau_sign", "double tau = (aqq - app) / (2.0 * apq);",
     "double tau = (app - aqq) / (2.0 * apq);",
     ["test_pair_random_2x2", "test_known_spectrum"]),
    ("approach1", "t = 1.0 / (tau + sqrt(1.0 + tau * tau));",
     "t = -tau + sqrt(tau * tau + 1.0);",
     ["test_small_angle_appendix_a"]),
    ("larger_root", "t = 1.0 / (tau - sqrt(1.0 + tau * tau));",
     "t = (tau - sqrt(1.0 + tau * tau));",
     ["test_pair_random_2x2"]),
    ("row_rot_sign", "A[IDX(p, j, n)] = c * ap - s * aq;",
     "A[IDX(p, j, n)] = c * ap + s * aq;",
     ["test_rotation_off_identity", "test_known_spectrum"]),
    ("v_rot_sign", "V[IDX(i, p, n)] = c * vp - s * vq;",
     "V[IDX(i, p, n)] = c * vp + s * vq;",
     ["test_known_spectrum"]),
    ("off_half", "if (i != j)\n                acc += A[IDX(i, j, n)] * A[IDX(i, j, n)];",
     "if (i < j)\n                acc += A[IDX(i, j, n)] * A[IDX(i, j, n)];",
     ["test_rotation_off_identity"]),
    ("sort_desc", "while (j >= 0 && D[perm[j]] > D[k]) {",
     "while (j >= 0 && D[perm[j]] < D[k]) {",
     ["test_diagonal_input", "test_known_spectrum"]),
    ("no_signfix", "double sg = tmp[IDX(imax, src, n)] < 0.0 ? -1.0 : 1.0;",
     "double sg = 1.0;",
     ["test_brute_force_vs_lapack"]),
    ("ns_2I", "M[IDX(i, j, n)] = (i == j ? 3.0 : 0.0) - acc;",
     "M[IDX(i, j, n)] = (i == j ? 2.0 : 0.0) - acc;",
     ["test_newton_schulz_scalar_map"]),
    ("ns_xxt", "acc += X[IDX(k, i, n)] * X[IDX(k, j, n)];\n                M[IDX(i, j, n)]",
     "acc += X[IDX(i, k, n)] * X[IDX(j, k, n)];\n                M[IDX(i, j, n)]",
     ["test_newton_schulz_scalar_map"]),
    ("qtaq_transposed", "acc += Q[IDX(k, i, n)] * T[IDX(k, j, n)];",
     "acc += Q[IDX(i, k, n)] * T[IDX(k, j, n)];",
     ["test_qtaq_vs_library"]),
    ("adjoint_gap_sign", "double gap = W[j] - W[i];", "double gap = W[i] - W[j];",
     ["test_backward_central_fd"]),
    ("adjoint_no_sym", "double m = 0.5 * (dA[IDX(i, j, n)] + dA[IDX(j, i, n)]);\n"
     "            dA[IDX(i, j, n)] = m;\n            dA[IDX(j, i, n)] = m;",
     "(void)0;", ["test_backward_central_fd"]),
    ("adjoint_vtdv", "acc += V[IDX(k, i, n)] * dV[IDX(k, j, n)];",
     "acc += V[IDX(i, k, n)] * dV[IDX(k, j, n)];",
     ["test_backward_central_fd"]),
    ("rows_skip_last", "for (int64_t q = p + 1; q < n; ++q) {\n            double apq = A[IDX(p, q, n)], app",
     "for (int64_t q = p + 1; q < n - 1; ++q) {\n            double apq = A[IDX(p, q, n)], app",
     ["test_jacobi_rows_is_one_sweep"]),
    ("rows_no_v", "orc_rotate(n, A, V, p, q, c, s);\n                ++rotations;\n            }\n        }\n    return rotations;",
     "orc_rotate(n, A, NULL, p, q, c, s);\n                ++rotations;\n            }\n        }\n    return rotations;",
     ["test_jacobi_rows_is_one_sweep"]),
    ("rayleigh_no_norm", "long double q = vv > 0.0L ? vy / vv : 0.0L;",
     "long double q = vy;", ["test_rayleigh_quadratic_and_scale_free"]),
    ("rayleigh_transposed", "acc += (long double)A[IDX(i, j, n)] * v[j];",
     "acc += (long double)A[IDX(j, i, n)] * v[i];", ["test_rayleigh_exact_eigenvectors"]),
    ("house_branch", "if (x[0] >= 0.0)\n        v[0] = x[0] + mu;",
     "if (x[0] < 0.0)\n        v[0] = x[0] + mu;", ["test_house_worked_example"]),
    ("house_beta", "*beta = 2.0 / (v[0] * v[0] + sigma);", "*beta = 1.0 / (v[0] * v[0] + sigma);",
     ["test_house_worked_example"]),
    ("qr_q_update_transposed", "acc += Q[IDX(i, k + j, n)] * v[j];",
     "acc += Q[IDX(k + j, i, n)] * v[j];", ["test_householder_qr_identities"]),
    ("qr_a_update_full", "A[IDX(k + i, k + j, n)] -= (beta * v[i]) * w[j];",
     "A[IDX(k + i, k + j, n)] -= (beta * v[j]) * w[i];", ["test_householder_qr_identities"]),
    ("chol_no_sqrt", "double rii = sqrt(d);", "double rii = d;", ["test_cholesky_known_factor"]),
    ("chol_wrong_index", "g -= R[IDX(k, i, n)] * R[IDX(k, j, n)];",
     "g -= R[IDX(k, i, n)] * R[IDX(k, i, n)];", ["test_cholesky_known_factor"]),
    ("cholqr_solve", "acc -= Q[IDX(i, k, n)] * R[IDX(k, j, n)];",
     "acc -= Q[IDX(i, k, n)] * R[IDX(j, k, n)];", ["test_cholesky_qr_identities"]),
    ("half_spacing", "    int q = (e - 1) - 10;   /* exponent of the spacing */",
     "    int q = (e - 1) - 11;   /* exponent of the spacing */", ["test_round_half_definition"]),
    ("half_subnormal", "        q = -24;            /* subnormal spacing */",
     "        q = -25;            /* subnormal spacing */", ["test_round_half_definition"]),
    ("half_no_round_cols", "A[IDX(i, p, n)] = (float)orc_round_half((double)(c * ap - s * aq));",
     "A[IDX(i, p, n)] = (c * ap - s * aq);", ["test_half_stage_bounds"]),
    ("ns_count_linear", "        err = err * err;", "        err = err * e;",
     ["test_ns_iteration_count_low_precision"]),
    ("rayleigh_res_unscaled", "res[k] = vv > 0.0L ? (double)sqrtl(rr / vv) : 0.0;",
     "res[k] = (double)sqrtl(rr);", ["test_rayleigh_quadratic_and_scale_free"]),
]


@pytest.fixture(scope="module")
def src_text():
    with open(SRC) as f:
        return f.read()


def _build(tmp_path, text, name):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"lib{name}.so"
    c.write_text(text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                           "-ffp-contract=off", "-o", str(so), str(c), "-lm"])
    return str(so)


@pytest.mark.parametrize("name,orig,mut,catchers", MUTANTS,
                         ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, src_text, name, orig, mut, catchers):
    assert src_text.count(orig) == 1, f"mutation site for {name} not unique"
    so = _build(tmp_path, src_text.replace(orig, mut), name)
    saved_lib, saved_path = oracle._lib, oracle._LIB
    try:
        oracle._lib = None
        oracle._LIB = so
        oracle._load()
        caught = []
        for pin in catchers:
            fn = getattr(pins, pin)
            params = _params_for(pin)
            for args in params:
                try:
                    fn(oracle, *args)
                except (AssertionError, ValueError, FloatingPointError):
                    caught.append(pin)
                    break
        assert caught, f"mutant {name} survived pins {catchers}"
    finally:
        oracle._lib, oracle._LIB = saved_lib, saved_path


def _params_for(pin):
    marks = getattr(getattr(pins, pin), "pytestmark", [])
    for m in marks:
        if m.name == "parametrize":
            names, values = m.args[0], m.args[1]
            return [v if isinstance(v, tuple) else (v,) for v in values]
    return [()]


def test_unmutated_source_passes(tmp_path, src_text):
    """Control: the same build path without a mutation passes every pin."""
    so = _build(tmp_path, src_text, "control")
    saved_lib, saved_path = oracle._lib, oracle._LIB
    try:
        oracle._lib = None
        oracle._LIB = so
        oracle._load()
        for _, _, _, catchers in MUTANTS:
            for pin in catchers:
                for args in _params_for(pin):
                    getattr(pins, pin)(oracle, *args)
    finally:
        oracle._lib, oracle._LIB = saved_lib, saved_path
