"""The pins must catch plausible mistakes in the oracle.

Each case copies oracle/householder.c, plants one mistake by a textual edit
(a flipped sign, a dropped term, a transposed index, a reversed loop, an
off-by-one), compiles the copy on the CPU, routes the oracle module through it
and checks that at least one pin from test_oracle_pins.py fails.
"""
import inspect
import os
import tempfile

import numpy as np

import pytest

import oracle
import tests.test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "householder.c")

MUTATIONS = {
    "flipped_reflector_sign": ("double beta = (alpha >= 0.0) ? -norm : norm;",
                               "double beta = (alpha >= 0.0) ? norm : -norm;"),
    "wrong_vector_scale": ("double scale = 1.0 / (alpha - beta);",
                           "double scale = 1.0 / (alpha + beta);"),
    "dropped_unit_term_in_dot": ("double w = AT(C, j, k, ldc);", "double w = 0.0;"),
    "dropped_tau_in_T": ("AT(T, i, j, ldt) = -tau[j] * s;", "AT(T, i, j, ldt) = -s;"),
    "transposed_T_index": ("s += AT(T, i, k, ldt) * g[k];", "s += AT(T, k, i, ldt) * g[k];"),
    "reversed_apply_order": ("for (int64_t j = n - 1; j >= 0; --j)",
                             "for (int64_t j = 0; j < n; ++j)"),
    "off_by_one_back_substitution": ("for (int64_t k = i + 1; k < n; ++k)\n                s -= AT(R, i, k, ldr)",
                                     "for (int64_t k = i + 2; k < n; ++k)\n                s -= AT(R, i, k, ldr)"),
}


def _pin_suite():
    yield lambda: pins.test_golden_3x2_worked_example()
    yield lambda: pins.test_single_column_closed_form()
    yield lambda: pins.test_matches_lapack_dgeqrt(64, 17, 2)
    yield lambda: pins.test_thin_q_matches_lapack_dorgqr(50, 9, 5)
    yield lambda: pins.test_t_closed_form(30, 12, 1)
    yield lambda: pins.test_g1_to_g4_invariants(64, 64, 13)
    yield lambda: pins.test_g7_exact_gram_identity(9, 8, 2)
    yield lambda: pins.test_lstsq_matches_scipy(120, 50, 4, 4)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "planted.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        lib = oracle.open_library(oracle.compile_source(path, os.path.join(d, "planted.so")))
        oracle.use_library(lib)
        try:
            failures = 0
            for check in _pin_suite():
                try:
                    check()
                except (AssertionError, ZeroDivisionError, RuntimeError, ValueError,
                        FloatingPointError):
                    failures += 1
        finally:
            oracle.use_library(None)
    assert failures > 0, "planted mistake %r passed every pin" % name


# Mistakes planted in the backward-error measure (plain numpy in
# oracle/__init__.py): the function's source is edited, re-executed, and the
# beta pins must fail.
BETA_MUTATIONS = {
    "residual_in_numerator": ("return float(np.linalg.norm(A.T @ r) / den)",
                              "return float(np.linalg.norm(r) / den)"),
    "dropped_residual_term": ("den = nA * (nA * np.linalg.norm(x) + np.linalg.norm(r))",
                              "den = nA * (nA * np.linalg.norm(x))"),
    "spectral_norm_of_A": ("nA = np.linalg.norm(A)", "nA = np.linalg.norm(A, 2)"),
    "residual_sign": ("r = b - A @ x", "r = b + A @ x"),
    "missing_outer_norm": ("den = nA * (nA * np.linalg.norm(x) + np.linalg.norm(r))",
                           "den = (nA * np.linalg.norm(x) + np.linalg.norm(r))"),
}


def _beta_pin_suite():
    yield lambda: pins.test_backward_error_golden_3x2()
    yield lambda: pins.test_backward_error_properties()


@pytest.mark.parametrize("name", sorted(BETA_MUTATIONS))
def test_beta_pins_catch_planted_mistake(name, monkeypatch):
    old, new = BETA_MUTATIONS[name]
    src = inspect.getsource(oracle.backward_error)
    assert src.count(old) == 1, "mutation anchor not found exactly once"
    ns = {"np": np}
    exec(src.replace(old, new), ns)
    monkeypatch.setattr(oracle, "backward_error", ns["backward_error"])
    failures = 0
    for check in _beta_pin_suite():
        try:
            check()
        except (AssertionError, ZeroDivisionError, FloatingPointError):
            failures += 1
    assert failures > 0, "planted mistake %r passed every beta pin" % name
