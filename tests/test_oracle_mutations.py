"""Sensitivity of the oracle pins: each plausible mistake planted in a copy of
the oracle (a dropped term, a wrong factor, sign or index, a transposed
operand) must make at least one pin fail.  Runs on the CPU only."""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, original text, planted mistake)
MUTATIONS = [
    ("laplacian_coefficient", "q[4] = M * (lP * g0 + (4.0 * l + 6.0) * P * g1",
     "q[4] = M * (lP * g0 + (4.0 * l + 4.0) * P * g1"),
    ("gradient_factor", "q[1 + x] = M * (dP[x] * g0 + 2.0 * d[x] * P * g1)",
     "q[1 + x] = M * (dP[x] * g0 + d[x] * P * g1)"),
    ("hessian_diagonal_term", "if (x == y) h += 2.0 * P * g1;", ""),
    ("radial_derivative_sign", "g1 += -g * e;", "g1 += g * e;"),
    ("third_derivative_sign", "g3 += -g * g * g * e;", "g3 += g * g * g * e;"),
    ("primitive_normalisation", "pow(4.0 * g, 0.5 * l)", "pow(4.0 * g, 1.0 * l)"),
    ("shell_normalisation", "dfl / pow(2.0 * al, (double)l)", "dfl / pow(al, (double)l)"),
    ("cartesian_factor", "ao_factor[ao++] = sqrt(dfl /", "ao_factor[ao++] = (dfl /"),
    ("gradlap_g2_coefficient", "((8.0 * l + 20.0) * d[x] * P", "((8.0 * l + 12.0) * d[x] * P"),
    ("gradlap_g3_coefficient", "8.0 * u * d[x] * P * g3", "4.0 * u * d[x] * P * g3"),
    ("component_order", "for (int bb = l - aa; bb >= 0; --bb) {\n            if (idx == i)",
     "for (int bb = 0; bb <= l - aa; ++bb) {\n            if (idx == i)"),
    ("nuclear_gradient_sign", "np_[ao_nucleus[k] * 6 + i] -= t;", "np_[ao_nucleus[k] * 6 + i] += t;"),
    ("hessian_index_table", "{{5, 6, 7}, {6, 8, 9}, {7, 9, 10}}", "{{5, 6, 7}, {6, 8, 10}, {7, 9, 10}}"),
    ("contraction_transposed", "const double* cn = coef + (size_t)n * (size_t)ao_num;",
     "const double* cn = coef + (size_t)n;"),
    ("cutoff_log_base", "(B - 1.0) * log(2.0)", "(B - 1.0) * log10(2.0)"),
]

# pins run against each mutant (a subset of test_oracle_pins, fast enough for the CPU suite)
CHECKS = [
    lambda: pins.test_normalised_s_primitive_closed_form(0.7, 0.1),
    lambda: pins.test_normalised_p_primitive_closed_form(5.0),
    pins.test_cartesian_order_and_normalisation_factor_table,
    pins.test_derivatives_match_brute_force_products,
    pins.test_contraction_matches_library_and_identity,
    pins.test_cutoff_is_strict_on_the_exponent_argument,
    lambda: pins.test_self_overlap_by_quadrature(1, [0.15, 2.0, 60.0]),
    lambda: pins.test_contraction_weights_are_quadrature_normalised_primitives(1),
    pins.test_adjoint_dcoef_is_w_transpose_ao,
    pins.test_adjoint_finite_differences_and_sum_rule,
]


@pytest.fixture(scope="module", autouse=True)
def _restore():
    yield
    oracle.use_library(None)


@pytest.mark.parametrize("name,orig,bad", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, orig, bad):
    src = open(SRC).read()
    assert src.count(orig) >= 1, f"mutation anchor not found: {name}"
    mutant = tmp_path / "oracle_mutant.c"
    mutant.write_text(src.replace(orig, bad, 1))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", str(mutant), "-o", str(lib), "-lm"])
    oracle.use_library(str(lib))
    caught = []
    try:
        for chk in CHECKS:
            try:
                chk()
            except (AssertionError, RuntimeError, ValueError, FloatingPointError):
                caught.append(chk)
                break
    finally:
        oracle.use_library(None)
    assert caught, f"no pin caught the planted mistake '{name}'"


def test_unmutated_copy_passes_every_check(tmp_path):
    lib = tmp_path / "liboracle_copy.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", SRC, "-o", str(lib), "-lm"])
    oracle.use_library(str(lib))
    try:
        for chk in CHECKS:
            chk()
    finally:
        oracle.use_library(None)
