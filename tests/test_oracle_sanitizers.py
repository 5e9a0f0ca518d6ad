"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, CPU): a sanitized build of oracle.c runs a subset of the
pins in a child process with the sanitizer runtime preloaded.  Any heap or
stack overflow, use after free, or undefined behaviour (signed overflow,
misaligned or out-of-range access, invalid shift) aborts the child.  A copy
with a planted one-element heap overflow must be caught, so the test also
shows that the sanitizer is active."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

PINS = """
import sys
sys.path.insert(0, {root!r})
import oracle
oracle.use_library({lib!r})
from tests import test_oracle_pins as pins
from tests import test_oracle_products_pins as prod
pins.test_normalised_s_primitive_closed_form(0.7, 0.1)
pins.test_normalised_p_primitive_closed_form(5.0)
pins.test_cartesian_order_and_normalisation_factor_table()
pins.test_derivatives_match_brute_force_products()
pins.test_contraction_matches_library_and_identity()
pins.test_cutoff_is_strict_on_the_exponent_argument()
pins.test_adjoint_dcoef_is_w_transpose_ao()
pins.test_adjoint_finite_differences_and_sum_rule()
prod.test_equals_literal_adjoint("tiny_spdf", 3, 53.0)
print("PINS_OK")
"""


def runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def build(src_text, out):
    src = out + ".c"
    with open(src, "w") as fh:
        fh.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-ffp-contract=off", src, "-o", out, "-lm"])


def run_pins(lib):
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime("libasan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return subprocess.run([sys.executable, "-c", PINS.format(root=ROOT, lib=lib)], capture_output=True,
                          text=True, env=env, timeout=600)


@pytest.mark.skipif(runtime("libasan.so") is None, reason="no AddressSanitizer runtime")
def test_oracle_pins_clean_under_address_and_ub_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    build(open(SRC).read(), lib)
    r = run_pins(lib)
    assert r.returncode == 0 and "PINS_OK" in r.stdout, r.stderr[-3000:]
    assert "runtime error" not in r.stderr, r.stderr[-3000:]


@pytest.mark.skipif(runtime("libasan.so") is None, reason="no AddressSanitizer runtime")
def test_sanitizer_catches_a_planted_overflow(tmp_path):
    src = open(SRC).read()
    anchor = "double* ns = (double*)malloc(sizeof(double) * (size_t)(shell_num > 0 ? shell_num : 1));"
    assert anchor in src
    bad = src.replace(anchor, "double* ns = (double*)malloc(sizeof(double) * (size_t)(shell_num - 1));", 1)
    lib = str(tmp_path / "liboracle_overflow.so")
    build(bad, lib)
    r = run_pins(lib)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr
