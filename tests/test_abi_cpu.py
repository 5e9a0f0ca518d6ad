"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host-only paths behave (no GPU compute here)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2512_16677_amd as qmk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "qmk.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qmk_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = qmk.load_library()
    names = header_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", qmk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (qmk_\w+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)
    assert set(names) == set(qmk.EXPORTED)


def test_status_strings():
    lib = qmk.load_library()
    assert lib.qmk_status_string(0) == b"QMK_OK"
    assert lib.qmk_status_string(qmk.QMK_SIZE) == b"QMK_SIZE"
    assert lib.qmk_status_string(qmk.QMK_INVALID_ARG_BASE + 3) == b"QMK_INVALID_ARG"
    assert lib.qmk_status_string(12345) == b"QMK_UNKNOWN_STATUS"


def test_null_context_is_rejected_without_touching_a_device():
    lib = qmk.load_library()
    assert lib.qmk_set_precision(None, 53, 0) == qmk.QMK_INVALID_CONTEXT
    assert lib.qmk_get_mo_vgl(None, None, 0, 0, None) == qmk.QMK_INVALID_CONTEXT
    assert lib.qmk_ctx_destroy(None) == qmk.QMK_INVALID_CONTEXT
    assert lib.qmk_ctx_create(None, 0) == qmk.QMK_INVALID_ARG_BASE + 1


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="host without GPU only")
def test_create_without_gpu_reports_an_error():
    lib = qmk.load_library()
    h = ctypes.c_void_p()
    st = lib.qmk_ctx_create(ctypes.byref(h), 0)
    assert st != qmk.QMK_OK
    assert len(lib.qmk_last_error(None)) > 0
