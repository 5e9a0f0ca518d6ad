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


def test_binding_checks_array_sizes_before_any_library_call():
    """The library reads and writes caller arrays through plain pointers, so
    the binding rejects arrays whose sizes do not match before it calls the
    library at all (here a stand-in library that fails on any call)."""
    import numpy as np

    class NoCalls:
        def __getattr__(self, name):
            raise AssertionError(f"the library was called: {name}")

    c = object.__new__(qmk.Context)
    c._h = ctypes.c_void_p()  # nothing to destroy
    c._lib = NoCalls()
    c.device = 0
    coord = np.zeros((2, 5, 3))
    with pytest.raises(ValueError):
        c.set_point(coord[:, :, :2].copy())                 # not [walk, elec, 3]
    with pytest.raises(ValueError):
        c.set_point(coord.reshape(-1)[:-3].copy(), 2, 5)    # 27 values for 30
    with pytest.raises(ValueError):
        c.set_point(np.zeros((3, 9)), 2, 5, transp="T")     # 27 values for 30
    sh_nuc, sh_l = np.zeros(3, np.int64), np.array([0, 1, 2], np.int32)
    off, ex, co = np.array([0, 2, 3, 5], np.int64), np.ones(5), np.ones(5)
    for bad in [dict(shell_prim_offset=off[:-1]), dict(coefficient=co[:-1]),
                dict(shell_nucleus=sh_nuc[:-1]), dict(prim_factor=np.ones(4)),
                dict(shell_factor=np.ones(4)), dict(ao_factor=np.ones(9))]:
        args = dict(shell_nucleus=sh_nuc, shell_ang_mom=sh_l, shell_prim_offset=off, exponent=ex,
                    coefficient=co)
        args.update(bad)
        with pytest.raises(ValueError):
            c.set_basis(**args)
    with pytest.raises(ValueError):
        c.set_mo_coef(np.ones(10))
    with pytest.raises(ValueError):
        c.set_mo_cusp(np.ones(3), np.ones(2))
    # consistent arrays get through to the library
    with pytest.raises(AssertionError, match="qmk_set_basis"):
        c.set_basis(sh_nuc, sh_l, off, ex, co, ao_factor=np.ones(10))
    with pytest.raises(AssertionError, match="qmk_set_point"):
        c.set_point(coord)


def test_batch_run_checks_every_tensor_before_the_library_call():
    """qmk_batch_run takes plain pointers without sizes, so Batch.run checks
    each output, weight and gradient tensor (device, contiguity, element type,
    element count) and raises before calling the library (a stand-in library
    that fails on any call)."""
    import torch

    class NoCalls:
        def __getattr__(self, name):
            raise AssertionError(f"the library was called: {name}")

    class FakeCtx:
        device = 0

        def __init__(self, walk, elec, mo, ao, nucl):
            self._d = dict(walk_num=walk, elec_num=elec, mo_num=mo, ao_num=ao, nucl_num=nucl)

        def dims(self):
            return dict(self._d)

    class FakeTensor:
        """Stands for a CUDA tensor (no GPU here)."""

        def __init__(self, numel, dtype=torch.float64, cuda=True, contiguous=True):
            self._n, self.dtype, self.is_cuda, self._c = numel, dtype, cuda, contiguous
            self.device = "cuda:0"

        def numel(self):
            return self._n

        def is_contiguous(self):
            return self._c

        def data_ptr(self):
            return 4096

    b = object.__new__(qmk.Batch)
    b._h = ctypes.c_void_p()
    b._lib = NoCalls()
    b.contexts = [FakeCtx(2, 3, 4, 6, 2), FakeCtx(1, 5, 2, 3, 1)]
    f64, f32 = torch.float64, torch.float32
    outs = [FakeTensor(2 * 3 * 5 * 4), FakeTensor(1 * 5 * 5 * 2)]
    ws = [FakeTensor(2 * 3 * 5 * 4), FakeTensor(1 * 5 * 5 * 2)]
    grads = [{"d_coef": FakeTensor(24), "d_elec": FakeTensor(18), "d_nucl": FakeTensor(6)},
             {"d_coef": FakeTensor(6), "d_elec": FakeTensor(15), "d_nucl": FakeTensor(3)}]
    bad_cases = [
        dict(outs=[outs[0]]),                                            # one tensor short
        dict(outs=[outs[0], FakeTensor(49)]),                            # wrong size
        dict(outs=[outs[0], FakeTensor(50, dtype=f32)], dtype=f64),      # wrong element type
        dict(outs=[outs[0], FakeTensor(50, cuda=False)]),                # host tensor
        dict(outs=[outs[0], FakeTensor(50, contiguous=False)]),          # strided view
        dict(outs=outs, ws=[ws[0], FakeTensor(50, dtype=f32)]),          # weights of another type
        dict(outs=outs, ws=[ws[0], FakeTensor(51)]),                     # weights of another size
        dict(outs=outs, ws=ws, grads=[grads[0], dict(grads[1], d_coef=FakeTensor(7))]),
        dict(outs=outs, ws=ws, grads=[grads[0], dict(grads[1], d_elec=FakeTensor(15, dtype=f32))]),
        dict(outs=outs, ws=ws, grads=[grads[0], dict(grads[1], d_nucl=FakeTensor(4))]),
        dict(outs=outs, ws=ws, grads=[grads[0], dict(grads[1], d_other=FakeTensor(3))]),
        dict(outs=outs, ws=ws, grads=[grads[0]]),
    ]
    for kw in bad_cases:
        with pytest.raises(ValueError):
            b.run(**kw)
    # consistent tensors (and a skipped gradient) get through to the library
    with pytest.raises(AssertionError, match="qmk_batch_run"):
        b.run(outs=outs, ws=ws, grads=[grads[0], dict(grads[1], d_nucl=None)])
