"""Python binding of the MI355X AO -> MO value/gradient/Laplacian library.

A thin ctypes layer over ``libqmk.so`` (C ABI in ``include/qmk.h``): it only
marshals arguments.  Every step of the computation runs in the library's
HIP kernels; there is no CPU fallback -- importing :class:`Context` without a
built library raises.  PyTorch supplies device memory and the current HIP
stream.

Typical use (mirrors the call sequence of the QMCkl paper, Section 5.1)::

    ctx = Context()
    ctx.set_nucleus(R)                  # [nucl, 3]
    ctx.set_basis(shell_nucleus, shell_ang_mom, shell_prim_offset, exponent, coefficient)
    ctx.set_mo_coef(C)                  # [mo, ao]
    ctx.set_point(r)                    # [walk, elec, 3], numpy or CUDA tensor
    mo = ctx.get_mo_vgl()               # CUDA tensor [walk, elec, 5, mo]
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqmk.so")
# tile shapes chosen by the library's autotuner on an MI355X for the shapes of
# the shipped workloads (read-only; new shapes are timed on first use)
TILE_TABLE = os.path.join(_HERE, "tiles_gfx950.json")

QMK_OK = 0
QMK_INVALID_CONTEXT = 1
QMK_NOT_SET = 2
QMK_SIZE = 3
QMK_OUT_OF_MEMORY = 4
QMK_HIP_ERROR = 5
QMK_NONFINITE = 6
QMK_UNSUPPORTED = 7
QMK_INVALID_ARG_BASE = 100

MODES = {"fp64": 0, "mixed_f32": 1, "mixed_bf16x3": 2}
QMK_F64, QMK_F32 = 0, 1

EXPORTED = [
    "qmk_status_string", "qmk_last_error", "qmk_ctx_create", "qmk_ctx_destroy",
    "qmk_set_precision", "qmk_set_nucleus", "qmk_set_basis", "qmk_set_mo_coef",
    "qmk_set_point", "qmk_get_dims", "qmk_get_ao_vgl", "qmk_get_mo_vgl", "qmk_get_mo_vgl_noalloc",
    "qmk_get_mo_value", "qmk_get_density", "qmk_set_mo_cusp", "qmk_set_screening",
    "qmk_get_screening_density", "qmk_det_adj", "qmk_jastrow_een_terms", "qmk_jastrow_een",
    "qmk_mo_vgl_adjoint", "qmk_get_launch_count", "qmk_set_timing", "qmk_get_timing",
    "qmk_get_tile_count", "qmk_set_tile", "qmk_set_ao_retention",
    "qmk_batch_create", "qmk_batch_destroy", "qmk_batch_last_error", "qmk_batch_run",
]

KERNEL_CLASSES = ["ao", "mo", "gbar", "ao_adjoint", "dcoef", "reduce", "density", "cusp", "sort", "det",
                  "jastrow", "jastrow_p", "convert"]

_lib = None


class QmkError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


def load_library(path: str = LIB_PATH):
    """Load libqmk.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libqmk.so not built at {path}: run paper_2512_16677_amd/build.py "
                          "(there is no CPU fallback)")
    if "QMK_TUNE_TABLE" not in os.environ and os.path.exists(TILE_TABLE):
        os.environ["QMK_TUNE_TABLE"] = TILE_TABLE
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "qmk_status_string": ([I32], ctypes.c_char_p),
        "qmk_last_error": ([P], ctypes.c_char_p),
        "qmk_ctx_create": ([ctypes.POINTER(P), I32], I32),
        "qmk_ctx_destroy": ([P], I32),
        "qmk_set_precision": ([P, I32, I32], I32),
        "qmk_set_nucleus": ([P, I64, P], I32),
        "qmk_set_basis": ([P, I64, I64, P, P, P, P, P, P, P, P], I32),
        "qmk_set_mo_coef": ([P, I64, I64, P], I32),
        "qmk_set_point": ([P, ctypes.c_char, I64, I64, P, I32], I32),
        "qmk_get_dims": ([P, P, P, P, P, P], I32),
        "qmk_get_ao_vgl": ([P, P, I64, I32, P], I32),
        "qmk_get_mo_vgl": ([P, P, I64, I32, P], I32),
        "qmk_get_mo_vgl_noalloc": ([P, P, I64, I32, P], I32),
        "qmk_get_mo_value": ([P, P, I64, I32, P], I32),
        "qmk_get_density": ([P, P, I64, P, I64, P], I32),
        "qmk_set_mo_cusp": ([P, I64, P, P], I32),
        "qmk_set_screening": ([P, I32], I32),
        "qmk_set_ao_retention": ([P, I32], I32),
        "qmk_get_screening_density": ([P, P], I32),
        "qmk_det_adj": ([P, I64, I64, P, P, P, P], I32),
        "qmk_jastrow_een_terms": ([I64, P], I32),
        "qmk_jastrow_een": ([P, I64, D, I64, P, P, P], I32),
        "qmk_mo_vgl_adjoint": ([P, P, I32, P, P, P, P], I32),
        "qmk_get_launch_count": ([P, P], I32),
        "qmk_set_timing": ([P, I32], I32),
        "qmk_get_timing": ([P, I32, P, P], I32),
        "qmk_get_tile_count": ([P, P], I32),
        "qmk_set_tile": ([P, I32, I32], I32),
        "qmk_batch_create": ([ctypes.POINTER(P), P, I64], I32),
        "qmk_batch_destroy": ([P], I32),
        "qmk_batch_last_error": ([P], ctypes.c_char_p),
        "qmk_batch_run": ([P, P, I32, P, P, P, P, P], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def jastrow_een_terms(nord: int) -> int:
    """Number of three-body Jastrow terms of order nord."""
    n = ctypes.c_int64()
    st = load_library().qmk_jastrow_een_terms(int(nord), ctypes.byref(n))
    if st != QMK_OK:
        raise QmkError(st, "invalid nord")
    return n.value


def _np(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(a.data_ptr())  # torch tensor


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """One QMCkl-style context (not thread-safe; one per host thread)."""

    _in_version = 0
    _cfg_version = 0

    def __init__(self, device: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        st = self._lib.qmk_ctx_create(ctypes.byref(h), int(device))
        if st != QMK_OK:
            raise QmkError(st, self._lib.qmk_last_error(None).decode())
        self._h = h
        self.device = int(device)
        self._keep = None  # device coordinates the library points into
        # bumped by every set_* call: the autograd function compares them
        # between forward and backward (inputs: nuclei, C, points; config:
        # precision, basis, cusp, screening)
        self._in_version = 0
        self._cfg_version = 0

    # ------------------------------------------------------------------ util
    def _check(self, st: int):
        if st != QMK_OK:
            raise QmkError(st, self._lib.qmk_last_error(self._h).decode())

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.qmk_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------- set
    def set_precision(self, bits: int = 53, mode: str = "fp64"):
        self._cfg_version += 1
        self._check(self._lib.qmk_set_precision(self._h, int(bits), MODES[mode]))

    def set_nucleus(self, coord):
        c = _np(coord, np.float64).reshape(-1, 3)
        self._in_version += 1
        self._check(self._lib.qmk_set_nucleus(self._h, c.shape[0], _ptr(c)))

    def set_basis(self, shell_nucleus, shell_ang_mom, shell_prim_offset, exponent, coefficient,
                  prim_factor=None, shell_factor=None, ao_factor=None):
        sn = _np(shell_nucleus, np.int64)
        sl = _np(shell_ang_mom, np.int32)
        so = _np(shell_prim_offset, np.int64)
        ex = _np(exponent, np.float64)
        co = _np(coefficient, np.float64)
        pf = None if prim_factor is None else _np(prim_factor, np.float64)
        sf = None if shell_factor is None else _np(shell_factor, np.float64)
        af = None if ao_factor is None else _np(ao_factor, np.float64)
        # the library takes shell_num and prim_num from two of the arrays and
        # reads the others at those lengths: check them here
        n_sh, n_pr = sl.size, ex.size
        n_ao = int(sum((l + 1) * (l + 2) // 2 for l in np.clip(sl.reshape(-1), 0, None)))
        for name, a, n in [("shell_nucleus", sn, n_sh), ("shell_prim_offset", so, n_sh + 1),
                           ("coefficient", co, n_pr), ("prim_factor", pf, n_pr),
                           ("shell_factor", sf, n_sh), ("ao_factor", af, n_ao)]:
            if a is not None and a.size != n:
                raise ValueError(f"{name} holds {a.size} values, {n} expected")
        self._cfg_version += 1
        self._check(self._lib.qmk_set_basis(self._h, sl.shape[0], ex.shape[0], _ptr(sn), _ptr(sl),
                                            _ptr(so), _ptr(ex), _ptr(co), _ptr(pf), _ptr(sf),
                                            _ptr(af)))

    def set_mo_coef(self, coef):
        c = _np(coef, np.float64)
        if c.ndim != 2:
            raise ValueError("coef must have shape [mo_num, ao_num]")
        self._in_version += 1
        self._check(self._lib.qmk_set_mo_coef(self._h, c.shape[0], c.shape[1], _ptr(c)))

    def set_point(self, coord, walk_num: Optional[int] = None, elec_num: Optional[int] = None,
                  transp: str = "N"):
        """coord: numpy array (copied) or CUDA float64 tensor (referenced, kept
        alive here).  Shape [walk, elec, 3] for 'N', [3, walk*elec] for 'T'."""
        shape = tuple(coord.shape)
        if walk_num is None or elec_num is None:
            if transp != "N" or len(shape) != 3:
                raise ValueError("give walk_num and elec_num for this layout")
            if shape[2] != 3:
                raise ValueError("coordinates must have shape [walk, elec, 3]")
            walk_num, elec_num = shape[0], shape[1]
        # the library reads 3 walk_num elec_num values through a plain pointer
        size = int(np.prod(shape, dtype=np.int64))
        if size != 3 * int(walk_num) * int(elec_num):
            raise ValueError(f"coordinates hold {size} values, 3 * walk_num * elec_num = "
                             f"{3 * int(walk_num) * int(elec_num)} expected")
        self._in_version += 1
        if isinstance(coord, np.ndarray):
            c = _np(coord, np.float64)
            self._check(self._lib.qmk_set_point(self._h, transp.encode(), int(walk_num),
                                                int(elec_num), _ptr(c), 0))
            self._keep = None
        else:
            import torch
            if not (coord.is_cuda and coord.dtype == torch.float64 and coord.is_contiguous()):
                raise ValueError("device coordinates must be a contiguous CUDA float64 tensor")
            self._check(self._lib.qmk_set_point(self._h, transp.encode(), int(walk_num),
                                                int(elec_num), _ptr(coord), 1))
            self._keep = coord

    # ------------------------------------------------------------------- get
    def dims(self) -> Dict[str, int]:
        v = [ctypes.c_int64() for _ in range(5)]
        self._check(self._lib.qmk_get_dims(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(["nucl_num", "ao_num", "mo_num", "walk_num", "elec_num"], [x.value for x in v]))

    def launch_count(self) -> int:
        v = ctypes.c_int64()
        self._check(self._lib.qmk_get_launch_count(self._h, ctypes.byref(v)))
        return v.value

    def set_timing(self, enable: bool = True):
        """Bracket every kernel launch with HIP events on its stream (resets sums)."""
        self._check(self._lib.qmk_set_timing(self._h, 1 if enable else 0))

    def timing(self) -> Dict[str, Dict[str, float]]:
        """Summed device time (ms) and launch count per kernel class."""
        out = {}
        for i, name in enumerate(KERNEL_CLASSES):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            self._check(self._lib.qmk_get_timing(self._h, i, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = {"ms": ms.value, "launches": n.value}
        return out

    def tile_count(self) -> int:
        v = ctypes.c_int32()
        self._check(self._lib.qmk_get_tile_count(self._h, ctypes.byref(v)))
        return v.value

    def set_tile(self, kernel: str, tile: int):
        """Force MFMA tile `tile` for kernel class 'mo', 'gbar', 'dcoef', 'density' or
        'jastrow_p' (-1: autotune)."""
        self._check(self._lib.qmk_set_tile(self._h, KERNEL_CLASSES.index(kernel), int(tile)))

    def _out(self, out, shape, dtype):
        import torch
        if out is None:
            out = torch.empty(shape, dtype=dtype, device=f"cuda:{self.device}")
        if not (out.is_cuda and out.is_contiguous() and out.dtype in (torch.float64, torch.float32)):
            raise ValueError("output must be a contiguous CUDA float64/float32 tensor")
        return out, (QMK_F32 if out.dtype == torch.float32 else QMK_F64)

    def get_ao_vgl(self, out=None, dtype=None, stream=None):
        import torch
        d = self.dims()
        out, dt = self._out(out, (d["walk_num"], d["elec_num"], 5, d["ao_num"]), dtype or torch.float64)
        self._check(self._lib.qmk_get_ao_vgl(self._h, _ptr(out), out.numel(), dt, _stream(stream)))
        return out

    def get_mo_vgl(self, out=None, dtype=None, stream=None):
        import torch
        d = self.dims()
        out, dt = self._out(out, (d["walk_num"], d["elec_num"], 5, d["mo_num"]), dtype or torch.float64)
        self._check(self._lib.qmk_get_mo_vgl(self._h, _ptr(out), out.numel(), dt, _stream(stream)))
        return out

    def get_mo_vgl_noalloc(self, out, stream=None):
        """mo_vgl into the caller's tensor `out` through the entry point that
        allocates nothing (its AO array lives in the library's fixed 64 MiB
        per-GPU scratch; see qmk_get_mo_vgl_noalloc)."""
        if out is None:
            raise ValueError("the no-allocation call writes into a caller tensor: pass out")
        d = self.dims()
        out, dt = self._out(out, (d["walk_num"], d["elec_num"], 5, d["mo_num"]), None)
        self._check(self._lib.qmk_get_mo_vgl_noalloc(self._h, _ptr(out), out.numel(), dt, _stream(stream)))
        return out

    def set_mo_cusp(self, charge=None, r_cusp=None):
        """Switch the MO cusp correction on (charges and radii per nucleus) or
        off (r_cusp None)."""
        self._cfg_version += 1
        if r_cusp is None:
            self._check(self._lib.qmk_set_mo_cusp(self._h, 0, None, None))
            return
        z = _np(charge, np.float64).reshape(-1)
        r = _np(r_cusp, np.float64).reshape(-1)
        if z.shape != r.shape:
            raise ValueError("charge and r_cusp must have one value per nucleus each")
        self._check(self._lib.qmk_set_mo_cusp(self._h, r.shape[0], _ptr(z), _ptr(r)))

    def set_screening(self, enable: bool = True):
        """Screened (block-sparse) forward contraction on or off."""
        self._cfg_version += 1
        self._check(self._lib.qmk_set_screening(self._h, 1 if enable else 0))

    def set_ao_retention(self, retain: bool = True):
        """Whether the adjoint's dC product reads the forward pass's AO array of
        the same points (True, the default) or evaluates the AO values again
        (False); the outputs are the same either way."""
        self._check(self._lib.qmk_set_ao_retention(self._h, 1 if retain else 0))

    def screening_density(self) -> float:
        """Fraction of (64-point block, 16-AO chunk) pairs with a non-zero AO
        in the last screened evaluation."""
        v = ctypes.c_double()
        self._check(self._lib.qmk_get_screening_density(self._h, ctypes.byref(v)))
        return v.value

    def jastrow_een(self, nord: int, kappa: float, c, out=None, stream=None):
        """Three-body Jastrow factor of every walker: CUDA float64 tensor
        [walk].  c: host array [n_terms, nucl] (jastrow_een_terms order)."""
        import torch
        d = self.dims()
        cc = _np(c, np.float64)
        if cc.ndim != 2 or cc.shape[1] != d["nucl_num"]:
            raise ValueError("c must have shape [n_terms, nucl_num]")
        if out is None:
            out = torch.empty((d["walk_num"],), dtype=torch.float64, device=f"cuda:{self.device}")
        if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() < d["walk_num"]:
            raise ValueError("out must be a contiguous float64 tensor of walk_num elements")
        self._check(self._lib.qmk_jastrow_een(self._h, int(nord), float(kappa), cc.shape[0], _ptr(cc),
                                              _ptr(out), _stream(stream)))
        return out

    def det_adj(self, a, stream=None):
        """Determinants and adjugates of a CUDA float64 tensor [..., n, n]:
        returns (det [...], adj [..., n, n])."""
        import torch
        if not (a.is_cuda and a.dtype == torch.float64 and a.dim() >= 2 and a.shape[-1] == a.shape[-2]):
            raise ValueError("a must be a CUDA float64 tensor [..., n, n]")
        a = a.contiguous()
        n = a.shape[-1]
        batch = a.numel() // (n * n)
        det = torch.empty(a.shape[:-2], dtype=torch.float64, device=a.device)
        adj = torch.empty_like(a)
        self._check(self._lib.qmk_det_adj(self._h, n, batch, _ptr(a), _ptr(det), _ptr(adj), _stream(stream)))
        return det, adj

    def get_mo_value(self, out=None, dtype=None, stream=None):
        """MO values only: CUDA tensor [walk, elec, mo]."""
        import torch
        d = self.dims()
        out, dt = self._out(out, (d["walk_num"], d["elec_num"], d["mo_num"]), dtype or torch.float64)
        self._check(self._lib.qmk_get_mo_value(self._h, _ptr(out), out.numel(), dt, _stream(stream)))
        return out

    def get_density(self, occ, out=None, stream=None):
        """rho = sum_n occ[n] phi_n^2 at every point: CUDA float64 tensor
        [walk, elec].  occ: mo_num occupation numbers (host)."""
        import torch
        d = self.dims()
        o = _np(occ, np.float64).reshape(-1)
        if out is None:
            out = torch.empty((d["walk_num"], d["elec_num"]), dtype=torch.float64,
                              device=f"cuda:{self.device}")
        if not (out.is_cuda and out.is_contiguous() and out.dtype == torch.float64):
            raise ValueError("out must be a contiguous CUDA float64 tensor")
        self._check(self._lib.qmk_get_density(self._h, _ptr(o), o.shape[0], _ptr(out), out.numel(),
                                              _stream(stream)))
        return out

    def adjoint(self, w, d_coef=True, d_elec=True, d_nucl=True, out=None, stream=None):
        """Gradients of sum(w * mo_vgl).  w: CUDA tensor [walk, elec, 5, mo]
        (float64 or float32).  Returns a dict of CUDA float64 tensors."""
        import torch
        d = self.dims()
        if not (w.is_cuda and w.is_contiguous() and w.dtype in (torch.float64, torch.float32)):
            raise ValueError("w must be a contiguous CUDA float64/float32 tensor")
        if w.numel() != d["walk_num"] * d["elec_num"] * 5 * d["mo_num"]:
            raise ValueError("w has the wrong number of elements")
        dev = f"cuda:{self.device}"
        res = dict(out or {})
        if d_coef and "d_coef" not in res:
            res["d_coef"] = torch.empty((d["mo_num"], d["ao_num"]), dtype=torch.float64, device=dev)
        if d_elec and "d_elec" not in res:
            res["d_elec"] = torch.empty((d["walk_num"], d["elec_num"], 3), dtype=torch.float64, device=dev)
        if d_nucl and "d_nucl" not in res:
            res["d_nucl"] = torch.empty((d["nucl_num"], 3), dtype=torch.float64, device=dev)
        # the library writes these through plain pointers: check them here
        sizes = {"d_coef": d["mo_num"] * d["ao_num"], "d_elec": d["walk_num"] * d["elec_num"] * 3,
                 "d_nucl": d["nucl_num"] * 3}
        for k, t in res.items():
            if k not in sizes:
                raise ValueError(f"unknown output {k!r}")
            if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float64):
                raise ValueError(f"{k} must be a contiguous CUDA float64 tensor")
            if t.numel() != sizes[k]:
                raise ValueError(f"{k} holds {t.numel()} values, {sizes[k]} expected")
        self._check(self._lib.qmk_mo_vgl_adjoint(
            self._h, _ptr(w), QMK_F32 if w.dtype == torch.float32 else QMK_F64,
            _ptr(res.get("d_coef")), _ptr(res.get("d_elec")), _ptr(res.get("d_nucl")),
            _stream(stream)))
        return res

    # ------------------------------------------------------------ helpers
    @classmethod
    def from_system(cls, s, device: int = 0, bits: int = 53, mode: str = "fp64",
                    points_on_device: bool = False):
        """Context filled from a synthetic system (see the ``synth`` module)."""
        c = cls(device)
        c.set_precision(bits, mode)
        c.set_nucleus(s.nucl_coord)
        c.set_basis(s.shell_nucleus, s.shell_ang_mom, s.shell_prim_offset, s.exponent, s.coefficient)
        c.set_mo_coef(s.mo_coef)
        if points_on_device:
            import torch
            c.set_point(torch.from_numpy(np.ascontiguousarray(s.elec_coord)).to(f"cuda:{device}"))
        else:
            c.set_point(s.elec_coord)
        return c


class Batch:
    """Several contexts evaluated together in one HIP-graph launch of
    persistent kernels (see qmk_batch_run)."""

    def __init__(self, contexts):
        self._lib = load_library()
        self.contexts = list(contexts)
        arr = (ctypes.c_void_p * len(self.contexts))(*[c.handle.value for c in self.contexts])
        h = ctypes.c_void_p()
        st = self._lib.qmk_batch_create(ctypes.byref(h), arr, len(self.contexts))
        if st != QMK_OK:
            raise QmkError(st, "qmk_batch_create failed")
        self._h = h

    def _check(self, st):
        if st != QMK_OK:
            raise QmkError(st, self._lib.qmk_batch_last_error(self._h).decode())

    def run(self, outs=None, dtype=None, ws=None, grads=None, stream=None):
        """outs: list of CUDA tensors [walk, elec, 5, mo] (allocated if None);
        ws: optional list of weight tensors (same shapes and dtype);
        grads: optional list of dicts with 'd_coef', 'd_elec', 'd_nucl'
        tensors (allocated when ws is given and grads is None).

        The library takes plain pointers without sizes here, so every tensor
        is checked (device, contiguity, element type, element count) before
        the call; a mismatch raises ValueError and nothing is launched."""
        import torch
        dtype = dtype or (outs[0].dtype if outs else torch.float64)
        if dtype not in (torch.float64, torch.float32):
            raise ValueError("dtype must be torch.float64 or torch.float32")
        dims = [c.dims() for c in self.contexts]
        n = len(self.contexts)
        if outs is None:
            outs = [torch.empty((d["walk_num"], d["elec_num"], 5, d["mo_num"]), dtype=dtype,
                                device=f"cuda:{c.device}") for d, c in zip(dims, self.contexts)]

        def need(t, what, numel, dt):
            if t is None or not (t.is_cuda and t.is_contiguous() and t.dtype == dt):
                raise ValueError(f"{what} must be a contiguous CUDA tensor of dtype {dt}")
            if t.numel() != numel:
                raise ValueError(f"{what} holds {t.numel()} values, {numel} expected")

        if len(outs) != n:
            raise ValueError(f"outs holds {len(outs)} tensors for {n} contexts")
        for i, (t, d) in enumerate(zip(outs, dims)):
            need(t, f"outs[{i}]", d["walk_num"] * d["elec_num"] * 5 * d["mo_num"], dtype)
        P = ctypes.c_void_p
        o = (P * n)(*[t.data_ptr() for t in outs])
        w_arr = dc = de = dn = None
        if ws is not None:
            if len(ws) != n:
                raise ValueError(f"ws holds {len(ws)} tensors for {n} contexts")
            for i, (t, d) in enumerate(zip(ws, dims)):
                need(t, f"ws[{i}]", d["walk_num"] * d["elec_num"] * 5 * d["mo_num"], dtype)
            if grads is None:
                grads = [{"d_coef": torch.empty((d["mo_num"], d["ao_num"]), dtype=torch.float64, device=t.device),
                          "d_elec": torch.empty((d["walk_num"], d["elec_num"], 3), dtype=torch.float64, device=t.device),
                          "d_nucl": torch.empty((d["nucl_num"], 3), dtype=torch.float64, device=t.device)}
                         for d, t in zip(dims, outs)]
            if len(grads) != n:
                raise ValueError(f"grads holds {len(grads)} entries for {n} contexts")
            for i, (g, d) in enumerate(zip(grads, dims)):
                sizes = {"d_coef": d["mo_num"] * d["ao_num"], "d_elec": d["walk_num"] * d["elec_num"] * 3,
                         "d_nucl": d["nucl_num"] * 3}
                for k, t in g.items():
                    if k not in sizes:
                        raise ValueError(f"grads[{i}]: unknown output {k!r}")
                    if t is not None:
                        need(t, f"grads[{i}][{k!r}]", sizes[k], torch.float64)
            w_arr = (P * n)(*[t.data_ptr() for t in ws])

            def col(k):
                return (P * n)(*[(g[k].data_ptr() if g.get(k) is not None else None) for g in grads])
            dc, de, dn = col("d_coef"), col("d_elec"), col("d_nucl")
        self._check(self._lib.qmk_batch_run(self._h, o, QMK_F32 if dtype == torch.float32 else QMK_F64,
                                            w_arr, dc, de, dn, _stream(stream)))
        return (outs, grads) if ws is not None else outs

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.qmk_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd():
    import torch

    class MoVgl(torch.autograd.Function):
        """mo_vgl(C, R_nucl, R_elec) with a hand-written adjoint.

        forward(ctx, qctx, C [mo,ao], R_nucl [nucl,3], R_elec [walk,elec,3])
        -> [walk, elec, 5, mo].  C and R_nucl are copied to the context (host
        round trip, small arrays); R_elec stays on the device.  backward
        calls the library's adjoint, which recomputes AO derivatives up to
        third order instead of storing them.

        One context may serve several graphs: forward keeps host copies of C
        and R_nucl and the device coordinates, and backward puts them back
        into the context when another forward (or any set_* call of the
        inputs) ran in between, so every graph gets the gradients of its own
        inputs.  A change of precision, basis, cusp or screening settings in
        between is an error."""

        @staticmethod
        def forward(ctx, qctx: Context, C, R_nucl, R_elec):
            nucl = R_nucl.detach().double().cpu().numpy().copy()
            coef = C.detach().double().cpu().numpy().copy()
            qctx.set_nucleus(nucl)
            qctx.set_mo_coef(coef)
            r = R_elec.detach().to(torch.float64).contiguous()
            qctx.set_point(r)
            mo = qctx.get_mo_vgl()
            ctx.qctx = qctx
            ctx.devices = (C.device, R_nucl.device, R_elec.device)
            ctx.host_inputs = (nucl, coef)
            ctx.versions = (qctx._in_version, qctx._cfg_version)
            ctx.save_for_backward(r)
            return mo

        @staticmethod
        def backward(ctx, grad):
            qctx = ctx.qctx
            in_v, cfg_v = ctx.versions
            if qctx._cfg_version != cfg_v:
                raise RuntimeError("the context's precision, basis, cusp or screening settings changed "
                                   "between forward and backward")
            if qctx._in_version != in_v:
                (r,) = ctx.saved_tensors
                nucl, coef = ctx.host_inputs
                qctx.set_nucleus(nucl)
                qctx.set_mo_coef(coef)
                qctx.set_point(r)
                ctx.versions = (qctx._in_version, qctx._cfg_version)
            g = qctx.adjoint(grad.contiguous(), d_coef=ctx.needs_input_grad[1],
                             d_elec=ctx.needs_input_grad[3], d_nucl=ctx.needs_input_grad[2])
            dc, dn, de = g.get("d_coef"), g.get("d_nucl"), g.get("d_elec")
            dc = None if dc is None else dc.to(ctx.devices[0])
            dn = None if dn is None else dn.to(ctx.devices[1])
            de = None if de is None else de.to(ctx.devices[2])
            return None, dc, dn, de

    return MoVgl


def mo_vgl(qctx: Context, C, R_nucl, R_elec):
    """Differentiable mo_vgl through the library (torch.autograd)."""
    return _autograd().apply(qctx, C, R_nucl, R_elec)
