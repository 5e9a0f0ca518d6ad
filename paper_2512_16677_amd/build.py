"""Builds libqmk.so (HIP for gfx950) in-tree.

Every HIP source is compiled with hipcc for gfx950 only; packed FP32 vector
instructions are disabled for the device code.  Objects go to
``_build/`` at the repository root; the shared library lands next to this
file so the Python binding finds it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libqmk.so")
BUILD_DIR = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Per-unit code generation flags.  The FP32 products (units 4-6, whose FP32
# accumulators are converted to FP64 on output), the density and Jastrow
# products (units 7 and 10, whose epilogues do arithmetic on the
# accumulators) and the BF16x3 units accumulate in vector registers, so that
# the accumulators are not copied between register files on every K step (and
# the large tiles do not spill).  The FP64 units store the accumulation
# registers directly and are faster without it.
VGPR_ACC = ["-mllvm", "-amdgpu-mfma-vgpr-form"]
UNIT_FLAGS = {u: VGPR_ACC for u in (4, 5, 6, 7, 10)}

# (source, extra defines, object name): the MFMA product sources are compiled
# once per (precision, product) unit so that their many tile instantiations
# build in parallel.
SOURCES = [("context.cpp", [], None), ("batch.cpp", [], None), ("tuner.cpp", [], None),
           ("ao_kernels.hip", [], None), ("adjoint_kernels.hip", [], None),
           ("cusp_kernels.hip", [], None), ("sort_kernels.hip", [], None),
           ("det_kernels.hip", [], None), ("jastrow_kernels.hip", [], None), ("convert_kernels.hip", [], None),
           ("noalloc.hip", [], None),
           ("gemm_kernels.hip", [], None)]
SOURCES += [("gemm_kernels.hip", [f"-DQMK_GEMM_UNIT={u}"] + UNIT_FLAGS.get(u, []), f"gemm_kernels_u{u}")
            for u in range(1, 11)]
SOURCES += [("gemm_bf16p.hip", [], None)]
SOURCES += [("gemm_bf16p.hip", [f"-DQMK_GEMM_UNIT={u}"] + VGPR_ACC, f"gemm_bf16p_u{u}") for u in range(1, 4)]

DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(item) -> str:
    src, defs, name = item
    obj = os.path.join(BUILD_DIR, (name or os.path.basename(src)) + ".o")
    cmd = [HIPCC] + COMMON + DEVICE_FLAGS + defs + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4, 16)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC] + DEVICE_FLAGS + ["-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
