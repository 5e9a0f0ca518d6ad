"""Benchmark: mo_vgl electron-evaluations per second, forward + adjoint.

One step = one pass of the whole hot path over one batch of walkers:
set_point (fresh device coordinates, so the AO stage really runs), the AO
stage, the AO -> MO contraction into mo_vgl[walk, elec, 5, mo], and the
adjoint of sum(W * mo_vgl) with respect to the MO coefficients, the
electron coordinates and the nuclear coordinates.  Inputs are seeded and
synthetic and already resident in HBM when the timed region starts.

Workload (default): 40 C + 40 H in a 20-bohr cube, 800 Cartesian AOs,
400 MOs, 280 electrons, 512 walkers (143,360 points per step).

Prints ONE JSON line.  Run `python bench.py --help` for options.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "mo_vgl electron-evals/s (fwd+adjoint), mixed vs FP64 GPU at stated error"
PEAKS = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "fp64_TFLOPs": 78.6,
    "fp32_TFLOPs": 157.3,
    "bf16_TFLOPs": 2500.0,
}
MODE_DTYPE = {"fp64": "f64", "mixed_f32": "f32", "mixed_bf16x3": "bf16x3"}
# precision modes whose contraction has a screened (block-sparse) form
SCREENED_MODES = {"fp64": True, "mixed_f32": True, "mixed_bf16x3": True}
# useful-flop ceiling of each mode's contraction: the dense MFMA peak of its
# datatype (BF16x3 issues three bf16 products per useful one)
MODE_PEAK_TF = {"fp64": PEAKS["fp64_TFLOPs"], "mixed_f32": PEAKS["fp32_TFLOPs"],
                "mixed_bf16x3": PEAKS["bf16_TFLOPs"] / 3.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--walkers", type=int, default=512)
    ap.add_argument("--mode", default="fp64", choices=list(MODE_DTYPE))
    ap.add_argument("--variants", default="mixed_f32,mixed_bf16x3",
                    help="comma list of extra precision modes to time and compare with FP64")
    ap.add_argument("--mixed-bits", type=int, default=53,
                    help="precision parameter B of the mixed variants (cutoff of the exponentials)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--workload", default="medium", choices=["medium", "batch96", "density", "large", "det", "jastrow", "cusp"],
                    help="medium: one 80-atom molecule; batch96: 96 molecules of uneven sizes; "
                         "density: electron density of a 1114-AO molecule on a 100^3 grid; "
                         "large: 7500-AO system, dense vs screened contraction; "
                         "det: batched determinants and adjugates of small matrices; "
                         "jastrow: three-body Jastrow factor of the 80-atom molecule")
    ap.add_argument("--cpu-walkers", type=int, default=96,
                    help="walkers in the oracle's timed sample")
    ap.add_argument("--cpu-points", type=int, default=1000000,
                    help="grid points in the oracle's timed sample (density workload)")
    ap.add_argument("--cpu-walkers-1t", type=int, default=8,
                    help="walkers in the oracle's one-thread timed sample")
    ap.add_argument("--quick", action="store_true",
                    help="default workload only: skip the batch and 7500-AO workloads of the default line")
    ap.add_argument("--counter-summary", nargs="+", metavar="ARG",
                    help="no GPU work: MODE DB [DB ...]: sums of every counter of rocprofv3 databases of a "
                         "medium-workload run per product class (forward, G-bar, dL/dC), with derived ratios")
    ap.add_argument("--kernel-counter-summary", nargs="+", metavar="DB",
                    help="no GPU work: per kernel name, dispatch count and mean per dispatch of every counter "
                         "of rocprofv3 databases")
    ap.add_argument("--traffic-summary", nargs=5, metavar=("MODE", "FETCH_DB", "WRITE_DB", "COPY_FETCH_DB",
                                                            "COPY_WRITE_DB"),
                    help="no GPU work: summarise rocprofv3 FETCH_SIZE / WRITE_SIZE databases of a medium-workload "
                         "run in MODE and of a --copy-calibration run into per-class HBM bytes")
    return ap.parse_args()


def make_workload(walkers: int):
    import synth
    return synth.medium(walkers=walkers)


def run_gpu(s, mode: str, steps: int, warmup: int, bits: int, keep_outputs: bool = False):
    import torch
    import paper_2512_16677_amd as qmk

    dev = torch.device("cuda:0")
    ctx = qmk.Context.from_system(s, bits=bits, mode=mode)
    # two coordinate sets on the device; alternating them bumps the time stamp
    r0 = torch.from_numpy(np.ascontiguousarray(s.elec_coord)).to(dev)
    r1 = (r0 + 1e-3).contiguous()
    g = torch.Generator(device=dev)
    g.manual_seed(1234)
    w = torch.randn((s.walk_num, s.elec_num, 5, s.mo_num), generator=g, device=dev,
                    dtype=torch.float64)
    mo = torch.empty((s.walk_num, s.elec_num, 5, s.mo_num), device=dev, dtype=torch.float64)
    grads = {
        "d_coef": torch.empty((s.mo_num, s.ao_num), device=dev, dtype=torch.float64),
        "d_elec": torch.empty((s.walk_num, s.elec_num, 3), device=dev, dtype=torch.float64),
        "d_nucl": torch.empty((s.nucl_num, 3), device=dev, dtype=torch.float64),
    }

    def step(i):
        ctx.set_point(r0 if i % 2 == 0 else r1)
        ctx.get_mo_vgl(out=mo)
        ctx.adjoint(w, out=grads)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    # events between steps on the launch stream give the per-step spread
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        step(i)
        ev[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = ctx.timing()
    ctx.set_timing(False)
    ms = (t1 - t0) * 1e3 / steps
    per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    timing["_step_ms"] = {"min": per[0], "median": per[len(per) // 2], "max": per[-1]}
    # the same step with AO retention off: the adjoint evaluates the AO
    # array again instead of reading the forward pass's (not the timed value)
    ctx.set_ao_retention(False)
    n_re = max(3, steps // 2)
    step(0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i in range(n_re):
        step(i)
    torch.cuda.synchronize()
    timing["_recompute_ms"] = (time.perf_counter() - t2) * 1e3 / n_re
    ctx.set_ao_retention(True)
    outs = None
    if keep_outputs:  # one more (untimed) step on the first coordinate set
        ctx.set_point(r0)
        ctx.get_mo_vgl(out=mo)
        ctx.adjoint(w, out=grads)
        torch.cuda.synchronize()
        outs = {"mo": mo, **grads}
    ctx.close()
    return ms, timing, outs


def errors_vs(ref, got, quantile=True):
    """Mixed vs FP64 GPU results over the whole workload: row-normwise relative
    error of mo_vgl per component (max over points of max_n|diff| / max_n|ref|)
    and normwise error of each gradient (max|diff| / max|ref|)."""
    import torch
    e = {}
    num = (got["mo"] - ref["mo"]).abs().amax(dim=-1)
    den = ref["mo"].abs().amax(dim=-1).clamp_min(1e-300)
    r = (num / den).reshape(-1, 5)
    e["value"] = float(r[:, 0].max())
    e["gradient"] = float(r[:, 1:4].max())
    e["laplacian"] = float(r[:, 4].max())
    if quantile:
        e["laplacian_p999"] = float(torch.quantile(r[:, 4].float(), 0.999))
    for k in ("d_coef", "d_elec", "d_nucl"):
        e[k] = float((got[k] - ref[k]).abs().max() / ref[k].abs().max().clamp_min(1e-300))
    return e


KERNEL_SOURCES = {  # files whose change invalidates a kernel class's counter figures
    "mo": ["gemm_impl.h", "gemm_kernels.hip", "gemm_bf16p.hip", "qmk_internal.h", "context.cpp",
           "tiles_gfx950.json"],
    "ao": ["ao_kernels.hip", "qmk_internal.h", "context.cpp"],
    "ao_adjoint": ["adjoint_kernels.hip", "qmk_internal.h", "context.cpp"],
}
KERNEL_SOURCES["gbar"] = KERNEL_SOURCES["dcoef"] = KERNEL_SOURCES["mo"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_ch80_800ao.txt")


def sources_digest(name: str) -> str:
    import hashlib
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2512_16677_amd")
    for f in KERNEL_SOURCES[name]:
        path = os.path.join(pkg, "csrc", f)
        if not os.path.exists(path):
            path = os.path.join(pkg, f)
        with open(path, "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(mode: str, name: str):
    """HBM bytes per launch of kernel class `name`, from the committed
    hardware-counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by what
    the counter reads for a plain copy of known size).  None when the summary
    has no entry or the kernel's sources changed since it was taken."""
    if name not in KERNEL_SOURCES or not os.path.exists(TRAFFIC_FILE):
        return None
    want = sources_digest(name)
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if not line.startswith("traffic:"):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if kv.get("mode") == mode and kv.get("class") == name:
                return float(kv["bytes"]) if kv.get("sources") == want else None
    return None


def kernel_roofline(s, mode, timing):
    """Per-kernel algorithmic rates.  Contractions: 2*5*P*K*N flop per launch.
    AO stage: 5*K*P*bytes(element) written + 24*P read per launch; its adjoint
    reads the AO-sized G-bar and writes 24 B per point."""
    P, K, N = s.point_num, s.ao_num, s.mo_num
    flop = 2.0 * 5 * P * K * N
    esz = 8 if mode == "fp64" else 4
    out = {}
    for name in ("mo", "gbar", "dcoef"):
        t = timing[name]
        if t["launches"]:
            avg = t["ms"] / t["launches"]
            out[name] = {"avg_ms": avg, "launches": t["launches"], "flop": flop,
                         "TFLOPs": flop / (avg * 1e-3) / 1e12}
    for name, nbytes in (("ao", 5.0 * K * P * esz + 24.0 * P),
                         ("ao_adjoint", 5.0 * K * P * esz + 48.0 * P)):
        t = timing[name]
        if t["launches"]:
            avg = t["ms"] / t["launches"]
            out[name] = {"avg_ms": avg, "launches": t["launches"], "bytes": nbytes,
                         "GBps": nbytes / (avg * 1e-3) / 1e9}
    if timing["reduce"]["launches"]:
        out["reduce"] = {"avg_ms": timing["reduce"]["ms"] / timing["reduce"]["launches"],
                         "launches": timing["reduce"]["launches"]}
    t = timing.get("convert", {"launches": 0})
    if t["launches"]:  # W read in FP64, written as FP32 or as two bf16 planes: 12 B per element
        avg = t["ms"] / t["launches"]
        nbytes = 12.0 * P * 5 * N
        out["convert"] = {"avg_ms": avg, "launches": t["launches"], "bytes": nbytes,
                          "GBps": nbytes / (avg * 1e-3) / 1e9}
    return out


def dominant_roofline(mode, kr, traffic_lookup=True):
    """Roofline entry for the kernel class with the largest share of step time
    (the committed HBM counter figures belong to the medium workload, so other
    workloads pass traffic_lookup=False)."""
    peak_key = {"fp64": "fp64_TFLOPs", "mixed_f32": "fp32_TFLOPs", "mixed_bf16x3": "bf16_TFLOPs"}[mode]
    cands = {k: v for k, v in kr.items() if k not in ("reduce", "convert")}
    name = max(cands, key=lambda k: cands[k]["avg_ms"] * cands[k]["launches"])
    d = cands[name]
    traffic = measured_traffic(mode, name) if traffic_lookup else None
    if "TFLOPs" in d:
        # BF16x3 issues three products per element; the algorithmic rate counts one
        roof = {"bound": "mfma", "achieved": d["TFLOPs"], "peak": PEAKS[peak_key], "unit": "TFLOP/s",
                "frac": d["TFLOPs"] / PEAKS[peak_key]}
    else:
        roof = {"bound": "hbm", "achieved": d["GBps"], "peak": PEAKS["hbm_GBps"], "unit": "GB/s",
                "frac": d["GBps"] / PEAKS["hbm_GBps"]}
    roof.update({"traffic": traffic, "kernel": name, "avg_ms": d["avg_ms"],
                 "traffic_unit": "bytes per launch (FETCH_SIZE, WRITE_SIZE scaled by a copy kernel)",
                 "per_kernel": kr})
    return roof


def cpu_baseline(walkers: int, threads: int = 0):
    """The FP64 oracle, forward + adjoint, on a bounded sample of the workload.
    threads = 0: the oracle's default (all host cores); otherwise the sample
    runs in a child process limited to that many OpenMP threads."""
    import oracle
    import synth
    if threads:
        import subprocess
        code = ("import json, sys; sys.path.insert(0, %r); import bench; "
                "print(json.dumps(bench.cpu_baseline(%d)))" % (ROOT, walkers))
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                             timeout=900, check=True).stdout
        res = json.loads(out.strip().splitlines()[-1])
        res["cores"] = threads
        return res
    s = synth.medium(walkers=walkers)
    w = synth.adjoint_weights(s, seed=1)
    n_threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    oracle.mo_vgl(s)
    oracle.adjoint(s, w, with_abs=False)
    dt = time.perf_counter() - t0
    return {"value": s.point_num / dt, "unit": "e-evals/s", "cores": n_threads, "kind": "oracle",
            "sample": f"{walkers} walkers x {s.elec_num} electrons of the same 800-AO/400-MO "
                      f"system (forward + adjoint), {dt:.1f} s", "cpu_model": cpu_model()}


def cpu_model() -> str:
    """Model of the host CPU as lscpu reports it: the model name plus the
    BIOS model name, family, model and stepping when present (some virtual
    machines report only a short model name); else /proc/cpuinfo's model
    name, or an empty string."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=30).stdout
        f = {}
        for ln in out.splitlines():
            if ":" in ln:
                k, v = ln.split(":", 1)
                f.setdefault(k.strip(), v.strip())
        if f.get("Model name"):
            extra = [f"{k.lower()} {f[k]}" for k in ("CPU family", "Model", "Stepping") if f.get(k)]
            bios = f.get("BIOS Model name", "")
            name = f["Model name"] + (f" / BIOS: {bios}" if bios and bios != f["Model name"] else "")
            return name + (f" ({', '.join(extra)})" if extra else "")
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def run_batch(mols, mode, steps, warmup, bits, batched=True, keep_outputs=False):
    """Forward + adjoint of every molecule per step, as one batch (one graph
    launch) or as a loop of single-context calls.  Returns ms per step and,
    with keep_outputs, the outputs of one more step on the first coordinates
    (mo_vgl widened to FP64 and the three gradients, per molecule)."""
    import torch
    import paper_2512_16677_amd as qmk
    dev = torch.device("cuda:0")
    dt = torch.float64 if mode == "fp64" else torch.float32
    ctxs = [qmk.Context.from_system(m, bits=bits, mode=mode) for m in mols]
    r = [[torch.from_numpy(np.ascontiguousarray(m.elec_coord)).to(dev)] for m in mols]
    for x in r:
        x.append((x[0] + 1e-3).contiguous())
    g = torch.Generator(device=dev)
    g.manual_seed(99)
    ws = [torch.randn((m.walk_num, m.elec_num, 5, m.mo_num), generator=g, device=dev, dtype=torch.float64).to(dt)
          for m in mols]
    outs = [torch.empty_like(w) for w in ws]
    grads = [{"d_coef": torch.empty((m.mo_num, m.ao_num), dtype=torch.float64, device=dev),
              "d_elec": torch.empty((m.walk_num, m.elec_num, 3), dtype=torch.float64, device=dev),
              "d_nucl": torch.empty((m.nucl_num, 3), dtype=torch.float64, device=dev)} for m in mols]
    b = qmk.Batch(ctxs) if batched else None

    def step(i):
        for c, x in zip(ctxs, r):
            c.set_point(x[i % 2])
        if batched:
            b.run(outs=outs, dtype=dt, ws=ws, grads=grads)
        else:
            for c, o, w, gr in zip(ctxs, outs, ws, grads):
                c.get_mo_vgl(out=o)
                c.adjoint(w, out=gr)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    kept = None
    if keep_outputs:
        step(0)
        torch.cuda.synchronize()
        kept = [{"mo": o.double(), **{k: v.clone() for k, v in gr.items()}} for o, gr in zip(outs, grads)]
    if b:
        b.close()
    for c in ctxs:
        c.close()
    return (ms, kept) if keep_outputs else ms


def batch_errors(ref, got):
    """Mixed vs FP64 batch outputs: the largest row-normwise error of mo_vgl
    per component over every molecule's points, and the largest normwise
    error of each gradient over the molecules."""
    e = {}
    for rm, gm in zip(ref, got):
        one = errors_vs(rm, gm, quantile=False)
        for k, v in one.items():
            e[k] = max(e.get(k, 0.0), v)
    return e


def batch_oracle_sample(mols, bits, outs, n_points=8):
    """Row-normwise error of sampled mo_vgl rows of three molecules (first,
    middle, last) against the oracle at the same B."""
    import oracle
    from tests.helpers import component_errors
    worst = {}
    for m in (0, len(mols) // 2, len(mols) - 1):
        s = mols[m]
        idx = np.linspace(0, s.point_num - 1, n_points).astype(np.int64)
        rows = outs[m]["mo"].reshape(s.point_num, 5, s.mo_num)[idx].cpu().numpy()
        e = component_errors(rows, oracle.mo_vgl(s, points=s.points()[idx], B=bits))
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
    return worst


def batch_workload(a, modes):
    """The 96-molecule batch: e-evals/s per mode, the fraction of the summed
    per-molecule MFMA ceilings, the speedup over a loop of single-context
    calls, and the mixed forms' errors against the FP64 batch and the oracle."""
    import synth
    import torch
    mols = synth.molecule_batch(96, seed=0)
    pts = sum(m.point_num for m in mols)
    flop = sum(3 * 2.0 * 5 * m.point_num * m.ao_num * m.mo_num for m in mols)  # fwd + 2 adjoint products
    res = {}
    ref = None
    for mode in modes:
        bits = 53 if mode == "fp64" else a.mixed_bits
        ms_b, kept = run_batch(mols, mode, a.steps, a.warmup, bits, batched=True, keep_outputs=True)
        ms_l = run_batch(mols, mode, max(2, a.steps // 4), 1, bits, batched=False)
        peak = MODE_PEAK_TF[mode] * 1e12
        res[mode] = {"value": pts / (ms_b * 1e-3), "unit": "e-evals/s", "ms_per_step": ms_b, "bits": bits,
                     "ceiling_frac": (flop / peak) / (ms_b * 1e-3),
                     "unbatched_ms_per_step": ms_l, "batching_speedup": ms_l / ms_b}
        if mode == "fp64":
            ref = kept
            res[mode]["oracle_sample_error"] = batch_oracle_sample(mols, bits, kept)
        else:
            if ref is not None:
                res[mode]["error_vs_fp64_gpu"] = batch_errors(ref, kept)
            res[mode]["oracle_sample_error"] = batch_oracle_sample(mols, bits, kept)
            res[mode]["speedup_vs_fp64_batch"] = res["fp64"]["ms_per_step"] / ms_b if "fp64" in res else None
        del kept
        torch.cuda.empty_cache()
    del ref
    torch.cuda.empty_cache()
    return {"workload": "batch96: 96 C/H molecules, 4-60 atoms, 8-128 walkers each, one persistent-kernel "
                        "HIP graph per step; forward + adjoint",
            "points_per_step": pts, "molecules": len(mols),
            "ao_range": [min(m.ao_num for m in mols), max(m.ao_num for m in mols)],
            "ceiling_definition": "sum over molecules of 3 x 2 x 5 x P x K x N flop at the mode's dense MFMA "
                                  "peak (BF16x3: a third of the bf16 peak), divided by the measured step",
            "modes": res}


def main_batch(a):
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    modes = ["fp64"] + [v for v in a.variants.split(",") if v]
    bw = batch_workload(a, modes)
    res = bw["modes"]
    line = {"metric": METRIC, "value": res["fp64"]["value"], "unit": "e-evals/s", "n_gpus": 1,
            "steps": a.steps, "warmup": a.warmup, "ms_per_step": res["fp64"]["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {k: v for k, v in bw.items() if k != "modes"},
            "modes": res}
    print(json.dumps(line))


def run_density(s, occ, mode, steps, warmup, bits):
    """get_density on fresh grid coordinates every step (so the AO stage runs)."""
    import torch
    import paper_2512_16677_amd as qmk
    dev = torch.device("cuda:0")
    ctx = qmk.Context.from_system(s, bits=bits, mode=mode)
    r0 = torch.from_numpy(np.ascontiguousarray(s.elec_coord)).to(dev)
    r1 = (r0 + 1e-3).contiguous()
    rho = torch.empty((s.walk_num, s.elec_num), dtype=torch.float64, device=dev)

    def step(i):
        ctx.set_point(r0 if i % 2 == 0 else r1)
        ctx.get_density(occ, out=rho)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    timing = ctx.timing()
    ctx.close()
    return ms, timing


def main_density(a):
    import synth
    s = synth.peptide_like()
    occ = s.meta["occ"]
    P, K, No = s.point_num, s.ao_num, int(np.count_nonzero(occ))
    flop = 2.0 * P * K * No
    res = {}
    for mode in ["fp64"] + [v for v in a.variants.split(",") if v == "mixed_f32"]:
        bits = 53 if mode == "fp64" else a.mixed_bits
        ms, t = run_density(s, occ, mode, a.steps, a.warmup, bits)
        esz = 8 if mode == "fp64" else 4
        per = {}
        for name in ("ao", "density", "reduce"):
            if t[name]["launches"]:
                per[name] = {"avg_ms": t[name]["ms"] / t[name]["launches"], "launches": t[name]["launches"]}
        per["ao"]["GBps"] = (K * P * esz + 24.0 * P) / (per["ao"]["avg_ms"] * 1e-3) / 1e9
        per["density"]["TFLOPs"] = flop / (per["density"]["avg_ms"] * 1e-3) / 1e12
        res[mode] = {"value": P / (ms * 1e-3), "ms_per_step": ms, "per_kernel": per}
    d = res["fp64"]["per_kernel"]
    dom = "density" if d["density"]["avg_ms"] >= d["ao"]["avg_ms"] else "ao"
    roof = ({"bound": "mfma", "achieved": d["density"]["TFLOPs"], "peak": PEAKS["fp64_TFLOPs"],
             "unit": "TFLOP/s", "frac": d["density"]["TFLOPs"] / PEAKS["fp64_TFLOPs"]} if dom == "density" else
            {"bound": "hbm", "achieved": d["ao"]["GBps"], "peak": PEAKS["hbm_GBps"], "unit": "GB/s",
             "frac": d["ao"]["GBps"] / PEAKS["hbm_GBps"]})
    roof.update({"kernel": dom, "traffic": None})
    line = {"metric": "density grid points/s (value-only AOs, MO product with fused sum of squares)",
            "value": res["fp64"]["value"], "unit": "points/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": res["fp64"]["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"peptide_like: 104 atoms (C34 N11 O10 H48 Cu), {K} AOs, "
                                   f"{No} doubly occupied of {s.mo_num} MOs, 100^3 grid",
                       "points_per_step": P},
            "roofline": roof, "modes": res,
            "paper_context": "Section 5.4: density of a 1114-AO, 218-occupied-MO molecule on a 100^3 "
                             "grid in 5.0 s (FP64) / 3.7 s (FP32) on 18 cores of an i7-13850HX, "
                             "including file input and cube output"}
    if not a.no_cpu_baseline:
        import oracle
        n = a.cpu_points
        pts = s.points()[:: max(1, P // n)][:n]
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        oracle.density(s, occ, points=pts)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": len(pts) / dt, "unit": "points/s", "cores": threads,
                                "kind": "oracle",
                                "sample": (f"the whole {len(pts)}-point grid" if len(pts) == P else
                                           f"{len(pts)} evenly strided grid points of the same system")
                                          + f", FP64, {dt:.1f} s"}
    print(json.dumps(line))


def large_workload(a):
    """The 7500-AO / 1050-MO system at 64 walkers: forward + adjoint with the
    dense and the screened contraction, per precision mode (FP64 at B = 53,
    the mixed modes at B = 24), each with the roofline of its dominant kernel
    class; the mixed forms' errors against the FP64 GPU path and, on sampled
    rows, against the oracle at their own B."""
    import torch
    import oracle
    import synth
    import paper_2512_16677_amd as qmk
    from tests.helpers import component_errors
    s = synth.large(walkers=64)
    P, K, N = s.point_num, s.ao_num, s.mo_num
    dev = torch.device("cuda:0")
    r0 = torch.from_numpy(np.ascontiguousarray(s.elec_coord)).to(dev)
    r1 = (r0 + 1e-3).contiguous()
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    w64 = torch.randn((s.walk_num, s.elec_num, 5, N), generator=g, device=dev, dtype=torch.float64)
    idx = np.linspace(0, P - 1, 8).astype(np.int64)
    steps, warmup = max(2, a.steps // 4), max(1, a.warmup // 2)
    res = {}
    ref = None
    for mode, bits in (("fp64", 53), ("mixed_f32", 24), ("mixed_bf16x3", 24)):
        ctx = qmk.Context.from_system(s, bits=bits, mode=mode)
        dt = torch.float64 if mode == "fp64" else torch.float32
        w = w64.to(dt)
        mo = torch.empty((s.walk_num, s.elec_num, 5, N), dtype=dt, device=dev)
        grads = {"d_coef": torch.empty((N, K), dtype=torch.float64, device=dev),
                 "d_elec": torch.empty((s.walk_num, s.elec_num, 3), dtype=torch.float64, device=dev),
                 "d_nucl": torch.empty((s.nucl_num, 3), dtype=torch.float64, device=dev)}
        out = {}
        for screened in (False, True):
            if screened and not SCREENED_MODES.get(mode, False):
                out["screened"] = None  # this mode has no screened product; the dense one runs
                continue
            ctx.set_screening(screened)
            key = "screened" if screened else "dense"

            def step(i):
                ctx.set_point(r0 if i % 2 == 0 else r1)
                ctx.get_mo_vgl(out=mo)
                ctx.adjoint(w, out=grads)

            for i in range(warmup):
                step(i)
            torch.cuda.synchronize()
            ctx.set_timing(True)
            t0 = time.perf_counter()
            for i in range(steps):
                step(i)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            t = ctx.timing()
            ctx.set_timing(False)
            kr = kernel_roofline(s, mode, t)
            out[key] = {"fwd_adjoint_ms": ms, "value": P / (ms * 1e-3), "unit": "e-evals/s",
                        "roofline": dominant_roofline(mode, kr, traffic_lookup=False)}
            if screened:
                out[key]["screening_density"] = ctx.screening_density()
                # the screened product skips all-zero AO chunks: its rate against the dense
                # product's flops is an effective rate, and can exceed the peak
                rl = out[key]["roofline"]
                rl["effective_frac"] = rl.pop("frac")
                rl["note"] = ("achieved and effective_frac count the dense product's flops; the screened "
                              "product skips all-zero AO chunks, so effective_frac is not a fraction of "
                              "the work it executes")
            if not screened:
                step(0)
                torch.cuda.synchronize()
                got = {"mo": mo.double().clone(), **{k: v.clone() for k, v in grads.items()}}
                rows = got["mo"].reshape(P, 5, N)[torch.from_numpy(idx).to(dev)].cpu().numpy()
                out["oracle_sample_error"] = component_errors(rows, oracle.mo_vgl(s, points=s.points()[idx],
                                                                                  B=bits))
                if mode == "fp64":
                    ref = got
                else:
                    out["error_vs_fp64_gpu"] = errors_vs(ref, got)
                    out["error_vs_fp64_gpu"]["note"] = "FP64 at B = 53, this mode at B = 24 (cutoff included)"
                    del got
        out["bits"] = bits
        if out.get("screened"):
            out["screened_speedup"] = out["dense"]["fwd_adjoint_ms"] / out["screened"]["fwd_adjoint_ms"]
        ctx.close()
        del mo, w, grads
        torch.cuda.empty_cache()
        res[mode] = out
    del ref, w64
    torch.cuda.empty_cache()
    return {"workload": f"ch300_7500ao: 150 C + 150 H in a 35-bohr cube, {K} AOs, {N} MOs, "
                        f"{s.elec_num} electrons, 64 walkers; forward + adjoint",
            "points_per_step": P, "steps": steps, "warmup": warmup, "modes": res}


def main_large(a):
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    lw = large_workload(a)
    res = lw["modes"]
    line = {"metric": "mo_vgl electron-evals/s (fwd+adjoint), dense vs screened contraction",
            "value": res["fp64"]["screened"]["value"], "unit": "e-evals/s", "n_gpus": 1,
            "steps": lw["steps"], "warmup": lw["warmup"], "ms_per_step": res["fp64"]["screened"]["fwd_adjoint_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": lw["workload"], "points_per_step": lw["points_per_step"]},
            "modes": res}
    print(json.dumps(line))


def main_det(a):
    """Determinant + adjugate of 2^24 random n x n matrices, n = 2, 3, 4, and
    2^16 matrices of n = 16 (LU path); one launch per step."""
    import torch
    import paper_2512_16677_amd as qmk
    ctx = qmk.Context()
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    res = {}
    for n, batch in ((2, 1 << 24), (3, 1 << 24), (4, 1 << 24), (16, 1 << 16)):
        A = torch.randn((batch, n, n), generator=g, device="cuda", dtype=torch.float64)
        det = torch.empty((batch,), dtype=torch.float64, device="cuda")
        adj = torch.empty_like(A)
        ctx._check(ctx._lib.qmk_det_adj(ctx._h, n, batch, qmk._ptr(A), qmk._ptr(det), qmk._ptr(adj),
                                        qmk._stream(None)))
        for _ in range(a.warmup):
            ctx._check(ctx._lib.qmk_det_adj(ctx._h, n, batch, qmk._ptr(A), qmk._ptr(det), qmk._ptr(adj),
                                            qmk._stream(None)))
        torch.cuda.synchronize()
        ctx.set_timing(True)
        for _ in range(a.steps):
            ctx._check(ctx._lib.qmk_det_adj(ctx._h, n, batch, qmk._ptr(A), qmk._ptr(det), qmk._ptr(adj),
                                            qmk._stream(None)))
        t = ctx.timing()["det"]
        ms = t["ms"] / t["launches"]
        nbytes = batch * (2 * n * n + 1) * 8.0
        res[f"n{n}"] = {"batch": batch, "avg_ms": ms, "matrices_per_s": batch / (ms * 1e-3),
                        "GBps": nbytes / (ms * 1e-3) / 1e9}
        del A, adj, det
        torch.cuda.empty_cache()
    ctx.close()
    d4 = res["n4"]
    line = {"metric": "4x4 determinant+adjugate matrices/s", "value": d4["matrices_per_s"],
            "unit": "matrices/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": d4["avg_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "2^24 random 4x4 FP64 matrices (also n = 2, 3; n = 16 by LU)"},
            "roofline": {"bound": "hbm", "achieved": d4["GBps"], "peak": PEAKS["hbm_GBps"], "unit": "GB/s",
                         "frac": d4["GBps"] / PEAKS["hbm_GBps"], "traffic": None, "kernel": "det_adj_small<4>"},
            "sizes": res}
    print(json.dumps(line))


def main_jastrow(a):
    """Three-body Jastrow factor of the ch80_800ao molecule (80 nuclei, 280
    electrons) for `walkers` walkers at expansion order 5: rescaled distances,
    the P product on MFMA and the contraction, one call per step."""
    import torch
    import oracle
    import synth
    import paper_2512_16677_amd as qmk
    nord, kappa = 5, 0.6
    s = synth.medium(walkers=a.walkers)
    rng = np.random.default_rng(0)
    c = rng.normal(scale=0.2, size=(qmk.jastrow_een_terms(nord), s.nucl_num))
    ctx = qmk.Context.from_system(s)
    out = torch.empty((s.walk_num,), dtype=torch.float64, device="cuda")
    for _ in range(1 + a.warmup):
        ctx.jastrow_een(nord, kappa, c, out=out)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ctx.jastrow_een(nord, kappa, c, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / a.steps
    tm = ctx.timing()
    ctx.close()
    W, ne, nn = s.walk_num, s.elec_num, s.nucl_num
    # the product: rows (m = 1..nord/2, nucleus), splits k = 0..nord-2
    M, nsplit = (nord // 2) * nn, nord - 1
    flops = 2.0 * W * nsplit * M * ne * ne
    p_ms = tm["jastrow_p"]["ms"] / tm["jastrow_p"]["launches"]
    tf = flops / (p_ms * 1e-3) / 1e12
    line = {"metric": "three-body Jastrow electron-evals/s", "value": W * ne / (ms * 1e-3),
            "unit": "electron-evals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"ch80_800ao: 40 C + 40 H, {ne} electrons, {W} walkers, "
                                   f"J_een order {nord}, kappa {kappa}"},
            "roofline": {"bound": "mfma", "achieved": tf, "peak": PEAKS["fp64_TFLOPs"], "unit": "TFLOP/s",
                         "frac": tf / PEAKS["fp64_TFLOPs"], "traffic": None,
                         "kernel": "gemm_kernel EPI 5 (P product, fused weights)"},
            "kernels_ms_per_step": {k: tm[k]["ms"] / a.steps for k in ("jastrow", "jastrow_p")}}
    if not a.no_cpu_baseline:
        n = max(1, min(a.cpu_walkers, W))
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        oracle.jastrow_een(s.elec_coord[:n], s.nucl_coord, kappa, nord, c)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": n * ne / dt, "unit": "electron-evals/s", "cores": threads,
                                "kind": "oracle", "sample": f"{n} walkers of the same workload"}
    print(json.dumps(line))


def main_cusp(a):
    """MO cusp correction (Section 3.3) on the medium workload (512 walkers,
    radii 0.25 bohr on C and 0.2 bohr on H): one step is set_point (fresh
    device coordinates), the AO stage, the forward contraction and the
    in-place cusp kernel.  The same steps without the correction are timed
    beside it.  The cusp kernel reads every point's coordinates and reads and
    writes the mo_vgl row of every point inside a sphere."""
    import torch
    import oracle
    import synth
    import paper_2512_16677_amd as qmk
    s = synth.medium(walkers=a.walkers)
    z = s.nucl_charge.astype(np.float64)
    rc = np.where(z > 1, 0.25, 0.2)
    dev = torch.device("cuda:0")
    coords = [np.ascontiguousarray(s.elec_coord), np.ascontiguousarray(s.elec_coord + 1e-3)]
    r = [torch.from_numpy(c).to(dev) for c in coords]
    ctx = qmk.Context.from_system(s)
    out = torch.empty((s.walk_num, s.elec_num, 5, s.mo_num), dtype=torch.float64, device=dev)

    def run(cusp):
        if cusp:
            ctx.set_mo_cusp(z, rc)
        else:
            ctx.set_mo_cusp(None)
        for i in range(1 + a.warmup):
            ctx.set_point(r[i % 2])
            ctx.get_mo_vgl(out=out)
        torch.cuda.synchronize()
        ctx.set_timing(False)
        ctx.set_timing(True)
        t0 = time.perf_counter()
        for i in range(a.steps):
            ctx.set_point(r[i % 2])
            ctx.get_mo_vgl(out=out)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / a.steps, ctx.timing()

    ms_off, _ = run(False)
    ms, tm = run(True)
    ctx.close()
    P, K, N = s.point_num, s.ao_num, s.mo_num

    def inside(c):
        d2 = ((c.reshape(-1, 1, 3) - s.nucl_coord[None]) ** 2).sum(-1)
        return int((d2 < rc[None] ** 2).any(axis=1).sum())

    n_in = sum(inside(coords[i % 2]) for i in range(a.steps)) / a.steps
    cusp_ms = tm["cusp"]["ms"] / tm["cusp"]["launches"]
    cusp_bytes = 24.0 * P + n_in * 2 * 5 * N * 8
    mo_ms = tm["mo"]["ms"] / tm["mo"]["launches"]
    tf = 2.0 * 5 * P * K * N / (mo_ms * 1e-3) / 1e12
    line = {"metric": "cusp-corrected mo_vgl electron-evals/s (forward)", "value": P / (ms * 1e-3),
            "unit": "e-evals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"ch80_800ao with MO cusp correction: 40 C + 40 H, {K} AOs, {N} MOs, "
                                   f"{s.walk_num} walkers x {s.elec_num} electrons, r_c 0.25 (C) / 0.2 (H) bohr"},
            "roofline": {"bound": "mfma", "achieved": tf, "peak": PEAKS["fp64_TFLOPs"], "unit": "TFLOP/s",
                         "frac": tf / PEAKS["fp64_TFLOPs"], "traffic": None,
                         "kernel": "gemm_kernel (forward product, the largest share of the step)"},
            "cusp_kernel": {"avg_ms": cusp_ms, "points_inside": n_in, "bytes": cusp_bytes,
                            "GBps": cusp_bytes / (cusp_ms * 1e-3) / 1e9,
                            "frac_hbm": cusp_bytes / (cusp_ms * 1e-3) / 1e9 / PEAKS["hbm_GBps"]},
            "without_cusp_ms_per_step": ms_off,
            "kernels_ms_per_step": {k: tm[k]["ms"] / a.steps for k in ("ao", "mo", "cusp")}}
    if not a.no_cpu_baseline:
        n = max(1, min(a.cpu_walkers, s.walk_num))
        sub = synth.medium(walkers=n)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        oracle.mo_vgl_cusp(sub, z, rc, points=np.ascontiguousarray(s.elec_coord[:n]).reshape(-1, 3))
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": n * s.elec_num / dt, "unit": "e-evals/s", "cores": threads,
                                "kind": "oracle", "sample": f"{n} walkers of the same workload (forward)"}
    print(json.dumps(line))


def copy_calibration():
    """A plain device-to-device copy of known size: under a hardware-counter
    profile its FETCH_SIZE / WRITE_SIZE give the factor that turns those
    counters into bytes."""
    import torch
    n = 1 << 27  # float64 elements: 1 GiB
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))


def _counter_rows(db: str, counter: str):
    """(dispatch id, kernel name, summed counter value) of every dispatch in a
    rocprofv3 database, in launch order."""
    import sqlite3
    c = sqlite3.connect(db)
    rows = c.execute("select dispatch_id, kernel_name, sum(value) from counters_collection "
                     "where counter_name = ? group by dispatch_id order by dispatch_id", (counter,)).fetchall()
    c.close()
    return rows


def _classify(name: str):
    """Kernel class of a dispatch of the medium step (None: not counted).
    Products are told apart by their order within a step (forward, G-bar,
    dC), since G-bar and dC may run the same kernel."""
    if "ao_vgl" in name:
        return "ao"
    if "ao_adjoint" in name:
        return "ao_adjoint"
    if "split_w" in name or "f64_to_f32" in name:
        return "convert"
    if "gemm" in name:
        return "product"
    return None


def kernel_counter_summary(*dbs):
    """Per kernel name: dispatches and the mean per dispatch of each counter."""
    import sqlite3
    for db in dbs:
        c = sqlite3.connect(db)
        rows = c.execute("select kernel_name, counter_name, count(distinct dispatch_id), sum(value) "
                         "from counters_collection group by kernel_name, counter_name").fetchall()
        c.close()
        print(f"# {db}")
        print(f"{'dispatches':>10s} {'counter':14s} {'mean per dispatch':>18s}  kernel")
        for name, counter, n, tot in sorted(rows, key=lambda r: -r[3]):
            print(f"{n:10d} {counter:14s} {tot / n:18.1f}  {name[:150]}")


def counter_summary(mode, *dbs):
    """Per product class (forward, G-bar, dL/dC, in launch order within a
    step), the sum over its dispatches of every counter in the databases."""
    import sqlite3
    tot = {}
    for db in dbs:
        c = sqlite3.connect(db)
        names = [r[0] for r in c.execute("select distinct counter_name from counters_collection")]
        c.close()
        for counter in names:
            k = 0
            for _, name, v in _counter_rows(db, counter):
                if _classify(name) != "product":
                    continue
                cls = ("mo", "gbar", "dcoef")[k % 3]
                k += 1
                tot.setdefault(cls, {}).setdefault(counter, 0.0)
                tot[cls][counter] += v
    print(f"mode {mode}: counter sums over the dispatches of each product class")
    for cls in ("mo", "gbar", "dcoef"):
        if cls not in tot:
            continue
        t = tot[cls]
        print(f"\n{cls}:")
        for k in sorted(t):
            print(f"    {k:28s} {t[k]:.4g}")
        if t.get("SQ_INSTS_MFMA"):
            if "SQ_INSTS_VALU" in t:
                print(f"    {'VALU instructions per MFMA':28s} {t['SQ_INSTS_VALU'] / t['SQ_INSTS_MFMA']:.2f}")
            if "SQ_INSTS_LDS" in t:
                print(f"    {'LDS instructions per MFMA':28s} {t['SQ_INSTS_LDS'] / t['SQ_INSTS_MFMA']:.2f}")
        if t.get("SQ_WAVE_CYCLES") and "SQ_WAIT_ANY" in t:
            print(f"    {'SQ_WAIT_ANY / SQ_WAVE_CYCLES':28s} {t['SQ_WAIT_ANY'] / t['SQ_WAVE_CYCLES']:.2f}")
        if t.get("SQ_INSTS_LDS") and "SQ_LDS_BANK_CONFLICT" in t:
            print(f"    {'LDS conflict cycles per LDS instruction':28s} "
                  f"{t['SQ_LDS_BANK_CONFLICT'] / t['SQ_INSTS_LDS']:.2f}")


def traffic_summary(mode, fetch_db, write_db, cfetch_db, cwrite_db):
    """Per-class HBM bytes per launch from counter databases (KiB per dispatch),
    each counter scaled by what it reads for the 1 GiB copy."""
    def copy_kib(db, counter):
        v = [x for _, n, x in _counter_rows(db, counter) if "copyBuffer" in n or "copy" in n.lower()]
        return sum(v) / len(v)
    f_scale = (1 << 30) / (copy_kib(cfetch_db, "FETCH_SIZE") * 1024.0)
    w_scale = (1 << 30) / (copy_kib(cwrite_db, "WRITE_SIZE") * 1024.0)
    per = {}
    for db, counter in ((fetch_db, "FETCH_SIZE"), (write_db, "WRITE_SIZE")):
        k = 0
        for _, name, v in _counter_rows(db, counter):
            cls = _classify(name)
            if cls is None:
                continue
            if cls == "product":
                cls = ("mo", "gbar", "dcoef")[k % 3]
                k += 1
            per.setdefault(cls, {}).setdefault(counter, []).append((v, name))
    import synth
    s = make_workload(512)
    P, K, N = s.point_num, s.ao_num, s.mo_num
    # element bytes of the AO array / G-bar / C (bf16 planes: hi + lo), and of W
    # as the products read it (the medium step passes FP64 W and writes FP64
    # mo_vgl in every mode; the mixed modes convert W once per call)
    esz = 8 if mode == "fp64" else 4
    wsz = 8 if mode == "fp64" else 4
    ao = 5.0 * K * P * esz
    algo = {  # operands read once + results written once
        "ao": ao + 24.0 * P,
        "mo": ao + K * N * esz + 5.0 * P * N * 8,
        "gbar": 5.0 * P * N * wsz + K * N * esz + ao,
        "dcoef": 5.0 * P * N * wsz + ao + N * K * 8.0,
        "ao_adjoint": ao + 48.0 * P,
        "convert": 5.0 * P * N * (8 + 4),
    }
    lines = []
    for cls in ("ao", "mo", "gbar", "dcoef", "ao_adjoint", "convert"):
        if cls not in per or "FETCH_SIZE" not in per[cls] or "WRITE_SIZE" not in per[cls]:
            continue
        fk = sum(v for v, _ in per[cls]["FETCH_SIZE"]) / len(per[cls]["FETCH_SIZE"])
        wk = sum(v for v, _ in per[cls]["WRITE_SIZE"]) / len(per[cls]["WRITE_SIZE"])
        b = fk * 1024.0 * f_scale + wk * 1024.0 * w_scale
        kname = per[cls]["FETCH_SIZE"][0][1].split("(")[0][:60]
        src = sources_digest(cls) if cls in KERNEL_SOURCES else "-"
        lines.append({"class": cls, "fetch_kib": fk, "write_kib": wk, "bytes": b, "algorithmic": algo[cls],
                      "ratio": b / algo[cls], "launches": len(per[cls]["FETCH_SIZE"]), "kernel": kname,
                      "sources": src})
    print(f"# copy calibration: bytes = FETCH_SIZE x 1024 x {f_scale:.4f}, WRITE_SIZE x 1024 x {w_scale:.4f}")
    print(f"{'class':12s} {'FETCH KiB':>12s} {'WRITE KiB':>12s} {'HBM bytes':>11s} {'algorithmic':>11s} "
          f"{'ratio':>6s}  kernel")
    for d in lines:
        print(f"{d['class']:12s} {d['fetch_kib']:12.1f} {d['write_kib']:12.1f} {d['bytes']:11.4g} "
              f"{d['algorithmic']:11.4g} {d['ratio']:6.2f}  {d['kernel']}")
    print()
    for d in lines:
        if d["sources"] != "-":
            print(f"traffic: mode={mode} class={d['class']} bytes={d['bytes']:.6g} fetch_kib={d['fetch_kib']:.1f} "
                  f"write_kib={d['write_kib']:.1f} sources={d['sources']}")


def main():
    a = parse()
    if a.traffic_summary:
        traffic_summary(*a.traffic_summary)
        return
    if a.counter_summary:
        counter_summary(*a.counter_summary)
        return
    if a.kernel_counter_summary:
        kernel_counter_summary(*a.kernel_counter_summary)
        return
    if a.copy_calibration:
        copy_calibration()
        return
    if a.workload == "jastrow":
        if a.gpus != 1:
            print(json.dumps({"error": "one GPU only"}))
            sys.exit(2)
        main_jastrow(a)
        return
    if a.workload == "cusp":
        if a.gpus != 1:
            print(json.dumps({"error": "one GPU only"}))
            sys.exit(2)
        main_cusp(a)
        return
    if a.workload == "det":
        if a.gpus != 1:
            print(json.dumps({"error": "one GPU only"}))
            sys.exit(2)
        main_det(a)
        return
    if a.workload == "large":
        if a.gpus != 1:
            print(json.dumps({"error": "one GPU only"}))
            sys.exit(2)
        main_large(a)
        return
    if a.workload == "density":
        if a.gpus != 1:
            print(json.dumps({"error": "one GPU only"}))
            sys.exit(2)
        main_density(a)
        return
    if a.workload == "batch96":
        if a.gpus != 1:
            print(json.dumps({"error": "one GPU only"}))
            sys.exit(2)
        main_batch(a)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU "
                                   "sharding over walkers is described in the design notes, "
                                   "not built)"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    s = make_workload(a.walkers)
    bits = 53 if a.mode == "fp64" else a.mixed_bits
    variants_list = [v for v in a.variants.split(",") if v and v != a.mode]
    ms, timing, ref_out = run_gpu(s, a.mode, a.steps, a.warmup, bits,
                                  keep_outputs=bool(variants_list) and a.mode == "fp64")
    value = s.point_num / (ms * 1e-3)
    kr = kernel_roofline(s, a.mode, timing)
    roof = dominant_roofline(a.mode, kr)
    line = {
        "metric": METRIC, "value": value, "unit": "e-evals/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": MODE_DTYPE[a.mode], "data": "synthetic",
        "config": {"workload": f"ch80_800ao: 40 C + 40 H in a 20-bohr cube, {s.ao_num} AOs, "
                               f"{s.mo_num} MOs, {s.elec_num} electrons, {s.walk_num} walkers; "
                               "forward + adjoint", "points_per_step": s.point_num,
                   "bits": bits, "mode": a.mode,
                   "ao_values": "retained from the forward pass for dL/dC (memoised AO array of the "
                                "current points); AO derivatives up to third order recomputed for "
                                "dL/dR_elec and dL/dR_nucl"},
        "roofline": roof,
        "step_ms_spread": timing.get("_step_ms"),
        "ao_recompute_ms_per_step": timing.get("_recompute_ms"),
    }
    variants = {}
    for m in variants_list:
        vms, vt, vout = run_gpu(s, m, a.steps, a.warmup, a.mixed_bits, keep_outputs=ref_out is not None)
        peak_v = PEAKS[{"mixed_f32": "fp32_TFLOPs", "mixed_bf16x3": "bf16_TFLOPs", "fp64": "fp64_TFLOPs"}[m]]
        kv = kernel_roofline(s, m, vt)
        variants[m] = {"value": s.point_num / (vms * 1e-3), "unit": "e-evals/s", "ms_per_step": vms,
                       "step_ms_spread": vt.get("_step_ms"),
                       "ao_recompute_ms_per_step": vt.get("_recompute_ms"),
                       "speedup_vs_primary": ms / vms, "bits": a.mixed_bits,
                       "mo_gemm_frac_of_peak": (kv["mo"]["TFLOPs"] * (3 if m == "mixed_bf16x3" else 1) / peak_v)
                       if "mo" in kv else None,
                       "roofline": dominant_roofline(m, kv)}
        if vout is not None:
            variants[m]["error_vs_fp64_gpu"] = errors_vs(ref_out, vout)
            variants[m]["oracle_sample_error"] = oracle_sample(s, vout, a.mixed_bits)
        del vout
        torch.cuda.empty_cache()
    if variants:
        line["variants"] = variants
    if ref_out is not None:
        line["oracle_sample_error"] = oracle_sample(s, ref_out, bits)
    del ref_out
    torch.cuda.empty_cache()
    if not a.quick:
        line["workloads"] = {
            "batch96": batch_workload(a, ["fp64"] + variants_list),
            "ch300_7500ao": large_workload(a),
        }
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(a.cpu_walkers)
        line["cpu_baseline_1thread"] = cpu_baseline(a.cpu_walkers_1t, threads=1)
    print(json.dumps(line))


def oracle_sample(s, out, bits, n_points=16):
    """Errors of sampled rows against the oracle at the same B: row-normwise
    mo_vgl per component, and dLoss/dR_elec of those points relative to the
    sum of |terms| (the weights of those rows are regenerated from the
    benchmark's seed)."""
    import torch
    import oracle
    from tests.helpers import component_errors, grad_err
    P, N = s.point_num, s.mo_num
    idx = np.linspace(0, P - 1, n_points).astype(np.int64)
    it = torch.from_numpy(idx).to(out["mo"].device)
    rows = out["mo"].reshape(P, 5, N)[it].double().cpu().numpy()
    e = component_errors(rows, oracle.mo_vgl(s, points=s.points()[idx], B=bits))
    g = torch.Generator(device=out["mo"].device)
    g.manual_seed(1234)
    w = torch.randn((s.walk_num, s.elec_num, 5, N), generator=g, device=out["mo"].device, dtype=torch.float64)
    w_rows = w.reshape(P, 5, N)[it].cpu().numpy()
    del w
    r = oracle.adjoint(s, w_rows, points=s.points()[idx], B=bits)
    e["d_elec_rows"] = grad_err(out["d_elec"].reshape(P, 3)[it].cpu().numpy(), r["d_elec"], r["d_elec_abs"])
    e["points"] = int(n_points)
    return e


if __name__ == "__main__":
    main()
