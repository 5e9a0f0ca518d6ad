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
    outs = None
    if keep_outputs:  # one more (untimed) step on the first coordinate set
        ctx.set_point(r0)
        ctx.get_mo_vgl(out=mo)
        ctx.adjoint(w, out=grads)
        torch.cuda.synchronize()
        outs = {"mo": mo, **grads}
    ctx.close()
    return ms, timing, outs


def errors_vs(ref, got):
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
    e["laplacian_p999"] = float(torch.quantile(r[:, 4].float(), 0.999))
    for k in ("d_coef", "d_elec", "d_nucl"):
        e[k] = float((got[k] - ref[k]).abs().max() / ref[k].abs().max().clamp_min(1e-300))
    return e


KERNEL_SOURCES = {  # files whose change invalidates a kernel class's counter figures
    "mo": ["gemm_impl.h", "gemm_kernels.hip", "gemm_bf16.hip", "qmk_internal.h", "context.cpp",
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
    return out


def dominant_roofline(mode, kr):
    """Roofline entry for the kernel class with the largest share of step time."""
    peak_key = {"fp64": "fp64_TFLOPs", "mixed_f32": "fp32_TFLOPs", "mixed_bf16x3": "bf16_TFLOPs"}[mode]
    cands = {k: v for k, v in kr.items() if k != "reduce"}
    name = max(cands, key=lambda k: cands[k]["avg_ms"] * cands[k]["launches"])
    d = cands[name]
    traffic = measured_traffic(mode, name)
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


def cpu_baseline(walkers: int):
    """The FP64 oracle, forward + adjoint, on a bounded sample of the workload."""
    import oracle
    import synth
    s = synth.medium(walkers=walkers)
    w = synth.adjoint_weights(s, seed=1)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    oracle.mo_vgl(s)
    oracle.adjoint(s, w, with_abs=False)
    dt = time.perf_counter() - t0
    return {"value": s.point_num / dt, "unit": "e-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{walkers} walkers x {s.elec_num} electrons of the same 800-AO/400-MO "
                      f"system (forward + adjoint), {dt:.1f} s", "cpu_model": cpu_model()}


def cpu_model() -> str:
    """Model name of the host CPU (Linux), or an empty string."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def run_batch(mols, mode, steps, warmup, bits, batched=True):
    """Forward + adjoint of every molecule per step, as one batch (one graph
    launch) or as a loop of single-context calls."""
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
    ws = [torch.randn((m.walk_num, m.elec_num, 5, m.mo_num), generator=g, device=dev, dtype=dt) for m in mols]
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
    if b:
        b.close()
    for c in ctxs:
        c.close()
    return ms


def main_batch(a):
    import synth
    mols = synth.molecule_batch(96, seed=0)
    pts = sum(m.point_num for m in mols)
    res = {}
    for mode in ["fp64"] + [v for v in a.variants.split(",") if v]:
        bits = 53 if mode == "fp64" else a.mixed_bits
        ms_b = run_batch(mols, mode, a.steps, a.warmup, bits, batched=True)
        ms_l = run_batch(mols, mode, max(2, a.steps // 2), 1, bits, batched=False)
        res[mode] = {"value": pts / (ms_b * 1e-3), "ms_per_step": ms_b,
                     "unbatched_ms_per_step": ms_l, "batching_speedup": ms_l / ms_b}
    line = {"metric": METRIC, "value": res["fp64"]["value"], "unit": "e-evals/s", "n_gpus": 1,
            "steps": a.steps, "warmup": a.warmup, "ms_per_step": res["fp64"]["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "batch96: 96 C/H molecules, 4-60 atoms, 8-128 walkers each, "
                                   "one persistent-kernel HIP graph per step; forward + adjoint",
                       "points_per_step": pts, "molecules": len(mols),
                       "ao_range": [min(m.ao_num for m in mols), max(m.ao_num for m in mols)]},
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


def main_large(a):
    """The 7500-AO / 1050-MO system at 64 walkers: forward (dense and screened
    contraction) and forward + adjoint, per precision mode."""
    import torch
    import synth
    import paper_2512_16677_amd as qmk
    s = synth.large(walkers=64)
    P, K, N = s.point_num, s.ao_num, s.mo_num
    dev = torch.device("cuda:0")
    r0 = torch.from_numpy(np.ascontiguousarray(s.elec_coord)).to(dev)
    r1 = (r0 + 1e-3).contiguous()
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    res = {}
    for mode, bits in (("fp64", 53), ("mixed_f32", 24), ("mixed_bf16x3", 24)):
        ctx = qmk.Context.from_system(s, bits=bits, mode=mode)
        dt = torch.float64 if mode == "fp64" else torch.float32
        mo = torch.empty((s.walk_num, s.elec_num, 5, N), dtype=dt, device=dev)
        out = {}
        for screened in (False, True):
            if screened and mode == "mixed_bf16x3":
                continue
            ctx.set_screening(screened)
            for i in range(a.warmup):
                ctx.set_point(r0 if i % 2 == 0 else r1)
                ctx.get_mo_vgl(out=mo)
            torch.cuda.synchronize()
            ctx.set_timing(True)
            t0 = time.perf_counter()
            for i in range(a.steps):
                ctx.set_point(r0 if i % 2 == 0 else r1)
                ctx.get_mo_vgl(out=mo)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / a.steps
            t = ctx.timing()
            key = "screened" if screened else "dense"
            out[key] = {"forward_ms": ms, "e_evals_per_s": P / (ms * 1e-3),
                        "mo_ms": t["mo"]["ms"] / max(1, t["mo"]["launches"]),
                        "ao_ms": t["ao"]["ms"] / max(1, t["ao"]["launches"])}
            if screened:
                out[key]["sort_ms"] = t["sort"]["ms"] / max(1, t["sort"]["launches"])
                out[key]["screening_density"] = ctx.screening_density()
            # forward + adjoint of sum(W * mo_vgl)
            w = torch.randn((s.walk_num, s.elec_num, 5, N), generator=g, device=dev, dtype=dt)
            for i in range(a.warmup):
                ctx.set_point(r0 if i % 2 == 0 else r1)
                ctx.get_mo_vgl(out=mo)
                ctx.adjoint(w)
            torch.cuda.synchronize()
            ctx.set_timing(True)
            t0 = time.perf_counter()
            for i in range(a.steps):
                ctx.set_point(r0 if i % 2 == 0 else r1)
                ctx.get_mo_vgl(out=mo)
                ctx.adjoint(w)
            torch.cuda.synchronize()
            ms2 = (time.perf_counter() - t0) * 1e3 / a.steps
            t = ctx.timing()
            out[key]["fwd_adjoint_ms"] = ms2
            out[key]["fwd_adjoint_e_evals_per_s"] = P / (ms2 * 1e-3)
            out[key]["per_kernel_ms"] = {k: v["ms"] / v["launches"] for k, v in t.items() if v["launches"]}
            del w
            torch.cuda.empty_cache()
        if "screened" in out:
            out["forward_speedup"] = out["dense"]["forward_ms"] / out["screened"]["forward_ms"]
            out["fwd_adjoint_speedup"] = out["dense"]["fwd_adjoint_ms"] / out["screened"]["fwd_adjoint_ms"]
        out["mo_dense_TFLOPs"] = 2.0 * 5 * P * K * N / (out["dense"]["mo_ms"] * 1e-3) / 1e12
        ctx.close()
        del mo
        torch.cuda.empty_cache()
        res[mode] = out
    line = {"metric": "mo_vgl electron-evals/s (fwd+adjoint), dense vs screened contraction",
            "value": res["fp64"]["screened"]["fwd_adjoint_e_evals_per_s"], "unit": "e-evals/s", "n_gpus": 1,
            "steps": a.steps, "warmup": a.warmup, "ms_per_step": res["fp64"]["screened"]["fwd_adjoint_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"ch300_7500ao: 150 C + 150 H in a 35-bohr cube, {K} AOs, {N} MOs, "
                                   f"{s.elec_num} electrons, 64 walkers; forward + adjoint",
                       "points_per_step": P},
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


def main():
    a = parse()
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
                   "bits": bits, "mode": a.mode},
        "roofline": roof,
        "step_ms_spread": timing.get("_step_ms"),
    }
    variants = {}
    for m in variants_list:
        vms, vt, vout = run_gpu(s, m, a.steps, a.warmup, a.mixed_bits, keep_outputs=ref_out is not None)
        peak_v = PEAKS[{"mixed_f32": "fp32_TFLOPs", "mixed_bf16x3": "bf16_TFLOPs", "fp64": "fp64_TFLOPs"}[m]]
        kv = kernel_roofline(s, m, vt)
        variants[m] = {"value": s.point_num / (vms * 1e-3), "unit": "e-evals/s", "ms_per_step": vms,
                       "step_ms_spread": vt.get("_step_ms"),
                       "speedup_vs_primary": ms / vms, "bits": a.mixed_bits,
                       "mo_gemm_frac_of_peak": (kv["mo"]["TFLOPs"] * (3 if m == "mixed_bf16x3" else 1) / peak_v)
                       if "mo" in kv else None,
                       "roofline": dominant_roofline(m, kv)}
        if vout is not None:
            variants[m]["error_vs_fp64_gpu"] = errors_vs(ref_out, vout)
        del vout
        torch.cuda.empty_cache()
    if variants:
        line["variants"] = variants
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(a.cpu_walkers)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
