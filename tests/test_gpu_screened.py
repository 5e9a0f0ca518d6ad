"""Screened (block-sparse) forward contraction (Section 3.2, sparsity of the
AOs) through the C ABI.

Only exact zeros of the AO array are skipped, so the screened product must
equal the dense product bit for bit (compared with ==, which treats the two
zeros as equal), and therefore the oracle to the FP64 tolerance."""
import json

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import component_errors, grad_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def qmk():
    import paper_2512_16677_amd as q
    return q


def dense_and_screened(s, bits=53, mode="fp64", dtype=None, tile=None):
    q = qmk()
    ctx = q.Context.from_system(s, bits=bits, mode=mode)
    if tile is not None:
        ctx.set_tile("mo", tile)
    dense = ctx.get_mo_vgl(dtype=dtype)
    ctx.set_screening(True)
    scr = ctx.get_mo_vgl(dtype=dtype)
    frac = ctx.screening_density()
    ctx.close()
    return dense, scr, frac


@pytest.mark.parametrize("system", ["water_like", "medium", "large"])
def test_screened_equals_dense_and_oracle(system):
    s = {"water_like": lambda: synth.water_like(walkers=5),
         "medium": lambda: synth.medium(walkers=2),
         "large": lambda: synth.large(walkers=1)}[system]()
    dense, scr, frac = dense_and_screened(s)
    print(json.dumps({"system": system, "screening_density": frac}))
    assert 0.0 < frac <= 1.0
    assert bool((dense == scr).all())
    if system != "large":
        e = component_errors(scr.cpu().numpy().reshape(-1, 5, s.mo_num), oracle.mo_vgl(s))
        for k, v in e.items():
            assert v <= 1e-12, (k, v)


def test_screened_skips_work_on_the_large_system():
    """Sorted 64-point blocks of the 7500-AO system use far from every AO
    chunk (the screening density is well below 1) and the result still
    equals the dense product; sampled rows match the oracle."""
    s = synth.large(walkers=8)
    dense, scr, frac = dense_and_screened(s, bits=24, mode="mixed_f32")
    print(json.dumps({"large_B24_screening_density": frac}))
    assert frac < 0.6
    assert bool((dense == scr).all())
    idx = np.arange(0, s.point_num, 997)
    rows = scr.reshape(s.point_num, 5, s.mo_num)[torch.from_numpy(idx).cuda()].cpu().numpy()
    for k, v in component_errors(rows, oracle.mo_vgl(s, points=s.points()[idx], B=24)).items():
        assert v <= 2e-5, (k, v)


def test_screened_every_tile_shape():
    s = synth.medium(walkers=1)
    q = qmk()
    ctx = q.Context.from_system(s, bits=24)
    dense = ctx.get_mo_vgl()
    ctx.set_screening(True)
    for t in range(ctx.tile_count()):
        ctx.set_tile("mo", t)
        assert bool((ctx.get_mo_vgl() == dense).all()), t
    ctx.close()


@pytest.mark.parametrize("mode,dtype", [("mixed_f32", "f32"), ("mixed_f32", "f64"), ("fp64", "f32")])
def test_screened_mixed_and_output_types(mode, dtype):
    s = synth.medium(walkers=1)
    dt = torch.float32 if dtype == "f32" else torch.float64
    dense, scr, _ = dense_and_screened(s, bits=24, mode=mode, dtype=dt)
    assert scr.dtype == dt
    assert bool((dense == scr).all())


def test_screened_new_points_cusp_and_other_calls():
    """New points re-sort; the cusp correction applies on top; the AO array,
    MO values and the adjoint keep the dense path."""
    q = qmk()
    s = synth.water_like(walkers=6)
    z = s.nucl_charge.astype(np.float64)
    rc = np.array([0.25, 0.2, 0.2])
    ctx = q.Context.from_system(s)
    ctx.set_screening(True)
    ctx.set_mo_cusp(z, rc)
    for shift in (0.0, 0.37):
        pts = np.ascontiguousarray(s.elec_coord + shift)
        ctx.set_point(pts)
        got = ctx.get_mo_vgl().cpu().numpy().reshape(-1, 5, s.mo_num)
        ref = oracle.mo_vgl_cusp(s, z, rc, points=pts.reshape(-1, 3))
        for k, v in component_errors(got, ref).items():
            assert v <= 1e-12, (k, v)
    ctx.set_mo_cusp(None)
    w = torch.from_numpy(synth.adjoint_weights(s, seed=1)).cuda()
    g = ctx.adjoint(w)
    r = oracle.adjoint(s, w.cpu().numpy(), points=pts.reshape(-1, 3))
    assert grad_err(g["d_coef"].cpu().numpy(), r["d_coef"], r["d_coef_abs"]) <= 1e-11
    ao = ctx.get_ao_vgl().cpu().numpy().reshape(-1, 5, s.ao_num)
    for k, v in component_errors(ao, oracle.ao_vgl(s, points=pts.reshape(-1, 3))).items():
        assert v <= 1e-12, (k, v)
    ctx.close()


def adjoint_pair(s, mode="fp64", bits=53, wdtype=torch.float64):
    q = qmk()
    w = torch.from_numpy(synth.adjoint_weights(s, seed=4)).to(dtype=wdtype).cuda()
    ctx = q.Context.from_system(s, bits=bits, mode=mode)
    dense = {k: v.clone() for k, v in ctx.adjoint(w).items()}
    ctx.set_screening(True)
    scr = {k: v.clone() for k, v in ctx.adjoint(w).items()}
    scr2 = ctx.adjoint(w)
    ctx.close()
    return w, dense, scr, scr2


@pytest.mark.parametrize("system", ["water_like", "medium", "large"])
def test_screened_adjoint_matches_dense_and_oracle(system):
    """Electron gradients equal the dense ones bit for bit (each G-bar row is
    the same sum); dL/dC and the nuclear gradients sum over points in sorted
    order and agree to rounding; repeated calls are bitwise identical."""
    s = {"water_like": lambda: synth.water_like(walkers=5),
         "medium": lambda: synth.medium(walkers=2),
         "large": lambda: synth.large(walkers=1)}[system]()
    w, dense, scr, scr2 = adjoint_pair(s)
    assert bool((scr["d_elec"] == dense["d_elec"]).all())
    for k in ("d_coef", "d_nucl"):
        num = (scr[k] - dense[k]).abs().max().item()
        assert num <= 1e-12 * dense[k].abs().max().item(), (k, num)
    for k in scr:
        assert torch.equal(scr[k], scr2[k]), k
    if system != "large":
        r = oracle.adjoint(s, w.cpu().numpy())
        for k in ("d_coef", "d_elec", "d_nucl"):
            got = scr[k].cpu().numpy().reshape(r[k].shape)
            assert grad_err(got, r[k], r[k + "_abs"]) <= 1e-11, k


@pytest.mark.parametrize("wdtype", [torch.float64, torch.float32])
def test_screened_adjoint_mixed_fp32(wdtype):
    s = synth.large(walkers=2)
    _, dense, scr, _ = adjoint_pair(s, mode="mixed_f32", bits=24, wdtype=wdtype)
    assert bool((scr["d_elec"] == dense["d_elec"]).all())
    for k in ("d_coef", "d_nucl"):
        num = (scr[k] - dense[k]).abs().max().item()
        assert num <= 1e-6 * dense[k].abs().max().item(), (k, num)


def test_screened_adjoint_every_tile_shape():
    s = synth.medium(walkers=1)
    q = qmk()
    w = torch.from_numpy(synth.adjoint_weights(s, seed=6)).cuda()
    ctx = q.Context.from_system(s, bits=24)
    dense = {k: v.clone() for k, v in ctx.adjoint(w).items()}
    ctx.set_screening(True)
    for t in range(ctx.tile_count()):
        ctx.set_tile("gbar", t)
        ctx.set_tile("dcoef", t)
        g = ctx.adjoint(w)
        assert bool((g["d_elec"] == dense["d_elec"]).all()), t
        for k in ("d_coef", "d_nucl"):
            assert (g[k] - dense[k]).abs().max().item() <= 1e-12 * dense[k].abs().max().item(), (t, k)
    ctx.close()


@pytest.mark.parametrize("mode,screened", [("fp64", False), ("fp64", True), ("mixed_bf16x3", False)])
def test_mo_subset_matches_oracle(mode, screened):
    """A subset of the MOs (Section 3.2: unoccupied MOs are left out of the
    product) is computed by setting only those rows of C: mo_vgl and the
    gradients equal the oracle's with the same rows, for a subset that is not
    a multiple of any tile width (37 of 400 MOs, every other one among the
    first 74)."""
    q = qmk()
    s = synth.medium(walkers=1)
    rows = np.arange(0, 74, 2)
    C_sub = np.ascontiguousarray(s.mo_coef[rows])
    bits = 53 if mode == "fp64" else 24
    ctx = q.Context.from_system(s, bits=bits, mode=mode)
    ctx.set_mo_coef(C_sub)
    if screened:
        ctx.set_screening(True)
    assert ctx.dims()["mo_num"] == len(rows)
    mo = ctx.get_mo_vgl().cpu().numpy().reshape(-1, 5, len(rows))
    rng = np.random.default_rng(12)
    w = rng.standard_normal((s.walk_num, s.elec_num, 5, len(rows)))
    g = {k: v.cpu().numpy() for k, v in ctx.adjoint(torch.from_numpy(w).cuda()).items()}
    ctx.close()
    ref = oracle.mo_vgl(s, coef=C_sub, B=bits)
    r = oracle.adjoint(s, w, coef=C_sub, B=bits)
    tol = 1e-12 if mode == "fp64" else 1e-4
    gtol = 1e-11 if mode == "fp64" else 1e-3
    for k, v in component_errors(mo, ref).items():
        assert v <= tol, (k, v)
    for k in ("d_coef", "d_elec", "d_nucl"):
        assert grad_err(g[k].reshape(r[k].shape), r[k], r[k + "_abs"]) <= gtol, k


@pytest.mark.parametrize("system", ["medium", "large"])
def test_screened_bf16x3_equals_dense_and_oracle(system):
    """The BF16x3 screened products: forward rows and electron gradients
    equal the dense BF16x3 ones bit for bit (the same non-zero terms in the
    same order), dL/dC and the nuclear gradients agree to FP32 rounding, and
    both match the oracle at the BF16x3 tolerance."""
    s = synth.medium(walkers=2) if system == "medium" else synth.large(walkers=1)
    dense, scr, frac = dense_and_screened(s, bits=24, mode="mixed_bf16x3", dtype=torch.float32)
    print(json.dumps({"system": system, "bf16x3_screening_density": frac}))
    assert bool((dense == scr).all())
    w, gd, gs, gs2 = adjoint_pair(s, mode="mixed_bf16x3", bits=24)
    assert bool((gs["d_elec"] == gd["d_elec"]).all())
    for k in ("d_coef", "d_nucl"):
        num = (gs[k] - gd[k]).abs().max().item()
        assert num <= 1e-6 * gd[k].abs().max().item(), (k, num)
    for k in gs:
        assert torch.equal(gs[k], gs2[k]), k
    ref_mo = oracle.mo_vgl(s, B=24) if system == "medium" else None
    if ref_mo is not None:
        for k, v in component_errors(scr.double().cpu().numpy().reshape(-1, 5, s.mo_num), ref_mo).items():
            assert v <= 1e-4, (k, v)
    r = oracle.adjoint_products(s, w.cpu().numpy(), B=24)
    for k in ("d_coef", "d_elec", "d_nucl"):
        assert grad_err(gs[k].cpu().numpy().reshape(r[k].shape), r[k], r[k + "_abs"]) <= 1e-3, k


def test_screened_bf16x3_every_tile_shape():
    s = synth.medium(walkers=1)
    q = qmk()
    w = torch.from_numpy(synth.adjoint_weights(s, seed=6)).cuda()
    ctx = q.Context.from_system(s, bits=24, mode="mixed_bf16x3")
    dense = ctx.get_mo_vgl(dtype=torch.float32).clone()
    gdense = {k: v.clone() for k, v in ctx.adjoint(w).items()}
    ctx.set_screening(True)
    for t in range(ctx.tile_count()):
        for k in ("mo", "gbar", "dcoef"):
            ctx.set_tile(k, t)
        assert bool((ctx.get_mo_vgl(dtype=torch.float32) == dense).all()), t
        g = ctx.adjoint(w)
        assert bool((g["d_elec"] == gdense["d_elec"]).all()), t
        for k in ("d_coef", "d_nucl"):
            assert (g[k] - gdense[k]).abs().max().item() <= 1e-6 * gdense[k].abs().max().item(), (t, k)
    ctx.close()


@pytest.mark.parametrize("mode", ["fp64", "mixed_f32", "mixed_bf16x3"])
def test_screened_reevaluation_after_points_move(mode):
    """The screened AO array is not rewritten where a (64-point block, 16-AO
    chunk) is inactive: the store pass writes zeros only where the previous
    evaluation had the chunk active.  Consecutive screened evaluations at
    points that sort into different blocks (electrons moved by several bohr,
    then moved back) each equal the dense product bit for bit, and the
    adjoint agrees with the dense one."""
    q = qmk()
    s = synth.medium(walkers=3)
    bits = 53 if mode == "fp64" else 24
    rng = np.random.default_rng(11)
    sets = [s.elec_coord, s.elec_coord + rng.normal(scale=3.0, size=s.elec_coord.shape), s.elec_coord]
    dense = q.Context.from_system(s, bits=bits, mode=mode)
    scr = q.Context.from_system(s, bits=bits, mode=mode)
    scr.set_screening(True)
    w = torch.from_numpy(synth.adjoint_weights(s, seed=4)).cuda()
    if mode != "fp64":
        w = w.float()
    tol = 1e-12 if mode == "fp64" else 1e-5
    for pts in sets:
        pts = np.ascontiguousarray(pts)
        for c in (dense, scr):
            c.set_point(pts)
        a = dense.get_mo_vgl()
        b = scr.get_mo_vgl()
        assert bool((a == b).all())
        ga = {k: v.clone() for k, v in dense.adjoint(w).items()}
        gb = scr.adjoint(w)
        for k in ("d_coef", "d_elec", "d_nucl"):
            assert (ga[k] - gb[k]).abs().max().item() <= tol * ga[k].abs().max().item(), k
    dense.close()
    scr.close()
