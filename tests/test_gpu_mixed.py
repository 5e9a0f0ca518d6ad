"""Mixed-precision modes against the FP64 oracle.

No error figure for reduced precision is given by the paper, so these
tolerances are stated here from the arithmetic (parity unpinned by the
paper): row-normwise relative error per component of mo_vgl, and error of
the gradients relative to the absolute sums of their terms.  The oracle is
run at the same precision parameter B as the library (B = 24), so the
numbers isolate the arithmetic; the B = 53 comparison adds the effect of the
looser cutoff and is reported, not asserted.
"""
import json

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import component_errors, grad_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# stated per-output tolerances (row-normwise relative error of mo_vgl)
TOL = {
    "mixed_f32": {"value": 2e-6, "gradient": 2e-6, "laplacian": 2e-6, "grad": 1e-5},
    "mixed_bf16x3": {"value": 1e-4, "gradient": 1e-4, "laplacian": 1e-4, "grad": 1e-3},
}


def run(s, mode, w=None):
    import paper_2512_16677_amd as q
    ctx = q.Context.from_system(s, bits=24, mode=mode)
    mo = ctx.get_mo_vgl().cpu().numpy().reshape(-1, 5, s.mo_num)
    g = None
    if w is not None:
        g = {k: v.cpu().numpy() for k, v in ctx.adjoint(torch.from_numpy(w).cuda()).items()}
    ctx.close()
    return mo, g


@pytest.mark.parametrize("mode", list(TOL))
@pytest.mark.parametrize("system", ["water_like", "medium"])
def test_mixed_forward_error(mode, system):
    s = synth.water_like(walkers=32) if system == "water_like" else synth.medium(walkers=2)
    mo, _ = run(s, mode)
    e24 = component_errors(mo, oracle.mo_vgl(s, B=24))
    e53 = component_errors(mo, oracle.mo_vgl(s, B=53))
    print(json.dumps({"mode": mode, "system": system, "vs_B24": e24, "vs_B53": e53}))
    for k in ("value", "gradient", "laplacian"):
        assert e24[k] <= TOL[mode][k], (k, e24[k])


@pytest.mark.parametrize("mode", list(TOL))
def test_mixed_adjoint_error(mode):
    s = synth.medium(walkers=2)
    w = synth.adjoint_weights(s, seed=9)
    _, g = run(s, mode, w)
    r = oracle.adjoint(s, w, B=24)
    e = {k: grad_err(g[k].reshape(r[k].shape), r[k], r[k + "_abs"]) for k in ("d_coef", "d_elec", "d_nucl")}
    print(json.dumps({"mode": mode, "adjoint_vs_B24": e}))
    for k, v in e.items():
        assert v <= TOL[mode]["grad"], (k, v)


@pytest.mark.parametrize("mode", list(TOL))
def test_mixed_every_tile_shape(mode):
    """Every tile shape of the mode's own table (the BF16x3 table has shapes
    the FP64/FP32 one does not) gives the oracle's result at the stated
    tolerance, forward and adjoint."""
    import paper_2512_16677_amd as q
    s = synth.medium(walkers=1)
    w = synth.adjoint_weights(s, seed=5)
    ref_mo = oracle.mo_vgl(s, B=24)
    ref = oracle.adjoint(s, w, B=24)
    wt = torch.from_numpy(w).cuda()
    ctx = q.Context.from_system(s, bits=24, mode=mode)
    tried = 0
    for t in range(ctx.tile_count()):
        try:
            for k in ("mo", "gbar", "dcoef"):
                ctx.set_tile(k, t)
        except q.QmkError:
            continue  # does not fit in LDS
        tried += 1
        mo = ctx.get_mo_vgl().cpu().numpy().reshape(-1, 5, s.mo_num)
        e = component_errors(mo, ref_mo)
        for k in ("value", "gradient", "laplacian"):
            assert e[k] <= TOL[mode][k], (t, k, e[k])
        g = ctx.adjoint(wt)
        for k in ("d_coef", "d_elec", "d_nucl"):
            err = grad_err(g[k].cpu().numpy().reshape(ref[k].shape), ref[k], ref[k + "_abs"])
            assert err <= TOL[mode]["grad"], (t, k, err)
    assert tried == ctx.tile_count()
    ctx.close()


def test_forced_tile_of_another_precision_is_an_error():
    """A tile index forced in BF16x3 mode that the FP64 table does not have
    is reported as an argument error after a switch to FP64, not launched."""
    import paper_2512_16677_amd as q
    s = synth.water_like(walkers=2)
    ctx = q.Context.from_system(s, bits=24, mode="mixed_bf16x3")
    n_bf = ctx.tile_count()
    ctx.set_tile("mo", n_bf - 1)
    ctx.get_mo_vgl()
    ctx.set_precision(53, "fp64")
    assert ctx.tile_count() < n_bf
    with pytest.raises(q.QmkError) as e:
        ctx.get_mo_vgl()
    assert e.value.status == q.QMK_INVALID_ARG_BASE + 3
    with pytest.raises(q.QmkError):
        ctx.set_tile("mo", n_bf - 1)
    ctx.set_tile("mo", -1)
    ctx.get_mo_vgl()
    ctx.close()


def test_fp32_mode_rounds_fp64_weights_like_fp32_weights():
    """In the FP32 mode FP64 weights are rounded to FP32 once before the
    products, so they give exactly the gradients of their FP32-rounded
    copy."""
    import paper_2512_16677_amd as q
    s = synth.medium(walkers=2)
    w = synth.adjoint_weights(s, seed=3)
    ctx = q.Context.from_system(s, bits=24, mode="mixed_f32")
    g64 = {k: v.cpu().numpy() for k, v in ctx.adjoint(torch.from_numpy(w).cuda()).items()}
    g32 = {k: v.cpu().numpy() for k, v in ctx.adjoint(torch.from_numpy(w.astype(np.float32)).cuda()).items()}
    ctx.close()
    for k in ("d_coef", "d_elec", "d_nucl"):
        np.testing.assert_array_equal(g64[k], g32[k])


def test_fp32_mode_accepts_unaligned_fp64_weights():
    """W as a contiguous view that starts one element into its storage (8-byte
    but not 32-byte aligned) takes the conversion's element-wise path and
    gives the gradients of an aligned copy."""
    import paper_2512_16677_amd as q
    s = synth.water_like(walkers=3)
    w = synth.adjoint_weights(s, seed=6)
    base = torch.zeros(w.size + 1, dtype=torch.float64, device="cuda")
    base[1:] = torch.from_numpy(w.reshape(-1)).cuda()
    w_view = base[1:].view(w.shape)
    assert w_view.data_ptr() % 32 != 0
    ctx = q.Context.from_system(s, bits=24, mode="mixed_f32")
    g1 = {k: v.cpu().numpy() for k, v in ctx.adjoint(w_view).items()}
    g2 = {k: v.cpu().numpy() for k, v in ctx.adjoint(torch.from_numpy(w).cuda()).items()}
    ctx.close()
    for k in ("d_coef", "d_elec", "d_nucl"):
        np.testing.assert_array_equal(g1[k], g2[k])
