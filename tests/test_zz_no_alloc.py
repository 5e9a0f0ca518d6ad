"""The entry point that allocates nothing (qmk_get_mo_vgl_noalloc) against
qmk_get_mo_vgl, through the C ABI: FP64 at 1e-12 row-normwise, the mixed
modes at their stated tolerances; two calls in a row on one context, the
second with fewer points, so the second call runs on the scratch array the
first one left; and its error paths (too large for the scratch, device
copies not yet built, cusp correction on)."""
import json

import numpy as np
import pytest

import synth
from tests.helpers import component_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed_f32": 2e-6, "mixed_bf16x3": 1e-4}


def qmk():
    import paper_2512_16677_amd as q
    return q


@pytest.mark.parametrize("mode", ["fp64", "mixed_f32", "mixed_bf16x3"])
@pytest.mark.parametrize("system", ["water_like", "medium"])
def test_noalloc_matches_get_mo_vgl_on_two_calls(mode, system):
    q = qmk()
    s = synth.water_like(walkers=96) if system == "water_like" else synth.medium(walkers=4)
    bits = 53 if mode == "fp64" else 24
    ctx = q.Context.from_system(s, bits=bits, mode=mode)
    sizes = (s.walk_num, s.walk_num // 3)          # the second call is smaller
    shift = (0.0, 0.21)
    for walk, dx in zip(sizes, shift):
        pts = np.ascontiguousarray(s.elec_coord[:walk] + dx)
        ctx.set_point(torch.from_numpy(pts).cuda())
        dt = torch.float64 if mode == "fp64" else torch.float32
        ref = ctx.get_mo_vgl(dtype=dt).clone()
        got = torch.full_like(ref, float("nan"))
        ctx.get_mo_vgl_noalloc(got)
        torch.cuda.synchronize()
        e = component_errors(got.double().cpu().numpy().reshape(-1, 5, s.mo_num),
                             ref.double().cpu().numpy().reshape(-1, 5, s.mo_num))
        print(json.dumps({"system": system, "mode": mode, "walkers": walk, "err": e}))
        for k, v in e.items():
            assert v <= TOL[mode], (walk, k, v)
    ctx.close()


def test_noalloc_error_paths():
    q = qmk()
    s = synth.medium(walkers=64)  # 896 x 5 x 17920 doubles: beyond the 64 MiB scratch
    ctx = q.Context.from_system(s)
    out = torch.empty((s.walk_num, s.elec_num, 5, s.mo_num), dtype=torch.float64, device="cuda")
    with pytest.raises(q.QmkError) as e:
        ctx.get_mo_vgl_noalloc(out)          # device copies not built yet
    assert e.value.status == q.QMK_NOT_SET
    ctx.get_mo_vgl(out=out)
    with pytest.raises(q.QmkError) as e:
        ctx.get_mo_vgl_noalloc(out)          # AO array larger than the scratch
    assert e.value.status == q.QMK_SIZE
    ctx.set_point(s.elec_coord[:2])
    small = out.reshape(-1)[: 2 * s.elec_num * 5 * s.mo_num].view(2, s.elec_num, 5, s.mo_num)
    with pytest.raises(q.QmkError) as e:
        ctx._check(ctx._lib.qmk_get_mo_vgl_noalloc(ctx._h, q._ptr(small), small.numel() - 1, q.QMK_F64,
                                                   q._stream(None)))
    assert e.value.status == q.QMK_SIZE
    ctx.get_mo_vgl_noalloc(small)
    ctx.set_mo_cusp(s.nucl_charge.astype(np.float64), np.full(s.nucl_num, 0.2))
    with pytest.raises(q.QmkError) as e:
        ctx.get_mo_vgl_noalloc(small)
    assert e.value.status == q.QMK_UNSUPPORTED
    ctx.close()
