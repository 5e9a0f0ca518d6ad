"""Every tile shape of the FP64 and FP32 products on shapes that take each
branch of their direct global-to-LDS K loop: whole K steps, a partial last
K step staged through registers, reads into the padded rows of internal
operands (odd point and MO counts), and weights whose rows cannot be loaded
in 16-byte pieces (odd MO counts in FP64, FP32 weights with an MO count that
is not a multiple of four), which the adjoint copies into padded rows first.
Forward and adjoint against the oracle: FP64 at 1e-12 (rows) / 1e-11
(gradients), FP32 at its stated tolerances with the oracle at the same B.
(The register-staged loop that operands without unit stride or padding
take is exercised by the batch tests: a batch reads each molecule's weights
in place.)

Shapes (P points, K AOs, N MOs; the forward product is P x N over K, G-bar
K x P over N, dC N x K over P):
  3 C + 5 H, 3 walkers:  P = 69, K = 70, N = 35  (odd P and N, partial steps)
  5 C + 9 H, 4 walkers:  P = 156, K = 120, N = 60 (all extents multiples of
                         four; every K extent ends in a partial step)
"""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import component_errors, grad_err, rownorm_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = [(3, 5, 3), (5, 9, 4)]
F32_TOL = {"value": 2e-6, "gradient": 2e-6, "laplacian": 2e-6, "grad": 1e-5}


@pytest.mark.parametrize("mode", ["fp64", "mixed_f32", "mixed_f32_wf32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_every_tile_on_ragged_shapes(mode, shape):
    import paper_2512_16677_amd as q
    n_c, n_h, walkers = shape
    s = synth.ch_cluster(n_c, n_h, 10.0, walkers, seed=7)
    assert (s.walk_num * s.elec_num, s.ao_num, s.mo_num) in ((69, 70, 35), (156, 120, 60))
    bits = 53 if mode == "fp64" else 24
    w = synth.adjoint_weights(s, seed=8)
    if mode == "mixed_f32_wf32":
        # FP32 weights from the caller; the oracle takes the same rounded values
        w = w.astype(np.float32)
        mode = "mixed_f32"
    ref_mo = oracle.mo_vgl(s, B=bits)
    ref = oracle.adjoint(s, w.astype(np.float64), B=bits)
    wt = torch.from_numpy(w).cuda()
    ctx = q.Context.from_system(s, bits=bits, mode=mode)
    tried = 0
    for t in range(ctx.tile_count()):
        try:
            for k in ("mo", "gbar", "dcoef"):
                ctx.set_tile(k, t)
        except q.QmkError:
            continue  # does not fit in LDS
        tried += 1
        mo = ctx.get_mo_vgl().cpu().numpy().reshape(-1, 5, s.mo_num)
        g = ctx.adjoint(wt)
        if mode == "fp64":
            assert rownorm_err(mo, ref_mo).max() <= 1e-12, t
            gtol = 1e-11
        else:
            e = component_errors(mo, ref_mo)
            for k in ("value", "gradient", "laplacian"):
                assert e[k] <= F32_TOL[k], (t, k, e[k])
            gtol = F32_TOL["grad"]
        for k in ("d_coef", "d_elec", "d_nucl"):
            err = grad_err(g[k].cpu().numpy().reshape(ref[k].shape), ref[k], ref[k + "_abs"])
            assert err <= gtol, (t, k, err)
    assert tried == ctx.tile_count()
    ctx.close()
