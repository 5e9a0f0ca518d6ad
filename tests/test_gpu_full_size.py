"""Parity at the full workload sizes, in the launch configuration the
benchmark times.

The oracle cannot evaluate a whole full-size step in test time, so these
tests compare outputs it can compute one by one (mo_vgl rows and electron
gradients at sampled points), and check properties that hold at any size:
  * linearity of mo_vgl in C: sum(W * mo_vgl) = <C, dLoss/dC>;
  * translation invariance: the nuclear and electron gradients sum to zero;
  * central differences (h = 1e-5) of the GPU's own loss on random entries.

Systems: the 80-atom, 800-AO / 400-MO system with 280 electrons at 512
walkers (forward + adjoint) and at 256 walkers (differentiation check), and
the 300-atom, 7500-AO / 1050-MO system with 1050 electrons at 64 walkers in
FP64 and both mixed modes.
"""
import json

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import component_errors, grad_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
N_SAMPLE = 48


def qmk():
    import paper_2512_16677_amd as q
    return q


def sample_points(P, seed, n=N_SAMPLE):
    rng = np.random.default_rng(seed)
    idx = rng.choice(P, size=n - 2, replace=False)
    return np.unique(np.concatenate([[0, P - 1], idx]))


def test_medium_full_size_forward_adjoint():
    """512 walkers x 280 electrons (143,360 points), FP64: sampled rows of
    mo_vgl and of dLoss/dR_elec vs the oracle; dLoss/dC through linearity;
    dLoss/dR_nuc through the translation sum rule."""
    q = qmk()
    s = synth.medium(walkers=512)
    P = s.point_num
    ctx = q.Context.from_system(s, bits=53, mode="fp64")
    mo = ctx.get_mo_vgl()  # [walk, elec, 5, mo]
    g = torch.Generator(device="cuda")
    g.manual_seed(1234)
    w = torch.randn(mo.shape, generator=g, device="cuda", dtype=torch.float64)
    grads = ctx.adjoint(w)

    idx = sample_points(P, seed=11)
    pts = s.points()[idx]
    mo_rows = mo.reshape(P, 5, s.mo_num)[torch.from_numpy(idx).cuda()].cpu().numpy()
    e = component_errors(mo_rows, oracle.mo_vgl(s, points=pts))
    w_rows = w.reshape(P, 5, s.mo_num)[torch.from_numpy(idx).cuda()].cpu().numpy()
    r = oracle.adjoint(s, w_rows, points=pts)
    de = grad_err(grads["d_elec"].reshape(P, 3)[torch.from_numpy(idx).cuda()].cpu().numpy(),
                  r["d_elec"], r["d_elec_abs"])

    loss = torch.sum(w * mo).item()
    loss_abs = torch.sum((w * mo).abs()).item()
    C = torch.from_numpy(s.mo_coef).cuda()
    lin = abs(loss - torch.sum(C * grads["d_coef"]).item()) / loss_abs

    tot = grads["d_nucl"].sum(0) + grads["d_elec"].reshape(-1, 3).sum(0)
    scale = grads["d_nucl"].abs().sum(0) + grads["d_elec"].reshape(-1, 3).abs().sum(0)
    rule = float((tot.abs() / scale).max())
    print(json.dumps({"mo_rows": e, "d_elec_rows": de, "linearity": lin, "sum_rule": rule}))
    ctx.close()
    for k, v in e.items():
        assert v <= TOL64, (k, v)
    assert de <= 1e-11
    assert lin <= 1e-12
    assert rule <= 1e-11


def test_medium_256_walkers_central_differences():
    """dLoss/dC, dLoss/dR_elec, dLoss/dR_nuc vs central differences of the
    GPU forward (h = 1e-5) on 32 random entries.  The difference quotient is
    summed as sum(W * (mo(+h) - mo(-h))) / 2h, so that the rows a
    perturbation leaves unchanged cancel exactly."""
    q = qmk()
    s = synth.medium(walkers=256)
    ctx = q.Context.from_system(s, bits=53, mode="fp64")
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    shape = (s.walk_num, s.elec_num, 5, s.mo_num)
    w = torch.randn(shape, generator=g, device="cuda", dtype=torch.float64)
    ctx.get_mo_vgl()
    grads = {k: v.cpu().numpy() for k, v in ctx.adjoint(w).items()}

    def mo_at(nucl=None, coef=None, elec=None):
        ctx.set_nucleus(s.nucl_coord if nucl is None else nucl)
        ctx.set_mo_coef(s.mo_coef if coef is None else coef)
        ctx.set_point(s.elec_coord if elec is None else elec)
        return ctx.get_mo_vgl().clone()

    h = 1e-5

    def fd(**kw_pm):
        (name, (base, e)), = kw_pm.items()
        plus = mo_at(**{name: base + e})
        minus = mo_at(**{name: base - e})
        return float(torch.sum(w * (plus - minus)).item()) / (2 * h)

    rng = np.random.default_rng(5)
    worst = {}
    for _ in range(11):
        n, k = int(rng.integers(s.mo_num)), int(rng.integers(s.ao_num))
        e = np.zeros_like(s.mo_coef)
        e[n, k] = h
        d = abs(fd(coef=(s.mo_coef, e)) - grads["d_coef"][n, k]) / np.abs(grads["d_coef"]).max()
        worst["d_coef"] = max(worst.get("d_coef", 0.0), d)
    for _ in range(11):
        wk, el, i = (int(rng.integers(s.walk_num)), int(rng.integers(s.elec_num)),
                     int(rng.integers(3)))
        e = np.zeros_like(s.elec_coord)
        e[wk, el, i] = h
        d = abs(fd(elec=(s.elec_coord, e)) - grads["d_elec"][wk, el, i]) / np.abs(grads["d_elec"]).max()
        worst["d_elec"] = max(worst.get("d_elec", 0.0), d)
    for _ in range(10):
        A, i = int(rng.integers(s.nucl_num)), int(rng.integers(3))
        e = np.zeros_like(s.nucl_coord)
        e[A, i] = h
        d = abs(fd(nucl=(s.nucl_coord, e)) - grads["d_nucl"][A, i]) / np.abs(grads["d_nucl"]).max()
        worst["d_nucl"] = max(worst.get("d_nucl", 0.0), d)
    print(json.dumps({"fd_normwise": worst}))
    ctx.close()
    # truncation h^2 f'''/6 and rounding eps |mo| / h both stay below 1e-7
    # of the largest entry for exponents up to 1e4 at these electron distances
    for k, v in worst.items():
        assert v <= 1e-6, (k, v)


MIXED_TOL_LARGE = {  # row-normwise, vs the oracle at the same B = 24
    "mixed_f32": {"value": 2e-5, "gradient": 2e-5, "laplacian": 2e-5},
    "mixed_bf16x3": {"value": 2e-4, "gradient": 2e-4, "laplacian": 2e-4},
}


@pytest.mark.parametrize("mode", ["fp64", "mixed_f32", "mixed_bf16x3"])
def test_large_sampled_rows(mode):
    """7500 AOs, 1050 MOs, 64 walkers x 1050 electrons (67,200 points):
    sampled rows of mo_vgl against the oracle.  The mixed tolerances grow
    with the contraction length K = 7500 (FP32 rounding of the AO operand and
    of the accumulation, about sqrt(K) u relative to the row norm)."""
    q = qmk()
    s = synth.large(walkers=64)
    bits = 53 if mode == "fp64" else 24
    ctx = q.Context.from_system(s, bits=bits, mode=mode)
    P = s.point_num
    mo = ctx.get_mo_vgl(dtype=torch.float64 if mode == "fp64" else torch.float32)
    idx = sample_points(P, seed=3, n=24)
    rows = mo.reshape(P, 5, s.mo_num)[torch.from_numpy(idx).cuda()].double().cpu().numpy()
    ctx.close()
    del mo
    torch.cuda.empty_cache()
    e = component_errors(rows, oracle.mo_vgl(s, points=s.points()[idx], B=bits))
    print(json.dumps({"mode": mode, "large_rows": e}))
    for k, v in e.items():
        assert v <= (TOL64 if mode == "fp64" else MIXED_TOL_LARGE[mode][k]), (k, v)
