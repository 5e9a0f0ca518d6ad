"""MO cusp correction (Section 3.3) through the C ABI vs the FP64 oracle.

Points are the walkers' electrons plus points placed inside and around every
cusp sphere (radii 0.2-0.3 bohr), so that many rows are corrected.  FP64:
row-normwise error <= 1e-12.  Mixed FP32: the stated forward tolerance of the
FP32 contraction, 2e-6, against the oracle at the same B."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import component_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def qmk():
    import paper_2512_16677_amd as q
    return q


def cusp_points(s, rc, per_nucleus=24, seed=0):
    rng = np.random.default_rng(seed)
    pts = [s.points()]
    for A in range(s.nucl_num):
        e = rng.normal(size=(per_nucleus, 3))
        e /= np.linalg.norm(e, axis=1, keepdims=True)
        r = rc[A] * rng.uniform(0.001, 1.3, size=(per_nucleus, 1))
        pts.append(s.nucl_coord[A] + r * e)
    return np.ascontiguousarray(np.concatenate(pts))


def charges_and_radii(s, r=0.25):
    z = s.nucl_charge.astype(np.float64)
    rc = np.where(z > 1, r, 0.8 * r)
    return z, rc


@pytest.mark.parametrize("system", ["water_like", "medium"])
def test_cusp_matches_oracle_fp64(system):
    q = qmk()
    s = synth.water_like(walkers=4) if system == "water_like" else synth.medium(walkers=1)
    z, rc = charges_and_radii(s)
    pts = cusp_points(s, rc)
    ctx = q.Context.from_system(s)
    ctx.set_mo_cusp(z, rc)
    ctx.set_point(pts.reshape(1, -1, 3))
    got = ctx.get_mo_vgl().cpu().numpy().reshape(-1, 5, s.mo_num)
    ref = oracle.mo_vgl_cusp(s, z, rc, points=pts)
    e = component_errors(got, ref)
    # the correction really acts: the corrected rows differ from the plain MOs
    plain = oracle.mo_vgl(s, points=pts)
    assert np.abs(ref - plain).max() > 1e-3 * np.abs(plain).max()
    for k, v in e.items():
        assert v <= 1e-12, (k, v)
    # switched off: the plain MOs again
    ctx.set_mo_cusp(None)
    got0 = ctx.get_mo_vgl().cpu().numpy().reshape(-1, 5, s.mo_num)
    for k, v in component_errors(got0, plain).items():
        assert v <= 1e-12, (k, v)
    ctx.close()


@pytest.mark.parametrize("mode", ["mixed_f32", "mixed_bf16x3"])
def test_cusp_mixed_modes(mode):
    q = qmk()
    s = synth.water_like(walkers=4)
    z, rc = charges_and_radii(s)
    pts = cusp_points(s, rc, seed=1)
    ctx = q.Context.from_system(s, bits=24, mode=mode)
    ctx.set_mo_cusp(z, rc)
    ctx.set_point(pts.reshape(1, -1, 3))
    got = ctx.get_mo_vgl(dtype=torch.float32).cpu().numpy().reshape(-1, 5, s.mo_num)
    ctx.close()
    tol = 2e-6 if mode == "mixed_f32" else 1e-4
    for k, v in component_errors(got, oracle.mo_vgl_cusp(s, z, rc, points=pts, B=24)).items():
        assert v <= tol, (k, v)


def test_cusp_tables_follow_coefficients_and_nuclei():
    q = qmk()
    s = synth.water_like(walkers=2)
    z, rc = charges_and_radii(s, 0.2)
    pts = cusp_points(s, rc, seed=2)
    ctx = q.Context.from_system(s)
    ctx.set_mo_cusp(z, rc)
    ctx.set_point(pts.reshape(1, -1, 3))
    ctx.get_mo_vgl()
    C2 = np.ascontiguousarray(s.mo_coef[:, ::-1])
    ctx.set_mo_coef(C2)
    got = ctx.get_mo_vgl().cpu().numpy().reshape(-1, 5, s.mo_num)
    for k, v in component_errors(got, oracle.mo_vgl_cusp(s, z, rc, points=pts, coef=C2)).items():
        assert v <= 1e-12, (k, v)
    ctx.close()


def test_cusp_errors():
    q = qmk()
    s = synth.water_like(walkers=2)
    z, _ = charges_and_radii(s)
    ctx = q.Context.from_system(s)
    with pytest.raises(q.QmkError) as e:
        ctx.set_mo_cusp(z, -np.ones(s.nucl_num))
    assert e.value.status == q.QMK_INVALID_ARG_BASE + 4
    ctx.set_mo_cusp(z, np.full(s.nucl_num, 1.5))  # spheres overlap (O-H distance 1.8 bohr)
    with pytest.raises(q.QmkError) as e:
        ctx.get_mo_vgl()
    assert e.value.status == q.QMK_INVALID_ARG_BASE + 4
    ctx.set_mo_cusp(z, np.full(s.nucl_num, 0.2))
    ctx.get_mo_vgl()
    w = torch.zeros((s.walk_num, s.elec_num, 5, s.mo_num), dtype=torch.float64, device="cuda")
    for call in (lambda: ctx.adjoint(w), lambda: ctx.get_density(np.ones(s.mo_num)),
                 lambda: ctx.get_mo_value()):
        with pytest.raises(q.QmkError) as e:
            call()
        assert e.value.status == q.QMK_UNSUPPORTED
    ctx.close()
