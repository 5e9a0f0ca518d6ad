"""Three-body Jastrow factor through the C ABI vs the FP64 oracle.

Tolerance: every term of J is a product of rescaled distances in (0, 1] and a
coefficient, so the rounding error of any summation order is bounded relative
to J_abs, the same sum with |c| (the oracle with the coefficients' absolute
values); the P product and the contraction run in FP64: 1e-12 J_abs.
"""
import json

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def qmk():
    import paper_2512_16677_amd as q
    return q


def coefficients(nord, nn, seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(scale=0.2, size=(len(oracle.een_terms(nord)), nn))


def reference(s, kappa, nord, c):
    ref = oracle.jastrow_een(s.elec_coord, s.nucl_coord, kappa, nord, c)
    ref_abs = oracle.jastrow_een(s.elec_coord, s.nucl_coord, kappa, nord, np.abs(c))
    return ref, ref_abs


def test_term_count_matches_oracle():
    q = qmk()
    for nord in range(2, 9):
        assert q.jastrow_een_terms(nord) == len(oracle.een_terms(nord))


@pytest.mark.parametrize("system,nord", [("water_like", 2), ("water_like", 3), ("water_like", 4),
                                         ("water_like", 5), ("water_like", 6), ("water_like", 7),
                                         ("water_like", 8), ("medium", 5)])
def test_jastrow_een_matches_oracle(system, nord):
    q = qmk()
    s = synth.water_like(walkers=7) if system == "water_like" else synth.medium(walkers=2)
    kappa = 0.6
    c = coefficients(nord, s.nucl_num, seed=nord)
    ctx = q.Context.from_system(s)
    j = ctx.jastrow_een(nord, kappa, c).cpu().numpy()
    j2 = ctx.jastrow_een(nord, kappa, c).cpu().numpy()
    ctx.close()
    ref, ref_abs = reference(s, kappa, nord, c)
    err = float(np.max(np.abs(j - ref) / ref_abs))
    print(json.dumps({"system": system, "nord": nord, "jastrow_err": err}))
    assert err <= 1e-12
    np.testing.assert_array_equal(j, j2)  # deterministic


def test_jastrow_een_every_tile_and_every_mode():
    """Every tile of the P product gives the oracle's J; the precision mode of
    the context does not change the (FP64) Jastrow."""
    q = qmk()
    s = synth.water_like(walkers=5)
    nord, kappa = 4, 0.9
    c = coefficients(nord, s.nucl_num, seed=11)
    ref, ref_abs = reference(s, kappa, nord, c)
    ctx = q.Context.from_system(s)
    for t in range(ctx.tile_count()):
        ctx.set_tile("jastrow_p", t)
        j = ctx.jastrow_een(nord, kappa, c).cpu().numpy()
        assert np.all(np.abs(j - ref) <= 1e-12 * ref_abs), t
    ctx.close()
    for mode in ("mixed_f32", "mixed_bf16x3"):
        ctx = q.Context.from_system(s, bits=24, mode=mode)
        j = ctx.jastrow_een(nord, kappa, c).cpu().numpy()
        ctx.close()
        assert np.all(np.abs(j - ref) <= 1e-12 * ref_abs), mode


def test_jastrow_een_one_electron_is_zero_and_new_points_are_used():
    q = qmk()
    s = synth.water_like(walkers=3)
    nord, kappa = 3, 1.0
    c = coefficients(nord, s.nucl_num, seed=5)
    ctx = q.Context.from_system(s)
    one = s.elec_coord[:, :1, :].copy()
    ctx.set_point(one)
    j = ctx.jastrow_een(nord, kappa, c)
    assert torch.count_nonzero(j).item() == 0
    # moving the electrons changes J to the oracle's value at the new points
    rng = np.random.default_rng(2)
    moved = s.elec_coord + rng.normal(scale=0.3, size=s.elec_coord.shape)
    ctx.set_point(moved)
    j = ctx.jastrow_een(nord, kappa, c).cpu().numpy()
    ctx.close()
    ref = oracle.jastrow_een(moved, s.nucl_coord, kappa, nord, c)
    ref_abs = oracle.jastrow_een(moved, s.nucl_coord, kappa, nord, np.abs(c))
    assert np.all(np.abs(j - ref) <= 1e-12 * ref_abs)


def test_jastrow_een_rejects_bad_arguments():
    q = qmk()
    s = synth.water_like(walkers=2)
    ctx = q.Context.from_system(s)
    c = coefficients(3, s.nucl_num)
    for nord, kappa, cc, status in [(1, 1.0, c, q.QMK_INVALID_ARG_BASE + 2),
                                    (9, 1.0, c, q.QMK_INVALID_ARG_BASE + 2),
                                    (3, 0.0, c, q.QMK_INVALID_ARG_BASE + 3),
                                    (3, float("nan"), c, q.QMK_INVALID_ARG_BASE + 3),
                                    (4, 1.0, c, q.QMK_INVALID_ARG_BASE + 4)]:
        with pytest.raises(q.QmkError) as e:
            ctx.jastrow_een(nord, kappa, cc)
        assert e.value.status == status
    bad = c.copy()
    bad[1, 2] = np.inf
    with pytest.raises(q.QmkError) as e:
        ctx.jastrow_een(3, 1.0, bad)
    assert e.value.status == q.QMK_NONFINITE
    host = torch.empty(2, dtype=torch.float64)
    with pytest.raises(q.QmkError) as e:
        ctx.jastrow_een(3, 1.0, c, out=host)
    assert e.value.status == q.QMK_INVALID_ARG_BASE + 6
    ctx.close()


def test_jastrow_een_new_coefficients_and_order_are_used():
    """The coefficient tables are cached between calls: a change of c or of
    the order must reach the kernels."""
    q = qmk()
    s = synth.water_like(walkers=4)
    kappa = 0.8
    ctx = q.Context.from_system(s)
    for nord, seed in [(4, 1), (4, 2), (6, 3), (4, 1)]:
        c = coefficients(nord, s.nucl_num, seed=seed)
        j = ctx.jastrow_een(nord, kappa, c).cpu().numpy()
        ref, ref_abs = reference(s, kappa, nord, c)
        assert np.all(np.abs(j - ref) <= 1e-12 * ref_abs), (nord, seed)
    with pytest.raises(ValueError):
        ctx.jastrow_een(4, kappa, coefficients(4, s.nucl_num + 1))
    with pytest.raises(ValueError):
        ctx.jastrow_een(4, kappa, coefficients(4, s.nucl_num), out=torch.empty(1, dtype=torch.float64,
                                                                               device="cuda"))
    ctx.close()


def test_jastrow_een_many_electrons_and_nuclei_transposed_points():
    """600 electrons (more than one 512-electron LDS chunk of the e-e
    kernel), 70 nuclei (two 64-nucleus blocks of the e-n kernels), points
    given transposed ([3][walk * elec], on the device); no basis is needed."""
    q = qmk()
    rng = np.random.default_rng(8)
    nn, ne, W = 70, 600, 1
    nucl = rng.uniform(-6.0, 6.0, size=(nn, 3))
    elec = nucl[rng.integers(nn, size=(W, ne))] + rng.normal(size=(W, ne, 3))
    nord, kappa = 5, 0.7
    c = coefficients(nord, nn, seed=9)
    ctx = q.Context()
    ctx.set_nucleus(nucl)
    pts = torch.from_numpy(np.ascontiguousarray(elec.reshape(-1, 3).T)).cuda()
    ctx.set_point(pts, W, ne, transp="T")
    j = ctx.jastrow_een(nord, kappa, c).cpu().numpy()
    ctx.close()
    ref = oracle.jastrow_een(elec, nucl, kappa, nord, c)
    ref_abs = oracle.jastrow_een(elec, nucl, kappa, nord, np.abs(c))
    err = float(np.max(np.abs(j - ref) / ref_abs))
    print(json.dumps({"ne": ne, "nn": nn, "jastrow_err": err}))
    assert err <= 1e-12


def test_jastrow_een_full_size_sampled():
    """The timed Jastrow workload at its full size (medium molecule: 80 nuclei,
    280 electrons; 512 walkers; order 5, kappa 0.6, the same seeded
    coefficients), in the launch configuration that is timed; the oracle
    checks the first, a middle and the last walker.  Every J is finite and a
    repeated call gives the same bits."""
    q = qmk()
    nord, kappa = 5, 0.6
    s = synth.medium(walkers=512)
    c = np.random.default_rng(0).normal(scale=0.2, size=(q.jastrow_een_terms(nord), s.nucl_num))
    ctx = q.Context.from_system(s)
    j = ctx.jastrow_een(nord, kappa, c).cpu().numpy()
    j2 = ctx.jastrow_een(nord, kappa, c).cpu().numpy()
    ctx.close()
    assert np.all(np.isfinite(j))
    np.testing.assert_array_equal(j, j2)
    idx = [0, 257, 511]
    elec = s.elec_coord[idx]
    ref = oracle.jastrow_een(elec, s.nucl_coord, kappa, nord, c)
    ref_abs = oracle.jastrow_een(elec, s.nucl_coord, kappa, nord, np.abs(c))
    err = float(np.max(np.abs(j[idx] - ref) / ref_abs))
    print(json.dumps({"walkers": s.walk_num, "sampled": idx, "jastrow_err": err}))
    assert err <= 1e-12
