"""HIP path vs the FP64 oracle, element by element on the same seeded inputs,
through the C ABI (FP64 mode: row-normwise relative error <= 1e-12)."""
import copy

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import component_errors, grad_err, rownorm_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def qmk():
    import paper_2512_16677_amd as q
    return q


def run_forward(s, points_on_device=False, transp="N"):
    q = qmk()
    ctx = q.Context.from_system(s, points_on_device=points_on_device)
    if transp == "T":
        pts = np.ascontiguousarray(s.points().T)
        ctx.set_point(pts, s.walk_num, s.elec_num, transp="T")
    ao = ctx.get_ao_vgl().cpu().numpy()
    mo = ctx.get_mo_vgl().cpu().numpy()
    ctx.close()
    return ao, mo


def test_water_like_full():
    s = synth.water_like()  # 3 nuclei, 25 AOs, 25 MOs, 128 walkers x 10 electrons
    ao, mo = run_forward(s)
    ref_ao = oracle.ao_vgl(s)
    ref_mo = oracle.mo_vgl_from_ao(ref_ao, s.mo_coef)
    e_ao = rownorm_err(ao.reshape(-1, 5, s.ao_num), ref_ao)
    e_mo = rownorm_err(mo.reshape(-1, 5, s.mo_num), ref_mo)
    print("water_like ao", e_ao.max(), "mo", e_mo.max())
    assert e_ao.max() <= TOL
    assert e_mo.max() <= TOL


@pytest.mark.parametrize("walkers", [1, 3])
def test_medium_subset(walkers):
    """80 atoms, 800 AOs, 400 MOs: several GEMM tiles plus ragged tails
    (280 and 840 points, K = 800, N = 400)."""
    s = synth.medium(walkers=walkers)
    ao, mo = run_forward(s)
    ref_ao = oracle.ao_vgl(s)
    ref_mo = oracle.mo_vgl_from_ao(ref_ao, s.mo_coef)
    assert rownorm_err(ao.reshape(-1, 5, s.ao_num), ref_ao).max() <= TOL
    assert rownorm_err(mo.reshape(-1, 5, s.mo_num), ref_mo).max() <= TOL


def test_transposed_and_device_points():
    s = synth.water_like(walkers=7)
    ref = oracle.mo_vgl(s)
    _, mo_t = run_forward(s, transp="T")
    _, mo_d = run_forward(s, points_on_device=True)
    assert rownorm_err(mo_t.reshape(-1, 5, s.mo_num), ref).max() <= TOL
    assert rownorm_err(mo_d.reshape(-1, 5, s.mo_num), ref).max() <= TOL


def test_float32_output_is_rounded_fp64():
    q = qmk()
    s = synth.water_like(walkers=5)
    ctx = q.Context.from_system(s)
    mo64 = ctx.get_mo_vgl().cpu().numpy()
    mo32 = ctx.get_mo_vgl(dtype=torch.float32).cpu().numpy()
    np.testing.assert_array_equal(mo32, mo64.astype(np.float32))


def test_single_point_and_lower_precision_cutoff():
    q = qmk()
    s = synth.medium(walkers=1)
    s.elec_coord = s.elec_coord[:, :1, :].copy()  # one point
    for bits in (53, 24, 10):
        ctx = q.Context.from_system(s, bits=bits)
        mo = ctx.get_mo_vgl().cpu().numpy()
        ref = oracle.mo_vgl(s, B=bits)
        assert rownorm_err(mo.reshape(-1, 5, s.mo_num), ref).max() <= TOL, bits
        ctx.close()


def test_nucleus_without_shells_and_unsorted_primitives():
    q = qmk()
    s = synth.tiny_system([0, 1, 2, 3], n_prim=4, seed=3, walkers=9, elec=6, n_nuc=3)
    # drop the shells of nucleus 1 and shuffle the primitives of each shell
    keep = s.shell_nucleus != 1
    offs = s.shell_prim_offset
    ex, co, new_off = [], [], [0]
    rng = np.random.default_rng(0)
    for sh in np.nonzero(keep)[0]:
        idx = np.arange(offs[sh], offs[sh + 1])
        rng.shuffle(idx)
        ex.append(s.exponent[idx])
        co.append(s.coefficient[idx])
        new_off.append(new_off[-1] + len(idx))
    s.shell_nucleus = s.shell_nucleus[keep]
    s.shell_ang_mom = s.shell_ang_mom[keep]
    s.shell_prim_offset = np.array(new_off, dtype=np.int64)
    s.exponent = np.concatenate(ex)
    s.coefficient = np.concatenate(co)
    s.mo_coef = np.random.default_rng(1).normal(size=(7, s.ao_num))
    ctx = q.Context.from_system(s)
    mo = ctx.get_mo_vgl().cpu().numpy()
    ref = oracle.mo_vgl(s)
    assert rownorm_err(mo.reshape(-1, 5, s.mo_num), ref).max() <= TOL
    w = torch.from_numpy(synth.adjoint_weights(s, seed=3)).cuda()
    g = ctx.adjoint(w)
    r = oracle.adjoint(s, w.cpu().numpy())
    assert grad_err(g["d_nucl"].cpu().numpy(), r["d_nucl"], r["d_nucl_abs"]) <= 1e-11
    assert np.all(g["d_nucl"].cpu().numpy()[1] == 0.0)


def test_time_stamps_recompute_only_when_points_change():
    q = qmk()
    s = synth.water_like(walkers=4)
    ctx = q.Context.from_system(s)
    ctx.get_mo_vgl()
    n1 = ctx.launch_count()
    ctx.get_mo_vgl()
    n2 = ctx.launch_count()
    assert n2 - n1 == 1  # contraction only: the AO array is still valid
    ctx.set_point(s.elec_coord)
    ctx.get_mo_vgl()
    assert ctx.launch_count() - n2 == 2  # AO stage + contraction
    ctx.set_mo_coef(s.mo_coef * 2.0)
    n3 = ctx.launch_count()
    mo = ctx.get_mo_vgl().cpu().numpy()
    assert ctx.launch_count() - n3 == 1
    ref = oracle.mo_vgl(s, coef=s.mo_coef * 2.0)
    assert rownorm_err(mo.reshape(-1, 5, s.mo_num), ref).max() <= TOL


@pytest.mark.parametrize("mode,screened", [("fp64", False), ("fp64", True), ("mixed_bf16x3", False),
                                           ("mixed_bf16x3", True)])
def test_ao_retention_off_recomputes_and_matches(mode, screened):
    """With AO retention off the adjoint evaluates the AO array again (one
    more AO launch, or sort + bitmap + AO launches when screened) and its
    outputs are bitwise those of the default (retained) adjoint."""
    q = qmk()
    s = synth.medium(walkers=2)
    ctx = q.Context.from_system(s, bits=53 if mode == "fp64" else 24, mode=mode)
    ctx.set_screening(screened)
    w = torch.from_numpy(synth.adjoint_weights(s, seed=8)).cuda()
    if mode != "fp64":
        w = w.float()
    ctx.get_mo_vgl()
    g_keep = {k: v.clone() for k, v in ctx.adjoint(w).items()}
    n_keep = ctx.launch_count()
    ctx.adjoint(w)
    per_keep = ctx.launch_count() - n_keep
    ctx.set_ao_retention(False)
    n0 = ctx.launch_count()
    g_again = ctx.adjoint(w)
    per_again = ctx.launch_count() - n0
    assert per_again > per_keep, (per_again, per_keep)
    for k in ("d_coef", "d_elec", "d_nucl"):
        assert bool((g_again[k] == g_keep[k]).all()), k
    with pytest.raises(q.QmkError) as e:
        ctx._check(ctx._lib.qmk_set_ao_retention(ctx._h, 2))
    assert e.value.status == q.QMK_INVALID_ARG_BASE + 2
    ctx.close()


def test_error_codes():
    q = qmk()
    ctx = q.Context()
    with pytest.raises(q.QmkError) as e:
        ctx.get_mo_vgl(out=torch.empty(10, dtype=torch.float64, device="cuda"))
    s = synth.water_like(walkers=2)
    ctx.set_nucleus(s.nucl_coord)
    with pytest.raises(q.QmkError) as e:
        ctx.set_basis(s.shell_nucleus + 5, s.shell_ang_mom, s.shell_prim_offset, s.exponent,
                      s.coefficient)
    assert e.value.status == q.QMK_INVALID_ARG_BASE + 4
    ctx.set_basis(s.shell_nucleus, s.shell_ang_mom, s.shell_prim_offset, s.exponent, s.coefficient)
    ctx.set_point(s.elec_coord)
    with pytest.raises(q.QmkError) as e:
        ctx.get_mo_vgl(out=torch.empty(10, dtype=torch.float64, device="cuda"))
    assert e.value.status == q.QMK_NOT_SET  # no MO coefficients yet
    ctx.set_mo_coef(s.mo_coef)
    with pytest.raises(q.QmkError) as e:
        ctx.get_mo_vgl(out=torch.empty(10, dtype=torch.float64, device="cuda"))
    assert e.value.status == q.QMK_SIZE
    bad = s.elec_coord.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(q.QmkError) as e:
        ctx.set_point(bad)
    assert e.value.status == q.QMK_NONFINITE
    ctx.get_mo_vgl()  # the context is still valid after errors
    ctx.close()


def test_empty_points_and_wrong_buffer_sizes_are_rejected():
    """Empty point sets are argument errors that leave the context's points in
    place; coordinate arrays and adjoint outputs whose size does not match the
    dimensions never reach the library (it reads and writes them through plain
    pointers); nothing is launched for any of them."""
    import ctypes
    q = qmk()
    s = synth.water_like(walkers=2)
    ctx = q.Context.from_system(s)
    ref = ctx.get_mo_vgl().cpu().numpy()
    n0 = ctx.launch_count()
    for shape, status in [((0, s.elec_num, 3), q.QMK_INVALID_ARG_BASE + 3),
                          ((s.walk_num, 0, 3), q.QMK_INVALID_ARG_BASE + 4)]:
        with pytest.raises(q.QmkError) as e:
            ctx.set_point(np.zeros(shape))
        assert e.value.status == status
    pts = torch.from_numpy(np.ascontiguousarray(s.elec_coord.reshape(-1, 3).T)).cuda()
    with pytest.raises(ValueError):
        ctx.set_point(pts[:, :-1].contiguous(), s.walk_num, s.elec_num, transp="T")
    with pytest.raises(ValueError):
        ctx.set_point(s.elec_coord[:, :, :2].copy())
    with pytest.raises(ValueError):
        ctx.set_point(s.elec_coord.reshape(-1)[:-3].copy(), s.walk_num, s.elec_num)
    # more than 2^31 points: refused before the pointer is used
    assert ctx._lib.qmk_set_point(ctx._h, b"T", 1 << 16, (1 << 15) + 1,
                                  ctypes.c_void_p(pts.data_ptr()), 1) == q.QMK_INVALID_ARG_BASE + 3
    w = torch.ones((s.walk_num, s.elec_num, 5, s.mo_num), dtype=torch.float64, device="cuda")
    for bad in [{"d_coef": torch.empty(3, dtype=torch.float64, device="cuda")},
                {"d_elec": torch.empty((s.walk_num, s.elec_num, 3), dtype=torch.float32, device="cuda")},
                {"d_nucl": torch.empty((s.nucl_num, 3), dtype=torch.float64)},
                {"d_x": torch.empty(3, dtype=torch.float64, device="cuda")}]:
        with pytest.raises(ValueError):
            ctx.adjoint(w, out=bad)
    with pytest.raises(ValueError):
        ctx.set_mo_cusp(np.ones(s.nucl_num), np.ones(s.nucl_num - 1))
    with pytest.raises(ValueError):
        ctx.set_basis(s.shell_nucleus, s.shell_ang_mom, s.shell_prim_offset[:-1], s.exponent,
                      s.coefficient)
    with pytest.raises(ValueError):
        ctx.set_basis(s.shell_nucleus, s.shell_ang_mom, s.shell_prim_offset, s.exponent,
                      s.coefficient[:-1])
    with pytest.raises(ValueError):
        ctx.set_basis(s.shell_nucleus, s.shell_ang_mom, s.shell_prim_offset, s.exponent,
                      s.coefficient, ao_factor=np.ones(s.ao_num + 1))
    with pytest.raises(ValueError):
        ctx.set_mo_coef(s.mo_coef.reshape(-1))
    assert ctx.launch_count() == n0
    np.testing.assert_array_equal(ctx.get_mo_vgl().cpu().numpy(), ref)
    assert ctx.dims()["walk_num"] == s.walk_num
    ctx.close()


# ---------------------------------------------------------------- adjoint
@pytest.mark.parametrize("system", ["water_like", "medium"])
def test_adjoint_matches_oracle(system):
    q = qmk()
    s = synth.water_like(walkers=16) if system == "water_like" else synth.medium(walkers=2)
    w = synth.adjoint_weights(s, seed=7)
    ctx = q.Context.from_system(s)
    ctx.get_mo_vgl()
    g = ctx.adjoint(torch.from_numpy(w).cuda())
    r = oracle.adjoint(s, w)
    e = {k: grad_err(g[k].cpu().numpy().reshape(r[k].shape), r[k], r[k + "_abs"])
         for k in ("d_coef", "d_elec", "d_nucl")}
    print(system, e)
    for k, v in e.items():
        assert v <= 1e-11, (k, v)
    # deterministic: bitwise repeat
    g2 = ctx.adjoint(torch.from_numpy(w).cuda())
    for k in g:
        assert torch.equal(g[k], g2[k]), k


def test_adjoint_finite_differences_and_sum_rule():
    """Central differences (h = 1e-5) of sum(W * mo_vgl) computed by the GPU
    forward, on random entries of C, R_elec and R_nucl."""
    q = qmk()
    s = synth.water_like(walkers=4)
    w = synth.adjoint_weights(s, seed=5)
    wt = torch.from_numpy(w).cuda()
    ctx = q.Context.from_system(s)
    g = {k: v.cpu().numpy() for k, v in ctx.adjoint(wt).items()}

    def loss(nucl=None, coef=None, elec=None):
        ctx.set_nucleus(s.nucl_coord if nucl is None else nucl)
        ctx.set_mo_coef(s.mo_coef if coef is None else coef)
        ctx.set_point(s.elec_coord if elec is None else elec)
        return float(torch.sum(wt * ctx.get_mo_vgl()).item())

    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(8):
        A, i = int(rng.integers(s.nucl_num)), int(rng.integers(3))
        e = np.zeros_like(s.nucl_coord)
        e[A, i] = h
        fd = (loss(nucl=s.nucl_coord + e) - loss(nucl=s.nucl_coord - e)) / (2 * h)
        assert fd == pytest.approx(g["d_nucl"][A, i], rel=1e-6, abs=1e-6 * np.abs(g["d_nucl"]).max())
    for _ in range(8):
        wk, el, i = int(rng.integers(s.walk_num)), int(rng.integers(s.elec_num)), int(rng.integers(3))
        e = np.zeros_like(s.elec_coord)
        e[wk, el, i] = h
        fd = (loss(elec=s.elec_coord + e) - loss(elec=s.elec_coord - e)) / (2 * h)
        assert fd == pytest.approx(g["d_elec"][wk, el, i], rel=1e-5, abs=1e-6 * np.abs(g["d_elec"]).max())
    for _ in range(8):
        n, k = int(rng.integers(s.mo_num)), int(rng.integers(s.ao_num))
        e = np.zeros_like(s.mo_coef)
        e[n, k] = h
        fd = (loss(coef=s.mo_coef + e) - loss(coef=s.mo_coef - e)) / (2 * h)
        assert fd == pytest.approx(g["d_coef"][n, k], rel=1e-6, abs=1e-8 * np.abs(g["d_coef"]).max())
    tot = g["d_nucl"].sum(axis=0) + g["d_elec"].reshape(-1, 3).sum(axis=0)
    scale = np.abs(g["d_nucl"]).sum(axis=0) + np.abs(g["d_elec"]).reshape(-1, 3).sum(axis=0)
    assert np.all(np.abs(tot) <= 1e-11 * scale)


def test_autograd_function():
    q = qmk()
    s = synth.water_like(walkers=3)
    ctx = q.Context.from_system(s)
    C = torch.tensor(s.mo_coef, requires_grad=True)
    Rn = torch.tensor(s.nucl_coord, requires_grad=True)
    Re = torch.tensor(s.elec_coord, device="cuda", requires_grad=True)
    mo = q.mo_vgl(ctx, C, Rn, Re)
    w = torch.from_numpy(synth.adjoint_weights(s, seed=2)).cuda()
    (mo * w).sum().backward()
    r = oracle.adjoint(s, w.cpu().numpy())
    assert grad_err(C.grad.cpu().numpy(), r["d_coef"], r["d_coef_abs"]) <= 1e-11
    assert grad_err(Rn.grad.cpu().numpy(), r["d_nucl"], r["d_nucl_abs"]) <= 1e-11
    assert grad_err(Re.grad.cpu().numpy().reshape(-1, 3), r["d_elec"], r["d_elec_abs"]) <= 1e-11


def test_autograd_two_graphs_on_one_context():
    """Two forwards with different C, nuclei and electrons on one context,
    then the backward passes in reverse order and again in forward order:
    each graph gets the oracle gradients of its own inputs (the binding puts
    a graph's inputs back into the context when another forward ran in
    between).  A precision change between forward and backward is an
    error."""
    q = qmk()
    s = synth.water_like(walkers=3)
    ctx = q.Context.from_system(s)
    rng = np.random.default_rng(31)
    inputs, outs = [], []
    for g in range(2):
        C0 = s.mo_coef + (0.1 * g) * rng.normal(size=s.mo_coef.shape)
        R0 = s.nucl_coord + (0.05 * g) * rng.normal(size=s.nucl_coord.shape)
        E0 = s.elec_coord + (0.2 * g) * rng.normal(size=s.elec_coord.shape)
        C = torch.tensor(C0, requires_grad=True)
        Rn = torch.tensor(R0, requires_grad=True)
        Re = torch.tensor(E0, device="cuda", requires_grad=True)
        inputs.append((C0, R0, E0, C, Rn, Re))
        outs.append(q.mo_vgl(ctx, C, Rn, Re))
    ws = [torch.from_numpy(synth.adjoint_weights(s, seed=40 + g)).cuda() for g in range(2)]
    for order in ((1, 0), (0, 1)):
        for g in order:
            C0, R0, E0, C, Rn, Re = inputs[g]
            for t in (C, Rn, Re):
                t.grad = None
            (outs[g] * ws[g]).sum().backward(retain_graph=True)
            sg = copy.copy(s)
            sg.nucl_coord, sg.mo_coef, sg.elec_coord = R0, C0, E0
            r = oracle.adjoint(sg, ws[g].cpu().numpy())
            assert grad_err(C.grad.cpu().numpy(), r["d_coef"], r["d_coef_abs"]) <= 1e-11, (order, g)
            assert grad_err(Rn.grad.cpu().numpy(), r["d_nucl"], r["d_nucl_abs"]) <= 1e-11, (order, g)
            assert grad_err(Re.grad.cpu().numpy().reshape(-1, 3), r["d_elec"], r["d_elec_abs"]) <= 1e-11, \
                (order, g)
    ctx.set_precision(53, "mixed_f32")
    with pytest.raises(RuntimeError, match="changed between forward and backward"):
        (outs[0] * ws[0]).sum().backward()
    ctx.close()


def test_every_tile_shape_matches_oracle():
    """The autotuner may pick any tile shape: each one must give the oracle's
    result (forward contraction, W C product and split-K W^T ao product)."""
    q = qmk()
    s = synth.medium(walkers=1)  # 280 points, 800 AOs, 400 MOs
    w = synth.adjoint_weights(s, seed=4)
    ref_mo = oracle.mo_vgl(s)
    ref = oracle.adjoint(s, w)
    wt = torch.from_numpy(w).cuda()
    ctx = q.Context.from_system(s)
    tried = 0
    for t in range(ctx.tile_count()):
        try:
            for k in ("mo", "gbar", "dcoef"):
                ctx.set_tile(k, t)
        except q.QmkError:
            continue  # does not fit in LDS
        tried += 1
        mo = ctx.get_mo_vgl().cpu().numpy().reshape(-1, 5, s.mo_num)
        assert rownorm_err(mo, ref_mo).max() <= TOL, t
        g = ctx.adjoint(wt)
        for k in ("d_coef", "d_elec", "d_nucl"):
            e = grad_err(g[k].cpu().numpy().reshape(ref[k].shape), ref[k], ref[k + "_abs"])
            assert e <= 1e-11, (t, k, e)
    assert tried >= 6
    ctx.close()


def test_host_buffers_are_rejected_before_any_launch():
    """Pageable host memory as a buffer argument returns an argument error
    and enqueues nothing.  Every call also carries a second invalid argument
    that is checked after the pointer (too small a size, a wrong length, an
    unknown dtype), so that it would stop before any kernel even if the
    pointer check let the host buffer through; the device-pointer set_point
    comes last and nothing runs after it."""
    import ctypes
    q = qmk()
    s = synth.water_like(walkers=2)
    ctx = q.Context.from_system(s)
    n0 = ctx.launch_count()
    host = np.zeros(16)
    hp = host.ctypes.data_as(ctypes.c_void_p)
    lib = ctx._lib
    assert lib.qmk_get_mo_vgl(ctx._h, hp, 1, q.QMK_F64, None) == q.QMK_INVALID_ARG_BASE + 2
    assert lib.qmk_get_ao_vgl(ctx._h, hp, 1, q.QMK_F64, None) == q.QMK_INVALID_ARG_BASE + 2
    assert lib.qmk_get_mo_value(ctx._h, hp, 1, q.QMK_F64, None) == q.QMK_INVALID_ARG_BASE + 2
    occ = np.zeros(s.mo_num + 1)  # wrong length as well
    assert lib.qmk_get_density(ctx._h, occ.ctypes.data_as(ctypes.c_void_p), occ.shape[0], hp, 1,
                               None) == q.QMK_INVALID_ARG_BASE + 4
    assert lib.qmk_mo_vgl_adjoint(ctx._h, hp, 99, None, None, None, None) == q.QMK_INVALID_ARG_BASE + 2
    assert "device can access" in lib.qmk_last_error(ctx._h).decode()
    assert ctx.launch_count() == n0
    assert lib.qmk_set_point(ctx._h, b"N", 1, 1, hp, 1) == q.QMK_INVALID_ARG_BASE + 5
    ctx.close()
