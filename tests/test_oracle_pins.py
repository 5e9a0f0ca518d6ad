"""Pins of the FP64 oracle against what the mathematics fixes.

None of these tests re-types the oracle's formulas: each checks it against a
closed form, a quadrature, finite differences, a brute-force derivative built
a different way (products of 1-D polynomial derivatives), an invariance, or a
library routine.  The paper prints no AO or MO values, so there is no printed
worked example to compare with.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def one_shell_system(l, gammas, coefs, centre=(0.0, 0.0, 0.0), pts=None):
    g = np.asarray(gammas, dtype=float)
    a = np.asarray(coefs, dtype=float)
    s = synth.System(
        name="one_shell",
        nucl_coord=np.array([centre], dtype=float),
        nucl_charge=np.array([1], dtype=np.int32),
        shell_nucleus=np.array([0], dtype=np.int64),
        shell_ang_mom=np.array([l], dtype=np.int32),
        shell_prim_offset=np.array([0, len(g)], dtype=np.int64),
        exponent=g,
        coefficient=a,
        mo_coef=np.eye(synth.N_CART[l]),
        elec_coord=np.zeros((1, 1, 3)) if pts is None else np.asarray(pts, float).reshape(1, -1, 3),
    )
    return s


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("gam", [0.1, 0.7, 3.0, 250.0, 1e4])
@pytest.mark.parametrize("a", [0.1, 1.0])
def test_normalised_s_primitive_closed_form(gam, a):
    """A normalised s Gaussian is (2g/pi)^(3/4) exp(-g r^2): value at the
    nucleus (2g/pi)^(3/4), zero gradient, Laplacian (4 g^2 r^2 - 6 g) times
    the value, independent of the contraction coefficient."""
    s = one_shell_system(0, [gam], [a])
    r = np.array([[0.0, 0.0, 0.0], [0.05, -0.02, 0.01], [0.3, 0.2, -0.1]])
    out = oracle.ao_derivs(s, r, B=0.0)
    norm = (2 * gam / math.pi) ** 0.75
    u = np.sum(r ** 2, axis=1)
    val = norm * np.exp(-gam * u)
    np.testing.assert_allclose(out[:, 0, 0], val, rtol=1e-14, atol=0)
    np.testing.assert_allclose(out[:, 1:4, 0], -2 * gam * r * val[:, None], rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(out[:, 4, 0], (4 * gam ** 2 * u - 6 * gam) * val, rtol=1e-13)
    assert out[0, 4, 0] == pytest.approx(-6 * gam * norm, rel=1e-14)


@pytest.mark.parametrize("gam", [0.2, 5.0, 800.0])
def test_normalised_p_primitive_closed_form(gam):
    """p_x of one primitive: (2g/pi)^(3/4) (4g)^(1/2) x exp(-g r^2); its
    x-derivative at the nucleus equals (2g/pi)^(3/4) (4g)^(1/2)."""
    s = one_shell_system(1, [gam], [0.37])
    r = np.array([[0.0, 0.0, 0.0], [0.03, 0.01, -0.02]])
    out = oracle.ao_derivs(s, r, B=0.0)
    c = (2 * gam / math.pi) ** 0.75 * math.sqrt(4 * gam)
    assert out[0, 1, 0] == pytest.approx(c, rel=1e-14)
    assert out[0, 0, 0] == 0.0
    e = np.exp(-gam * np.sum(r[1] ** 2))
    assert out[1, 0, 0] == pytest.approx(c * r[1, 0] * e, rel=1e-14)
    assert out[1, 0, 1] == pytest.approx(c * r[1, 1] * e, rel=1e-14)  # p_y
    assert out[1, 0, 2] == pytest.approx(c * r[1, 2] * e, rel=1e-14)  # p_z


def test_one_primitive_independent_of_coefficient():
    r = np.random.default_rng(3).normal(size=(7, 3))
    for l in range(4):
        a = oracle.ao_derivs(one_shell_system(l, [1.3], [0.11]), r, B=0.0, nq=14)
        b = oracle.ao_derivs(one_shell_system(l, [1.3], [0.93]), r, B=0.0, nq=14)
        scale = np.max(np.abs(a), axis=(0, 2), keepdims=True)
        np.testing.assert_allclose(a / scale, b / scale, rtol=0, atol=1e-14)


def test_cartesian_order_and_normalisation_factor_table():
    """d-shell components are xx xy xz yy yz zz (x power descending); the
    mixed ones carry sqrt(3) relative to the axis ones, the f-shell xyz
    carries sqrt(15)."""
    _, _, m2 = oracle.normalisation(one_shell_system(2, [1.0], [1.0]))
    np.testing.assert_allclose(m2, [1, math.sqrt(3), math.sqrt(3), 1, math.sqrt(3), 1], rtol=1e-15)
    _, _, m3 = oracle.normalisation(one_shell_system(3, [1.0], [1.0]))
    np.testing.assert_allclose(m3, [1, math.sqrt(5), math.sqrt(5), math.sqrt(5), math.sqrt(15),
                                    math.sqrt(5), 1, math.sqrt(5), math.sqrt(5), 1], rtol=1e-15)
    # the xy component is x*y times the radial part
    s = one_shell_system(2, [0.8], [1.0])
    r = np.array([[0.3, -0.4, 0.2]])
    v = oracle.ao_derivs(s, r, B=0.0)[0, 0]
    np.testing.assert_allclose(v[1] / v[0], math.sqrt(3) * r[0, 1] / r[0, 0], rtol=1e-14)
    np.testing.assert_allclose(v[4] / v[3], math.sqrt(3) * r[0, 2] / r[0, 1], rtol=1e-14)


# ---------------------------------------------------------------- quadrature
def _sinh_rule(c=0.002, h=0.15, tmax=10.5):
    t = np.arange(-tmax, tmax + 1e-12, h)
    x = c * np.sinh(t)
    w = c * np.cosh(t) * h
    return x, w


def test_quadrature_rule_itself():
    """The 1-D rule integrates x^(2n) exp(-alpha x^2) to 1e-10 relative over
    the exponent range of the bases (2 g from 0.2 to 2e4)."""
    x, w = _sinh_rule()
    for alpha in [0.2, 1.0, 37.0, 2e4]:
        for n in range(4):
            exact = math.gamma(n + 0.5) / alpha ** (n + 0.5)
            num = np.sum(w * x ** (2 * n) * np.exp(-alpha * x * x))
            assert num == pytest.approx(exact, rel=1e-10)


@pytest.mark.parametrize("l,gam", [
    (0, [0.1, 0.9, 15.0, 300.0, 9000.0]),
    (1, [0.15, 2.0, 60.0]),
    (2, [0.3, 4.0]),
    (3, [0.5, 1.2, 9.0]),
])
def test_self_overlap_by_quadrature(l, gam):
    """Numerical overlap of the oracle's AOs on a tensor grid (the overlap
    check idea of Section 5.3): every Cartesian AO has unit norm, and the
    overlaps between components match the Gaussian moments."""
    rng = np.random.default_rng(l)
    coef = rng.uniform(0.1, 1.0, size=len(gam))
    s = one_shell_system(l, gam, coef)
    x, w = _sinh_rule()
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    W3 = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
    v = oracle.ao_derivs(s, pts, B=0.0)[:, 0, :]
    S = (v * W3[:, None]).T @ v
    np.testing.assert_allclose(np.diag(S), 1.0, rtol=2e-9)
    # off-diagonal: two components overlap iff every summed power is even;
    # for unit-norm AOs, <x^a..|x^a'..> / sqrt(<..><..>) is a ratio of
    # Gaussian moments (2n-1)!! that does not depend on the exponents.
    comps = [(a, b, l - a - b) for a in range(l, -1, -1) for b in range(l - a, -1, -1)]

    def dfact(n):
        return 1.0 if n <= 0 else n * dfact(n - 2)

    def mom(e):
        return dfact(e - 1) if e % 2 == 0 else 0.0

    for i, ci in enumerate(comps):
        for j, cj in enumerate(comps):
            e = [ci[q] + cj[q] for q in range(3)]
            num = mom(e[0]) * mom(e[1]) * mom(e[2])
            den = math.sqrt(mom(2 * ci[0]) * mom(2 * ci[1]) * mom(2 * ci[2]) *
                            mom(2 * cj[0]) * mom(2 * cj[1]) * mom(2 * cj[2]))
            assert S[i, j] == pytest.approx(num / den, rel=2e-9, abs=1e-12)


# ----------------------------------------------- brute-force 1-D derivatives
def _poly_derivs(n, gam, t, order=3):
    """d^m/dt^m of t^n exp(-g t^2) for m = 0..order, as polynomials times the
    exponential: p_{m+1} = p_m' - 2 g t p_m."""
    from numpy.polynomial import polynomial as Pl
    p = np.zeros(n + 1)
    p[n] = 1.0
    out = []
    e = np.exp(-gam * t * t)
    for m in range(order + 1):
        out.append(Pl.polyval(t, p) * e)
        p = Pl.polysub(Pl.polyder(p), Pl.polymulx(p) * 2 * gam) if len(p) > 1 else -2 * gam * Pl.polymulx(p)
    return out


def _brute_force(sys_, pts):
    """AO value, gradient, Hessian, Laplacian and gradient of the Laplacian
    from products of 1-D derivatives of x^a exp(-g x^2) (no cutoff)."""
    f, ns, m = oracle.normalisation(sys_)
    K = sys_.ao_num
    P = pts.shape[0]
    out = np.zeros((P, 14, K))
    ao = 0
    hpairs = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for s in range(sys_.shell_num):
        l = int(sys_.shell_ang_mom[s])
        R = sys_.nucl_coord[sys_.shell_nucleus[s]]
        d = pts - R
        comps = [(a, b, l - a - b) for a in range(l, -1, -1) for b in range(l - a, -1, -1)]
        for (a, b, c) in comps:
            acc = np.zeros((P, 14))
            for k in range(sys_.shell_prim_offset[s], sys_.shell_prim_offset[s + 1]):
                g = sys_.exponent[k]
                cp = sys_.coefficient[k] * f[k] * ns[s]
                D = [_poly_derivs(e, g, d[:, ax]) for ax, e in enumerate((a, b, c))]

                def term(mx, my, mz):
                    return D[0][mx] * D[1][my] * D[2][mz]

                acc[:, 0] += cp * term(0, 0, 0)
                for i in range(3):
                    mm = [0, 0, 0]
                    mm[i] = 1
                    acc[:, 1 + i] += cp * term(*mm)
                for q, (i, j) in enumerate(hpairs):
                    mm = [0, 0, 0]
                    mm[i] += 1
                    mm[j] += 1
                    acc[:, 5 + q] += cp * term(*mm)
                for i in range(3):
                    for j in range(3):
                        mm = [0, 0, 0]
                        mm[i] += 1
                        mm[j] += 2
                        acc[:, 11 + i] += cp * term(*mm)
            acc[:, 4] = acc[:, 5] + acc[:, 8] + acc[:, 10]
            out[:, :, ao] = m[ao] * acc
            ao += 1
    return out


def test_derivatives_match_brute_force_products():
    """Gradient, Hessian, Laplacian (= trace of the Hessian) and gradient of
    the Laplacian agree with the 1-D product construction to ~1e-13."""
    s = synth.tiny_system([0, 1, 2, 3, 0, 2], n_prim=3, seed=5, gamma_range=(-0.7, 1.3))
    pts = np.random.default_rng(9).normal(scale=0.8, size=(40, 3))
    a = oracle.ao_derivs(s, pts, B=0.0, nq=14)
    b = _brute_force(s, pts)
    scale = np.max(np.abs(b), axis=(0, 2), keepdims=True)
    np.testing.assert_allclose(a / scale, b / scale, rtol=0, atol=5e-14)


def test_gradient_laplacian_third_order_by_finite_differences():
    """Central differences: gradient of the value, Hessian of the gradient,
    gradient of the Laplacian from the Laplacian (h = 1e-4/sqrt(g_max))."""
    s = synth.water_like(walkers=1)
    pts = s.points()
    h = 1e-4 / math.sqrt(float(np.max(s.exponent)))
    h = max(h, 2e-6)
    a = oracle.ao_derivs(s, pts, B=0.0, nq=14)
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        ap = oracle.ao_derivs(s, pts + e, B=0.0, nq=14)
        am = oracle.ao_derivs(s, pts - e, B=0.0, nq=14)
        fd = (ap - am) / (2 * h)
        for src, dst in [(0, 1 + i), (4, 11 + i)]:
            ref = a[:, dst]
            sc = np.max(np.abs(ref)) + 1e-300
            assert np.max(np.abs(fd[:, src] - ref)) / sc < 1e-6, (src, dst)
        hrow = {0: [5, 6, 7], 1: [6, 8, 9], 2: [7, 9, 10]}[i]
        for j in range(3):
            ref = a[:, hrow[j]]
            sc = np.max(np.abs(ref)) + 1e-300
            assert np.max(np.abs(fd[:, 1 + j] - ref)) / sc < 1e-6


# ------------------------------------------------------------ invariances
def test_rigid_translation_invariance_of_mo_vgl():
    s = synth.water_like(walkers=4)
    ref = oracle.mo_vgl(s)
    t = np.array([3.7, -1.25, 0.4])
    s2 = synth.water_like(walkers=4)
    s2.nucl_coord = s.nucl_coord + t
    moved = oracle.mo_vgl(s2, points=s.points() + t)
    # row-normwise per (point, component)
    num = np.max(np.abs(moved - ref), axis=2)
    den = np.maximum(np.max(np.abs(ref), axis=2), 1e-300)
    assert np.max(num / den) < 1e-12


def test_contraction_matches_library_and_identity():
    s = synth.water_like(walkers=3)
    ao = oracle.ao_vgl(s)
    mo = oracle.mo_vgl_from_ao(ao, s.mo_coef)
    np.testing.assert_allclose(mo, np.einsum("pck,nk->pcn", ao, s.mo_coef), rtol=1e-12, atol=1e-13)
    np.testing.assert_array_equal(oracle.mo_vgl_from_ao(ao, np.eye(s.ao_num)), ao)
    c2 = np.random.default_rng(1).normal(size=s.mo_coef.shape)
    lin = oracle.mo_vgl_from_ao(ao, 2.0 * s.mo_coef - 0.5 * c2)
    np.testing.assert_allclose(lin, 2.0 * mo - 0.5 * oracle.mo_vgl_from_ao(ao, c2), rtol=1e-12, atol=1e-12)


# ----------------------------------------------------------------- cutoff
def test_cutoff_is_strict_on_the_exponent_argument():
    """A primitive contributes iff g u < (B-1) ln 2 (natural log, strict)."""
    B = 20.0
    T = (B - 1) * math.log(2.0)
    g = 2.0
    s = one_shell_system(0, [g], [1.0])
    r_in = math.sqrt(T / g) * (1 - 1e-9)
    r_out = math.sqrt(T / g) * (1 + 1e-9)
    v = oracle.ao_derivs(s, np.array([[r_in, 0, 0], [r_out, 0, 0]]), B=B)
    assert v[0, 0, 0] > 0
    assert np.all(v[1] == 0.0)


def test_cutoff_error_bound():
    """|unscreened - screened| is at most sum_k |a f N M P| 2^-(B-1) for the
    value and sum_k |a f N M| (|dP| + 2 g |d_i| |P|) 2^-(B-1) for the
    gradient; with small B the cut is visible."""
    s = synth.tiny_system([0, 1, 2], n_prim=4, seed=2, gamma_range=(-1.0, 2.0))
    pts = np.random.default_rng(4).normal(scale=1.5, size=(300, 3))
    B = 12.0
    full = oracle.ao_derivs(s, pts, B=0.0)
    cut = oracle.ao_derivs(s, pts, B=B)
    assert np.max(np.abs(full - cut)) > 0
    f, ns, m = oracle.normalisation(s)
    eps = 2.0 ** -(B - 1)
    ao = 0
    for sh in range(s.shell_num):
        l = int(s.shell_ang_mom[sh])
        d = pts - s.nucl_coord[s.shell_nucleus[sh]]
        ks = range(s.shell_prim_offset[sh], s.shell_prim_offset[sh + 1])
        csum = sum(abs(s.coefficient[k] * f[k] * ns[sh]) for k in ks)
        gsum = sum(abs(s.coefficient[k] * f[k] * ns[sh]) * s.exponent[k] for k in ks)
        comps = [(a, b, l - a - b) for a in range(l, -1, -1) for b in range(l - a, -1, -1)]
        for (a, b, c) in comps:
            P = np.abs(d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** c)
            bound = m[ao] * csum * P * eps
            assert np.all(np.abs(full[:, 0, ao] - cut[:, 0, ao]) <= bound * (1 + 1e-12) + 1e-300)
            e = (a, b, c)
            for i in range(3):
                ei = list(e)
                dP = np.zeros(len(pts)) if ei[i] == 0 else ei[i] * np.abs(d[:, i]) ** (ei[i] - 1)
                ei[i] = 0
                others = np.abs(d[:, 0] ** ei[0] * d[:, 1] ** ei[1] * d[:, 2] ** ei[2])
                gb = m[ao] * (csum * dP * others + 2 * gsum * np.abs(d[:, i]) * P) * eps
                assert np.all(np.abs(full[:, 1 + i, ao] - cut[:, 1 + i, ao]) <= gb * (1 + 1e-12) + 1e-300)
            ao += 1


# ---------------------------------------------------------------- adjoint
def _loss(sys_, w, pts=None, coef=None, nucl=None):
    s = sys_
    if nucl is not None:
        import copy
        s = copy.copy(sys_)
        s.nucl_coord = nucl
    mo = oracle.mo_vgl(s, points=pts, coef=coef, B=0.0)
    return math.fsum((w * mo).ravel())


def test_adjoint_dcoef_is_w_transpose_ao():
    s = synth.water_like(walkers=3)
    w = synth.adjoint_weights(s, seed=1).reshape(-1, 5, s.mo_num)
    g = oracle.adjoint(s, w, B=0.0)
    ao = oracle.ao_vgl(s, B=0.0)
    np.testing.assert_allclose(g["d_coef"], np.einsum("pcn,pck->nk", w, ao), rtol=1e-11, atol=1e-12)


def test_adjoint_finite_differences_and_sum_rule():
    s = synth.water_like(walkers=2)
    w = synth.adjoint_weights(s, seed=2).reshape(-1, 5, s.mo_num)
    g = oracle.adjoint(s, w, B=0.0)
    rng = np.random.default_rng(11)
    h = 1e-5
    pts = s.points()
    # electron coordinates: 12 random entries
    for _ in range(12):
        p, i = int(rng.integers(pts.shape[0])), int(rng.integers(3))
        # only point p moves: restrict the loss to its rows for accuracy
        e = np.zeros_like(pts)
        e[p, i] = h
        lp = _loss(s, w[p:p + 1], pts=(pts + e)[p:p + 1])
        lm = _loss(s, w[p:p + 1], pts=(pts - e)[p:p + 1])
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(g["d_elec"][p, i], rel=1e-6, abs=1e-6 * g["d_elec_abs"][p, i])
    # nuclear coordinates
    for A in range(s.nucl_num):
        for i in range(3):
            e = np.zeros_like(s.nucl_coord)
            e[A, i] = h
            fd = (_loss(s, w, nucl=s.nucl_coord + e) - _loss(s, w, nucl=s.nucl_coord - e)) / (2 * h)
            assert fd == pytest.approx(g["d_nucl"][A, i], rel=1e-6, abs=1e-6 * g["d_nucl_abs"][A, i])
    # MO coefficients: the loss is linear in C, so the FD is exact up to rounding
    for _ in range(8):
        n, k = int(rng.integers(s.mo_num)), int(rng.integers(s.ao_num))
        e = np.zeros_like(s.mo_coef)
        e[n, k] = h
        fd = (_loss(s, w, coef=s.mo_coef + e) - _loss(s, w, coef=s.mo_coef - e)) / (2 * h)
        assert fd == pytest.approx(g["d_coef"][n, k], rel=1e-6, abs=1e-8 * g["d_coef_abs"][n, k])
    # translating everything leaves the loss unchanged
    tot = g["d_nucl"].sum(axis=0) + g["d_elec"].sum(axis=0)
    scale = g["d_nucl_abs"].sum(axis=0) + g["d_elec_abs"].sum(axis=0)
    assert np.all(np.abs(tot) <= 1e-11 * scale)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_contraction_weights_are_quadrature_normalised_primitives(l):
    """A contracted shell is the unit-norm combination sum_k a_k phi_k of
    primitives phi_k that are themselves unit-norm.  Each phi_k is normalised
    here by numerical quadrature (no closed form), so the relative weights of
    the primitives are fixed independently of the oracle's factors."""
    gam = np.array([0.3, 1.7, 9.0])
    a = np.array([0.8, 0.35, 0.6])
    s = one_shell_system(l, gam, a)
    x, w = _sinh_rule()
    pts = np.random.default_rng(l).normal(scale=0.7, size=(25, 3))
    got = oracle.ao_derivs(s, pts, B=0.0)[:, 0, 0]  # axis component x^l
    # 1-D quadrature of x^(2l) exp(-2 g x^2) and exp(-2 g x^2) gives each primitive's norm
    norms = np.array([np.sqrt(np.sum(w * x ** (2 * l) * np.exp(-2 * g * x * x)) *
                              np.sum(w * np.exp(-2 * g * x * x)) ** 2) for g in gam])
    prim = pts[:, 0:1] ** l * np.exp(-np.sum(pts ** 2, axis=1, keepdims=True) * gam[None, :]) / norms
    combo = prim @ a
    # normalise the combination by quadrature of its square (cross overlaps numerically)
    ov = 0.0
    for i in range(3):
        for j in range(3):
            gi, gj = gam[i], gam[j]
            ov += a[i] * a[j] / (norms[i] * norms[j]) * (
                np.sum(w * x ** (2 * l) * np.exp(-(gi + gj) * x * x)) *
                np.sum(w * np.exp(-(gi + gj) * x * x)) ** 2)
    np.testing.assert_allclose(got, combo / np.sqrt(ov), rtol=1e-9, atol=1e-14)
