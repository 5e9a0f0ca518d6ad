"""Pins of `oracle.adjoint_products`, the oracle's gradients with the long
sums (over MOs, and over points and components) taken as library matrix
products, point chunk by point chunk.  It is the form the full-size parity
tests use, so it is pinned to the literal `oracle.adjoint` (itself pinned by
finite differences, the sum rule and the W^T ao identity) and, directly, to
the sum rule and to finite differences of the oracle's forward pass."""
import math

import numpy as np
import pytest

import oracle
import synth

GRADS = ("d_coef", "d_elec", "d_nucl")


def rel_to_abs(got, ref, ref_abs):
    return float(np.max(np.abs(got - ref) / np.maximum(ref_abs, 1e-300)))


@pytest.mark.parametrize("system,chunk", [("water_like", 7), ("water_like", None),
                                          ("tiny_spdf", 3), ("medium1", 101)])
@pytest.mark.parametrize("B", [53.0, 24.0])
def test_equals_literal_adjoint(system, chunk, B):
    """Same gradients and absolute sums as the literal loops (to rounding),
    with ragged point chunks; the forward rows equal oracle.mo_vgl."""
    s = {"water_like": lambda: synth.water_like(walkers=4),
         "tiny_spdf": lambda: synth.tiny_system([0, 1, 2, 3], walkers=3),
         "medium1": lambda: synth.medium(walkers=1)}[system]()
    w = synth.adjoint_weights(s, seed=8)
    lit = oracle.adjoint(s, w, B=B)
    got = oracle.adjoint_products(s, w, B=B, with_mo=True, chunk=chunk)
    for k in GRADS:
        assert got[k].shape == lit[k].shape
        assert rel_to_abs(got[k], lit[k], lit[k + "_abs"]) <= 1e-13, k
        assert rel_to_abs(got[k + "_abs"], lit[k + "_abs"], lit[k + "_abs"]) <= 1e-13, k
    mo = oracle.mo_vgl(s, B=B)
    err = np.max(np.abs(got["mo"] - mo), axis=-1) / np.maximum(np.max(np.abs(mo), axis=-1), 1e-300)
    assert float(err.max()) <= 1e-13


def test_sum_rule_and_finite_differences():
    """Translating nuclei and electrons together leaves the loss unchanged,
    and central differences of the forward pass reproduce sampled entries."""
    s = synth.water_like(walkers=2)
    w = synth.adjoint_weights(s, seed=3).reshape(-1, 5, s.mo_num)
    g = oracle.adjoint_products(s, w, B=0.0, chunk=5)
    tot = g["d_nucl"].sum(axis=0) + g["d_elec"].sum(axis=0)
    scale = g["d_nucl_abs"].sum(axis=0) + g["d_elec_abs"].sum(axis=0)
    assert np.all(np.abs(tot) <= 1e-11 * scale)

    pts = s.points()
    h = 1e-5

    def loss(points=None, nucl=None, coef=None):
        import copy
        t = s
        if nucl is not None:
            t = copy.copy(s)
            t.nucl_coord = nucl
        mo = oracle.mo_vgl(t, points=pts if points is None else points, coef=coef, B=0.0)
        return math.fsum((w * mo).ravel())

    rng = np.random.default_rng(4)
    for _ in range(6):
        p, i = int(rng.integers(pts.shape[0])), int(rng.integers(3))
        e = np.zeros_like(pts)
        e[p, i] = h
        fd = (loss(points=pts + e) - loss(points=pts - e)) / (2 * h)
        assert fd == pytest.approx(g["d_elec"][p, i], rel=1e-6, abs=1e-6 * g["d_elec_abs"][p, i])
    for A in range(s.nucl_num):
        e = np.zeros_like(s.nucl_coord)
        e[A, 1] = h
        fd = (loss(nucl=s.nucl_coord + e) - loss(nucl=s.nucl_coord - e)) / (2 * h)
        assert fd == pytest.approx(g["d_nucl"][A, 1], rel=1e-6, abs=1e-6 * g["d_nucl_abs"][A, 1])
    for _ in range(4):
        n, k = int(rng.integers(s.mo_num)), int(rng.integers(s.ao_num))
        e = np.zeros_like(s.mo_coef)
        e[n, k] = h
        fd = (loss(coef=s.mo_coef + e) - loss(coef=s.mo_coef - e)) / (2 * h)
        assert fd == pytest.approx(g["d_coef"][n, k], rel=1e-6, abs=1e-8 * g["d_coef_abs"][n, k])


def test_chunking_does_not_change_electron_gradients():
    """Electron gradients and forward rows are per point: every chunking gives
    them bit for bit; the point sums (dC, nuclear gradients) agree to rounding."""
    s = synth.water_like(walkers=6)
    w = synth.adjoint_weights(s, seed=5)
    a = oracle.adjoint_products(s, w, with_mo=True, chunk=1)
    b = oracle.adjoint_products(s, w, with_mo=True, chunk=13)
    np.testing.assert_array_equal(a["d_elec"], b["d_elec"])
    np.testing.assert_array_equal(a["mo"], b["mo"])
    for k in ("d_coef", "d_nucl"):
        assert rel_to_abs(a[k], b[k], b[k + "_abs"]) <= 1e-14
