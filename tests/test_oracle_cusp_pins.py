"""Pins of the oracle's MO cusp correction (Section 3.3) against what the
construction must satisfy, checked numerically and not by re-typing its
formulas: the electron-nucleus cusp of the corrected orbital (finite
differences around the nucleus), continuity of value, gradient and Laplacian
across the sphere, and no change outside the spheres.

Reading (the paper names continuity of values and gradients plus the cusp
condition for four coefficients): the fourth condition is continuity of the
second radial derivative, so that the Laplacian of mo_vgl is continuous."""
import numpy as np
import pytest

import oracle
import synth


def system():
    s = synth.water_like(walkers=1)
    return s, np.array([8.0, 1.0, 1.0]), np.array([0.25, 0.15, 0.15])


def test_cusp_condition_at_each_nucleus():
    """Spherical average of the radial derivative at R_A equals -Z_A times
    the corrected orbital at R_A: one-sided differences along +-x, +-y, +-z
    (the p-type and off-centre parts cancel between opposite directions),
    Richardson-extrapolated over steps h and h/2 to remove the O(h) term
    h lap(phi)/6 of the smooth part."""
    s, z, rc = system()
    h = 1e-5
    dirs = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    for A in range(s.nucl_num):
        R = s.nucl_coord[A]
        pts = np.concatenate([R[None, :], R + h * dirs, R + 0.5 * h * dirs])
        v = oracle.mo_vgl_cusp(s, z, rc, points=pts)[:, 0, :]  # [13, mo]
        d1 = np.mean((v[1:7] - v[0]) / h, axis=0)
        d2 = np.mean((v[7:13] - v[0]) / (0.5 * h), axis=0)
        slope = 2.0 * d2 - d1
        scale = np.abs(z[A] * v[0]) + np.abs(slope) + 1e-3 * np.abs(v).max()
        np.testing.assert_array_less(np.abs(slope + z[A] * v[0]), 1e-6 * scale)


def test_corrected_orbital_is_smooth_across_the_sphere():
    """Value, gradient and Laplacian just inside and just outside r_A agree
    (the outside values are the uncorrected MOs)."""
    s, z, rc = system()
    rng = np.random.default_rng(3)
    eps = 1e-9
    for A in range(s.nucl_num):
        e = rng.normal(size=(4, 3))
        e /= np.linalg.norm(e, axis=1, keepdims=True)
        inner = s.nucl_coord[A] + rc[A] * (1 - eps) * e
        outer = s.nucl_coord[A] + rc[A] * (1 + eps) * e
        a = oracle.mo_vgl_cusp(s, z, rc, points=inner)
        b = oracle.mo_vgl_cusp(s, z, rc, points=outer)
        np.testing.assert_array_equal(b, oracle.mo_vgl_cusp(s, z, np.zeros(3), points=outer))
        scale = np.abs(b).max(axis=2, keepdims=True)
        assert np.all(np.abs(a - b) <= 1e-6 * scale)


def test_no_change_outside_the_spheres_or_without_radii():
    s, z, rc = system()
    pts = s.points()
    r = np.linalg.norm(pts[:, None, :] - s.nucl_coord[None], axis=2)
    outside = np.all(r >= rc[None, :], axis=1)
    assert outside.sum() > 0
    plain = oracle.mo_vgl(s, points=pts)
    got = oracle.mo_vgl_cusp(s, z, rc, points=pts)
    np.testing.assert_allclose(got[outside], plain[outside], rtol=1e-13, atol=1e-13 * np.abs(plain).max())
    np.testing.assert_allclose(oracle.mo_vgl_cusp(s, z, np.zeros(3), points=pts), plain,
                               rtol=1e-13, atol=1e-13 * np.abs(plain).max())


def test_s_only_orbital_becomes_the_polynomial():
    """With one s shell on one nucleus and that AO as the MO, phi - phi^s is
    zero, so inside the sphere the corrected orbital is the cubic itself:
    its value at the nucleus is f0 and its slope there is -Z f0."""
    from tests.test_oracle_pins import one_shell_system
    s = one_shell_system(0, [0.4, 3.0, 50.0], [0.3, 0.5, 0.2])
    z, rc = np.array([2.0]), np.array([0.4])
    f = oracle.cusp_coefficients(s, z, rc)[0][0]
    assert f[1] == pytest.approx(-z[0] * f[0], rel=1e-12)
    v = oracle.mo_vgl_cusp(s, z, rc, points=np.zeros((1, 3)))[0, 0, 0]
    assert v == pytest.approx(f[0], rel=1e-14)
