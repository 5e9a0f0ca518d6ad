"""Pins of the oracle's MO values and electron density (Section 5.4, density of
a determinant as a sum of squared orbitals) against what the mathematics
fixes: a closed form, the electron count by quadrature, and invariance under
orthogonal mixing of equally occupied orbitals."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.test_oracle_pins import _sinh_rule, one_shell_system


@pytest.mark.parametrize("gam", [0.3, 4.0, 900.0])
def test_density_of_one_s_gaussian(gam):
    """One normalised s Gaussian as the only orbital, occupation 2:
    rho(r) = 2 (2g/pi)^(3/2) exp(-2 g r^2)."""
    r = np.array([[0.0, 0.0, 0.0], [0.02, -0.01, 0.03], [0.4, 0.1, -0.2]])
    s = one_shell_system(0, [gam], [0.6], pts=r)
    rho = oracle.density(s, np.array([2.0]), points=r, B=0.0)
    exact = 2.0 * (2 * gam / math.pi) ** 1.5 * np.exp(-2 * gam * np.sum(r ** 2, axis=1))
    np.testing.assert_allclose(rho, exact, rtol=1e-13, atol=0)


def _s_and_p_on_one_centre(gs, gp):
    """One nucleus with an s shell (exponents gs) and a p shell (exponents gp)."""
    gs, gp = np.asarray(gs, float), np.asarray(gp, float)
    rng = np.random.default_rng(1)
    return synth.System(
        name="s_and_p",
        nucl_coord=np.zeros((1, 3)),
        nucl_charge=np.array([5], dtype=np.int32),
        shell_nucleus=np.array([0, 0], dtype=np.int64),
        shell_ang_mom=np.array([0, 1], dtype=np.int32),
        shell_prim_offset=np.array([0, len(gs), len(gs) + len(gp)], dtype=np.int64),
        exponent=np.concatenate([gs, gp]),
        coefficient=rng.uniform(0.1, 1.0, size=len(gs) + len(gp)),
        mo_coef=np.eye(4),
        elec_coord=np.zeros((1, 1, 3)),
    )


def test_density_integrates_to_the_electron_count():
    """Orthonormal orbitals built from one s and one p shell on the same
    centre (s is orthogonal to p by parity, p_x, p_y, p_z are mutually
    orthogonal): phi1 = s, phi2 = (p_x + p_z)/sqrt(2), phi3 = p_y with
    occupations (2, 2, 1) integrate to 5 electrons; the numerical integral of
    rho on a tensor grid gives that count."""
    s = _s_and_p_on_one_centre([0.2, 1.5, 40.0], [0.3, 2.5])
    # AO order: s, then p_x, p_y, p_z (Cartesian order x^a y^b z^c, a descending)
    C = np.zeros((3, 4))
    C[0, 0] = 1.0
    C[1, 1] = C[1, 3] = 1.0 / math.sqrt(2.0)
    C[2, 2] = 1.0
    x, w = _sinh_rule()
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    W3 = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
    rho = oracle.density(s, np.array([2.0, 2.0, 1.0]), points=pts, B=0.0, coef=C)
    assert float(np.sum(W3 * rho)) == pytest.approx(5.0, rel=2e-9)


def test_density_invariant_under_mixing_of_equally_occupied_orbitals():
    """rho depends on the occupied space only: replacing the occupied
    orbitals by Q times them, Q orthogonal, leaves rho unchanged; orbitals of
    zero occupation do not contribute."""
    s = synth.medium(walkers=1)
    pts = s.points()[:64]
    rng = np.random.default_rng(4)
    n_occ = 12
    occ = np.zeros(s.mo_num)
    occ[:n_occ] = 2.0
    rho, rho_abs = oracle.density(s, occ, points=pts, with_abs=True)
    Q, _ = np.linalg.qr(rng.normal(size=(n_occ, n_occ)))
    C2 = s.mo_coef.copy()
    C2[:n_occ] = Q @ s.mo_coef[:n_occ]
    C2[n_occ:] = rng.normal(size=C2[n_occ:].shape)  # virtual orbitals changed freely
    rho2 = oracle.density(s, occ, points=pts, coef=C2)
    assert np.all(np.abs(rho2 - rho) <= 1e-12 * rho_abs)
    assert np.all(rho > 0)


def test_mo_value_is_the_value_row():
    """mo_value is the value component of mo_vgl, which the contraction pins
    cover; here only the slicing is checked on a tiny system."""
    s = synth.tiny_system([0, 1, 2], n_prim=2, seed=1, walkers=2, elec=3)
    v = oracle.mo_value(s)
    full = oracle.mo_vgl(s)
    assert v.shape == (s.point_num, s.mo_num)
    np.testing.assert_array_equal(v, full[:, 0, :])
