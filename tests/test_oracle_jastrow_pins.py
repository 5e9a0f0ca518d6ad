"""Pins of the oracle's three-body Jastrow factor (Section 3.5): the
intermediate-matrix form of the same sum (the reformulation the paper derives),
a hand-written two-electron case, invariances and linearity in the
coefficients."""
import math

import numpy as np
import pytest

import oracle


def p_form(elec, nucl, kappa, nord, c):
    """The same J through P^{k,m}_{ia} = sum_{j != i} rt_ij^k Rt_ja^m and
    J = sum_t sum_a c[t,a] sum_i Rt_ia^((p-k+l)/2) P^{k,(p-k-l)/2}_{ia}."""
    out = []
    for x in elec:
        r = np.linalg.norm(x[:, None] - x[None], axis=2)
        rt = np.exp(-kappa * r)
        np.fill_diagonal(rt, 0.0)
        Rt = np.exp(-kappa * np.linalg.norm(x[:, None] - nucl[None], axis=2))
        J = 0.0
        for t, (p, k, l) in enumerate(oracle.een_terms(nord)):
            m = (p - k - l) // 2
            rk = rt ** k if k > 0 else (1.0 - np.eye(len(x)))
            P = rk @ (Rt ** m)                    # [elec, nucl]
            J += float(np.sum(c[t] * np.sum(Rt ** ((p - k + l) // 2) * P, axis=0)))
        out.append(J)
    return np.array(out)


def system(seed, walkers=3, ne=7, nn=3, nord=5):
    rng = np.random.default_rng(seed)
    nucl = rng.uniform(-2, 2, size=(nn, 3))
    elec = nucl[rng.integers(nn, size=(walkers, ne))] + rng.normal(size=(walkers, ne, 3))
    c = rng.normal(size=(len(oracle.een_terms(nord)), nn))
    return elec, nucl, c


@pytest.mark.parametrize("nord", [2, 3, 5, 6])
def test_pairwise_sum_equals_intermediate_matrix_form(nord):
    elec, nucl, c = system(nord, nord=nord)
    a = oracle.jastrow_een(elec, nucl, 0.8, nord, c)
    b = p_form(elec, nucl, 0.8, nord, c)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


def test_two_electrons_one_term_by_hand():
    """nord = 2 has terms (p,k,l) = (2,0,0), (2,1,1); with only c for (2,1,1):
    J = c rt_12 (Rt_1 + Rt_2) (Rt_1 Rt_2)^0."""
    assert oracle.een_terms(2) == [(2, 0, 0), (2, 1, 1)]
    elec = np.array([[[0.3, 0.0, 0.0], [0.0, 1.1, -0.4]]])
    nucl = np.zeros((1, 3))
    kappa = 0.7
    c = np.array([[0.0], [1.3]])
    r12 = math.dist(elec[0, 0], elec[0, 1])
    R1, R2 = np.linalg.norm(elec[0], axis=1)
    ref = 1.3 * math.exp(-kappa * r12) * (math.exp(-kappa * R1) + math.exp(-kappa * R2))
    assert oracle.jastrow_een(elec, nucl, kappa, 2, c)[0] == pytest.approx(ref, rel=1e-14)
    # the (2,0,0) term alone: c Rt_1 Rt_2 + c Rt_2 Rt_1 ... (l = 0 gives 1 + 1)
    c = np.array([[0.5], [0.0]])
    ref = 0.5 * 2.0 * math.exp(-kappa * R1) * math.exp(-kappa * R2)
    assert oracle.jastrow_een(elec, nucl, kappa, 2, c)[0] == pytest.approx(ref, rel=1e-14)


def test_invariances_and_linearity():
    elec, nucl, c = system(11)
    J = oracle.jastrow_een(elec, nucl, 0.9, 5, c)
    perm = np.random.default_rng(2).permutation(elec.shape[1])
    np.testing.assert_allclose(oracle.jastrow_een(elec[:, perm], nucl, 0.9, 5, c), J, rtol=1e-12)
    shift = np.array([0.4, -1.3, 2.2])
    np.testing.assert_allclose(oracle.jastrow_een(elec + shift, nucl + shift, 0.9, 5, c), J, rtol=1e-12)
    np.testing.assert_allclose(oracle.jastrow_een(elec, nucl, 0.9, 5, 2.5 * c), 2.5 * J, rtol=1e-13)
    # far away nuclei: every term carries Rt factors -> 0
    assert np.all(np.abs(oracle.jastrow_een(elec, nucl + 400.0, 0.9, 5, c)) < 1e-100)
