"""Pins of the oracle's determinant and adjugate (Section 3.4) against the
permutation (Leibniz) formula, the identity A adj(A) = det(A) I, closed forms
and the singular case."""
import itertools

import numpy as np
import pytest

import oracle


def leibniz(a):
    n = a.shape[0]
    total, absum = 0.0, 0.0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        t = np.prod([a[i, perm[i]] for i in range(n)])
        total += -t if inv % 2 else t
        absum += abs(t)
    return total, absum


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_det_matches_permutation_formula(n):
    rng = np.random.default_rng(n)
    a = rng.normal(size=(6, n, n))
    det, _ = oracle.det_adj(a)
    for b in range(6):
        ref, scale = leibniz(a[b])
        assert abs(det[b] - ref) <= 1e-13 * scale


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 9])
def test_adjugate_identity(n):
    rng = np.random.default_rng(10 + n)
    a = rng.normal(size=(5, n, n))
    det, adj = oracle.det_adj(a)
    for b in range(5):
        res = a[b] @ adj[b] - det[b] * np.eye(n)
        assert np.abs(res).max() <= 1e-12 * np.abs(a[b]).max() * np.abs(adj[b]).max() * n


def test_two_by_two_closed_form_and_triangular():
    a = np.array([[[3.0, -2.0], [5.0, 7.0]]])
    det, adj = oracle.det_adj(a)
    assert det[0] == pytest.approx(31.0, rel=1e-15)
    np.testing.assert_allclose(adj[0], [[7.0, 2.0], [-5.0, 3.0]], rtol=1e-15)
    u = np.triu(np.random.default_rng(1).normal(size=(4, 4)))
    assert oracle.det_adj(u[None])[0][0] == pytest.approx(np.prod(np.diag(u)), rel=1e-13)


@pytest.mark.parametrize("n", [3, 4])
def test_singular_matrix_has_rank_one_adjugate(n):
    """A of rank n-1: det = 0, adj(A) != 0 has rank 1 and A adj(A) = 0."""
    rng = np.random.default_rng(n)
    a = rng.normal(size=(n, n))
    a[-1] = a[0] + 2.0 * a[1]
    det, adj = oracle.det_adj(a[None])
    assert abs(det[0]) <= 1e-13 * np.abs(a).max() ** n
    assert np.abs(adj[0]).max() > 1e-3
    assert np.linalg.matrix_rank(adj[0], tol=1e-10 * np.abs(adj[0]).max()) == 1
    assert np.abs(a @ adj[0]).max() <= 1e-12 * np.abs(a).max() * np.abs(adj[0]).max()
