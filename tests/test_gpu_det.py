"""Batched determinant and adjugate (Section 3.4) through the C ABI vs the
oracle.  Tolerances: n <= 4 (explicit cofactors), each entry within 1e-13 of
its Hadamard scale (the product of the row norms it is built from); n >= 5
(LU with pivoting, well-conditioned inputs), 1e-11 relative."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def ctx():
    import paper_2512_16677_amd as q
    return q.Context()


def hadamard_scales(a):
    rn = np.linalg.norm(a, axis=-1)                      # [b, n]
    det_scale = np.prod(rn, axis=-1)
    adj_scale = det_scale[:, None] / np.maximum(rn, 1e-300)  # drop row i -> adj_{j i}
    return det_scale, adj_scale[:, None, :]


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_small_matrices_match_oracle(n):
    rng = np.random.default_rng(n)
    a = rng.normal(size=(1037, n, n))
    a[:20, -1] = a[:20, 0] - 0.5 * a[:20, min(1, n - 1)]  # some singular matrices
    c = ctx()
    det, adj = c.det_adj(torch.from_numpy(a).cuda())
    c.close()
    rdet, radj = oracle.det_adj(a)
    ds, as_ = hadamard_scales(a)
    assert np.all(np.abs(det.cpu().numpy() - rdet) <= 1e-13 * ds + 1e-300)
    assert np.all(np.abs(adj.cpu().numpy() - radj) <= 1e-13 * as_ + 1e-300)


@pytest.mark.parametrize("n", [5, 8, 17, 32])
def test_lu_path_matches_oracle(n):
    rng = np.random.default_rng(100 + n)
    a = rng.normal(size=(70, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)
    c = ctx()
    det, adj = c.det_adj(torch.from_numpy(a).cuda())
    c.close()
    rdet, radj = oracle.det_adj(a)
    np.testing.assert_allclose(det.cpu().numpy(), rdet, rtol=1e-11)
    g = adj.cpu().numpy()
    assert np.abs(g - radj).max() <= 1e-11 * np.abs(radj).max()


def test_det_errors_and_empty_batch():
    import paper_2512_16677_amd as q
    c = ctx()
    det, adj = c.det_adj(torch.zeros((0, 3, 3), dtype=torch.float64, device="cuda"))
    assert det.numel() == 0
    for n in (33,):
        with pytest.raises(q.QmkError) as e:
            c.det_adj(torch.zeros((2, n, n), dtype=torch.float64, device="cuda"))
        assert e.value.status == q.QMK_INVALID_ARG_BASE + 2
    c.close()
