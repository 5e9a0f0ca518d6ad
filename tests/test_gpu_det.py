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


@pytest.mark.parametrize("n", [5, 8, 16, 32])
def test_lu_path_singular_matrices_match_cofactors(n):
    """Exactly singular matrices on the LU path (a repeated row, a zero
    column: rank n - 1; two zero rows: rank n - 2): det is 0 and the adjugate
    is the oracle's transposed cofactor matrix, finite, within 1e-10 of its
    largest entry (zero for rank n - 2)."""
    rng = np.random.default_rng(300 + n)
    a = rng.normal(size=(12, n, n))
    a[0:4, 3] = a[0:4, 1]          # repeated row
    a[4:8, :, 2] = 0.0             # zero column
    a[8:12, 0] = 0.0               # two zero rows
    a[8:12, n - 1] = 0.0
    c = ctx()
    det, adj = c.det_adj(torch.from_numpy(a).cuda())
    c.close()
    det = det.cpu().numpy()
    g = adj.cpu().numpy()
    rdet, radj = oracle.det_adj(a)
    assert np.all(det == 0.0), det
    assert np.all(np.isfinite(g))
    for b in range(8):
        assert np.abs(g[b] - radj[b]).max() <= 1e-10 * np.abs(radj[b]).max(), b
    assert np.all(g[8:] == 0.0)
    assert np.abs(radj[8:]).max() <= 1e-12 * np.abs(radj[:8]).max()


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


@pytest.mark.parametrize("n,batch", [(2, 1 << 24), (3, 1 << 24), (4, 1 << 24), (16, 1 << 16)])
def test_full_size_sampled_and_adjugate_identity(n, batch):
    """The timed determinant workload at full size (standard-normal matrices
    drawn on the device): sampled matrices (the first, the last and 62 in
    between) against the oracle, and A adj(A) = det(A) I for every matrix of
    the batch.  For n <= 4 the residual bound follows the cofactor error
    bound used above (Hadamard scales); for the LU path it is the backward
    error form c n u |A| |adj| with growth allowed for, and the sampled
    comparison is scaled by the condition number."""
    c = ctx()
    g = torch.Generator(device="cuda")
    g.manual_seed(3 + n)
    A = torch.randn((batch, n, n), generator=g, device="cuda", dtype=torch.float64)
    det, adj = c.det_adj(A)
    c.close()
    assert bool(torch.isfinite(det).all()) and bool(torch.isfinite(adj).all())
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    R = (torch.bmm(A, adj) - det[:, None, None] * eye).abs()
    if n <= 4:
        rn = A.norm(dim=-1)
        ds = rn.prod(dim=-1)
        bound = 2e-13 * (n ** 0.5 * ds[:, None, None] * rn[:, :, None] / rn[:, None, :]
                         + torch.bmm(A.abs(), adj.abs())) + 1e-13 * ds[:, None, None] * eye
        assert bool((R <= bound).all())
    else:
        scale = A.norm(dim=(1, 2)) * adj.norm(dim=(1, 2))
        assert bool((R.amax(dim=(1, 2)) <= 1e-12 * scale).all())
    idx = np.unique(np.concatenate([[0, batch - 1], np.random.default_rng(n).integers(batch, size=62)]))
    a = A[torch.from_numpy(idx).cuda()].cpu().numpy()
    gd, ga = det.cpu().numpy()[idx], adj[torch.from_numpy(idx).cuda()].cpu().numpy()
    rdet, radj = oracle.det_adj(a)
    if n <= 4:
        ds, as_ = hadamard_scales(a)
        assert np.all(np.abs(gd - rdet) <= 1e-13 * ds + 1e-300)
        assert np.all(np.abs(ga - radj) <= 1e-13 * as_ + 1e-300)
    else:
        cond = np.linalg.cond(a)
        assert np.all(np.abs(gd - rdet) <= 1e-13 * n * cond * np.abs(rdet))
        err = np.abs(ga - radj).max(axis=(1, 2))
        assert np.all(err <= 1e-13 * n * cond * np.abs(radj).max(axis=(1, 2)))
