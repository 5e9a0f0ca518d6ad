"""Batched execution (persistent kernels + one HIP graph launch) against
solo runs of the same contexts and against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import rownorm_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def qmk():
    import paper_2512_16677_amd as q
    return q


def contexts(mols, mode="fp64", bits=53):
    q = qmk()
    return [q.Context.from_system(m, bits=bits, mode=mode, points_on_device=True) for m in mols]


def solo(ctx, w=None):
    mo = ctx.get_mo_vgl().clone()
    g = None if w is None else {k: v.clone() for k, v in ctx.adjoint(w).items()}
    return mo, g


def maxrel(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def mols():
    return synth.molecule_batch(n_mol=7, seed=3)


def test_batch_forward_matches_solo_and_oracle(mols):
    q = qmk()
    ctxs = contexts(mols)
    b = q.Batch(ctxs)
    outs = b.run()
    torch.cuda.synchronize()
    for m, c, o in zip(mols, ctxs, outs):
        ref, _ = solo(c)
        e = rownorm_err(o.cpu().numpy().reshape(-1, 5, m.mo_num), ref.cpu().numpy().reshape(-1, 5, m.mo_num))
        assert e.max() <= 1e-13, (m.name, e.max())
        # first walker against the oracle
        pts = m.points()[: m.elec_num]
        r = oracle.mo_vgl(m, points=pts)
        got = o.cpu().numpy().reshape(-1, 5, m.mo_num)[: m.elec_num]
        assert rownorm_err(got, r).max() <= 1e-12, m.name
    b.close()


def test_batch_replay_new_points_and_adjoint(mols):
    q = qmk()
    ctxs = contexts(mols)
    b = q.Batch(ctxs)
    ws = [torch.from_numpy(synth.adjoint_weights(m, seed=i)).cuda() for i, m in enumerate(mols)]
    b.run(ws=ws)  # first run: tiles timed, graph captured
    rng = np.random.default_rng(0)
    for rep in range(2):  # graph replays with new coordinates
        keep = []
        for m, c in zip(mols, ctxs):
            r = torch.from_numpy(m.elec_coord + rng.normal(scale=0.05, size=m.elec_coord.shape)).cuda()
            c.set_point(r)
            keep.append(r)
        outs, grads = b.run(ws=ws)
        torch.cuda.synchronize()
        for m, c, o, g, w in zip(mols, ctxs, outs, grads, ws):
            ref, rg = solo(c, w)
            assert maxrel(o, ref) <= 1e-13, m.name
            for k in ("d_coef", "d_elec", "d_nucl"):
                assert maxrel(g[k], rg[k]) <= 1e-11, (m.name, k, maxrel(g[k], rg[k]))
    b.close()


@pytest.mark.parametrize("mode,tol", [("mixed_f32", 1e-6), ("mixed_bf16x3", 1e-5)])
def test_batch_mixed_modes_match_solo(mols, mode, tol):
    q = qmk()
    ctxs = contexts(mols[:4], mode=mode)
    b = q.Batch(ctxs)
    ws = [torch.from_numpy(synth.adjoint_weights(m, seed=i)).float().cuda() for i, m in enumerate(mols[:4])]
    outs, grads = b.run(dtype=torch.float32, ws=ws)
    torch.cuda.synchronize()
    for m, c, o, g, w in zip(mols[:4], ctxs, outs, grads, ws):
        ref = c.get_mo_vgl(dtype=torch.float32)
        rg = c.adjoint(w)
        e = rownorm_err(o.cpu().numpy().reshape(-1, 5, m.mo_num), ref.cpu().numpy().reshape(-1, 5, m.mo_num))
        assert e.max() <= tol, (m.name, e.max())
        for k in ("d_coef", "d_elec", "d_nucl"):
            assert maxrel(g[k], rg[k]) <= 10 * tol, (m.name, k)
    b.close()


def test_batch_independent_of_molecule_order(mols):
    q = qmk()
    ctxs = contexts(mols)
    fwd = q.Batch(ctxs).run()
    rev = q.Batch(ctxs[::-1]).run()[::-1]
    torch.cuda.synchronize()
    for a, c in zip(fwd, rev):
        assert maxrel(a, c) <= 1e-13


def test_batch96_full_size_sampled():
    """The timed batch workload at full size (96 molecules of 4-60 atoms,
    8-128 walkers each, seed 0; forward + adjoint in one graph launch, FP64):
    every molecule's MOs and gradients equal its solo run, and the first
    walker of four sampled molecules (the smallest, the largest and two
    more) matches the oracle."""
    q = qmk()
    mols = synth.molecule_batch(96, seed=0)
    ctxs = contexts(mols)
    g = torch.Generator(device="cuda")
    g.manual_seed(99)
    ws = [torch.randn((m.walk_num, m.elec_num, 5, m.mo_num), generator=g, device="cuda",
                      dtype=torch.float64) for m in mols]
    b = q.Batch(ctxs)
    b.run(ws=ws)  # tiles timed, graph captured
    outs, grads = b.run(ws=ws)  # graph replay, as timed
    torch.cuda.synchronize()
    for m, c, o, gr, w in zip(mols, ctxs, outs, grads, ws):
        ref, rg = solo(c, w)
        assert maxrel(o, ref) <= 1e-13, m.name
        for k in ("d_coef", "d_elec", "d_nucl"):
            assert maxrel(gr[k], rg[k]) <= 1e-11, (m.name, k)
    size = [m.ao_num * m.point_num for m in mols]
    picks = sorted({int(np.argmin(size)), int(np.argmax(size)), 17, 60})
    for i in picks:
        m = mols[i]
        r = oracle.mo_vgl(m, points=m.points()[: m.elec_num])
        got = outs[i].cpu().numpy().reshape(-1, 5, m.mo_num)[: m.elec_num]
        assert rownorm_err(got, r).max() <= 1e-12, m.name
    b.close()
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("mode,tol,otol", [("mixed_f32", 1e-6, 4e-6), ("mixed_bf16x3", 1e-5, 1e-4)])
def test_batch96_mixed_full_size_sampled(mode, tol, otol):
    """The timed batch workload in the mixed modes (BF16x3: the pre-split
    planes path of every stage): every molecule's MOs and gradients equal its
    solo run within the mode's rounding (the solo products split the point
    range differently), and the first walker of four sampled molecules
    matches the oracle within the mode's bound (B = 53)."""
    q = qmk()
    mols = synth.molecule_batch(96, seed=0)
    ctxs = contexts(mols, mode=mode)
    g = torch.Generator(device="cuda")
    g.manual_seed(98)
    ws = [torch.randn((m.walk_num, m.elec_num, 5, m.mo_num), generator=g, device="cuda",
                      dtype=torch.float32) for m in mols]
    b = q.Batch(ctxs)
    b.run(dtype=torch.float32, ws=ws)  # tiles timed, graph captured
    outs, grads = b.run(dtype=torch.float32, ws=ws)  # graph replay, as timed
    torch.cuda.synchronize()
    for m, c, o, gr, w in zip(mols, ctxs, outs, grads, ws):
        ref = c.get_mo_vgl(dtype=torch.float32)
        rg = c.adjoint(w)
        e = rownorm_err(o.cpu().numpy().reshape(-1, 5, m.mo_num), ref.cpu().numpy().reshape(-1, 5, m.mo_num))
        assert e.max() <= tol, (m.name, e.max())
        for k in ("d_coef", "d_elec", "d_nucl"):
            assert maxrel(gr[k], rg[k]) <= 10 * tol, (m.name, k, maxrel(gr[k], rg[k]))
    size = [m.ao_num * m.point_num for m in mols]
    picks = sorted({int(np.argmin(size)), int(np.argmax(size)), 17, 60})
    for i in picks:
        m = mols[i]
        r = oracle.mo_vgl(m, points=m.points()[: m.elec_num])
        got = outs[i].cpu().numpy().reshape(-1, 5, m.mo_num)[: m.elec_num]
        assert rownorm_err(got, r).max() <= otol, (m.name, rownorm_err(got, r).max())
    b.close()
    for c in ctxs:
        c.close()
