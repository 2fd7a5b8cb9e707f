"""GPU parity of the overlap landscapes (gd_sweep_profile, peak analysis of
Section III-B) against the oracle: at every ranked pose, every rotamer side
turned by every multiple of the step, whole-ligand S and feasibility bit for
bit, and the side sizes."""
import numpy as np
import pytest

import oracle
import synth
from synth import configs
from tests import gpuutil
from tests.gpuutil import gpu


@pytest.fixture(scope="module")
def g():
    return gpuutil.gd()


@gpu
@pytest.mark.parametrize("knobs,step", [(dict(hp=10, repetitions=2), 3),
                                        (dict(hp=5, lp=90, threshold=0.4, repetitions=1, refine=True), 1)])
def test_profile_matches_oracle(g, knobs, step):
    import torch
    pts = configs.SINGLE.pocket_points()
    P, O = g.Pocket(pts, 0.5, 12.0), oracle.OraclePocket(pts, 0.5)
    ligs = synth.ligands(51, 0, 6, 14, 40, 1, 5, 0.0)
    q = synth.quaternions(8, 6)
    B = g.Batch(P, ligs, q, top_k=2, **knobs)
    res = B.dock(g.BATCHED)
    S, f, sz = g.sweep_profile(P, B, res, step=step)
    torch.cuda.synchronize()
    S, f, sz = S.cpu().numpy(), f.cpu().numpy(), sz.cpu().numpy()
    h = res.host()
    kn = oracle.knobs(**knobs)
    na = 360 // step
    for i in range(ligs.n):
        lig = ligs.ligand(i)
        r = oracle.dock(O, lig, kn, q)
        nr = ligs.n_rot(i)
        for kk in range(2):
            o = int(h["orient"][i, kk])
            for rr in range(B.max_rot):
                for side in (0, 1):
                    if rr >= nr:
                        assert not S[i, kk, rr, side].any() and not f[i, kk, rr, side].any()
                        assert sz[i, kk, rr, side] == 0
                        continue
                    size, So, fo = oracle.sweep_profile(O, lig, r.xyz[o], rr, side, step=step)
                    assert sz[i, kk, rr, side] == size, (i, kk, rr, side)
                    assert np.array_equal(S[i, kk, rr, side], So), (i, kk, rr, side)
                    assert np.array_equal(f[i, kk, rr, side] != 0, fo), (i, kk, rr, side)
                    assert len(So) == na


@gpu
def test_profile_guards(g):
    import torch
    pts = configs.SINGLE.pocket_points()
    P = g.Pocket(pts, 0.5, 12.0)
    ligs = synth.ligands(52, 0, 3, 14, 30, 1, 3, 0.0)
    B = g.Batch(P, ligs, synth.quaternions(9, 4), hp=10, top_k=1)
    res = B.alloc_outputs()
    res.recs.fill_(-1)  # no docking call: orientations out of range
    S, f, sz = g.sweep_profile(P, B, res, step=10)
    torch.cuda.synchronize()
    assert not S.any().item() and not f.any().item() and not sz.any().item()
    with pytest.raises(ValueError):
        g.sweep_profile(P, B, res, step=7)


@gpu
def test_profile_peaks_workload_sampled(g):
    """The peak-analysis launch (2,000 exploration ligands at the baseline
    knobs, 1-degree landscapes of every side at the best pose); 5 sampled
    ligands against the oracle, every rotamer side."""
    import torch
    from paper_1901_06363_amd import dse
    w = configs.DSE
    pts = w.pocket_points()
    P, O = g.Pocket(pts, 0.5, w.pad), oracle.OraclePocket(pts, 0.5)
    ligs = w.ligands(0, 2000)
    q = w.quaternions()
    b = dse.BASE_KNOBS
    B = g.Batch(P, ligs, q, top_k=1, **b)
    res = B.dock(g.BATCHED)
    S, f, sz = g.sweep_profile(P, B, res, step=1)
    torch.cuda.synchronize()
    S, f, sz = S.cpu().numpy(), f.cpu().numpy(), sz.cpu().numpy()
    h = res.host()
    kn = oracle.knobs(**b)
    rng = np.random.default_rng(4)
    for i in rng.choice(ligs.n, 5, replace=False):
        lig = ligs.ligand(int(i))
        o = int(h["orient"][i, 0])
        Xo = oracle.dock(O, lig, kn, q[o:o + 1]).xyz[0]
        for rr in range(ligs.n_rot(int(i))):
            for side in (0, 1):
                size, So, fo = oracle.sweep_profile(O, lig, Xo, rr, side, step=1)
                assert sz[i, 0, rr, side] == size
                assert np.array_equal(S[i, 0, rr, side], So), (i, rr, side)
                assert np.array_equal(f[i, 0, rr, side] != 0, fo), (i, rr, side)
