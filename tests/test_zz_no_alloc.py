"""The allocation-free scoring entry point (gd_score_poses_noalloc) against
gd_score_poses, through the C ABI: identical integer scores and bump flags
on two calls in a row (the second smaller, so the scratch holds stale data
from the first), and the capacity limit rejected before any device work."""
import numpy as np
import pytest

from synth import configs
from tests import gpuutil
from tests.gpuutil import gpu


def _docked(g, P, ligs, q, hp, k):
    from paper_1901_06363_amd.stream import poses_from_topk
    b = g.Batch(P, ligs, q, hp=hp, top_k=k)
    r = b.dock(g.BATCHED)
    return poses_from_topk(r, ligs)


@gpu
def test_noalloc_scoring_matches_the_allocating_call():
    import torch
    g = gpuutil.gd()
    w = configs.SCREEN
    P = g.Pocket(w.pocket_points(), 0.5, w.pad)
    q = w.quaternions(64)
    for first, count, k in ((0, 400, 6), (400, 37, 3)):
        ligs = w.ligands(first, count)
        pose_lig, px, py, pz = _docked(g, P, ligs, q, w.hp, k)
        # shake the poses so that some bump and scores spread
        rng = np.random.default_rng(first)
        for t in (px, py, pz):
            t += torch.tensor(rng.normal(0, 0.6, t.numel()).astype(np.float32), device="cuda")
        S_ref, c_ref = g.score_poses(P, ligs, pose_lig, px, py, pz)
        S = torch.full((len(pose_lig),), -7, dtype=torch.int32, device="cuda")
        c = torch.full((len(pose_lig),), 9, dtype=torch.uint8, device="cuda")
        g.score_poses_noalloc(P, ligs, pose_lig, px, py, pz, S, c)
        torch.cuda.synchronize()
        assert torch.equal(S, S_ref) and torch.equal(c, c_ref), first
        assert int(c_ref.sum()) > 0 and int(c_ref.sum()) < len(pose_lig)


@gpu
def test_noalloc_rejects_tables_beyond_the_scratch():
    import torch
    g = gpuutil.gd()
    d = configs.DSE
    P = g.Pocket(d.pocket_points(), 0.5, d.pad)
    ligs = d.ligands(0, 4000)  # about 20 MB of far-pair lists, beyond the 16 MiB scratch
    pose_lig = np.arange(8)
    n_at = int(np.diff(ligs.atom_off)[:8].sum())
    xyz = [torch.zeros(n_at, dtype=torch.float32, device="cuda") for _ in range(3)]
    S = torch.full((8,), -7, dtype=torch.int32, device="cuda")
    c = torch.full((8,), 9, dtype=torch.uint8, device="cuda")
    with pytest.raises(g.GdError) as ei:
        g.score_poses_noalloc(P, ligs, pose_lig, *xyz, S, c)
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((S == -7).all()) and bool((c == 9).all())  # nothing written
