"""GPU parity of the continuous Eq. 1 scorer (gd_overlap_continuous) against
the FP64 oracle.  Both sides widen the same FP32 coordinates, form each
squared distance with the same two fused multiply-adds, take exact minima and
sum each pose's atoms in index order, so every per-atom minimum, per-pose sum
and overlap must agree bit for bit."""
import numpy as np
import pytest

import oracle
from synth import configs
from tests import gpuutil
from tests.gpuutil import gpu


@pytest.fixture(scope="module")
def g():
    return gpuutil.gd()


def _run(g, P, counts, X):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda() if len(X) else torch.zeros((0, 3)).cuda()
    px, py, pz = (t[:, a].contiguous() for a in range(3))
    m, s, o = g.overlap_continuous(P, counts, px, py, pz)
    torch.cuda.synchronize()
    return m.cpu().numpy(), s.cpu().numpy(), o.cpu().numpy()


def _oracle(O, counts, X):
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    ms, ss, os_ = [], [], []
    for p in range(len(counts)):
        s, m, o = O.overlap_continuous(np.asarray(X[off[p]:off[p + 1]], np.float32).astype(np.float64))
        ms.append(m)
        ss.append(s)
        os_.append(o)
    return (np.concatenate(ms) if ms else np.zeros(0)), np.array(ss), np.array(os_)


def _same(a, b):
    assert a.shape == b.shape
    assert np.array_equal(a, b, equal_nan=True), np.nonzero(~((a == b) | (np.isnan(a) & np.isnan(b))))[0][:10]


@gpu
@pytest.mark.parametrize("seed", [0, 1])
def test_overlap_ragged_multi_block(g, seed):
    # ragged poses (an empty one, a one-atom one) over several 1,024-atom
    # blocks and a ragged tail; atoms spread inside and around the pocket
    w = configs.SINGLE
    pts = w.pocket_points()
    P, O = g.Pocket(pts, 0.5, 12.0), oracle.OraclePocket(pts, 0.5)
    rng = np.random.default_rng(seed)
    counts = np.concatenate([[0, 1], rng.integers(20, 81, size=60), [0, 128]])
    n = int(counts.sum())
    assert n > 3 * 1024
    X = (rng.normal(size=(n, 3)) * 9 + np.asarray(pts, np.float64).mean(0)).astype(np.float32)
    got = _run(g, P, counts, X)
    exp = _oracle(O, counts, X)
    for a, b in zip(got, exp):
        _same(a, b)
    assert np.isnan(got[2][0]) and got[1][0] == 0.0  # empty pose: sum 0, overlap NaN


@gpu
def test_overlap_edge_cases(g):
    import torch
    w = configs.SINGLE
    pts = np.asarray(w.pocket_points(), np.float32)
    P, O = g.Pocket(pts, 0.5, 12.0), oracle.OraclePocket(pts, 0.5)
    # no poses
    e = torch.zeros(0, dtype=torch.float32, device="cuda")
    m, s, o = g.overlap_continuous(P, [], e, e, e)
    assert m.numel() == 0 and s.numel() == 0 and o.numel() == 0
    # every atom on a pocket point: sum 0, overlap +inf; an atom far away
    X = np.vstack([pts[:5], pts[7:9], [[900.0, -900.0, 900.0]]]).astype(np.float32)
    counts = [5, 2, 1]
    got = _run(g, P, counts, X)
    exp = _oracle(O, counts, X)
    for a, b in zip(got, exp):
        _same(a, b)
    assert got[1][0] == 0.0 and np.isinf(got[2][0]) and np.isinf(got[2][1])
    # a pose of every size 1..128 in one call (odd tails in every position)
    rng = np.random.default_rng(5)
    counts = np.arange(1, 129)
    X = (rng.normal(size=(int(counts.sum()), 3)) * 6).astype(np.float32)
    got = _run(g, P, counts, X)
    exp = _oracle(O, counts, X)
    for a, b in zip(got, exp):
        _same(a, b)


@gpu
def test_overlap_rejects_bad_arguments(g):
    import torch
    w = configs.SINGLE
    P = g.Pocket(w.pocket_points(), 0.5, 12.0)
    x = torch.zeros(4, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        g.overlap_continuous(P, [5], x, x, x)  # coordinate rows missing
    with pytest.raises(ValueError):
        g.overlap_continuous(P, [-1, 5], x, x, x)
    with pytest.raises(TypeError):
        g.overlap_continuous(P, [4], x.double(), x.double(), x.double())


@gpu
def test_overlap_screen_topk_full_size_sampled(g):
    """Every top-8 pose of the 10,000-ligand screen (the rescoring launch the
    benchmark times); 200 sampled poses against the oracle."""
    import torch
    from paper_1901_06363_amd import stream
    w = configs.SCREEN
    pts = w.pocket_points()
    P, O = g.Pocket(pts, 0.5, 20.0), oracle.OraclePocket(pts, 0.5)
    ligs = w.ligands()
    b = g.Batch(P, ligs, w.quaternions(), hp=w.hp, top_k=w.top_k)
    res = b.dock(g.BATCHED)
    pose_lig, px, py, pz = stream.poses_from_topk(res, ligs)
    counts = np.diff(np.asarray(ligs.atom_off))[pose_lig]
    m, s, o = g.overlap_continuous(P, counts, px, py, pz)
    torch.cuda.synchronize()
    m, s, o = m.cpu().numpy(), s.cpu().numpy(), o.cpu().numpy()
    X = torch.stack([px, py, pz], 1).cpu().numpy()
    off = np.concatenate([[0], np.cumsum(counts)])
    rng = np.random.default_rng(11)
    for p in rng.choice(len(counts), 200, replace=False):
        so, mo, oo = O.overlap_continuous(X[off[p]:off[p + 1]].astype(np.float64))
        assert s[p] == so and o[p] == oo, p
        assert np.array_equal(m[off[p]:off[p + 1]], mo), p
    assert np.all(np.isfinite(s)) and np.all(s > 0)
