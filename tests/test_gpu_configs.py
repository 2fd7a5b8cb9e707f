"""GPU parity on the workloads at their real sizes, against the FP64 oracle.

Each workload runs in the launch configuration the benchmark uses (batched
persistent kernel, default tiling, distance-grid pad 20 A) over the whole
ligand set; the oracle checks sampled ligands one by one (full ranking of
every orientation: orientation, S, clash, chosen angles, coordinates), and
the per-ligand launches must return identical results to the batched form.

  screen   10,000 ligands x 512 orientations, 15-degree steps
  grid     the screen stream extended to 100,000 ligands x 4 pockets x knob
           grid {64, 256, 1024} orientations x {30, 15, 10} degrees
  large    1,000,000-ligand stream (rings, up to 120 atoms, 16 rotamers) in
           chunks of 65,536, top-8 refined on the density surrogate
  refine   4,096 ligands x top-64 poses, 50 ascent steps
"""
import numpy as np
import pytest

import oracle
import synth
from synth import configs
from tests import gpuutil
from tests.gpuutil import gpu

PAD = 20.0


@pytest.fixture(scope="module")
def g():
    return gpuutil.gd()


def _csr(xyz, ligs, k):
    """Rows (atoms of pose 0 of ligand 0, pose 1 of ligand 0, ...) of a host
    (n, k, max_atoms, 3) pose array."""
    nat = np.diff(ligs.atom_off)
    return np.concatenate([xyz[i, kk, :nat[i]] for i in range(len(nat)) for kk in range(k)])


def _check_refined(O, ligs, pose_lig, S0, c0, X_in, X_out, S, clash, acc, rng, n_sample=16):
    """Acceptance rule of the refinement on every pose.  A rejected pose comes
    back bit for bit and carries the exact score of its FP32 coordinates; that
    score equals the docking score (FP64 pose) except where rounding the pose to
    FP32 moved an atom across a cell face or the bump distance, which the oracle
    decides pose by pose.  An accepted pose is clash-free and scores strictly
    below its input."""
    off = np.concatenate([[0], np.cumsum(np.diff(ligs.atom_off)[pose_lig])])
    acc = acc.astype(bool)
    rows_acc = np.repeat(acc, np.diff(off))
    assert np.array_equal(X_out[~rows_acc], X_in[~rows_acc])
    assert not np.any(clash[acc])

    def oscore(p, X):
        sl = X[off[p]:off[p + 1]]
        Sx, cx = oracle.score_poses(O, ligs.ligand(int(pose_lig[p])), sl[None, :, 0], sl[None, :, 1], sl[None, :, 2])
        return int(Sx[0]), bool(cx[0])

    moved = np.nonzero(~acc & ((S != S0) | (clash != c0)))[0]
    assert len(moved) <= max(8, len(S) // 100), len(moved)
    for p in moved:
        assert oscore(p, X_in) == (int(S[p]), bool(clash[p])), p
    for p in rng.choice(np.nonzero(acc)[0], min(n_sample, int(acc.sum())), replace=False):
        assert oscore(p, X_out) == (int(S[p]), False), p
        assert S[p] < oscore(p, X_in)[0], p
    for p in rng.choice(len(S), n_sample, replace=False):
        assert oscore(p, X_out) == (int(S[p]), bool(clash[p])), p


def _assert_same(a, b, keys=("orient", "S", "clash", "angles", "xyz", "overlap")):
    for k in keys:
        assert np.array_equal(a[k], b[k]), k


@gpu
def test_screen_full_size_sampled(g):
    """All 10,000 screening ligands in one batched call; every 100th ligand
    against the oracle."""
    w = configs.SCREEN
    pts = w.pocket_points()
    P, O = g.Pocket(pts, 0.5, PAD), oracle.OraclePocket(pts, 0.5)
    ligs = w.ligands()
    q = w.quaternions()
    b = g.Batch(P, ligs, q, hp=w.hp, top_k=w.top_k)
    res = b.dock(g.BATCHED).host()
    assert res["counters"][0] == b.poses_expected == 1722466304
    idx = list(range(0, ligs.n, 100))
    sub = ligs.subset(idx)
    orc = gpuutil.oracle_dock_batch(O, sub, oracle.knobs(hp=w.hp), q)
    picked = {k: v[idx] for k, v in res.items() if k != "counters"}
    gpuutil.compare_full_ranking(picked, orc, sub)


@gpu
@pytest.mark.parametrize("pk", [0, 1, 2, 3])
def test_grid_knob_points(g, pk):
    """Every (orientations, step) point of the knob grid on one pocket: 128
    ligands spread over the 100,000-ligand stream, batched == per-ligand, and
    16 of them (a different 16 at every point) against the oracle."""
    w = configs.GRID
    pts = w.pocket_points(pk)
    P, O = g.Pocket(pts, 0.5, PAD), oracle.OraclePocket(pts, 0.5)
    idx = np.linspace(0, w.n_ligands - 1, 128).astype(int)
    ligs = synth.LigandBatch.from_list([w.ligands(int(i), 1).ligand(0) for i in idx])
    for n_o in w.extra["orient_grid"]:
        q = synth.quaternions(w.quat_seed, n_o)
        for hp in w.extra["step_grid"]:
            b = g.Batch(P, ligs, q, hp=hp, top_k=w.top_k)
            rb = b.dock(g.BATCHED).host()
            rp = b.dock(g.PER_LIGAND).host()
            _assert_same(rb, rp)
            assert rb["counters"][0] == rp["counters"][0] == b.poses_expected
            rng = np.random.default_rng(1000 * pk + 10 * hp + n_o)
            pick = sorted(rng.choice(ligs.n, 16, replace=False).tolist())
            sub = ligs.subset(pick)
            orc = gpuutil.oracle_dock_parallel(pts, sub, oracle.knobs(hp=hp), q)
            gpuutil.compare_full_ranking({k: v[pick] for k, v in rb.items() if k != "counters"}, orc, sub)


@gpu
def test_grid_full_stream_heaviest_point(g):
    """All 100,000 ligands of the grid stream against the largest pocket at the
    heaviest knob point (1024 orientations, 10-degree steps); 16 ligands
    spread over the stream against the oracle."""
    w = configs.GRID
    pts = w.pocket_points(3)
    P, O = g.Pocket(pts, 0.5, PAD), oracle.OraclePocket(pts, 0.5)
    ligs = w.ligands()
    q = synth.quaternions(w.quat_seed, 1024)
    b = g.Batch(P, ligs, q, hp=10, top_k=w.top_k)
    res = b.dock(g.BATCHED).host()
    assert res["counters"][0] == b.poses_expected
    idx = [int(i) for i in np.linspace(0, ligs.n - 1, 16)]
    sub = ligs.subset(idx)
    orc = gpuutil.oracle_dock_batch(O, sub, oracle.knobs(hp=10), q)
    gpuutil.compare_full_ranking({k: v[idx] for k, v in res.items() if k != "counters"}, orc, sub)


@gpu
def test_large_stream_chunks_with_refinement(g):
    """The large library streamed in chunks of 65,536 (one full chunk and the
    start of the next) with top-8 refinement: 8 ligands per chunk and 8 ring
    ligands of the first chunk against the oracle; every refined pose obeys
    the acceptance rule and sampled refined poses score as the oracle says."""
    from paper_1901_06363_amd.stream import screen
    w = configs.LARGE
    r = configs.REFINE.extra
    pts = w.pocket_points()
    P = g.Pocket(pts, 0.5, PAD, blur_sigma=r["blur_sigma"], blur_h=r["blur_h"])
    O = oracle.OraclePocket(pts, 0.5)
    q = w.quaternions()
    ropt = dict(steps=r["steps"], lr_t=r["lr_t"], lr_q=r["lr_q"], lr_tau=r["lr_tau"], max_dt=r["max_dt"],
                max_dtau=r["max_dtau"])
    n = w.chunk + 4096
    kn = oracle.knobs(hp=w.hp)
    seen = 0
    for item in screen(P, w.ligands, n, q, chunk=w.chunk, refine_poses=ropt, hp=w.hp, top_k=w.top_k):
        ligs, res = item["ligands"], item["result"]
        assert res["counters"][0] == item["poses"]
        rng = np.random.default_rng(item["first"])
        idx = sorted(set(rng.choice(ligs.n, 8, replace=False).tolist()))
        if item["first"] == 0:
            # ring ligands carry a ring closure: more bonds than atoms - 1
            ring = [i for i in range(ligs.n)
                    if (ligs.bond_off[i + 1] - ligs.bond_off[i]) > ligs.n_atoms(i) - 1][:8]
            assert len(ring) == 8
            idx = sorted(set(idx + ring))
        sub = ligs.subset(idx)
        orc = gpuutil.oracle_dock_batch(O, sub, kn, q)
        gpuutil.compare_full_ranking({k: v[idx] for k, v in res.items() if k != "counters"}, orc, sub)
        # refinement: acceptance rule on every pose, oracle rescoring on samples
        rf = item["refine"]
        _check_refined(O, ligs, rf["pose_lig"], res["S"].reshape(-1), res["clash"].reshape(-1),
                       _csr(res["xyz"], ligs, w.top_k), rf["xyz"], rf["S"], rf["clash"], rf["accepted"], rng)
        seen += 1
    assert seen == 2


@gpu
def test_refine_full_size_sampled(g):
    """4,096 ligands x top-64 docked poses, 50 ascent steps: the acceptance
    rule on every pose, exact rescoring of sampled poses against the oracle,
    and sampled ascent trajectories against the FP64 oracle ascent."""
    import torch
    from paper_1901_06363_amd.stream import poses_from_topk
    w = configs.REFINE
    e = w.extra
    pts = w.pocket_points()
    P = g.Pocket(pts, 0.5, w.pad, blur_sigma=e["blur_sigma"], blur_h=e["blur_h"])
    O = oracle.OraclePocket(pts, 0.5)
    OB = oracle.OracleBlur(O, e["blur_sigma"], 4.0, e["blur_h"])
    ligs = w.ligands()
    b = g.Batch(P, ligs, w.quaternions(), hp=w.hp, top_k=w.top_k)
    r = b.dock(g.BATCHED)
    h = r.host()
    pose_lig, px, py, pz = poses_from_topk(r, ligs)
    X0 = torch.stack([px, py, pz], 1).cpu().numpy()
    kw = dict(steps=e["steps"], lr_t=e["lr_t"], lr_q=e["lr_q"], lr_tau=e["lr_tau"], max_dt=e["max_dt"],
              max_dtau=e["max_dtau"])
    out = g.refine(P, ligs, pose_lig, px, py, pz, want_iterate=True, **kw)
    S, clash, acc = (out[k].cpu().numpy() for k in ("S", "clash", "accepted"))
    it = torch.stack(out["iterate"], 1).cpu().numpy()
    Xr = torch.stack([px, py, pz], 1).cpu().numpy()
    assert len(S) == 4096 * 64
    rng = np.random.default_rng(9)
    _check_refined(O, ligs, pose_lig, h["S"].reshape(-1), h["clash"].reshape(-1), X0, Xr, S, clash, acc, rng,
                   n_sample=48)
    off = np.concatenate([[0], np.cumsum(np.diff(ligs.atom_off)[pose_lig])])
    rows_acc = np.repeat(acc.astype(bool), np.diff(off))
    assert np.array_equal(Xr[rows_acc], it[rows_acc])
    # trajectories: FP32 ascent vs the FP64 oracle ascent from the same input
    # pose, within 1e-3 A unless the paths part at a certified face crossing
    rms, certified = [], []
    for p in rng.choice(len(pose_lig), 12, replace=False):
        li = int(pose_lig[p])
        sl = slice(off[p], off[p + 1])
        _, Xref, _ = OB.refine(ligs.ligand(li), X0[sl].astype(np.float64), **kw)
        r = np.sqrt(np.mean(np.sum((it[sl].astype(np.float64) - Xref) ** 2, axis=1)))
        rms.append(r)
        if r > 1e-3:
            def gpu_iterate(k, li=li, sl=sl):
                q = [torch.tensor(X0[sl, a].copy(), device="cuda") for a in range(3)]
                o = g.refine(P, ligs, np.array([li]), *q, want_iterate=True, **dict(kw, steps=k))
                return torch.stack(o["iterate"], 1).cpu().numpy()
            why, info = gpuutil.certify_split(OB, ligs.ligand(li), X0[sl], gpu_iterate, e["steps"],
                                              float(np.float32(e["blur_h"])), **{k: v for k, v in kw.items()
                                                                                if k != "steps"})
            assert why, ("uncertified split", int(p), info)
            certified.append((int(p), why, info["step"]))
    rms = np.array(rms)
    print("sampled trajectories: median RMSD %.2e, %d certified split(s) (pose, reason, step): %s"
          % (np.median(rms), len(certified), certified))
    assert np.median(rms) < 1e-5


@gpu
def test_autotune_keeps_results_and_caches(g, tmp_path):
    w = configs.SCREEN
    P = g.Pocket(w.pocket_points(), 0.5, PAD)
    ligs = w.ligands(0, 256)
    b = g.Batch(P, ligs, w.quaternions(), hp=w.hp, top_k=w.top_k)
    ref = b.dock(g.BATCHED).host()
    cache = str(tmp_path / "tiles.txt")
    t1 = b.autotune(reps=1, cache_path=cache)
    assert t1[0] in (1, 2, 4, 8) and t1[1] in (8, 16, 32) and t1[2] in (1, 2, 4, 8)
    assert b.tiling() == t1
    _assert_same(b.dock(g.BATCHED).host(), ref)
    b2 = g.Batch(P, ligs, w.quaternions(), hp=w.hp, top_k=w.top_k)
    assert b2.autotune(reps=1, cache_path=cache) == t1  # served from the cache
    _assert_same(b2.dock(g.PER_LIGAND).host(), ref)
