"""GPU parity of the docking path against the FP64 oracle (through the C ABI).

Bar: overlap counts S, bump flags, selected orientations and chosen angles
bit-exact; FP32 output coordinates within 1e-4 A of the oracle's FP64 pose.
"""
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


def _pockets(w, g):
    pts = w.pocket_points()
    return g.Pocket(pts, 0.5, 12.0), oracle.OraclePocket(pts, 0.5)


@gpu
@pytest.mark.parametrize("wname", ["single", "screen", "large"])
def test_distance_grid_equals_brute_force(g, wname):
    w = configs.ALL[wname]
    P, O = _pockets(w, g)
    inf = P.info()
    grid = P.read_grid()
    lo = np.array(inf["box_lo"])
    nx, ny, nz = inf["box_dim"]
    rng = np.random.default_rng(5)
    idx = np.stack([rng.integers(0, nx, 4000), rng.integers(0, ny, 4000), rng.integers(0, nz, 4000)], 1)
    # corners and faces of the box too
    idx = np.concatenate([idx, np.array([[0, 0, 0], [nx - 1, ny - 1, nz - 1], [0, ny - 1, nz // 2]])])
    for ix, iy, iz in idx:
        assert grid[iz, iy, ix] == O.D(ix + lo[0], iy + lo[1], iz + lo[2])
    assert inf["n_occupied"] == len(O.occupied())
    assert np.allclose(inf["centroid"], O.centroid, rtol=0, atol=0)


@gpu
@pytest.mark.parametrize("mode", [0, 1])
def test_single_ligand_full_ranking(g, mode):
    """256 orientations x 36 angles per fragment sweep, all orientations ranked."""
    w = configs.SINGLE
    P, O = _pockets(w, g)
    ligs = w.ligands()
    q = w.quaternions()
    kn = dict(hp=w.hp, top_k=256)
    b = g.Batch(P, ligs, q, **kn)
    res = b.dock(mode).host()
    orc = gpuutil.oracle_dock_batch(O, ligs, oracle.knobs(hp=w.hp), q)
    gpuutil.compare_full_ranking(res, orc, ligs)
    assert res["counters"][0] == b.poses_expected == 73984
    assert res["counters"][0] == sum(r.n_cand for r in orc)


@gpu
def test_screen_sample_parity(g):
    """A ragged sample of the screening workload (20-80 atoms, 2-12 rotatable
    bonds, 512 orientations, 15-degree steps), batched form, top-8."""
    w = configs.SCREEN
    P, O = _pockets(w, g)
    full = w.ligands(0, 1200)
    ligs = full.subset(range(0, 1200, 100))
    q = w.quaternions()
    b = g.Batch(P, ligs, q, hp=w.hp, top_k=8)
    res = b.dock(1).host()
    orc = gpuutil.oracle_dock_batch(O, ligs, oracle.knobs(hp=w.hp), q)
    gpuutil.compare_full_ranking(res, orc, ligs)
    assert res["counters"][0] == sum(r.n_cand for r in orc)


@gpu
@pytest.mark.parametrize("kn", [
    dict(hp=5, lp=90, threshold=0.3, repetitions=2),
    dict(hp=1, lp=45, threshold=0.6, refine=True),
    dict(hp=10, refine=True, repetitions=3),
    dict(hp=30, repetitions=1),
    dict(hp=2, lp=60, threshold=0.8, refine=True, repetitions=2),
])
def test_knob_settings_parity(g, kn):
    w = configs.SCREEN
    P, O = _pockets(w, g)
    ligs = w.ligands(0, 300).subset(range(0, 300, 60))
    q = synth.quaternions(11, 48)
    b = g.Batch(P, ligs, q, top_k=48, **kn)
    res = b.dock(1).host()
    orc = gpuutil.oracle_dock_batch(O, ligs, oracle.knobs(**kn), q)
    gpuutil.compare_full_ranking(res, orc, ligs)
    assert res["counters"][0] == b.poses_expected == sum(r.n_cand for r in orc)


@gpu
@pytest.mark.parametrize("mode", [0, 1])
def test_ragged_items_and_long_angle_records(g, mode):
    """Outputs are held per work item (up to 8 orientations of a ligand) and
    stored when 64 angle records or the item are complete: 37 orientations
    (a last item of 5), three repetitions (72 records per orientation for the
    ligand with 12 rotatable bonds, 12 for the one with 2, so stores fall
    inside and across orientations), against the oracle's full ranking."""
    w = configs.SCREEN
    P, O = _pockets(w, g)
    pool = w.ligands(0, 400)
    nrot = np.diff(np.asarray(pool.rot_off))
    pick = [int(np.argmax(nrot)), int(np.argmin(nrot))] + list(range(0, 400, 100))
    ligs = pool.subset(pick)
    q = synth.quaternions(23, 37)
    kn = dict(hp=30, repetitions=3)
    b = g.Batch(P, ligs, q, top_k=37, **kn)
    res = b.dock(mode).host()
    orc = gpuutil.oracle_dock_batch(O, ligs, oracle.knobs(**kn), q)
    gpuutil.compare_full_ranking(res, orc, ligs)
    assert res["counters"][0] == b.poses_expected == sum(r.n_cand for r in orc)


@gpu
def test_batched_equals_per_ligand_and_tilings(g):
    w = configs.SCREEN
    P, _ = _pockets(w, g)
    ligs = w.ligands(0, 64)
    q = w.quaternions(128)
    b = g.Batch(P, ligs, q, hp=w.hp, top_k=16)
    ref = b.dock(0).host()
    for t in [(4, 8, 4), (2, 8, 2), (8, 16, 8), (1, 32, 1), (4, 32, 8)]:
        b.set_tiling(*t)
        for mode in (0, 1):
            got = b.dock(mode).host()
            for k in ("orient", "S", "clash", "angles", "xyz", "overlap"):
                assert np.array_equal(got[k], ref[k]), (t, mode, k)
            assert got["counters"][0] == ref["counters"][0]


@gpu
def test_pairs_per_lane_on_heavy_ligands(g):
    """The heaviest ligands of the large library (most straddling pairs per
    sweep, where more pairs can survive the prune than the LDS list holds and
    the bump pass holds 1, 2, 4 or 8 pairs per lane): every tiling and both
    forms give identical results, and three of them match the oracle."""
    w = configs.LARGE
    P, O = _pockets(w, g)
    pool = w.ligands(0, 2048)
    n_atoms = np.diff(np.asarray(pool.atom_off))
    heavy = [int(i) for i in np.argsort(-n_atoms, kind="stable")[:12]]
    ligs = pool.subset(heavy)
    q = synth.quaternions(13, 32)
    b = g.Batch(P, ligs, q, hp=w.hp, top_k=32)
    ref = b.dock(1).host()
    for t in [(8, 32, 1), (8, 32, 2), (8, 32, 8), (4, 16, 8), (2, 8, 8)]:
        b.set_tiling(*t)
        for mode in (0, 1):
            got = b.dock(mode).host()
            for k in ("orient", "S", "clash", "angles", "xyz"):
                assert np.array_equal(got[k], ref[k]), (t, mode, k)
    sub = ligs.subset(range(3))
    b3 = g.Batch(P, sub, q, hp=w.hp, top_k=32)
    b3.set_tiling(8, 32, 8)
    orc = gpuutil.oracle_dock_batch(O, sub, oracle.knobs(hp=w.hp), q)
    gpuutil.compare_full_ranking(b3.dock(1).host(), orc, sub)


@gpu
def test_repeat_runs_are_identical(g):
    w = configs.SCREEN
    P, _ = _pockets(w, g)
    ligs = w.ligands(100, 32)
    q = w.quaternions(64)
    b = g.Batch(P, ligs, q, hp=w.hp, top_k=8)
    a = b.dock(1).host()
    for _ in range(3):
        c = b.dock(1).host()
        for k in ("orient", "S", "clash", "angles", "xyz"):
            assert np.array_equal(a[k], c[k])


@gpu
def test_edge_cases(g):
    """Rigid ligands (no rotatable bond), a 2-atom ligand, one orientation,
    top-1, ring ligands, atoms far outside the tabulated grid."""
    w = configs.SINGLE
    pts = w.pocket_points()
    O = oracle.OraclePocket(pts, 0.5)
    ligs = [synth.ligands(5, i, 1, 15, 60, 0, 16, 1.0).ligand(0) for i in range(6)]
    ligs.append(dict(x=np.array([0.0, 1.5], np.float32), y=np.zeros(2, np.float32), z=np.zeros(2, np.float32),
                     bonds=np.array([[0, 1]]), rot=np.zeros((0, 2), np.int32)))
    base = configs.SINGLE.ligands().ligand(0)
    ligs.append(dict(base, rot=np.zeros((0, 2), np.int32)))
    batch = synth.LigandBatch.from_list(ligs)
    for pad in (12.0, 0.0):  # pad 0: many atoms leave the tabulated box
        P = g.Pocket(pts, 0.5, pad)
        for no, k in ((1, 1), (24, 5)):
            q = synth.quaternions(3, no)
            b = g.Batch(P, batch, q, hp=15, top_k=k)
            res = b.dock(1).host()
            orc = gpuutil.oracle_dock_batch(O, batch, oracle.knobs(hp=15), q)
            gpuutil.compare_full_ranking(res, orc, batch)
            if pad == 0.0 and no == 24:
                assert res["counters"][2] > 0  # the brute-force path ran


@gpu
def test_score_poses_parity(g):
    w = configs.SCREEN
    pts = w.pocket_points()
    P = g.Pocket(pts, 0.5, 12.0)
    O = oracle.OraclePocket(pts, 0.5)
    ligs = w.ligands(0, 40)
    import torch
    rng = np.random.default_rng(3)
    pose_lig, rows = [], []
    for p in range(300):
        i = int(rng.integers(0, ligs.n))
        lig = ligs.ligand(i)
        X = np.stack([lig["x"], lig["y"], lig["z"]], 1) + pts.mean(0) + rng.normal(0, 3, 3).astype(np.float32)
        if p % 7 == 0:
            X = X * np.float32(0.6)  # squeeze: creates bumps
        if p % 11 == 0:
            X = X + np.float32(40.0)  # far outside the box
        pose_lig.append(i)
        rows.append(X.astype(np.float32))
    allx = np.concatenate(rows)
    px, py, pz = (torch.tensor(allx[:, k].copy(), device="cuda") for k in range(3))
    S, clash = g.score_poses(P, ligs, np.array(pose_lig), px, py, pz)
    S, clash = S.cpu().numpy(), clash.cpu().numpy()
    for p, (i, X) in enumerate(zip(pose_lig, rows)):
        s_ref, c_ref = oracle.score_poses(O, ligs.ligand(i), X[None, :, 0], X[None, :, 1], X[None, :, 2])
        assert S[p] == s_ref[0] and clash[p] == c_ref[0], p
    assert clash.any() and not clash.all()


@gpu
def test_invalid_inputs_write_nothing(g):
    w = configs.SINGLE
    P, _ = _pockets(w, g)
    lig = w.ligands().ligand(0)
    q = w.quaternions(8)
    bad = [
        (dict(hp=7), "integer divisor"),
        (dict(hp=10, threshold=1.5), "threshold"),
        (dict(hp=10, repetitions=0), "repetitions"),
        (dict(hp=10, top_k=9), "top_k"),
    ]
    for kn, msg in bad:
        with pytest.raises(g.GdError) as e:
            g.Batch(P, synth.LigandBatch.from_list([lig]), q, **kn)
        assert msg in str(e.value)
    L2 = dict(lig, bonds=lig["bonds"][:-1])
    with pytest.raises(g.GdError, match="disconnected"):
        g.Batch(P, synth.LigandBatch.from_list([L2]), q, hp=10, top_k=1)
    L3 = dict(lig, rot=np.array([[0, 0]]))
    with pytest.raises(g.GdError, match="rotamer"):
        g.Batch(P, synth.LigandBatch.from_list([L3]), q, hp=10, top_k=1)
    qq = q.copy()
    qq[3] *= 2
    with pytest.raises(g.GdError, match="unit quaternion"):
        g.Batch(P, synth.LigandBatch.from_list([lig]), qq, hp=10, top_k=1)
