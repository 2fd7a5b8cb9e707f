"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage or fact it relies on.  None of them re-types the
oracle's formulas: independent references come from scipy/numpy routines
(tests/refimpl.py), closed forms, hand-derived tables and invariants.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import synth
from synth import configs
from tests import refimpl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Eq. 2 / Eq. 3 (Section III-C): tile size of the iterative refinement

def test_tile_size_paper_example():
    # Section III-C: a 1-degree high-precision step gives an 18-degree tile,
    # i.e. 360/18 peels + 18 fine angles = 38 evaluations instead of 360.
    with open(os.path.join(GOLDEN, "tile_example.json")) as f:
        g = json.load(f)
    assert oracle.tile_size(g["hp_step"]) == g["tile"]
    assert 360 // g["tile"] + g["tile"] // g["hp_step"] == g["evaluations"]


@pytest.mark.parametrize("hp", sorted(refimpl.TILE_TABLE))
def test_tile_size_table(hp):
    x, y = refimpl.TILE_TABLE[hp]
    assert oracle.tile_size(hp) == x
    assert 360 // x + x // hp == y
    # Eq. 3: the continuous optimum sqrt(360 hp) = 6 sqrt(10) sqrt(hp); the
    # chosen admissible tile is never worse than any other admissible divisor
    xhat = 6 * np.sqrt(10) * np.sqrt(hp)
    assert abs(xhat - np.sqrt(360 * hp)) < 1e-9
    for x2 in range(hp, 361, hp):
        if 360 % x2 == 0:
            assert 360 / x2 + x2 / hp >= y


# --------------------------------------------------------------------------
# Eq. 1 on the lattice: the squared distance field D and the score S

def test_edt_single_point_closed_form():
    pts = np.array([[1.3, -0.7, 2.2]], np.float32)
    P = oracle.OraclePocket(pts, 0.5)
    c0 = np.floor(pts[0].astype(np.float64) / 0.5).astype(int)
    rng = np.random.default_rng(0)
    for _ in range(200):
        c = c0 + rng.integers(-30, 31, 3)
        assert P.D(*c) == int(((c - c0) ** 2).sum())


def test_edt_matches_scipy_exact_edt():
    pts = synth.pocket(1000, 1000, (8, 6, 5), configs.POCKET_CENTRE)
    P = oracle.OraclePocket(pts, 0.5)
    ref = refimpl.EdtTable(pts, 0.5, margin=20)
    assert np.array_equal(np.unique(P.occupied(), axis=0), ref.occ)
    rng = np.random.default_rng(1)
    dims = np.array(ref.D.shape)
    for _ in range(3000):
        ci = rng.integers(0, dims)
        c = ci + ref.lo
        assert P.D(*c) == ref.D[tuple(ci)]


def test_score_special_cases():
    pts = synth.pocket(1000, 1000, (8, 6, 5), configs.POCKET_CENTRE)
    P = oracle.OraclePocket(pts, 0.5)
    occ = P.occupied()
    # atoms at the centres of occupied cells score 0
    X = (occ[:25] + 0.5) * 0.5
    assert P.score_xyz(X) == 0
    # a one-atom ligand scores D of its cell
    ref = refimpl.EdtTable(pts, 0.5, margin=20)
    for x in [(20.1, 3.3, -1.2), (0.3, 0.2, 0.1), (-9.9, -7.1, 4.4)]:
        assert P.score_xyz(np.array([x])) == ref.score(np.array([x]))
    # overlap o = l / (h^2 S), S = 0 -> +inf (Eq. 1 divides by the sum)
    assert oracle.overlap(10, 40, 0.5) == pytest.approx(1.0)
    assert oracle.overlap(10, 0, 0.5) == float("inf")


CUBE = [np.array(p) for p in itertools.permutations(range(3))]


@pytest.mark.parametrize("perm", range(6))
@pytest.mark.parametrize("signs", range(8))
def test_score_invariant_under_cube_symmetries(perm, signs):
    """Joint signed permutations of ligand and pocket keep S exactly:
    permuting axes permutes cells; negation maps c -> -c-1 off the faces."""
    pts = synth.pocket(1000, 1000, (8, 6, 5), configs.POCKET_CENTRE).astype(np.float64)
    lig = configs.SINGLE.ligands().ligand(0)
    X = np.stack([lig["x"], lig["y"], lig["z"]], 1).astype(np.float64) + pts.mean(0)
    M = np.zeros((3, 3))
    M[np.arange(3), CUBE[perm]] = [(-1) ** ((signs >> k) & 1) for k in range(3)]
    P0 = oracle.OraclePocket(pts.astype(np.float32), 0.5)
    P1 = oracle.OraclePocket((pts @ M.T).astype(np.float32), 0.5)
    assert P1.score_xyz(X @ M.T) == P0.score_xyz(X)


def test_score_invariant_under_lattice_translation():
    pts = synth.pocket(1000, 1000, (8, 6, 5), configs.POCKET_CENTRE).astype(np.float64)
    lig = configs.SINGLE.ligands().ligand(0)
    X = np.stack([lig["x"], lig["y"], lig["z"]], 1).astype(np.float64) + pts.mean(0)
    t = np.array([3.0, -2.5, 7.5])  # a multiple of h = 0.5 in every axis
    P0 = oracle.OraclePocket(pts.astype(np.float32), 0.5)
    P1 = oracle.OraclePocket((pts + t).astype(np.float32), 0.5)
    assert P1.score_xyz(X + t) == P0.score_xyz(X)


# --------------------------------------------------------------------------
# Topology: rotamers are bridges (Section II), fragments (Alg. 1)

def test_topology_matches_scipy():
    L = synth.ligands(2, 0, 20, 20, 80, 2, 12)
    for i in range(L.n):
        lig = L.ligand(i)
        l = len(lig["x"])
        rc, dist, left = oracle.topology(lig)
        assert rc == oracle.OK
        assert np.array_equal(dist, refimpl.bond_distances(l, lig["bonds"]).astype(int))
        for r, (a, c) in enumerate(lig["rot"]):
            assert np.array_equal(left[r].astype(bool), refimpl.left_mask(l, lig["bonds"], a, c))


def test_topology_errors():
    lig = configs.SINGLE.ligands().ligand(0)
    bad = dict(lig)
    bad["bonds"] = lig["bonds"][:-1]  # drop a bond -> disconnected
    assert oracle.topology(bad)[0] == oracle.ERR_GRAPH
    bad = dict(lig)
    term = [int(b[1]) for b in lig["bonds"] if (lig["bonds"] == b[1]).sum() == 1][0]
    nb = [b for b in lig["bonds"] if term in b][0]
    bad["rot"] = np.array([nb])  # a terminal bond is not rotatable
    assert oracle.topology(bad)[0] == oracle.ERR_ROTAMER
    bad = dict(lig)
    bad["rot"] = np.array([[0, 31]]) if not any({0, 31} == set(b) for b in lig["bonds"]) else np.array([[0, 30]])
    assert oracle.topology(bad)[0] == oracle.ERR_ROTAMER  # not a bond


def test_ring_bonds_are_not_rotatable():
    L = synth.ligands(5, 0, 400, 15, 40, 0, 16, ring_frac=1.0)
    for i in range(L.n):
        lig = L.ligand(i)
        l = len(lig["x"])
        rc, _, _ = oracle.topology(lig)
        assert rc == oracle.OK
        for a, c in lig["rot"]:
            m = refimpl.left_mask(l, lig["bonds"], a, c)
            assert not m[c]  # removing the bond splits the graph


# --------------------------------------------------------------------------
# Pose counts implied by the knobs (Alg. 2, Eq. 2) -- closed form

def _closed_form_count(lig, k, n_orient):
    l = len(lig["x"])
    per_rep = 0
    for a, c in lig["rot"]:
        nl = int(refimpl.left_mask(l, lig["bonds"], a, c).sum())
        for size in (nl, l - nl):
            if size / l <= k.threshold:
                per_rep += 360 // k.lp_step
            elif k.refine:
                x, y = refimpl.TILE_TABLE[k.hp_step]
                per_rep += y
            else:
                per_rep += 360 // k.hp_step
    return n_orient * (k.repetitions * per_rep + 1)


@pytest.mark.parametrize("kn", [
    dict(hp=10), dict(hp=15), dict(hp=30, repetitions=2), dict(hp=5, lp=90, threshold=0.3),
    dict(hp=1, lp=45, threshold=0.6, refine=True), dict(hp=10, refine=True, repetitions=3),
    dict(hp=2, lp=90, threshold=0.8, refine=True)])
def test_pose_count_closed_form(kn):
    w = configs.SINGLE
    lig = synth.ligands(2, 3, 1, 20, 40, 3, 6).ligand(0)
    P = oracle.OraclePocket(w.pocket_points(), 0.5)
    k = oracle.knobs(**kn)
    q = synth.quaternions(5, 4)
    r = oracle.dock(P, lig, k, q, want_xyz=False)
    assert r.n_cand == _closed_form_count(lig, k, 4)


def test_single_workload_pose_count():
    # 256 orientations x (1 rep x 4 rotamers x 2 sides x 36 angles + 1) = 73,984
    w = configs.SINGLE
    lig = w.ligands().ligand(0)
    P = oracle.OraclePocket(w.pocket_points(), 0.5)
    r = oracle.dock(P, lig, oracle.knobs(**w.knob_dict()), w.quaternions(), want_xyz=False)
    assert r.n_cand == 256 * (4 * 2 * 36 + 1) == 73984


# --------------------------------------------------------------------------
# Kinematics: rigid placement and fragment rotation invariants

def _xyz(lig):
    return np.stack([lig["x"], lig["y"], lig["z"]], 1).astype(np.float64)


def test_placement_is_rigid_and_centred():
    lig = synth.ligands(2, 7, 1, 20, 80, 2, 12).ligand(0)
    x0 = _xyz(lig)
    d0 = np.linalg.norm(x0[:, None] - x0[None], axis=-1)
    centre = np.array([3.1, -1.2, 2.0])
    for q in synth.quaternions(3, 20):
        X = oracle.place(lig, q, centre)
        assert np.allclose(np.linalg.norm(X[:, None] - X[None], axis=-1), d0, atol=1e-12)
        assert np.allclose(X.mean(0), centre, atol=1e-12)
        # same rotation as scipy's quaternion convention (scalar-last there)
        R = refimpl.Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        assert np.allclose(X - centre, (x0 - x0.mean(0)) @ R.T, atol=1e-12)


def test_torsion_invariants():
    L = synth.ligands(2, 0, 5, 20, 60, 3, 8)
    rng = np.random.default_rng(4)
    for i in range(L.n):
        lig = L.ligand(i)
        l = len(lig["x"])
        X0 = _xyz(lig)
        b = lig["bonds"]
        bl0 = np.linalg.norm(X0[b[:, 0]] - X0[b[:, 1]], axis=1)
        dist = refimpl.bond_distances(l, b)
        ang = np.argwhere(dist == 2)
        d13_0 = np.linalg.norm(X0[ang[:, 0]] - X0[ang[:, 1]], axis=1)
        moves = [(r, s, int(rng.integers(0, 360))) for r in range(len(lig["rot"])) for s in (0, 1)]
        X = oracle.apply_torsions(lig, X0, moves)
        assert np.allclose(np.linalg.norm(X[b[:, 0]] - X[b[:, 1]], axis=1), bl0, atol=1e-10)
        assert np.allclose(np.linalg.norm(X[ang[:, 0]] - X[ang[:, 1]], axis=1), d13_0, atol=1e-10)
        # agrees with an independent rotation-vector implementation
        Y = X0.copy()
        for r, s, deg in moves:
            a, c = lig["rot"][r]
            m = refimpl.left_mask(l, b, a, c)
            Y = refimpl.rotate_fragment(Y, m if s == 0 else ~m, a, c, s, deg)
        assert np.allclose(X, Y, atol=1e-10)
        # 360/s steps of s compose to the identity
        for step in (10, 15, 30):
            Z = oracle.apply_torsions(lig, X0, [(0, 0, step)] * (360 // step))
            assert np.allclose(Z, X0, atol=1e-9)
        # left by theta and right by -theta give congruent ligands
        a = oracle.apply_torsions(lig, X0, [(0, 0, 70)])
        c = oracle.apply_torsions(lig, X0, [(0, 1, 290)])
        da = np.linalg.norm(a[:, None] - a[None], axis=-1)
        dc = np.linalg.norm(c[:, None] - c[None], axis=-1)
        assert np.allclose(da, dc, atol=1e-10)


# --------------------------------------------------------------------------
# The greedy sweep (Alg. 1/2) against independent brute force

def _tiny_case(seed, l, nrot):
    for s in range(seed, seed + 50):
        lig = configs.tiny_ligand(s, l, nrot)
        if len(lig["rot"]) == nrot:
            return lig
    raise RuntimeError("no tiny ligand with %d rotamers" % nrot)


def _setup_tiny(lig, pocket_n=300, axes=(4.0, 3.0, 2.5)):
    pts = synth.pocket(1100, pocket_n, axes, configs.POCKET_CENTRE)
    return oracle.OraclePocket(pts, 0.5), refimpl.EdtTable(pts, 0.5, margin=40)


def _independent_replay(lig, X0, angles):
    """Apply the greedy's own angle choices with scipy rotations."""
    l = len(lig["x"])
    X = X0.copy()
    for rep in angles:
        for r, (tl, tr) in enumerate(rep):
            a, c = lig["rot"][r]
            m = refimpl.left_mask(l, lig["bonds"], a, c)
            X = refimpl.rotate_fragment(X, m, a, c, 0, tl)
            X = refimpl.rotate_fragment(X, ~m, a, c, 1, tr)
    return X


@pytest.mark.parametrize("seed", range(4))
def test_greedy_endpoint_replays_exactly(seed):
    lig = _tiny_case(10 * seed, 10, 3)
    P, ref = _setup_tiny(lig)
    q = synth.quaternions(20 + seed, 16)
    k = oracle.knobs(hp=30, repetitions=2)
    res = oracle.dock(P, lig, k, q)
    dist = refimpl.bond_distances(len(lig["x"]), lig["bonds"])
    for o in range(len(q)):
        X0 = oracle.place(lig, q[o], P.centroid)
        X = _independent_replay(lig, X0, res.angles[o])
        assert np.allclose(X, res.xyz[o], atol=1e-9)
        if ref.face_margin(X) > 1e-7:
            assert ref.score(X) == res.S[o]
        assert refimpl.clash_flag(X, dist) == bool(res.clash[o])


@pytest.mark.parametrize("seed", range(4))
def test_single_rotamer_sweeps_are_exhaustive_minima(seed):
    """B = 1: the left sweep picks the earliest feasible minimiser of S over
    all left angles; the right sweep then does the same given the left choice."""
    lig = _tiny_case(100 + 10 * seed, 9, 1)
    P, ref = _setup_tiny(lig)
    l = len(lig["x"])
    dist = refimpl.bond_distances(l, lig["bonds"])
    a, c = lig["rot"][0]
    m = refimpl.left_mask(l, lig["bonds"], a, c)
    step = 10
    k = oracle.knobs(hp=step)
    q = synth.quaternions(40 + seed, 12)
    res = oracle.dock(P, lig, k, q)
    for o in range(len(q)):
        X0 = oracle.place(lig, q[o], P.centroid)
        tl, tr = res.angles[o][0][0]
        for side, base, chosen in ((0, X0, tl), (1, refimpl.rotate_fragment(X0, m, a, c, 0, tl), tr)):
            mask = m if side == 0 else ~m
            best = None
            for deg in range(0, 360, step):
                Y = refimpl.rotate_fragment(base, mask, a, c, side, deg)
                if ref.face_margin(Y[mask]) < 1e-7:
                    pytest.skip("atom on a cell face")
                if refimpl.cross_feasible(Y, mask, dist):
                    s = ref.score(Y)
                    if best is None or s < best[0]:
                        best = (s, deg)
            assert chosen == (0 if best is None else best[1])


@pytest.mark.parametrize("seed", range(3))
def test_greedy_never_beats_exhaustive_search(seed):
    """min over every clash-free combination of fragment angles <= greedy S."""
    lig = _tiny_case(200 + 10 * seed, 8, 2)
    P, ref = _setup_tiny(lig)
    l = len(lig["x"])
    dist = refimpl.bond_distances(l, lig["bonds"])
    step = 30
    q = synth.quaternions(60 + seed, 4)
    res = oracle.dock(P, lig, oracle.knobs(hp=step), q)
    masks = [refimpl.left_mask(l, lig["bonds"], a, c) for a, c in lig["rot"]]
    angs = range(0, 360, step)
    for o in range(len(q)):
        if res.clash[o]:
            continue
        X0 = oracle.place(lig, q[o], P.centroid)
        best = None
        for combo in itertools.product(angs, repeat=4):
            X = X0
            for r, (a, c) in enumerate(lig["rot"]):
                X = refimpl.rotate_fragment(X, masks[r], a, c, 0, combo[2 * r])
                X = refimpl.rotate_fragment(X, ~masks[r], a, c, 1, combo[2 * r + 1])
            if not refimpl.clash_flag(X, dist):
                s = ref.score(X)
                best = s if best is None else min(best, s)
        assert best is not None and best <= res.S[o]


def test_greedy_is_monotone_from_clash_free_start():
    """Refinement off: angle 0 (stay) is always a candidate, so from a
    clash-free placement every sweep is feasible at 0 and S never rises."""
    w = configs.SINGLE
    lig = w.ligands().ligand(0)
    P = oracle.OraclePocket(w.pocket_points(), 0.5)
    q = w.quaternions(64)
    res = oracle.dock(P, lig, oracle.knobs(hp=10, repetitions=2), q)
    dist = refimpl.bond_distances(len(lig["x"]), lig["bonds"])
    n_checked = 0
    for o in range(len(q)):
        X0 = oracle.place(lig, q[o], P.centroid)
        if refimpl.clash_flag(X0, dist):
            continue
        n_checked += 1
        assert res.clash[o] == 0
        assert res.S[o] <= P.score_xyz(X0)
    assert n_checked > 32


def test_rigid_only_ligand_ranks_placements():
    """B = 0: every orientation is just its rigid placement, ranked by (clash, S, index)."""
    w = configs.SINGLE
    lig = w.ligands().ligand(0)
    lig = dict(lig, rot=np.zeros((0, 2), np.int32))
    P = oracle.OraclePocket(w.pocket_points(), 0.5)
    q = w.quaternions(32)
    res = oracle.dock(P, lig, oracle.knobs(hp=10), q)
    assert res.n_cand == 32
    dist = refimpl.bond_distances(len(lig["x"]), lig["bonds"])
    ref = refimpl.EdtTable(w.pocket_points(), 0.5)
    keys = []
    for o in range(32):
        X0 = oracle.place(lig, q[o], P.centroid)
        assert res.S[o] == ref.score(X0)
        keys.append((int(refimpl.clash_flag(X0, dist)), ref.score(X0), o))
    top = oracle.topk(res.S, res.clash, 10)
    assert [kk[2] for kk in sorted(keys)[:10]] == list(top)


def test_topk_tie_break():
    S = np.array([5, 3, 3, 9, 3, 1], np.int64)
    clash = np.array([0, 0, 0, 0, 1, 1], np.uint8)
    assert list(oracle.topk(S, clash, 6)) == [1, 2, 0, 3, 5, 4]


def test_refinement_picks_within_best_tile():
    """Peel/tile (Alg. 2, refinement on): every chosen angle lies in a tile
    of size x, and the count of evaluations follows Eq. 2."""
    lig = _tiny_case(300, 10, 2)
    P, _ = _setup_tiny(lig)
    for hp in (1, 5, 10):
        k = oracle.knobs(hp=hp, refine=True)
        res = oracle.dock(P, lig, k, synth.quaternions(8, 6), want_xyz=False)
        x, y = refimpl.TILE_TABLE[hp]
        assert res.n_cand == 6 * (2 * len(lig["rot"]) * y + 1)
        assert np.all(res.angles % hp == 0)


def test_threshold_rule_is_inclusive():
    """Alg. 2 takes the coarse step when the relative fragment size is
    <= threshold; a fragment exactly at the threshold is coarse."""
    L = synth.ligands(2, 0, 200, 20, 20, 1, 1)
    for i in range(L.n):
        lig = L.ligand(i)
        if len(lig["rot"]) != 1:
            continue
        a, c = lig["rot"][0]
        nl = int(refimpl.left_mask(20, lig["bonds"], a, c).sum())
        small = min(nl, 20 - nl)
        if small * 4 % 20:  # want a size whose fraction is exact in binary
            continue
        thr = small / 20
        P = oracle.OraclePocket(configs.SINGLE.pocket_points(), 0.5)
        q = synth.quaternions(1, 2)
        at = oracle.dock(P, lig, oracle.knobs(hp=10, lp=90, threshold=thr), q, want_xyz=False)
        below = oracle.dock(P, lig, oracle.knobs(hp=10, lp=90, threshold=np.nextafter(np.float32(thr), 0)), q,
                            want_xyz=False)
        large = 20 - small
        assert at.n_cand == 2 * ((4 if large / 20 <= thr else 36) + 4 + 1)
        assert below.n_cand == 2 * (36 + 36 + 1)
        return
    pytest.skip("no ligand with an exactly representable fragment fraction")


def test_pocket_centroid_is_mean_of_points():
    pts = synth.pocket(1001, 4000, (12, 9, 7), configs.POCKET_CENTRE)
    P = oracle.OraclePocket(pts, 0.5)
    assert np.allclose(P.centroid, pts.astype(np.float64).mean(0), rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("hp", [1, 5, 10])
def test_refinement_matches_independent_two_level_search(seed, hp):
    """Alg. 2 with refinement: evaluate the central element of every tile of
    size x, keep the best tile (earliest on ties), then scan that tile with the
    fine step and keep its earliest best feasible angle."""
    lig = _tiny_case(400 + 10 * seed, 9, 1)
    P, ref = _setup_tiny(lig)
    l = len(lig["x"])
    dist = refimpl.bond_distances(l, lig["bonds"])
    a, c = lig["rot"][0]
    m = refimpl.left_mask(l, lig["bonds"], a, c)
    x, _ = refimpl.TILE_TABLE[hp]
    q = synth.quaternions(80 + seed, 8)
    res = oracle.dock(P, lig, oracle.knobs(hp=hp, refine=True), q)

    def best(base, mask, side, angles):
        out = None
        for deg in angles:
            Y = refimpl.rotate_fragment(base, mask, a, c, side, deg)
            if ref.face_margin(Y[mask]) < 1e-7:
                pytest.skip("atom on a cell face")
            if refimpl.cross_feasible(Y, mask, dist):
                s = ref.score(Y)
                if out is None or s < out[0]:
                    out = (s, deg)
        return out

    for o in range(len(q)):
        X0 = oracle.place(lig, q[o], P.centroid)
        tl, tr = res.angles[o][0][0]
        base = X0
        for side, chosen in ((0, tl), (1, tr)):
            mask = m if side == 0 else ~m
            centres = [t * x + (x // 2 // hp) * hp for t in range(360 // x)]
            pk = best(base, mask, side, centres)
            t_star = 0 if pk is None else centres.index(pk[1])
            fine = best(base, mask, side, [t_star * x + j * hp for j in range(x // hp)])
            assert chosen == (0 if fine is None else fine[1])
            base = refimpl.rotate_fragment(base, mask, a, c, side, int(chosen))


@pytest.mark.parametrize("seed", range(3))
def test_sweep_feasibility_tests_only_straddling_pairs(seed):
    """With a clash distance large enough that pairs inside one fragment
    already clash, a sweep is still tested only on the pairs that the rotation
    moves against each other (pairs within a side keep their distance)."""
    lig = _tiny_case(500 + 10 * seed, 18, 1)
    P, ref = _setup_tiny(lig)
    l = len(lig["x"])
    dist = refimpl.bond_distances(l, lig["bonds"])
    a, c = lig["rot"][0]
    m = refimpl.left_mask(l, lig["bonds"], a, c)
    cd = 3.0
    q = synth.quaternions(90 + seed, 8)
    res = oracle.dock(P, lig, oracle.knobs(hp=10, clash_dist=cd), q)
    saw_inner_clash = False
    for o in range(len(q)):
        base = oracle.place(lig, q[o], P.centroid)
        for side in (0, 1):
            mask = m if side == 0 else ~m
            chosen = res.angles[o][0][0][side]
            inner = refimpl.clash_flag(base[mask], dist[np.ix_(mask, mask)], cd=cd)
            out = None
            for deg in range(0, 360, 10):
                Y = refimpl.rotate_fragment(base, mask, a, c, side, deg)
                if ref.face_margin(Y[mask]) < 1e-7:
                    pytest.skip("atom on a cell face")
                if refimpl.cross_feasible(Y, mask, dist, cd=cd):
                    s = ref.score(Y)
                    if out is None or s < out[0]:
                        out = (s, deg)
            assert chosen == (0 if out is None else out[1])
            saw_inner_clash |= inner and out is not None
            base = refimpl.rotate_fragment(base, mask, a, c, side, int(chosen))
    if not saw_inner_clash:
        pytest.skip("no fragment with an inner clash at this clash distance")
