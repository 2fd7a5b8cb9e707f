"""Constructed edge cases of the FP32 fast path's exactness guards, against
the FP64 oracle (full ranking of every orientation, bit-exact).

The docking kernel scores candidates in FP32 and re-evaluates in FP64 every
candidate whose cell or bump decision lies within the rounding bound of a
boundary and that could still win its sweep.  These inputs put decisions
exactly on the boundaries and one float step either side of them:
  - atoms exactly on lattice cell faces and 2^-20 A (about 1e-6 A) off them
    in the pose the first sweeps start from (identity orientation, centroid
    placed exactly);
  - straddling far pairs exactly 2.0 A apart and 2 +- 2^-20 A;
  - pairs whose minimum distance over a full turn of the rotamer is 2.0 A
    plus offsets from 0 to +-2^-8 A (around the sweep's prune margin);
  - a ligand stretched 100-fold, so that moving atoms far outside the grid
    box carry fragment scores above 2^23 (the decision key is 64-bit).
Each case asserts that the FP64 re-evaluation actually ran (fallback
counter > 0)."""
import numpy as np
import pytest

import oracle
import synth
from tests import gpuutil
from tests.gpuutil import gpu

EPS = 2.0 ** -20  # about 1e-6 A, exactly representable
CNT_POSES, CNT_FALLBACK, CNT_OOB = 0, 1, 2


@pytest.fixture(scope="module")
def g():
    return gpuutil.gd()


def _chain_bonds(n):
    return np.array([[i, i + 1] for i in range(n - 1)], np.int32)


def _lig(X, bonds, rot):
    X = np.asarray(X, np.float64)
    x32 = X.astype(np.float32)
    assert np.array_equal(x32.astype(np.float64), X), "coordinates must be exact in FP32"
    return dict(x=x32[:, 0].copy(), y=x32[:, 1].copy(), z=x32[:, 2].copy(), bonds=np.asarray(bonds, np.int32),
                rot=np.asarray(rot, np.int32))


def _hairpin(dx_face=0.0, dy_pair=0.0):
    """16-atom hairpin chain: atoms 0-7 along +x (x = 1.25 i, z = 0.75 (i mod
    2)), atoms 8-15 back along -x at y = 2 A, so that atoms i and 15 - i
    (graph distance 15 - 2i > 3 for i <= 5) are exactly 2.0 A apart and every
    other far pair is at least 2.47 A apart.  Every even atom sits on a cell
    face in x, y = 0 and y = 2 are faces, and so is z = 0.
    dx_face moves atom 2 by +dx and atom 4 by -dx along x; dy_pair moves atom
    15 by -dy and atom 14 by +dy along y (pair (0,15) at 2 - dy, (1,14) at
    2 + dy).  The coordinate sums, hence the centroid, do not change."""
    X = np.zeros((16, 3))
    for i in range(8):
        X[i] = (1.25 * i, 0.0, 0.75 * (i % 2))
        X[15 - i] = (1.25 * i, 2.0, 0.75 * (i % 2))
    X[2, 0] += dx_face
    X[4, 0] -= dx_face
    X[15, 1] -= dy_pair
    X[14, 1] += dy_pair
    X += (3.5, -1.5, 2.5)  # a lattice translation keeps faces on faces
    return X


def _balanced_pocket(X, shift=0.25, far=30.0):
    """Pocket points whose FP64 centroid equals the ligand's exactly: one
    point per atom at X_i + (shift, shift, shift) (the atom's own cell holds
    it when the atom is on or above the cell's lower faces), and as many
    points at centroid - shift +- (far, 0, 0) to balance the sum."""
    n = len(X)
    m = X.sum(0) / n
    near = X + shift
    fx = np.array([far, 0.0, 0.0])
    fars = [m - shift + fx if k % 2 == 0 else m - shift - fx for k in range(n)]
    P = np.concatenate([near, np.array(fars)])
    P32 = P.astype(np.float32)
    assert np.array_equal(P32.astype(np.float64), P)
    assert np.array_equal(P32.astype(np.float64).sum(0) / len(P), m)  # exact in FP64
    return P32


def _quats(n_rand, seed):
    return np.concatenate([[[1.0, 0.0, 0.0, 0.0]], synth.quaternions(seed, n_rand)])


def _dock_and_compare(g, ligs, pts, q, hp, top_k=None):
    P = g.Pocket(pts, 0.5, 12.0)
    O = oracle.OraclePocket(pts, 0.5)
    top_k = top_k or len(q)
    b = g.Batch(P, ligs, q, hp=hp, top_k=top_k)
    res = b.dock(1).host()
    orc = gpuutil.oracle_dock_batch(O, ligs, oracle.knobs(hp=hp), q)
    gpuutil.compare_full_ranking(res, orc, ligs)
    assert res["counters"][CNT_POSES] == sum(r.n_cand for r in orc)
    # the per-ligand form takes the same decisions
    rp = b.dock(0).host()
    for k in ("orient", "S", "clash", "angles", "xyz"):
        assert np.array_equal(res[k], rp[k]), k
    return res, orc


HAIRPIN_CASES = [(0.0, 0.0), (EPS, 0.0), (0.0, EPS), (EPS, EPS)]
HAIRPIN_ROT = [[2, 3], [5, 6], [9, 10], [12, 13]]


@pytest.mark.parametrize("dx,dy", HAIRPIN_CASES)
def test_hairpin_inputs_are_as_designed(dx, dy):
    """(CPU) the constructed hairpin: far pairs at the bump distance, atoms on
    faces, a pocket whose FP64 centroid is the ligand's, exactly."""
    X = _hairpin(dx, dy)
    lig = _lig(X, _chain_bonds(16), HAIRPIN_ROT)
    rc, dist, _ = oracle.topology(lig)
    assert rc == 0
    pairs = [(i, 15 - i) for i in range(6)]
    assert all(dist[i, j] > 3 for i, j in pairs)
    d = [np.linalg.norm(X[i] - X[j]) for i, j in pairs]
    assert d[0] == 2.0 - dy and d[1] == 2.0 + dy and d[3] == 2.0 and d[5] == 2.0
    assert d[2] == d[4] == np.hypot(2.0, dx)
    # every other far pair is well clear of the bump distance
    far = [(i, j) for i in range(16) for j in range(i + 1, 16) if dist[i, j] > 3 and (i, j) not in pairs]
    assert min(np.linalg.norm(X[i] - X[j]) for i, j in far) > 2.4
    on = [0, 6, 9, 11, 13, 15]  # x on a face (atoms 2 and 4 too, unless moved)
    assert np.all(X[on, 0] / 0.5 == np.round(X[on, 0] / 0.5))
    leg = np.array([i if i < 8 else 15 - i for i in range(16)])
    assert np.all(X[:, 2] == 2.5 + 0.75 * (leg % 2))  # z = 2.5 is a face
    assert np.all(X[:, 1] == np.where(np.arange(16) < 8, -1.5, 0.5 - (np.arange(16) == 15) * dy + (np.arange(16) == 14) * dy))
    assert X[2, 0] - 6.0 == dx and X[4, 0] - 8.5 == -dx  # one float step off the faces x = 6.0 and 8.5
    _balanced_pocket(X)


@gpu
@pytest.mark.parametrize("dx,dy", HAIRPIN_CASES)
def test_atoms_on_cell_faces_and_pairs_at_the_bump_distance(g, dx, dy):
    X = _hairpin(dx, dy)
    lig = _lig(X, _chain_bonds(16), HAIRPIN_ROT)
    ligs = synth.LigandBatch.from_list([lig])
    pts = _balanced_pocket(X)
    res, orc = _dock_and_compare(g, ligs, pts, _quats(15, 31), hp=30)
    assert res["counters"][CNT_FALLBACK] > 0


def _touch(e, n=16):
    """Chain L(0)-a(1)-c(2)-r(3)-T(4)-f5..: the rotamer (a, c) lies on the x
    axis; L turns on a circle of radius 1 about it (axial -0.5), T sits at
    axial -0.5 and radius 3 - e on the far side, four bonds from L.  Over a
    full turn of either side the pair (L, T) comes closest, 2 - e A, at
    180 degrees from the start.  The rest of the chain runs away from L."""
    X = np.zeros((n, 3))
    X[0] = (-0.5, 0.0, 1.0)
    X[1] = (0.0, 0.0, 0.0)
    X[2] = (1.5, 0.0, 0.0)
    X[3] = (2.5, 1.0, 0.0)
    X[4] = (-0.5, 0.0, -3.0 + e)
    for k in range(5, n):
        X[k] = (-0.5 - 1.5 * (k - 4), 0.0, -3.0 - 0.25 * (k % 2))
    return X


TOUCH_OFFSETS = [0.0, EPS, -EPS, 2.0 ** -16, -2.0 ** -16, 2.0 ** -12, -2.0 ** -12, 2.0 ** -8, -2.0 ** -8]
TOUCH_ROT = [[1, 2], [3, 4], [7, 8]]


def test_touch_inputs_are_as_designed():
    """(CPU) the constructed touching pairs: over a full turn of the rotamer
    (1, 2) the pair (0, 4), four bonds apart, comes to 2 - e A."""
    for e in TOUCH_OFFSETS:
        X = _touch(e)
        lig = _lig(X, _chain_bonds(16), TOUCH_ROT)
        rc, dist, _ = oracle.topology(lig)
        assert rc == 0 and dist[0, 4] == 4
        # L and T share the axial coordinate; radial distances 1 and 3 - e from the x axis
        rL, rT = np.hypot(X[0, 1], X[0, 2]), np.hypot(X[4, 1], X[4, 2])
        assert X[0, 0] == X[4, 0] and rL == 1.0 and rT == 3.0 - e
        assert np.all(X[1:3, 1:] == 0.0)  # the rotamer's atoms on the axis


@gpu
def test_pairs_touching_the_bump_distance_over_a_turn(g):
    ligs = synth.LigandBatch.from_list([_lig(_touch(e), _chain_bonds(16), TOUCH_ROT) for e in TOUCH_OFFSETS])
    # pocket: points on the 180-degree image of L and around the chain, so
    # that turning L (or T) towards the contact scores well
    X0 = _touch(0.0)
    img = X0.copy()
    img[0] = (-0.5, 0.0, -1.0)
    pts = np.concatenate([img + 0.25, img - 0.25, img + (0.0, 0.25, -0.25)]).astype(np.float32)
    res, orc = _dock_and_compare(g, ligs, pts, _quats(63, 32), hp=10, top_k=16)
    assert res["counters"][CNT_FALLBACK] > 0


@gpu
def test_stretched_ligand_far_outside_the_grid(g):
    """Coordinates scaled 300-fold about the centroid: every atom lies far
    outside the tabulated box (exact brute-force lookups), every atom's D
    exceeds 2^23 / 3, so the fragments' S exceed 2^23, and the whole-ligand
    S stays below 2^31."""
    base = synth.ligands(9100, 0, 1, 36, 36, 6, 6).ligand(0)
    X = np.stack([base["x"], base["y"], base["z"]], 1).astype(np.float64)
    c = X.mean(0)
    Xs = ((X - c) * 300.0 + c).astype(np.float32)
    lig = dict(base, x=Xs[:, 0].copy(), y=Xs[:, 1].copy(), z=Xs[:, 2].copy())
    ligs = synth.LigandBatch.from_list([lig])
    pts = synth.pocket(1005, 64, (4.0, 3.0, 2.5), tuple(c))
    q = _quats(15, 33)
    res, orc = _dock_and_compare(g, ligs, pts, q, hp=30)
    S = orc[0].S
    assert S.max() < 2 ** 31 and np.all(S > 36 * 2 ** 23 // 3)
    assert res["counters"][CNT_OOB] > 0 and res["counters"][CNT_FALLBACK] > 0
