"""Pins of the oracle's continuous Eq. 1 (no lattice) and of the Eq. 5 /
Pareto host logic of the knob exploration.

Eq. 1 (Section III-A): o = l / sum_i min_j d^2(L_i, P_j).  Independent
references: exact rational arithmetic (fractions), closed forms, the lattice
reading of Eq. 1 (itself pinned elsewhere) at cell centres, and invariances.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth import configs


def _exact_sum(X, P):
    """Exact rational sum over atoms of the smallest squared distance."""
    tot = Fraction(0)
    for a in X:
        best = None
        for p in P:
            d = sum((Fraction(float(a[k])) - Fraction(float(p[k]))) ** 2 for k in range(3))
            best = d if best is None or d < best else best
        tot += best
    return tot


@pytest.mark.parametrize("seed", range(6))
def test_continuous_matches_exact_rationals(seed):
    # The FP64 sum must agree with the exact rational value within its
    # rounding bound: each squared distance errs by <= 4u d^2 (three
    # differences and two fused roundings), the minimum keeps that bound, and
    # l sequential additions add <= l u of the total (u = 2^-53).
    rng = np.random.default_rng(seed)
    P = (rng.normal(size=(int(rng.integers(1, 40)), 3)) * 5).astype(np.float32)
    X = rng.normal(size=(int(rng.integers(1, 12)), 3)) * 6
    pk = oracle.OraclePocket(P, 0.5)
    s, m, o = pk.overlap_continuous(X)
    exact = _exact_sum(X, P)
    u = 2.0 ** -53
    assert abs(Fraction(s) - exact) <= (6 + len(X)) * u * exact
    assert o == len(X) / s
    for i, a in enumerate(X):
        e = _exact_sum(a[None, :], P)
        assert abs(Fraction(float(m[i])) - e) <= 6 * u * e


def test_continuous_one_point_closed_form():
    # One pocket point: the minimum is the distance to it; offsets (3, 4, 0),
    # (1, 2, 2) and (0, 0, 0) give 25 + 9 + 0 = 34 exactly.
    p = np.array([[1.5, -2.25, 0.75]], np.float32)
    X = p.astype(np.float64) + np.array([[3, 4, 0], [1, 2, 2], [0, 0, 0]], np.float64)
    s, m, o = oracle.OraclePocket(p, 0.5).overlap_continuous(X)
    assert list(m) == [25.0, 9.0, 0.0]
    assert s == 34.0 and o == 3 / 34.0
    # every atom on a point: the sum is 0 and the overlap +inf
    s0, _, o0 = oracle.OraclePocket(p, 0.5).overlap_continuous(p.astype(np.float64))
    assert s0 == 0.0 and o0 == float("inf")


@pytest.mark.parametrize("seed", range(4))
def test_continuous_equals_lattice_score_at_cell_centres(seed):
    # With every point and atom at a cell centre ((c + 1/2) h), the smallest
    # squared distance is h^2 min |c - c'|^2 = h^2 D(c): continuous Eq. 1 and
    # its lattice reading agree exactly (all values are exact binary fractions).
    rng = np.random.default_rng(100 + seed)
    h = 0.5
    cells = rng.integers(-20, 20, size=(int(rng.integers(1, 30)), 3))
    P = ((cells + 0.5) * h).astype(np.float32)
    ac = rng.integers(-30, 30, size=(int(rng.integers(1, 20)), 3))
    X = (ac + 0.5) * h
    pk = oracle.OraclePocket(P, h)
    s, m, _ = pk.overlap_continuous(X)
    assert s == h * h * pk.score_xyz(X)
    for i, c in enumerate(ac):
        assert m[i] == h * h * pk.D(*c)


def test_continuous_invariances():
    # (a coarse lattice keeps the oracle's lattice memo small; the continuous
    # score does not use it)
    H = 8.0
    rng = np.random.default_rng(7)
    # integer coordinates: every difference and square is exact, so a joint
    # integer translation, an axis permutation or a point reordering leaves
    # each minimum and the sum bit-identical
    P = rng.integers(-50, 50, size=(60, 3)).astype(np.float32)
    X = rng.integers(-60, 60, size=(25, 3)).astype(np.float64)
    s0, m0, _ = oracle.OraclePocket(P, H).overlap_continuous(X)
    t = np.array([17, -9, 33])
    s1, m1, _ = oracle.OraclePocket(P + t, H).overlap_continuous(X + t)
    assert s1 == s0 and np.array_equal(m1, m0)
    for perm in itertools.permutations(range(3)):
        s2, m2, _ = oracle.OraclePocket(P[:, perm], H).overlap_continuous(X[:, perm])
        assert s2 == s0 and np.array_equal(m2, m0)
    s3, m3, _ = oracle.OraclePocket(P[rng.permutation(len(P))], H).overlap_continuous(X)
    assert s3 == s0 and np.array_equal(m3, m0)
    # adding a far point changes nothing; adding an atom's own position as a
    # point makes that atom's minimum 0
    s4, m4, _ = oracle.OraclePocket(np.vstack([P, [[500.0, 500.0, 500.0]]]), H).overlap_continuous(X)
    assert s4 == s0
    s5, m5, _ = oracle.OraclePocket(np.vstack([P, X[3:4].astype(np.float32)]), H).overlap_continuous(X)
    assert m5[3] == 0.0 and np.all(m5 <= m0)


def test_continuous_monotone_in_points():
    # A superset of points can only lower every minimum (min over a larger set).
    rng = np.random.default_rng(9)
    P = (rng.normal(size=(200, 3)) * 4).astype(np.float32)
    X = rng.normal(size=(30, 3)) * 5
    _, m_half, _ = oracle.OraclePocket(P[:100], 8.0).overlap_continuous(X)
    _, m_all, _ = oracle.OraclePocket(P, 8.0).overlap_continuous(X)
    assert np.all(m_all <= m_half)


# --------------------------------------------------------------------------
# Knob exploration host logic (Sections IV-B, V-B): design spaces, Eq. 5,
# top-1 % means and the Pareto front

def test_design_space_sizes_and_baseline():
    from paper_1901_06363_amd import dse
    flat, full = dse.configurations("flat"), dse.configurations("full")
    # full factorial sizes of the two spaces listed in Section V-B
    assert len(flat) == 8 * 3 and len(full) == 4 * 2 * 4 * 3 * 2
    assert len({tuple(sorted(c.items())) for c in full}) == len(full)
    # the baseline (hp 1, threshold 0, 3 repetitions, no refinement) is a
    # member of both spaces: once in flat, once per low-precision step in full
    assert sum(dse.is_baseline(c) for c in flat) == 1
    assert sum(dse.is_baseline(c) for c in full) == 2
    assert all(c["lp"] == c["hp"] and c["threshold"] == 0.0 and not c["refine"] for c in flat)


def test_eq5_degradation_closed_forms():
    from paper_1901_06363_amd import dse
    assert dse.degradation(5.0, 5.0) == 0.0
    assert abs(dse.degradation(0.977, 1.0) - 2.3) < 1e-12   # the 2.3 % of Section V-B's first step
    assert dse.degradation(1.1, 1.0) < 0                     # better than the baseline: negative
    # top 1 %: ceil(0.01 n) best values (at least one)
    s = np.arange(250, dtype=float)
    assert dse.top_fraction_mean(s) == np.mean([249, 248, 247])
    assert dse.top_fraction_mean([3.0, 1.0]) == 3.0
    assert dse.top_fraction_mean(s, frac=0.1) == np.mean(np.arange(225, 250))


@pytest.mark.parametrize("seed", range(5))
def test_pareto_front_against_brute_force(seed):
    from paper_1901_06363_amd import dse
    rng = np.random.default_rng(seed)
    n = 60
    t = rng.integers(0, 12, n).astype(float)   # ties on both axes on purpose
    d = rng.integers(0, 12, n).astype(float)
    keep = dse.pareto_front(t, d)
    # reference: sort by throughput descending, degradation ascending, and
    # keep a point when its degradation is strictly below all earlier ones
    # (points equal on both axes share their status)
    order = sorted(range(n), key=lambda i: (-t[i], d[i]))
    ref = np.zeros(n, bool)
    best = float("inf")
    for i in order:
        if d[i] < best:
            ref[i] = True
            best = d[i]
    for i in range(n):
        for j in range(n):
            if t[i] == t[j] and d[i] == d[j]:
                ref[i] = ref[i] or ref[j]
    assert np.array_equal(keep, ref)
    # every excluded point is dominated by a kept one
    for i in np.nonzero(~keep)[0]:
        assert np.any(keep & (t >= t[i]) & (d <= d[i]))


# --------------------------------------------------------------------------
# Overlap landscape of a rotamer side (peak analysis, Section III-B)

@pytest.mark.parametrize("seed", range(3))
def test_profile_argmin_is_every_sweeps_choice(seed):
    # Alg. 1 with a flat 1-degree step keeps the lowest S among the feasible
    # angles (ties to the earliest, none feasible -> 0): the landscape taken
    # at the pose before each sweep must reproduce every chosen angle
    lig = configs.tiny_ligand(20 + seed, 14, 3)
    pts = configs.SINGLE.pocket_points()
    O = oracle.OraclePocket(pts, 0.5)
    q = np.array([0.8, 0.2, -0.4, 0.4])
    q = q / np.linalg.norm(q)
    kn = oracle.knobs(hp=1, repetitions=1)
    r = oracle.dock(O, lig, kn, q[None, :])
    X = oracle.place(lig, q, O.centroid)
    moves = []
    nr = len(np.asarray(lig["rot"]).reshape(-1, 2))
    for rr in range(nr):
        for side in (0, 1):
            done = [m for m in moves if m[2] != 0]
            Xb = oracle.apply_torsions(lig, X, done) if done else X
            size, S, f = oracle.sweep_profile(O, lig, Xb, rr, side, step=1)
            assert 1 <= size < len(lig["x"])
            if f.any():
                best = int(np.flatnonzero(f)[np.argmin(S[f])])
            else:
                best = 0
            assert best == r.angles[0, 0, rr, side], (rr, side)
            moves.append((rr, side, best))
    # the final pose is the placement with every chosen rotation applied (a
    # sweep commits nothing for 0 degrees)
    nz = [m for m in moves if m[2] != 0]
    assert np.array_equal(oracle.apply_torsions(lig, X, nz) if nz else X, r.xyz[0])


def test_profile_subsampling_and_clash_limits():
    lig = configs.tiny_ligand(7, 16, 3)
    O = oracle.OraclePocket(configs.SINGLE.pocket_points(), 0.5)
    X = oracle.place(lig, np.array([1.0, 0, 0, 0]), O.centroid)
    n1, S1, f1 = oracle.sweep_profile(O, lig, X, 1, 0, step=1)
    n5, S5, f5 = oracle.sweep_profile(O, lig, X, 1, 0, step=5)
    assert n1 == n5 and np.array_equal(S5, S1[::5]) and np.array_equal(f5, f1[::5])
    # bump distance 0 never bumps (strict d^2 < 0); a 100 A distance bumps at
    # every angle (the ligand has straddling pairs more than 3 bonds apart)
    assert oracle.sweep_profile(O, lig, X, 1, 0, step=10, clash_dist=0.0)[2].all()
    assert not oracle.sweep_profile(O, lig, X, 1, 0, step=10, clash_dist=100.0)[2].any()
    with pytest.raises(oracle.OracleError):
        oracle.sweep_profile(O, lig, X, 1, 0, step=7)
    with pytest.raises(oracle.OracleError):
        oracle.sweep_profile(O, lig, X, 9, 0, step=1)
