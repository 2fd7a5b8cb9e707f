"""Pins of the oracle's smoothed surrogate and its analytic gradient.

Closed forms (a one-point pocket), trilinear identities, central finite
differences in FP64 (h = 1e-4, relative error 1e-3 per parameter group;
stencils in which an atom crosses a lattice face, where the trilinear
gradient jumps, are retried with h = 1e-7 and otherwise excluded and
counted), and an independent leaf-first forward-kinematics implementation.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import configs
from tests import refimpl

SIG, CUTS, BH = 0.6, 4.0, 0.375


def _blur(pts):
    P = oracle.OraclePocket(pts, 0.5)
    return P, oracle.OracleBlur(P, SIG, CUTS, BH)


def test_one_point_density_closed_form():
    pts = np.array([[0.31, -0.52, 0.77]], np.float32)
    _, B = _blur(pts)
    p = pts[0].astype(np.float64)
    sig = float(np.float32(SIG))
    cut = float(np.float32(CUTS)) * sig
    bh = float(np.float32(BH))
    for i in range(-8, 9):
        for j in (-3, 0, 2):
            for k in (-1, 1, 4):
                g = bh * np.array([i, j, k], np.float64)
                d2 = ((g - p) ** 2).sum()
                want = np.exp(-d2 / (2 * sig * sig)) if d2 <= cut * cut else 0.0
                assert B.node(i, j, k) == pytest.approx(want, rel=1e-14, abs=1e-300)


def test_trilinear_identities():
    pts = configs.SINGLE.pocket_points()
    _, B = _blur(pts)
    bh = float(np.float32(BH))
    rng = np.random.default_rng(0)
    c = np.floor(pts.mean(0) / bh).astype(int)
    for _ in range(50):
        n = c + rng.integers(-6, 7, 3)
        v, _ = B.interp(bh * n.astype(np.float64))
        assert v == pytest.approx(B.node(*n), rel=1e-12, abs=1e-15)
        # linear along an edge of the cell
        s = rng.random()
        x = bh * (n + np.array([s, 0.0, 0.0]))
        v, g = B.interp(x)
        want = (1 - s) * B.node(*n) + s * B.node(n[0] + 1, n[1], n[2])
        assert v == pytest.approx(want, rel=1e-10, abs=1e-12)
        assert g[0] == pytest.approx((B.node(n[0] + 1, n[1], n[2]) - B.node(*n)) / bh, rel=1e-10, abs=1e-10)


def _pose(lig, shift):
    X = np.stack([lig["x"], lig["y"], lig["z"]], 1).astype(np.float64)
    return X - X.mean(0) + shift


def _cells(X):
    return np.floor(X / float(np.float32(BH)))


def _fd_grad(B, lig, X0, prm, h):
    g = np.zeros(len(prm))
    crossed = np.zeros(len(prm), bool)
    _, _, Xc = B.surrogate(lig, X0, prm, want_grad=False)
    for k in range(len(prm)):
        for hh in (h, 1e-7):
            e = np.zeros(len(prm))
            e[k] = hh
            Fp, _, Xp = B.surrogate(lig, X0, prm + e, want_grad=False)
            Fm, _, Xm = B.surrogate(lig, X0, prm - e, want_grad=False)
            ok = np.array_equal(_cells(Xp), _cells(Xc)) and np.array_equal(_cells(Xm), _cells(Xc))
            if ok:
                g[k] = (Fp - Fm) / (2 * hh)
                break
        else:
            crossed[k] = True
    return g, crossed


@pytest.mark.parametrize("seed", range(6))
def test_gradient_matches_central_differences(seed):
    pts = configs.SINGLE.pocket_points()
    P, B = _blur(pts)
    lig = synth.ligands(4, seed, 1, 20, 40, 2, 8).ligand(0)
    rng = np.random.default_rng(seed)
    X0 = _pose(lig, pts.mean(0).astype(np.float64) + rng.normal(0, 1.0, 3))
    nr = len(lig["rot"])
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    prm = np.concatenate([rng.normal(0, 0.3, 3), q, rng.normal(0, 0.4, nr)])
    F, g, _ = B.surrogate(lig, X0, prm)
    fd, crossed = _fd_grad(B, lig, X0, prm, 1e-4)
    assert crossed.sum() <= 2, crossed
    for sl in (slice(0, 3), slice(3, 7), slice(7, 7 + nr)):
        keep = ~crossed[sl]
        a, b = g[sl][keep], fd[sl][keep]
        if len(a):
            assert np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-6) <= 1e-3, (sl, a, b)


def test_quaternion_gradient_is_tangent():
    pts = configs.SINGLE.pocket_points()
    P, B = _blur(pts)
    lig = synth.ligands(4, 11, 1, 20, 40, 2, 8).ligand(0)
    X0 = _pose(lig, pts.mean(0).astype(np.float64))
    rng = np.random.default_rng(1)
    for _ in range(10):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        prm = np.concatenate([rng.normal(0, 0.3, 3), q, rng.normal(0, 0.4, len(lig["rot"]))])
        _, g, _ = B.surrogate(lig, X0, prm)
        assert abs(np.dot(g[3:7], q)) <= 1e-10 * max(1.0, np.linalg.norm(g[3:7]))


def test_forward_kinematics_independent():
    """FK applied root first about current axes equals leaf-first rotations
    about the original axes (scipy rotation vectors), then the rigid motion."""
    pts = configs.SINGLE.pocket_points()
    _, B = _blur(pts)
    rng = np.random.default_rng(2)
    for i in range(6):
        lig = synth.ligands(4, 20 + i, 1, 20, 60, 3, 10).ligand(0)
        l = len(lig["x"])
        X0 = _pose(lig, pts.mean(0).astype(np.float64))
        nr = len(lig["rot"])
        order, near, far, mov = oracle.torsion_tree(lig)
        dist = refimpl.bond_distances(l, lig["bonds"])
        depth = dist[0][near]
        assert np.all(np.diff(depth[order]) >= 0)  # root first
        for r in range(nr):
            a, c = lig["rot"][r]
            m = refimpl.left_mask(l, lig["bonds"], a, c)
            assert np.array_equal(mov[r], ~m if m[0] else m)  # the side without atom 0 moves
        tau = rng.normal(0, 0.8, nr)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        t = rng.normal(0, 0.5, 3)
        _, _, X = B.surrogate(lig, X0, np.concatenate([t, q, tau]), want_grad=False)
        Y = X0.copy()
        for r in order[::-1]:  # leaf first, original axes
            k = X0[far[r]] - X0[near[r]]
            k /= np.linalg.norm(k)
            R = refimpl.Rotation.from_rotvec(tau[r] * k)
            Y[mov[r]] = X0[near[r]] + R.apply(Y[mov[r]] - X0[near[r]])
        c0 = X0.mean(0)
        Rq = refimpl.Rotation.from_quat([q[1], q[2], q[3], q[0]])
        Y = Rq.apply(Y - c0) + c0 + t
        assert np.allclose(X, Y, atol=1e-10)
        # identity parameters give back the input pose
        _, _, Xi = B.surrogate(lig, X0, np.concatenate([[0, 0, 0, 1, 0, 0, 0], np.zeros(nr)]), want_grad=False)
        assert np.allclose(Xi, X0, atol=1e-12)


def test_ascent_increases_the_surrogate():
    pts = configs.SINGLE.pocket_points()
    P, B = _blur(pts)
    rng = np.random.default_rng(3)
    ups = 0
    for i in range(8):
        lig = synth.ligands(4, 40 + i, 1, 20, 40, 2, 8).ligand(0)
        X0 = _pose(lig, pts.mean(0).astype(np.float64) + rng.normal(0, 1.5, 3))
        F0, _, _ = B.surrogate(lig, X0, np.concatenate([[0, 0, 0, 1, 0, 0, 0], np.zeros(len(lig["rot"]))]))
        prm, X, F = B.refine(lig, X0, steps=50)
        ups += F > F0
        # the refined pose is rigid-body + torsion motion of the input: bonds keep their length
        b = lig["bonds"]
        assert np.allclose(np.linalg.norm(X[b[:, 0]] - X[b[:, 1]], axis=1),
                           np.linalg.norm(X0[b[:, 0]] - X0[b[:, 1]], axis=1), atol=1e-9)
    assert ups >= 7


# --------------------------------------------------------------------------
# The ascent's step rule, pinned by its properties: given the gradient g at
# the current parameters (itself pinned by central differences above), one
# step moves t by lr_t g_t shortened along its own direction to length
# max_dt, puts q on the unit sphere in the direction of q + lr_q g_q, and
# moves each tau_b by lr_tau g_b clamped to [-max_dtau, max_dtau] on its own;
# a zero learning rate leaves every parameter and the pose unchanged.

def _f32(v):
    return float(np.float32(v))


def _step_cases():
    pts = configs.SINGLE.pocket_points()
    P, B = _blur(pts)
    rng = np.random.default_rng(21)
    for i in range(6):
        lig = synth.ligands(4, 80 + i, 1, 20, 48, 4, 10).ligand(0)
        X0 = _pose(lig, pts.mean(0).astype(np.float64) + rng.normal(0, 1.2, 3))
        nr = len(lig["rot"])
        p0 = np.concatenate([[0, 0, 0, 1, 0, 0, 0], np.zeros(nr)])
        yield B, lig, X0, p0


def test_ascent_zero_rate_is_the_identity():
    for B, lig, X0, p0 in _step_cases():
        F0, _, _ = B.surrogate(lig, X0, p0, want_grad=False)
        prm, X, F = B.refine(lig, X0, steps=7, lr_t=0.0, lr_q=0.0, lr_tau=0.0)
        assert np.array_equal(prm, p0)
        assert np.allclose(X, X0, rtol=0, atol=1e-12)
        assert F == pytest.approx(F0, rel=1e-14, abs=1e-300)


def test_ascent_translation_is_norm_clipped():
    n_clip = n_free = 0
    for B, lig, X0, p0 in _step_cases():
        _, g, _ = B.surrogate(lig, X0, p0)
        gt = g[:3]
        assert np.linalg.norm(gt) > 0
        # large rate: the step has length max_dt and the direction of g_t (a
        # per-component clip would bend it towards the diagonal)
        for lr_t, max_dt in ((10.0, 0.05), (1e-4, 100.0)):
            prm, _, _ = B.refine(lig, X0, steps=1, lr_t=lr_t, lr_q=0.0, lr_tau=0.0, max_dt=max_dt, max_dtau=0.0)
            d = prm[:3]
            want = _f32(lr_t) * gt
            if np.linalg.norm(want) > _f32(max_dt):
                n_clip += 1
                assert np.linalg.norm(d) == pytest.approx(_f32(max_dt), rel=1e-12)
                assert np.allclose(d / np.linalg.norm(d), gt / np.linalg.norm(gt), rtol=0, atol=1e-12)
            else:
                n_free += 1
                assert np.allclose(d, want, rtol=1e-12, atol=1e-18)
            assert np.array_equal(prm[3:], p0[3:])
        # every step of a longer clipped run has length max_dt
        prev = None
        for k in range(1, 4):
            prm, _, _ = B.refine(lig, X0, steps=k, lr_t=10.0, lr_q=0.0, lr_tau=0.0, max_dt=0.05, max_dtau=0.0)
            step = prm[:3] - (prev if prev is not None else 0.0)
            assert np.linalg.norm(step) == pytest.approx(_f32(0.05), rel=1e-9)
            prev = prm[:3].copy()
    assert n_clip == 6 and n_free == 6


def test_ascent_quaternion_is_renormalised():
    for B, lig, X0, p0 in _step_cases():
        _, g, _ = B.surrogate(lig, X0, p0)
        lr = 0.05
        prm, _, _ = B.refine(lig, X0, steps=1, lr_t=0.0, lr_q=lr, lr_tau=0.0, max_dt=0.0, max_dtau=0.0)
        q = p0[3:7] + _f32(lr) * g[3:7]
        assert np.linalg.norm(q) > 1 + 1e-9  # the tangent step leaves the sphere
        assert np.allclose(prm[3:7], q / np.linalg.norm(q), rtol=0, atol=1e-14)
        for k in range(1, 5):
            prm, X, _ = B.refine(lig, X0, steps=k, lr_t=0.0, lr_q=lr, lr_tau=0.0, max_dt=0.0, max_dtau=0.0)
            assert abs(np.linalg.norm(prm[3:7]) - 1.0) < 1e-14
            # a pure rotation about the centroid: distances to it are kept
            c0 = X0.mean(0)
            assert np.allclose(np.linalg.norm(X - c0, axis=1), np.linalg.norm(X0 - c0, axis=1), atol=1e-10)


def test_ascent_torsions_are_clamped_one_by_one():
    n_clamped = n_free = 0
    for B, lig, X0, p0 in _step_cases():
        _, g, _ = B.surrogate(lig, X0, p0)
        gtau = g[7:]
        lr = 1.0
        # a cap between the smallest and the largest |lr g_b|: some clamp, some do not
        a = np.sort(np.abs(_f32(lr) * gtau[gtau != 0]))
        assert len(a) >= 2
        cap = _f32(0.5 * (a[0] + a[-1]))
        prm, _, _ = B.refine(lig, X0, steps=1, lr_t=0.0, lr_q=0.0, lr_tau=lr, max_dt=0.0, max_dtau=cap)
        want = np.clip(_f32(lr) * gtau, -cap, cap)
        assert np.allclose(prm[7:], want, rtol=1e-12, atol=0)
        n_clamped += int(np.sum(np.abs(_f32(lr) * gtau) > cap))
        n_free += int(np.sum(np.abs(_f32(lr) * gtau) < cap))
        assert np.array_equal(prm[:7], p0[:7])
    assert n_clamped >= 6 and n_free >= 6


# --------------------------------------------------------------------------
# Clash-penalised surrogate: F - lam sum_{far pairs, d < c} (c^2 - d^2)^2

def _fd_grad_pen(B, lig, X0, prm, h, **kw):
    # the penalty is C1 in the coordinates; the density part needs the
    # stencil to stay inside its trilinear cells, as above
    g = np.zeros(len(prm))
    crossed = np.zeros(len(prm), bool)
    _, _, Xc = B.surrogate(lig, X0, prm, want_grad=False, **kw)
    for k in range(len(prm)):
        for hh in (h, 1e-7):
            e = np.zeros(len(prm))
            e[k] = hh
            Fp, _, Xp = B.surrogate(lig, X0, prm + e, want_grad=False, **kw)
            Fm, _, Xm = B.surrogate(lig, X0, prm - e, want_grad=False, **kw)
            if np.array_equal(_cells(Xp), _cells(Xc)) and np.array_equal(_cells(Xm), _cells(Xc)):
                g[k] = (Fp - Fm) / (2 * hh)
                break
        else:
            crossed[k] = True
    return g, crossed


@pytest.mark.parametrize("seed", range(4))
def test_clash_penalty_value_and_gradient(seed):
    pts = configs.SINGLE.pocket_points()
    P, B = _blur(pts)
    lig = synth.ligands(4, 10 + seed, 1, 20, 40, 2, 8).ligand(0)
    rng = np.random.default_rng(50 + seed)
    X0 = _pose(lig, pts.mean(0).astype(np.float64) + rng.normal(0, 1.0, 3))
    nr = len(lig["rot"])
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    prm = np.concatenate([rng.normal(0, 0.3, 3), q, rng.normal(0, 0.6, nr)])
    # a wide bump distance puts several far pairs inside the penalty band
    kw = dict(clash_weight=0.25, clash_dist=4.5, clash_min_bonds=4)
    F0, _, X = B.surrogate(lig, X0, prm)
    F1, g1, X1 = B.surrogate(lig, X0, prm, **kw)
    assert np.array_equal(X, X1)
    # value: an independent brute force over the bond-count distances
    _, dist, _ = oracle.topology(lig)
    iu = np.triu_indices(len(X), 1)
    far = dist[iu] >= 4
    d2 = ((X[iu[0]] - X[iu[1]]) ** 2).sum(1)
    band = far & (d2 < 4.5 ** 2)
    assert band.sum() >= 1
    pen = 0.25 * ((4.5 ** 2 - d2[band]) ** 2).sum()
    assert F1 == pytest.approx(F0 - pen, rel=1e-12, abs=1e-12)
    # gradient: central differences
    gfd, crossed = _fd_grad_pen(B, lig, X0, prm, 1e-5, **kw)
    ok = ~crossed
    assert ok.sum() >= len(prm) - 2
    assert np.allclose(g1[ok], gfd[ok], rtol=2e-4, atol=2e-4 * (1 + np.abs(g1).max()))
    # the weight 0 is the plain surrogate
    F2, g2, _ = B.surrogate(lig, X0, prm, clash_weight=0.0, clash_dist=4.5)
    F3, g3, _ = B.surrogate(lig, X0, prm)
    assert F2 == F3 and np.array_equal(g2, g3)


def test_penalised_ascent_has_fewer_bumps():
    # an aggressive torsion ascent on the plain surrogate ends with bumping
    # far pairs; the penalised one (weight 10) ends with at most half as many
    pts = configs.SINGLE.pocket_points()
    P, B = _blur(pts)
    plain = pen = 0
    for seed in range(12):
        lig = synth.ligands(4, 30 + seed, 1, 30, 50, 4, 8).ligand(0)
        X0 = _pose(lig, pts.mean(0).astype(np.float64))
        _, dist, _ = oracle.topology(lig)
        iu = np.triu_indices(len(X0), 1)
        far = dist[iu] >= 4

        def bumps(X):
            return int((far & (((X[iu[0]] - X[iu[1]]) ** 2).sum(1) < 4.0)).sum())
        _, Xa, _ = B.refine(lig, X0, steps=60, lr_tau=5e-3, max_dtau=0.2)
        _, Xb, _ = B.refine(lig, X0, steps=60, lr_tau=5e-3, max_dtau=0.2, clash_weight=10.0)
        plain += bumps(Xa)
        pen += bumps(Xb)
    assert plain >= 10 and 2 * pen <= plain
