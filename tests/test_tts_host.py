"""Pins of the time-to-solution model (Eq. 4, Section III-D) and the
budget-driven knob choice (Section V-D): host logic, no GPU."""
import numpy as np
import pytest

from paper_1901_06363_amd import tts


def test_features_are_the_seven_predictors():
    # Eq. 4: pocket points, mean atoms, mean rotamers and every interaction
    assert tts.FEATURES == ("p", "a", "r", "p*a", "p*r", "a*r", "p*a*r")
    assert list(tts.features(2, 3, 5)) == [2, 3, 5, 6, 10, 15, 30]


def _grid():
    P, A, R = [], [], []
    for p in (1000, 2000, 4000, 8000):
        for a, r in ((25, 3), (40, 6), (60, 9), (75, 11), (90, 14)):
            P.append(p)
            A.append(a + 0.1 * p / 1000)
            R.append(r + 0.05 * a / 10)
    return np.array(P, float), np.array(A), np.array(R)


def test_fit_recovers_planted_coefficients():
    P, A, R = _grid()
    alpha = np.array([1e-4, 2e-3, 3e-2, 4e-7, 5e-6, 6e-5, 7e-9])
    beta = 0.25
    y = np.array([alpha @ tts.features(p, a, r) + beta for p, a, r in zip(P, A, R)])
    m = tts.fit(P, A, R, y)
    assert np.allclose(m.alpha, alpha, rtol=1e-6, atol=1e-15)
    assert abs(m.beta - beta) < 1e-9
    assert m.r2 > 1 - 1e-12 and m.r2_adj > 1 - 1e-12 and m.n == len(P)
    # Eq. 4 scales the per-ligand time by the database size
    assert m.predict(3000, 50, 7, 1000) == pytest.approx(1000 * m.per_ligand(3000, 50, 7))


def test_r2_and_adjusted_r2_against_their_definitions():
    rng = np.random.default_rng(3)
    P, A, R = _grid()
    y = 1e-3 * A + 0.01 * R + rng.normal(0, 0.01, len(P))
    m = tts.fit(P, A, R, y)
    pred = np.array([m.per_ligand(p, a, r) for p, a, r in zip(P, A, R)])
    ss_res = ((y - pred) ** 2).sum()
    ss_tot = ((y - y.mean()) ** 2).sum()
    r2 = 1 - ss_res / ss_tot
    assert m.r2 == pytest.approx(r2, rel=1e-9)
    n, q = len(y), 7
    assert m.r2_adj == pytest.approx(1 - (1 - r2) * (n - 1) / (n - q - 1), rel=1e-9)
    # least squares: the residual is orthogonal to every predictor column
    X = np.stack([np.append(tts.features(p, a, r), 1.0) for p, a, r in zip(P, A, R)])
    Xs = X / np.abs(X).max(axis=0)
    assert np.all(np.abs(Xs.T @ (y - pred)) < 1e-8)


def test_fit_needs_enough_observations():
    with pytest.raises(ValueError):
        tts.fit([1, 2, 3], [1, 2, 3], [1, 2, 3], [1, 2, 3])


def _const_model(per_ligand_ms):
    return tts.LinearModel(np.zeros(7), per_ligand_ms, 1.0, 1.0, 8)


def test_budget_choice():
    k_fast, k_mid, k_slow = ("fast",), ("mid",), ("slow",)
    models = {k_fast: _const_model(1.0), k_mid: _const_model(2.0), k_slow: _const_model(4.0)}
    deg = {k_fast: 20.0, k_mid: 5.0, k_slow: 0.0}
    # 1,000 ligands: 1, 2 and 4 s predicted
    c = tts.choose(models, deg, 4000, 50, 8, 1000, budget_ms=5000)
    assert c["key"] == k_slow and c["completion"] == 1.0 and c["predicted_ms"] == 4000
    c = tts.choose(models, deg, 4000, 50, 8, 1000, budget_ms=2500)
    assert c["key"] == k_mid and c["degradation"] == 5.0
    c = tts.choose(models, deg, 4000, 50, 8, 1000, budget_ms=1000)
    assert c["key"] == k_fast and c["completion"] == 1.0
    # nothing fits: the fastest, finishing part of the database
    c = tts.choose(models, deg, 4000, 50, 8, 1000, budget_ms=250)
    assert c["key"] == k_fast and c["completion"] == 0.25
    # equal degradation: the faster of the two
    c = tts.choose(models, {k_fast: 1.0, k_mid: 1.0}, 4000, 50, 8, 1000, budget_ms=1e9)
    assert c["key"] == k_fast
    with pytest.raises(ValueError):
        tts.choose(models, {}, 4000, 50, 8, 1000, budget_ms=1)


def test_fit_models_groups_by_configuration():
    P, A, R = _grid()
    recs = []
    for cfg, slope in ((dict(hp=1, lp=45, threshold=0.0, repetitions=3, refine=False), 2e-3),
                       (dict(hp=5, lp=90, threshold=0.6, repetitions=1, refine=True), 1e-4)):
        for p, a, r in zip(P, A, R):
            recs.append(dict(cfg, p=p, a=a, r=r, nu=500, ms=500 * (slope * a * r + 0.1)))
    models = tts.fit_models(recs)
    assert set(models) == {(1, 45, 0.0, 3, False), (5, 90, 0.6, 1, True)}
    m = models[(1, 45, 0.0, 3, False)]
    assert m.per_ligand(2000, 50, 7) == pytest.approx(2e-3 * 50 * 7 + 0.1, rel=1e-6)


def test_floor_of_a_run():
    # t = max(c, nu u): below the size where the slowest work item decides,
    # the prediction is the floor; above it, Eq. 4
    P, A, R = _grid()
    cfg = dict(hp=3, lp=45, threshold=0.0, repetitions=2, refine=False)
    u = lambda p, a, r: 1e-3 * a * r + 1e-5 * p
    recs = [dict(cfg, p=p, a=a, r=r, nu=5000, ms=5000 * u(p, a, r)) for p, a, r in zip(P, A, R)]
    fl = tts.floors([dict(cfg, p=4000, a=50, r=7, nu=1000, ms=120.0)])
    assert fl == {tts.key(cfg): 120.0}
    m = tts.fit_models(recs, fl)[tts.key(cfg)]
    assert m.floor == 120.0
    p, a, r = 4000, 50, 7
    assert m.predict(p, a, r, 100) == 120.0
    assert m.predict(p, a, r, 10 ** 6) == pytest.approx(10 ** 6 * u(p, a, r), rel=1e-6)
    assert tts.fit_models(recs)[tts.key(cfg)].predict(p, a, r, 100) == pytest.approx(100 * u(p, a, r), rel=1e-6)


# --------------------------------------------------------------------------
# Peak analysis (Section III-B): delta overlap, peaks, widths and heights

def test_circular_runs():
    from paper_1901_06363_amd import peaks
    assert peaks.circular_runs([]) == []
    assert peaks.circular_runs([False, False]) == []
    assert peaks.circular_runs([True] * 5) == [(0, 5)]
    # a run across the wrap-around is one run
    assert sorted(peaks.circular_runs([True, True, False, True])) == [(3, 3)]
    assert sorted(peaks.circular_runs([True, False, True, False, False, True, True])) == [(2, 1), (5, 3)]


def test_analyse_side_closed_forms():
    from paper_1901_06363_amd import peaks
    th = np.arange(360)
    # one smooth bump: o = 2 + cos(theta - 100 deg); above the midpoint over
    # (10, 190) exclusive -> 179 angles, height 1
    o = 2 + np.cos(np.radians(th - 100))
    a = peaks.analyse_side(o, np.ones(360, bool))
    assert a["delta"] == pytest.approx(2.0) and len(a["peaks"]) == 1
    w, h, s = a["peaks"][0]
    assert w == 179 and h == pytest.approx(1.0) and s == 11
    # a bump across 0 degrees stays one peak
    a = peaks.analyse_side(2 + np.cos(np.radians(th)), np.ones(360, bool))
    assert len(a["peaks"]) == 1 and a["peaks"][0][0] == 179
    # an invalid (bumping) gap splits it; the part without the maximum is lower
    v = np.ones(360, bool)
    v[60:70] = False
    a = peaks.analyse_side(o, v)
    assert sorted(p[0] for p in a["peaks"]) == [49, 120]
    assert max(p[1] for p in a["peaks"]) == pytest.approx(1.0) and min(p[1] for p in a["peaks"]) < 1.0
    # two bumps of different heights: two peaks, heights 1 and (2.6 - 1) / 2;
    # a bump below half the delta is no peak
    o2 = np.where(np.abs(th - 90) < 20, 3.0, np.where(np.abs(th - 270) < 10, 2.6, 1.0))
    o2[200] = 1.9
    a = peaks.analyse_side(o2, np.ones(360, bool))
    got = sorted((p[0], round(p[1], 6)) for p in a["peaks"])
    assert got == [(19, 0.8), (39, 1.0)]
    # flat landscape: no peak; nothing valid: None; step scales widths
    assert peaks.analyse_side(np.ones(360), np.ones(360, bool))["peaks"] == []
    assert peaks.analyse_side(o, np.zeros(360, bool)) is None
    a5 = peaks.analyse_side(o[::5], np.ones(72, bool), step=5)
    assert a5["peaks"][0][0] == 5 * 35  # samples 15, 20, ..., 185


def test_analyse_and_summary_shapes():
    from paper_1901_06363_amd import peaks
    th = np.arange(360)
    S = np.full((1, 1, 2, 2, 360), 100, np.int64)
    S[0, 0, 0, 0] = 100 - np.round(20 * np.cos(np.radians(th))).astype(np.int64)  # one peak near 0
    f = np.ones_like(S, np.uint8)
    f[0, 0, 1, 1] = 0  # a side with no valid angle is skipped
    recs = peaks.analyse(S, f, np.array([[[[3, 9], [6, 6]]]]), [12], [2], np.array([[80]]))
    assert len(recs) == 3
    r0 = [r for r in recs if r["rotamer"] == 0 and r["side"] == 0][0]
    assert r0["rel_size"] == 0.25 and r0["n_peaks"] == 1
    # delta normalised by the final overlap l / (h^2 S_final)
    o = 12 / (0.25 * S[0, 0, 0, 0])
    assert r0["delta_norm"] == pytest.approx((o.max() - o.min()) / (12 / (0.25 * 80)))
    s = peaks.summarize(recs)
    assert s["sides"] == 3 and sum(b["sides"] for b in s["by_rel_size"]) == 3
