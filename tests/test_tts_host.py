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
