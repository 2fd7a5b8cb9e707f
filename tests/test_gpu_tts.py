"""The time-to-solution campaign on the GPU (Eq. 4): small campaign, one
regression per configuration, predictions and the budget choice."""
import numpy as np
import pytest

import synth
from synth import configs
from tests import gpuutil
from tests.gpuutil import gpu


@pytest.fixture(scope="module")
def g():
    return gpuutil.gd()


@gpu
def test_campaign_fit_and_choice(g):
    from paper_1901_06363_amd import tts
    pockets = []
    for k in (0, 1):
        pts = configs.GRID.pocket_points(k)
        pockets.append((g.Pocket(pts, 0.5, 20.0), len(pts)))
    sets = [synth.ligands(40 + i, 0, 48, lo, hi, bl, bh, 0.0)
            for i, (lo, hi, bl, bh) in enumerate(((20, 30, 2, 3), (30, 50, 2, 6), (40, 80, 4, 10), (60, 90, 2, 4),
                                                   (25, 45, 6, 9)))]
    q = synth.quaternions(3, 8)
    cfgs = [dict(hp=10, lp=10, threshold=0.0, repetitions=1, refine=False),
            dict(hp=5, lp=90, threshold=0.6, repetitions=2, refine=True)]
    recs = tts.campaign(pockets, sets, q, cfgs, top_k=1)
    assert len(recs) == 2 * 5 * 2
    assert all(r["ms"] > 0 and r["nu"] == 48 for r in recs)
    assert {r["p"] for r in recs} == {1000, 2000}
    models = tts.fit_models(recs)
    assert set(models) == {tts.key(c) for c in cfgs}
    for m in models.values():
        assert np.isfinite(m.r2) and m.n == 10
    # the fit reproduces its own observations on average within a factor of two
    obs = [r["ms"] / r["nu"] for r in recs if tts.key(r) == tts.key(cfgs[0])]
    m0 = models[tts.key(cfgs[0])]
    pred = [m0.per_ligand(r["p"], r["a"], r["r"]) for r in recs if tts.key(r) == tts.key(cfgs[0])]
    assert abs(np.mean(pred) - np.mean(obs)) <= 0.5 * np.mean(obs)
    deg = {tts.key(cfgs[0]): 0.0, tts.key(cfgs[1]): 10.0}
    a, r = tts.ligand_features(sets[2])
    big = tts.choose(models, deg, 2000, a, r, 1000, budget_ms=1e12)
    assert big["key"] == tts.key(cfgs[0]) and big["completion"] == 1.0
    tiny = tts.choose(models, deg, 2000, a, r, 1000, budget_ms=1e-6)
    assert tiny["completion"] < 1.0
