"""GPU parity of the knob exploration (Sections IV-B, V-B) against an
oracle-side pipeline: oracle docking (Alg. 2) of every ligand under every
configuration, its top-1 pose rounded to the FP32 the GPU returns, the
oracle's continuous Eq. 1, then Eq. 5 and the Pareto front written out here.
Per-ligand scores must agree bit for bit; means and degradations to 1e-12."""
import math

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


SPACE = dict(hp=[1, 10], lp=[90], threshold=[0.0, 0.6], repetitions=[1, 3], refine=[False, True])


def _oracle_scores(O, ligs, q, cfg):
    kn = oracle.knobs(hp=cfg["hp"], lp=cfg["lp"], threshold=cfg["threshold"], repetitions=cfg["repetitions"],
                      refine=cfg["refine"])
    scores, xyz = [], []
    for i in range(ligs.n):
        r = oracle.dock(O, ligs.ligand(i), kn, q)
        top = int(oracle.topk(r.S, r.clash, 1)[0])
        X = r.xyz[top].astype(np.float32)
        xyz.append(X)
        _, _, o = O.overlap_continuous(X.astype(np.float64))
        scores.append(o if r.clash[top] == 0 else 0.0)
    return np.array(scores), np.concatenate(xyz)


@gpu
def test_dse_matches_oracle_pipeline(g):
    import torch
    from paper_1901_06363_amd import dse
    w = configs.SCREEN
    pts = w.pocket_points()
    P, O = g.Pocket(pts, 0.5, 20.0), oracle.OraclePocket(pts, 0.5)
    ligs = synth.ligands(31, 0, 24, 18, 30, 2, 4, 0.0)
    q = synth.quaternions(5, 6)
    frac = 0.1  # top 10 % of 24 ligands: the best 3
    recs = dse.explore(P, ligs, q, space=SPACE, top_k=1, frac=frac)
    cfgs = dse.configurations(SPACE)
    assert len(recs) == len(cfgs) == 16
    means = []
    for rec, cfg in zip(recs, cfgs):
        assert all(rec[k] == cfg[k] for k in cfg)
        exp, X = _oracle_scores(O, ligs, q, cfg)
        got = dse.ligand_scores(P, ligs, q, cfg, top_k=1)
        px, py, pz = got["xyz"]
        Xg = torch.stack([px, py, pz], 1).cpu().numpy()
        assert np.array_equal(Xg, X), cfg            # same FP32 poses
        assert np.array_equal(got["score"], exp), cfg  # same continuous overlaps, bit for bit
        kk = max(1, math.ceil(frac * len(exp)))
        m = sum(sorted(exp.tolist(), reverse=True)[:kk]) / kk
        assert abs(rec["top_mean"] - m) <= 1e-12 * abs(m)
        means.append(m)
    base = [m for m, c in zip(means, cfgs) if c["hp"] == 1 and c["threshold"] == 0.0 and c["repetitions"] == 3
            and not c["refine"]][0]
    for rec, m in zip(recs, means):
        assert abs(rec["degradation"] - 100.0 * (1.0 - m / base)) <= 1e-9
        assert rec["time_ms"] > 0 and rec["atoms_per_s"] > 0
    assert any(r["degradation"] == 0.0 for r in recs)
    # front: no kept record is dominated, every dropped one is
    t = np.array([r["atoms_per_s"] for r in recs])
    d = np.array([r["degradation"] for r in recs])
    for i, r in enumerate(recs):
        dom = (t >= t[i]) & (d <= d[i]) & ((t > t[i]) | (d < d[i]))
        assert r["pareto"] == (not dom.any())


@gpu
def test_dse_baseline_added_when_missing(g):
    from paper_1901_06363_amd import dse
    w = configs.SCREEN
    P = g.Pocket(w.pocket_points(), 0.5, 20.0)
    ligs = synth.ligands(32, 0, 8, 18, 26, 2, 3, 0.0)
    q = synth.quaternions(6, 4)
    recs = dse.explore(P, ligs, q, space=dict(hp=[30], repetitions=[1]), top_k=2, frac=0.25)
    assert len(recs) == 2 and dse.is_baseline(recs[0]) and recs[0]["degradation"] == 0.0
    with pytest.raises(ValueError):
        dse.explore(P, ligs, q, space=dict(hp=[30], repetitions=[1]), include_baseline=False)


@gpu
@pytest.mark.parametrize("cfg", [dict(hp=1, lp=45, threshold=0.0, repetitions=3, refine=False),
                                 dict(hp=5, lp=90, threshold=0.8, repetitions=1, refine=True)])
def test_dse_full_size_sampled(g, cfg):
    """The exploration workload at its full size (20,000 ligands x 32
    orientations, the launch the exploration times) for the baseline and the
    fastest full-space configuration; 6 sampled ligands' scores against the
    oracle pipeline."""
    import torch
    from paper_1901_06363_amd import dse
    w = configs.DSE
    pts = w.pocket_points()
    P, O = g.Pocket(pts, 0.5, w.pad), oracle.OraclePocket(pts, 0.5)
    ligs = w.ligands()
    q = w.quaternions()
    got = dse.ligand_scores(P, ligs, q, cfg, top_k=1)
    assert len(got["score"]) == 20000 and got["feasible"].mean() > 0.99
    px, py, pz = got["xyz"]
    Xg = torch.stack([px, py, pz], 1).cpu().numpy()
    off = np.concatenate([[0], np.cumsum(np.diff(np.asarray(ligs.atom_off)))])
    rng = np.random.default_rng(3)
    idx = rng.choice(ligs.n, 6, replace=False)
    exp, X = _oracle_scores(O, ligs.subset(idx), q, cfg)
    xo = np.concatenate([[0], np.cumsum([ligs.n_atoms(int(i)) for i in idx])])
    for t, i in enumerate(idx):
        assert got["score"][i] == exp[t], i
        assert np.array_equal(Xg[off[i]:off[i + 1]], X[xo[t]:xo[t + 1]]), i
