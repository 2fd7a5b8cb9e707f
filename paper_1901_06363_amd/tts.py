"""Time-to-solution model (Eq. 4) and knob choice under a time budget
(Sections III-D, V-C and V-D).

Per knob configuration k the time to dock one ligand of a database is modelled
as a multivariate linear regression with interactions on the input's average
features

    x = (p, a, r, p a, p r, a r, p a r)

(p: pocket points, a: mean atoms per ligand, r: mean rotatable bonds per
ligand), t_ligand = alpha(k) . x + beta(k), and a database of nu ligands takes
t = nu (alpha(k) . x + beta(k)) (Eq. 4).  The coefficients are fitted per
configuration by least squares from a profiling campaign on the target GPU;
the accuracy of each configuration (its Eq. 5 degradation) comes from a
separate exploration, since it does not depend on the platform.  Given a time
budget the tuner picks the configuration with the lowest degradation whose
predicted time fits, or else the fastest one and the fraction of the database
it can finish.

On a GPU the run time of a database is proportional to its size only once
the device is full: every (ligand, block of orientations) work item runs on
one wave, so a small database takes as long as its slowest item, whatever
its size.  The model therefore takes the coefficients from runs large enough
to be throughput-bound and carries, per configuration, a floor c(k) (ms), the
time of a small run: t = max(c(k), nu (alpha(k) . x + beta(k))).  c = 0 gives
Eq. 4 as printed.
"""
from __future__ import annotations

import numpy as np

FEATURES = ("p", "a", "r", "p*a", "p*r", "a*r", "p*a*r")


def key(cfg) -> tuple:
    """Hashable identity of a knob configuration."""
    return (int(cfg["hp"]), int(cfg["lp"]), float(cfg["threshold"]), int(cfg["repetitions"]), bool(cfg["refine"]))


def features(p, a, r) -> np.ndarray:
    """The seven predictors of Eq. 4 for one input (pocket points p, mean atoms
    a, mean rotatable bonds r)."""
    p, a, r = float(p), float(a), float(r)
    return np.array([p, a, r, p * a, p * r, a * r, p * a * r])


def ligand_features(ligands):
    """(mean atoms, mean rotatable bonds) of a ligand batch (CSR offsets)."""
    at = np.diff(np.asarray(ligands.atom_off, np.int64))
    rt = np.diff(np.asarray(ligands.rot_off, np.int64))
    return float(at.mean()), float(rt.mean())


class LinearModel:
    """t_ligand = alpha . x + beta for one configuration, with its fit quality
    and the floor of a run (`floor`, ms)."""

    def __init__(self, alpha, beta, r2, r2_adj, n, floor=0.0):
        self.alpha, self.beta, self.r2, self.r2_adj, self.n = np.asarray(alpha, np.float64), float(beta), r2, r2_adj, n
        self.floor = float(floor)

    def per_ligand(self, p, a, r) -> float:
        return float(self.alpha @ features(p, a, r) + self.beta)

    def predict(self, p, a, r, nu) -> float:
        """Eq. 4 (with the floor of a run): time for nu ligands with these
        average features."""
        return max(self.floor, nu * self.per_ligand(p, a, r))


def fit(P, A, R, t_ligand) -> LinearModel:
    """Least-squares fit of Eq. 4's regression for one configuration from
    observations (pocket points, mean atoms, mean rotamers, time per ligand).
    Columns are scaled to unit maximum before solving for conditioning; the
    coefficients are returned in the original units.  R^2 and the adjusted
    R^2 (n - 1) / (n - q - 1) on q = 7 predictors are computed on the
    training observations."""
    X = np.stack([features(p, a, r) for p, a, r in zip(P, A, R)])
    y = np.asarray(t_ligand, np.float64)
    n, q = X.shape
    if n < q + 1:
        raise ValueError("need at least %d observations, got %d" % (q + 1, n))
    M = np.hstack([X, np.ones((n, 1))])
    scale = np.abs(M).max(axis=0)
    scale[scale == 0] = 1.0
    coef, *_ = np.linalg.lstsq(M / scale, y, rcond=None)
    coef = coef / scale
    res = y - M @ coef
    ss_res = float(res @ res)
    ss_tot = float(((y - y.mean()) ** 2).sum())
    r2 = 1.0 - ss_res / ss_tot if ss_tot > 0 else 1.0
    r2_adj = 1.0 - (1.0 - r2) * (n - 1) / (n - q - 1) if n > q + 1 else float("nan")
    return LinearModel(coef[:q], coef[q], r2, r2_adj, n)


def floors(records) -> dict:
    """Floor c(k) of every configuration: the kernel time of its run in
    `records` (small databases, where the slowest work item decides)."""
    return {key(r): float(r["ms"]) for r in records}


def fit_models(records, floor=None) -> dict:
    """One model per configuration from campaign records (dicts with the knob
    fields and p, a, r, nu, ms), fitted to ms / nu; `floor` (key -> c(k) ms)
    sets the models' floors."""
    groups = {}
    for rec in records:
        groups.setdefault(key(rec), []).append(rec)
    models = {}
    for k, v in groups.items():
        m = fit([g["p"] for g in v], [g["a"] for g in v], [g["r"] for g in v], [g["ms"] / g["nu"] for g in v])
        m.floor = (floor or {}).get(k, 0.0)
        models[k] = m
    return models


def choose(models, degradation, p, a, r, nu, budget_ms) -> dict:
    """Budget-driven knob choice.  `degradation` maps a configuration key to
    its Eq. 5 degradation (percent).  Among configurations whose predicted
    time for nu ligands fits the budget, the one with the lowest degradation
    wins (ties to the faster); if none fits, the fastest is taken and only
    part of the database is docked.  Returns the key, predicted_ms,
    degradation and completion (fraction of the nu ligands docked within the
    budget)."""
    cands = []
    for k, m in models.items():
        if k not in degradation:
            continue
        cands.append((k, m.predict(p, a, r, nu), degradation[k]))
    if not cands:
        raise ValueError("no configuration has both a model and a degradation")
    fits = [c for c in cands if c[1] <= budget_ms]
    if fits:
        k, t, d = min(fits, key=lambda c: (c[2], c[1]))
    else:
        k, t, d = min(cands, key=lambda c: (c[1], c[2]))
    return dict(key=k, predicted_ms=t, degradation=d, completion=min(1.0, budget_ms / t) if t > 0 else 1.0)


def campaign(pockets, ligand_sets, quats, configs, reps=1, warm=True, progress=None, **batch_kw) -> list:
    """Profiling campaign on the GPU: every configuration on every (pocket,
    ligand set); one record per run with the knobs, p, a, r, nu and the
    docking kernel's time in ms (HIP events around the kernel alone; the
    median of `reps` timed calls, after one untimed call when `warm`).
    `pockets` is a list of (Pocket, n_points)."""
    from . import BATCHED, _torch
    torch = _torch()
    recs = []
    n_runs = len(pockets) * len(ligand_sets) * len(configs)
    i = 0
    from .dse import prepared_batches
    for pi, (P, npts) in enumerate(pockets):
        for li, L in enumerate(ligand_sets):
            a, r = ligand_features(L)
            for cfg, B in prepared_batches(P, L, quats, configs, **batch_kw):
                out = B.alloc_outputs(want_angles=False, want_xyz=False)
                if warm:
                    B.dock(BATCHED, out)
                B.enable_timing(True)
                for _ in range(reps):
                    B.dock(BATCHED, out)
                torch.cuda.synchronize()
                ms = float(np.median(B.read_timing()))
                rec = dict(cfg, pocket=pi, ligset=li, p=npts, a=a, r=r, nu=B.n_ligands, ms=ms)
                recs.append(rec)
                i += 1
                if progress:
                    progress(i, n_runs, rec)
                del B, out
    return recs
