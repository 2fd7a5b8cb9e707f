"""Accuracy/time trade-off of the five knobs (Sections IV-B and V-B).

For every knob configuration of a design space the library is docked on the
GPU, each ligand's best pose (top-k by the exact lattice score, feasible
poses only) is re-scored with the continuous Eq. 1 over the raw pocket
points, and the configuration is summarised by

  * its time to solution (docking kernel + re-scoring kernels, HIP events)
    and throughput in ligand atoms per second (the paper's metric),
  * the mean continuous overlap of its top 1 % ligands, and the overlap
    degradation of Eq. 5 against the baseline configuration:
    (1 - mean_approx / mean_baseline) * 100,

and the Pareto front over (throughput up, degradation down) is marked.

Design spaces (full factorial, Section V-B):
  FLAT  high-precision step {1, 2, 3, 5, 10, 15, 45, 60} x repetitions {1, 2, 3}
  FULL  high-precision step {1, 2, 3, 5} x low-precision step {45, 90} x
        threshold {0, 0.3, 0.6, 0.8} x repetitions {1, 2, 3} x
        refinement {on, off}
Baseline: high-precision step 1, threshold 0, repetitions 3, no refinement
(the low-precision step is then unused).
"""
from __future__ import annotations

import itertools
import math
import threading

import numpy as np

from . import BATCHED, Batch, _torch
from ._ops import overlap_continuous

FLAT = dict(hp=[1, 2, 3, 5, 10, 15, 45, 60], repetitions=[1, 2, 3])
FULL = dict(hp=[1, 2, 3, 5], lp=[45, 90], threshold=[0.0, 0.3, 0.6, 0.8], repetitions=[1, 2, 3],
            refine=[True, False])
BASE_KNOBS = dict(hp=1, lp=1, threshold=0.0, repetitions=3, refine=False)
SPACES = {"flat": FLAT, "full": FULL}


def configurations(space) -> list:
    """Full factorial list of knob dicts (hp, lp, threshold, repetitions,
    refine) of a design space; knobs a space does not vary take the
    baseline's values (lp follows hp where the space has no lp)."""
    space = SPACES[space] if isinstance(space, str) else space
    names = list(space)
    out = []
    for vals in itertools.product(*(space[n] for n in names)):
        k = dict(zip(names, vals))
        cfg = dict(hp=k["hp"], lp=k.get("lp", k["hp"]), threshold=float(k.get("threshold", 0.0)),
                   repetitions=k.get("repetitions", BASE_KNOBS["repetitions"]), refine=bool(k.get("refine", False)))
        out.append(cfg)
    return out


def is_baseline(cfg) -> bool:
    """The most precise configuration: hp 1, threshold 0, 3 repetitions, no
    refinement (any low-precision step: with threshold 0 it is never used)."""
    return (cfg["hp"] == BASE_KNOBS["hp"] and cfg["threshold"] == 0.0 and cfg["repetitions"] == BASE_KNOBS["repetitions"]
            and not cfg["refine"])


def top_fraction_mean(scores, frac=0.01) -> float:
    """Mean of the best ceil(frac * n) scores (at least one)."""
    s = np.sort(np.asarray(scores, np.float64))[::-1]
    if len(s) == 0:
        raise ValueError("no scores")
    k = max(1, int(math.ceil(frac * len(s))))
    return float(np.mean(s[:k]))


def degradation(mean_approx, mean_orig) -> float:
    """Eq. 5: overlap degradation in percent."""
    return (1.0 - mean_approx / mean_orig) * 100.0


def pareto_front(throughput, degr) -> np.ndarray:
    """Boolean mask of the configurations no other configuration dominates
    (throughput at least as high and degradation at least as low, one of the
    two strictly)."""
    t = np.asarray(throughput, np.float64)
    d = np.asarray(degr, np.float64)
    n = len(t)
    keep = np.ones(n, bool)
    for i in range(n):
        dom = (t >= t[i]) & (d <= d[i]) & ((t > t[i]) | (d < d[i]))
        keep[i] = not dom.any()
    return keep


def _batch(pocket, ligands, quats, cfg, top_k, clash_dist, clash_min_bonds, stream=None):
    return Batch(pocket, ligands, quats, hp=cfg["hp"], lp=cfg["lp"], threshold=cfg["threshold"],
                 repetitions=cfg["repetitions"], refine=cfg["refine"], top_k=top_k, clash_dist=clash_dist,
                 clash_min_bonds=clash_min_bonds, stream=stream)


def prepared_batches(pocket, ligands, quats, cfgs, top_k=1, clash_dist=2.0, clash_min_bonds=4):
    """Yield (cfg, Batch) for every configuration, preparing the next batch on
    a host thread (uploads on a side stream) while the caller docks the
    current one."""
    torch = _torch()
    side = torch.cuda.Stream()

    def start(c):
        box = {}

        def run():
            try:
                box["b"] = _batch(pocket, ligands, quats, c, top_k, clash_dist, clash_min_bonds, side)
            except BaseException as e:  # re-raised in the consumer
                box["e"] = e
        th = threading.Thread(target=run)
        th.start()
        return box, th

    nxt = start(cfgs[0]) if cfgs else None
    for i, c in enumerate(cfgs):
        box, th = nxt
        th.join()
        if "e" in box:
            raise box["e"]
        nxt = start(cfgs[i + 1]) if i + 1 < len(cfgs) else None
        yield c, box["b"]


def ligand_scores(pocket, ligands, quats, cfg, top_k=1, clash_dist=2.0, clash_min_bonds=4, stream=None, batch=None):
    """Dock one configuration and re-score each ligand's top-k poses with the
    continuous Eq. 1.  Returns a dict: score (per ligand: the best continuous
    overlap among its feasible top-k poses, 0 when none is feasible), S and
    grid overlap of the best pose, per-pose continuous overlaps, the pose
    coordinates (device tensors), dock_ms, rescore_ms.  `batch` may bring
    the configuration's prepared Batch."""
    torch = _torch()
    from .stream import poses_from_topk
    B = batch if batch is not None else _batch(pocket, ligands, quats, cfg, top_k, clash_dist, clash_min_bonds,
                                               stream)
    B.enable_timing(True)
    out = B.alloc_outputs(want_angles=False, want_xyz=True)
    B.dock(BATCHED, out, stream=stream)
    pose_lig, px, py, pz = poses_from_topk(out, ligands)
    counts = np.diff(np.asarray(ligands.atom_off, np.int64))[pose_lig]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _, _, o = overlap_continuous(pocket, counts, px, py, pz)
    e1.record()
    torch.cuda.synchronize()
    dock_ms = B.read_timing()[-1]
    rescore_ms = e0.elapsed_time(e1)
    h = out.host()
    n = B.n_ligands
    o = o.cpu().numpy().reshape(n, top_k)
    feasible = h["clash"].reshape(n, top_k) == 0
    score = np.where(feasible, o, 0.0).max(axis=1)
    return dict(score=score, S=h["S"][:, 0], clash=h["clash"][:, 0], overlap_grid=h["overlap"][:, 0],
                overlap_cont=o, feasible=feasible, xyz=(px, py, pz), pose_lig=pose_lig, dock_ms=dock_ms,
                rescore_ms=rescore_ms, n_atoms=int(np.asarray(ligands.atom_off)[-1]))


def explore(pocket, ligands, quats, space="full", top_k=1, frac=0.01, include_baseline=True, progress=None,
            **score_kw) -> list:
    """Evaluate every configuration of a design space (and the baseline if the
    space lacks it).  Returns one record per configuration: the knobs, dock_ms,
    rescore_ms, time_ms, atoms_per_s, ligands_per_s, top_mean (mean continuous
    overlap of the top `frac` ligands), degradation (Eq. 5, percent) and
    pareto (on the front of throughput vs degradation)."""
    cfgs = configurations(space)
    if include_baseline and not any(is_baseline(c) for c in cfgs):
        cfgs = [dict(BASE_KNOBS)] + cfgs
    recs = []
    kw = {k: v for k, v in score_kw.items() if k in ("clash_dist", "clash_min_bonds")}
    for i, (c, B) in enumerate(prepared_batches(pocket, ligands, quats, cfgs, top_k=top_k, **kw)):
        r = ligand_scores(pocket, ligands, quats, c, top_k=top_k, batch=B, **score_kw)
        del B
        t = r["dock_ms"] + r["rescore_ms"]
        rec = dict(c, dock_ms=r["dock_ms"], rescore_ms=r["rescore_ms"], time_ms=t,
                   atoms_per_s=r["n_atoms"] / (t * 1e-3), ligands_per_s=len(r["score"]) / (t * 1e-3),
                   top_mean=top_fraction_mean(r["score"], frac), feasible=float(np.mean(r["feasible"][:, 0])))
        recs.append(rec)
        if progress:
            progress(i, len(cfgs), rec)
    base = [r for r in recs if is_baseline(r)]
    if not base:
        raise ValueError("no baseline configuration among the evaluated ones")
    b = base[0]["top_mean"]
    for r in recs:
        r["degradation"] = degradation(r["top_mean"], b)
    front = pareto_front([r["atoms_per_s"] for r in recs], [r["degradation"] for r in recs])
    for r, f in zip(recs, front):
        r["pareto"] = bool(f)
    return recs
