"""Peak analysis of overlap landscapes (Section III-B).

For one rotamer side turned about its bond, the landscape is the overlap
o(theta) = l / (h^2 S(theta)) of the whole ligand at every valid (bump-free)
angle.  Its delta overlap is max - min over the valid angles; a peak is a
maximal run of contiguous valid angles whose overlap exceeds the minimum by
more than half the delta (angles wrap around 360 degrees).  Per side the
analysis reports the delta normalised by the ligand's final overlap, the
relative fragment size, and per peak its width (degrees) and height
normalised by the delta (1 for the peak holding the maximum).  The GPU
supplies the landscapes (sweep_profile); this module is host post-processing.
"""
from __future__ import annotations

import numpy as np


def circular_runs(mask) -> list:
    """Maximal runs of True in a circular boolean array: (start, length), the
    last element adjacent to the first."""
    m = np.asarray(mask, bool)
    n = len(m)
    if n == 0 or not m.any():
        return []
    if m.all():
        return [(0, n)]
    start = int(np.flatnonzero(~m)[0]) + 1  # begin just after a False
    runs = []
    i = 0
    while i < n:
        j = (start + i) % n
        if m[j]:
            ln = 0
            while i < n and m[(start + i) % n]:
                ln += 1
                i += 1
            runs.append((j, ln))
        else:
            i += 1
    return runs


def overlap(S, l, h=0.5):
    """Eq. 1 on the lattice: o = l / (h^2 S), +inf for S = 0."""
    S = np.asarray(S, np.float64)
    with np.errstate(divide="ignore"):
        return l / (h * h * S)


def analyse_side(o, valid, step=1):
    """Delta overlap and peaks of one landscape; None when no angle is valid.
    Returns dict(delta, omin, omax, peaks=[(width_deg, height/delta, start_deg)])."""
    o = np.asarray(o, np.float64)
    v = np.asarray(valid, bool)
    if not v.any():
        return None
    omin, omax = float(o[v].min()), float(o[v].max())
    delta = omax - omin
    if not np.isfinite(delta) or delta <= 0:
        return dict(delta=0.0 if np.isfinite(delta) else delta, omin=omin, omax=omax, peaks=[])
    above = v & (o - omin > 0.5 * delta)
    peaks = []
    for s, ln in circular_runs(above):
        idx = (s + np.arange(ln)) % len(o)
        peaks.append((ln * step, (float(o[idx].max()) - omin) / delta, s * step))
    return dict(delta=delta, omin=omin, omax=omax, peaks=peaks)


def analyse(S, feasible, side_size, n_atoms, n_rot, final_S, step=1, h=0.5) -> list:
    """Per-side records of a batch of landscapes (host arrays shaped as
    sweep_profile returns them: S and feasible (n, k, R, 2, A), side_size
    (n, k, R, 2)); n_atoms and n_rot per ligand, final_S (n, k) the ranked
    poses' S.  Records: ligand, pose, rotamer, side, rel_size, delta_norm,
    n_peaks, peaks."""
    out = []
    n, k = S.shape[0], S.shape[1]
    for i in range(n):
        l = int(n_atoms[i])
        for kk in range(k):
            o_final = float(overlap(final_S[i, kk], l, h))
            for r in range(int(n_rot[i])):
                for side in (0, 1):
                    a = analyse_side(overlap(S[i, kk, r, side], l, h), feasible[i, kk, r, side] != 0, step)
                    if a is None or not np.isfinite(o_final) or o_final <= 0:
                        continue
                    out.append(dict(ligand=i, pose=kk, rotamer=r, side=side,
                                    rel_size=float(side_size[i, kk, r, side]) / l,
                                    delta_norm=a["delta"] / o_final, n_peaks=len(a["peaks"]), peaks=a["peaks"]))
    return out


def summarize(records, edges=(0.0, 0.2, 0.4, 0.6, 0.8, 1.0)) -> dict:
    """Distributions by relative fragment size (bins between `edges`): the
    normalised delta and the peak count (min, 25th, 50th, 75th percentile,
    max), and over all peaks the width of the peaks that hold their side's
    maximum (height 1) against the others."""
    q = (0, 25, 50, 75, 100)
    bins = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = [r for r in records if lo <= r["rel_size"] < hi or (hi == edges[-1] and r["rel_size"] == hi)]
        if not sel:
            bins.append(dict(rel_size=[lo, hi], sides=0))
            continue
        d = np.array([r["delta_norm"] for r in sel])
        npk = np.array([r["n_peaks"] for r in sel])
        bins.append(dict(rel_size=[lo, hi], sides=len(sel), delta_norm=[float(np.percentile(d, p)) for p in q],
                         n_peaks=[float(np.percentile(npk, p)) for p in q], single_peak=float(np.mean(npk == 1))))
    top = np.array([w for r in records for (w, ht, _) in r["peaks"] if ht >= 1.0])
    other = np.array([w for r in records for (w, ht, _) in r["peaks"] if ht < 1.0])
    hts = np.array([ht for r in records for (w, ht, _) in r["peaks"] if w <= 10])
    res = dict(sides=len(records), by_rel_size=bins)
    if len(top):
        res["max_peak_width_deg"] = [float(np.percentile(top, p)) for p in q]
        res["max_peak_wider_than_50deg"] = float(np.mean(top > 50))
    if len(other):
        res["other_peak_width_deg"] = [float(np.percentile(other, p)) for p in q]
    if len(hts):
        res["narrow_peaks_reaching_max"] = float(np.mean(hts >= 1.0))
    return res
