"""Shared helpers of the GPU parity tests (inputs come from synth only)."""
import numpy as np
import pytest

import oracle
import synth

gpu = pytest.mark.gpu


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gd():
    need_gpu()
    import paper_1901_06363_amd as g
    return g


def oracle_dock_batch(opocket, ligs, kn, quats):
    """Oracle endpoints of every ligand of a LigandBatch: list of DockResult."""
    return [oracle.dock(opocket, ligs.ligand(i), kn, quats) for i in range(ligs.n)]


def oracle_dock_parallel(pts, ligs, kn, quats, threads=None):
    """oracle_dock_batch over host threads (the oracle runs outside the
    interpreter lock), each thread with its own oracle pocket."""
    import os
    import threading
    from concurrent.futures import ThreadPoolExecutor
    threads = threads or max(1, min(16, os.cpu_count() or 1, ligs.n))
    local = threading.local()

    def one(i):
        if not hasattr(local, "pocket"):
            local.pocket = oracle.OraclePocket(pts, 0.5)
        return oracle.dock(local.pocket, ligs.ligand(i), kn, quats)
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, range(ligs.n)))


def compare_full_ranking(res_host, orc, ligs, atol_xyz=1e-4):
    """GPU top-k == oracle ranking of all orientations: orientation, S, clash,
    chosen angles and coordinates (FP32 vs FP64 within atol)."""
    k = res_host["orient"].shape[1]
    for i, r in enumerate(orc):
        top = oracle.topk(r.S, r.clash, k)
        assert np.array_equal(res_host["orient"][i], top), (i, res_host["orient"][i][:8], top[:8])
        assert np.array_equal(res_host["S"][i], r.S[top]), i
        assert np.array_equal(res_host["clash"][i], r.clash[top]), i
        l = ligs.n_atoms(i)
        nr = ligs.n_rot(i)
        if "angles" in res_host:
            ang = res_host["angles"][i][:, :, :nr, :]
            assert np.array_equal(ang.astype(np.int64), r.angles[top].astype(np.int64)), i
        if "xyz" in res_host:
            got = res_host["xyz"][i][:, :l, :].astype(np.float64)
            assert np.max(np.abs(got - r.xyz[top])) < atol_xyz, i
        ov = np.array([oracle.overlap(l, s, 0.5) for s in r.S[top]])
        assert np.array_equal(res_host["overlap"][i], ov), i


# Bound on the FP32 kernels' coordinate error: the parity bar on coordinates.
FP32_XYZ = 1e-4


def face_dist(X, bh):
    """Smallest distance of any coordinate of X to a face of the density
    lattice of spacing bh (planes at its multiples on every axis)."""
    u = np.asarray(X, np.float64) / bh
    f = u - np.floor(u)
    return float(np.min(np.minimum(f, 1.0 - f))) * bh


def certify_split(oblur, lig, X0, gpu_iterate, steps, bh, **kw):
    """A GPU ascent trajectory that parts from the oracle's FP64 one is
    excused for one of two reasons, both decided on the oracle at the first
    step k whose iterates differ by more than FP32_XYZ:
      face:  at the iterate step k's gradient was taken from, an atom of the
             oracle's path lies within FP32_XYZ plus the paths' separation of
             a face of the trilinear density, where the gradient jumps;
      chaos: the ascent map amplifies rounding-size differences: oracle runs
             of k steps from the same input moved by 4e-6 A per coordinate (a
             few FP32 ulps) end at least a tenth as far from the unperturbed
             run as the GPU iterate does.
    gpu_iterate(k) returns the GPU iterate after k steps.  Returns (reason or
    None, details)."""
    X0 = np.asarray(X0, np.float64)
    prev_o, prev_dev = X0, 0.0
    for k in range(1, steps + 1):
        _, Xo, _ = oblur.refine(lig, X0, steps=k, **kw)
        dev = float(np.max(np.abs(gpu_iterate(k) - Xo)))
        if dev > FP32_XYZ:
            info = dict(step=k, dev=dev, face=face_dist(prev_o, bh), prev_dev=prev_dev)
            if info["face"] < FP32_XYZ + prev_dev:
                return "face", info
            rng = np.random.default_rng(len(X0) + k)
            spread = 0.0
            for _ in range(4):
                Xp = X0 + rng.choice([-4e-6, 4e-6], size=X0.shape)
                _, Xq, _ = oblur.refine(lig, Xp, steps=k, **kw)
                spread = max(spread, float(np.max(np.abs(Xq - Xo))))
            info["oracle_spread"] = spread
            return ("chaos" if spread >= 0.1 * dev else None), info
        prev_o, prev_dev = Xo, dev
    return None, None
