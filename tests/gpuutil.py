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
