"""Exact pose scoring and the density-surrogate refinement (C-ABI marshalling)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _lig_desc(ligands):
    from . import _LigandArrays
    return ligands if isinstance(ligands, _LigandArrays) else _LigandArrays(ligands)


def score_poses(pocket, ligands, pose_lig, px, py, pz, clash_dist=2.0, clash_min_bonds=4, stream=None):
    """Exact S and bump flags of poses (device float32 CSR rows by pose)."""
    torch = _torch()
    lg = _lig_desc(ligands)
    pl = np.ascontiguousarray(pose_lig, dtype=np.int32)
    n = len(pl)
    S = torch.empty(n, dtype=torch.int32, device="cuda")
    clash = torch.empty(n, dtype=torch.uint8, device="cuda")
    _abi.check(_abi.load().gd_score_poses(pocket.handle, ctypes.byref(lg.desc), n, pl.ctypes.data_as(ctypes.c_void_p),
                                          _dp(px), _dp(py), _dp(pz), float(clash_dist), int(clash_min_bonds),
                                          _stream_ptr(stream), _dp(S), _dp(clash)))
    return S, clash


def surrogate_fwd(*a, **k):
    raise NotImplementedError("surrogate kernels are not in this build")


def surrogate_bwd(*a, **k):
    raise NotImplementedError("surrogate kernels are not in this build")


def refine(*a, **k):
    raise NotImplementedError("refinement kernels are not in this build")


class SurrogateScore:
    pass
