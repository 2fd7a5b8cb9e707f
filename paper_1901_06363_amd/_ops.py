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


def _pose_layout(lg, pose_lig):
    """(pose_lig as int32, total atoms of the poses, most rotamers of any
    pose's ligand); raises on a ligand index out of range."""
    pl = np.ascontiguousarray(pose_lig, dtype=np.int32).reshape(-1)
    nat = np.diff(np.asarray(lg.atom_off, dtype=np.int64))
    nrot = np.diff(np.asarray(lg.rot_off, dtype=np.int64))
    if len(pl) and (pl.min() < 0 or pl.max() >= len(nat)):
        raise ValueError("pose_lig holds a ligand index outside [0, %d)" % len(nat))
    if not len(pl):
        return pl, 0, 0
    return pl, int(nat[pl].sum()), int(nrot[pl].max())


def _check_rows(name, t, n_rows):
    """Format of a coordinate array the kernels read (and gd_refine writes)
    in place: contiguous float32 with at least n_rows elements."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.float32:
        raise TypeError("%s must be float32, got %s" % (name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous (a strided view would be read as consecutive rows)" % name)
    if t.numel() < n_rows:
        raise ValueError("%s holds %d values, the poses need %d" % (name, t.numel(), n_rows))


def _check_coords(px, py, pz, n_atoms):
    arrays = (("px", px), ("py", py), ("pz", pz))
    for name, t in arrays:
        _check_rows(name, t, n_atoms)
    for name, t in arrays:
        if not t.is_cuda:
            raise TypeError("%s must be a CUDA (HIP device) tensor" % name)


def _check_param(name, t, n, cols):
    """A per-pose parameter array on the GPU: shape (n,) when cols is None,
    (n, cols) for an int, (n, >= cols[0]) for a one-element tuple."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.dtype.is_floating_point:
        raise TypeError("%s must be floating point, got %s" % (name, t.dtype))
    if cols is None:
        ok, want = t.dim() == 1 and t.shape[0] == n, "(%d,)" % n
    elif isinstance(cols, tuple):
        ok, want = t.dim() == 2 and t.shape[0] == n and t.shape[1] >= cols[0], "(%d, >= %d)" % (n, cols[0])
    else:
        ok, want = t.dim() == 2 and tuple(t.shape) == (n, cols), "(%d, %d)" % (n, cols)
    if not ok:
        raise ValueError("%s must have shape %s, got %s" % (name, want, tuple(t.shape)))
    if not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP device) tensor" % name)


def score_poses(pocket, ligands, pose_lig, px, py, pz, clash_dist=2.0, clash_min_bonds=4, stream=None):
    """Exact S and bump flags of poses (device float32 CSR rows by pose)."""
    torch = _torch()
    lg = _lig_desc(ligands)
    pl, n_atoms, _ = _pose_layout(lg, pose_lig)
    _check_coords(px, py, pz, n_atoms)
    n = len(pl)
    S = torch.empty(n, dtype=torch.int32, device="cuda")
    clash = torch.empty(n, dtype=torch.uint8, device="cuda")
    _abi.check(_abi.load().gd_score_poses(pocket.handle, ctypes.byref(lg.desc), n, pl.ctypes.data_as(ctypes.c_void_p),
                                          _dp(px), _dp(py), _dp(pz), float(clash_dist), int(clash_min_bonds),
                                          _stream_ptr(stream), _dp(S), _dp(clash)))
    return S, clash


def score_poses_noalloc(pocket, ligands, pose_lig, px, py, pz, S_out, clash_out, clash_dist=2.0, clash_min_bonds=4,
                        stream=None):
    """score_poses into caller-owned device outputs (int32 S_out, uint8
    clash_out, one entry per pose) through the allocation-free entry point:
    the call's tables are staged in the library's static device scratch."""
    torch = _torch()
    lg = _lig_desc(ligands)
    pl, n_atoms, _ = _pose_layout(lg, pose_lig)
    _check_coords(px, py, pz, n_atoms)
    n = len(pl)
    for name, t, dt in (("S_out", S_out, torch.int32), ("clash_out", clash_out, torch.uint8)):
        if not isinstance(t, torch.Tensor) or t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
            raise ValueError("%s must be a contiguous %s CUDA tensor of at least %d elements" % (name, dt, n))
    _abi.check(_abi.load().gd_score_poses_noalloc(pocket.handle, ctypes.byref(lg.desc), n,
                                                  pl.ctypes.data_as(ctypes.c_void_p), _dp(px), _dp(py), _dp(pz),
                                                  float(clash_dist), int(clash_min_bonds), _stream_ptr(stream),
                                                  _dp(S_out), _dp(clash_out)))
    return S_out, clash_out


class OverlapLayout:
    """Device pose offsets of a fixed list of pose sizes, reusable across
    calls of overlap_continuous (no host-to-device copy per call)."""

    def __init__(self, counts):
        torch = _torch()
        cnt = np.ascontiguousarray(counts, dtype=np.int64)
        if np.any(cnt < 0):
            raise ValueError("negative atom count")
        off = np.zeros(len(cnt) + 1, np.int64)
        np.cumsum(cnt, out=off[1:])
        if off[-1] >= 2 ** 31:
            raise ValueError("more than 2^31 - 1 atoms in one call")
        self.n_poses, self.n_atoms = len(cnt), int(off[-1])
        self.pose_off = torch.from_numpy(off.astype(np.int32)).to("cuda")


def overlap_continuous(pocket, counts, px, py, pz, stream=None):
    """Eq. 1 on the pocket's raw points for poses given as device float32
    rows (px, py, pz) grouped by pose, ``counts[p]`` atoms for pose p (or an
    OverlapLayout of them).  Returns device float64 tensors (min_d2 per atom,
    sum per pose, overlap per pose)."""
    torch = _torch()
    lay = counts if isinstance(counts, OverlapLayout) else OverlapLayout(counts)
    n, n_atoms, pose_off = lay.n_poses, lay.n_atoms, lay.pose_off
    if n_atoms > 0 and (px.numel() < n_atoms or py.numel() < n_atoms or pz.numel() < n_atoms):
        raise ValueError("coordinate arrays shorter than the atom count")
    for t in (px, py, pz):
        if n_atoms > 0 and (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()):
            raise TypeError("coordinates must be contiguous float32 CUDA tensors")
    min_d2 = torch.empty(max(n_atoms, 1), dtype=torch.float64, device="cuda")
    s = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
    o = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
    _abi.check(_abi.load().gd_overlap_continuous(pocket.handle, n, _dp(pose_off), n_atoms, _dp(px), _dp(py), _dp(pz),
                                                 _stream_ptr(stream), _dp(min_d2), _dp(s), _dp(o)))
    return min_d2[:n_atoms], s[:n], o[:n]


def sweep_profile(pocket, batch, res, step=1, stream=None):
    """Overlap landscapes of every rotamer side at every ranked pose of the
    docking result `res` (the last dock call of `batch`).  Returns device
    tensors S (n, k, max_rot, 2, 360/step) int32, feasible (same, uint8) and
    side_size (n, k, max_rot, 2) int32."""
    torch = _torch()
    if step < 1 or 360 % step:
        raise ValueError("step must be an integer divisor of 360")
    n, k, rm = batch.n_ligands, batch.top_k, max(batch.max_rot, 1)
    na = 360 // step
    S = torch.empty((n, k, rm, 2, na), dtype=torch.int32, device="cuda")
    f = torch.empty((n, k, rm, 2, na), dtype=torch.uint8, device="cuda")
    sz = torch.empty((n, k, rm, 2), dtype=torch.int32, device="cuda")
    _abi.check(_abi.load().gd_sweep_profile(pocket.handle, batch._h, _dp(res.recs), int(step), _stream_ptr(stream),
                                            _dp(S), _dp(f), _dp(sz)))
    return S, f, sz


def _prm(t, q, tau, n, rmax):
    """Checked float32 copies of the parameters t (n, 3), q (n, 4) and tau
    (n, >= rmax; may be None or empty when no pose has a rotamer)."""
    torch = _torch()
    _check_param("t", t, n, 3)
    _check_param("q", q, n, 4)
    t = t.contiguous().float()
    q = q.contiguous().float()
    if tau is None or tau.numel() == 0:
        if rmax > 0:
            raise ValueError("tau is required: the poses' ligands have up to %d rotamers" % rmax)
        tau = torch.zeros((n, 1), dtype=torch.float32, device="cuda")
    _check_param("tau", tau, n, (max(rmax, 1),))
    tau = tau.contiguous().float()
    return t, q, tau, tau.shape[1]


def _penalty(clash_weight, clash_dist, clash_min_bonds):
    if not clash_weight:
        return None
    return ctypes.byref(_abi.BumpPenalty(float(clash_weight), float(clash_dist), int(clash_min_bonds)))


def surrogate_fwd(pocket, ligands, pose_lig, px, py, pz, t, q, tau, stream=None, clash_weight=0.0, clash_dist=2.0,
                  clash_min_bonds=4):
    """F(t, q, tau) per pose (device float32 (n,)); clash_weight > 0 subtracts
    the bump penalty."""
    torch = _torch()
    lg = _lig_desc(ligands)
    pl, n_atoms, rmax = _pose_layout(lg, pose_lig)
    _check_coords(px, py, pz, n_atoms)
    n = len(pl)
    t, q, tau, stride = _prm(t, q, tau, n, rmax)
    F = torch.empty(n, dtype=torch.float32, device="cuda")
    _abi.check(_abi.load().gd_surrogate_fwd(pocket.handle, ctypes.byref(lg.desc), n,
                                            pl.ctypes.data_as(ctypes.c_void_p), _dp(px), _dp(py), _dp(pz), _dp(t),
                                            _dp(q), _dp(tau), stride, _penalty(clash_weight, clash_dist,
                                                                               clash_min_bonds),
                                            _stream_ptr(stream), _dp(F)))
    return F


def surrogate_bwd(pocket, ligands, pose_lig, px, py, pz, t, q, tau, dF, stream=None, clash_weight=0.0,
                  clash_dist=2.0, clash_min_bonds=4):
    """dF/dt, dF/dq, dF/dtau scaled by the upstream gradient dF (per pose)."""
    torch = _torch()
    lg = _lig_desc(ligands)
    pl, n_atoms, rmax = _pose_layout(lg, pose_lig)
    _check_coords(px, py, pz, n_atoms)
    n = len(pl)
    t, q, tau, stride = _prm(t, q, tau, n, rmax)
    _check_param("dF", dF, n, None)
    dF = dF.contiguous().float()
    dt = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    dq = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    dtau = torch.empty((n, stride), dtype=torch.float32, device="cuda")
    _abi.check(_abi.load().gd_surrogate_bwd(pocket.handle, ctypes.byref(lg.desc), n,
                                            pl.ctypes.data_as(ctypes.c_void_p), _dp(px), _dp(py), _dp(pz), _dp(t),
                                            _dp(q), _dp(tau), stride,
                                            _penalty(clash_weight, clash_dist, clash_min_bonds), _dp(dF),
                                            _stream_ptr(stream), _dp(dt), _dp(dq), _dp(dtau)))
    return dt, dq, dtau


def refine(pocket, ligands, pose_lig, px, py, pz, steps=50, lr_t=0.002, lr_q=1e-5, lr_tau=5e-4, max_dt=0.1,
           max_dtau=0.05, clash_dist=2.0, clash_min_bonds=4, stream=None, want_iterate=False, time_kernel=False,
           clash_weight=0.0):
    """Gradient ascent on the surrogate, then exact rescoring; px/py/pz are
    overwritten with the refined pose where it is accepted.  With time_kernel
    the call waits for the ascent kernel and returns its duration (ms) as
    out["kernel_ms"].  clash_weight > 0 climbs the clash-penalised surrogate
    (bump penalty over the far pairs closer than clash_dist)."""
    torch = _torch()
    lg = _lig_desc(ligands)
    pl, n_atoms, _ = _pose_layout(lg, pose_lig)
    _check_coords(px, py, pz, n_atoms)  # written in place
    n = len(pl)
    kms = ctypes.c_float(0.0)
    opts = _abi.RefineOpts(int(steps), float(lr_t), float(lr_q), float(lr_tau), float(max_dt), float(max_dtau),
                           ctypes.pointer(kms) if time_kernel else None, float(clash_weight))
    F = torch.empty(n, dtype=torch.float32, device="cuda")
    S = torch.empty(n, dtype=torch.int32, device="cuda")
    clash = torch.empty(n, dtype=torch.uint8, device="cuda")
    acc = torch.empty(n, dtype=torch.uint8, device="cuda")
    it = [torch.empty_like(px) for _ in range(3)] if want_iterate else [None, None, None]
    _abi.check(_abi.load().gd_refine(pocket.handle, ctypes.byref(lg.desc), n, pl.ctypes.data_as(ctypes.c_void_p),
                                     _dp(px), _dp(py), _dp(pz), ctypes.byref(opts), float(clash_dist),
                                     int(clash_min_bonds), _stream_ptr(stream), _dp(F), _dp(S), _dp(clash), _dp(acc),
                                     _dp(it[0]), _dp(it[1]), _dp(it[2])))
    out = dict(F=F, S=S, clash=clash, accepted=acc)
    if time_kernel:
        out["kernel_ms"] = kms.value
    if want_iterate:
        out["iterate"] = it
    return out


def _make_autograd():
    torch = _torch()

    class SurrogateScore(torch.autograd.Function):
        """F = SurrogateScore.apply(t, q, tau, ctx_obj): differentiable in t, q and tau.

        ctx_obj = (pocket, ligands, pose_lig, px, py, pz) fixes the poses being
        refined; the backward kernel recomputes the pose from the parameters.
        A seventh element, a dict (clash_weight, clash_dist, clash_min_bonds),
        selects the clash-penalised surrogate.
        """

        @staticmethod
        def forward(ctx, t, q, tau, spec):
            pocket, ligands, pose_lig, px, py, pz = spec[:6]
            pen = spec[6] if len(spec) > 6 else {}
            ctx.spec = spec
            ctx.save_for_backward(t, q, tau)
            return surrogate_fwd(pocket, ligands, pose_lig, px, py, pz, t.detach(), q.detach(), tau.detach(), **pen)

        @staticmethod
        def backward(ctx, dF):
            t, q, tau = ctx.saved_tensors
            pocket, ligands, pose_lig, px, py, pz = ctx.spec[:6]
            pen = ctx.spec[6] if len(ctx.spec) > 6 else {}
            dt, dq, dtau = surrogate_bwd(pocket, ligands, pose_lig, px, py, pz, t.detach(), q.detach(), tau.detach(),
                                         dF, **pen)
            return dt, dq, dtau[:, :tau.shape[1]], None

    return SurrogateScore


class _LazyAutograd:
    _cls = None

    def __getattr__(self, name):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _make_autograd()
        return getattr(_LazyAutograd._cls, name)


SurrogateScore = _LazyAutograd()
