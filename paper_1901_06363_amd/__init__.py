"""MI355X-native geometric docking: Python binding of libgd.so.

The binding only marshals arguments: every step of docking, scoring and
refinement runs in the HIP kernels behind the C ABI declared in
``include/gd.h``.  PyTorch provides device memory and streams.  There is no
CPU fallback: importing the binding fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _abi
from ._abi import GdError  # noqa: F401

__all__ = ["Pocket", "Batch", "DockResult", "dock", "dock_batch", "DeviceLigands", "score_poses", "score_poses_noalloc",
           "refine", "surrogate_fwd", "surrogate_bwd", "SurrogateScore", "GdError", "lib_path"]

PER_LIGAND, BATCHED = 0, 1
CNT_POSES, CNT_FALLBACK, CNT_OOB, CNT_SWEEPS = 0, 1, 2, 3


def lib_path() -> str:
    return _abi.LIB_PATH


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Pocket:
    """Pocket point cloud on the device: distance grid and optional density grid."""

    def __init__(self, xyz, grid_h=0.5, pad=12.0, blur_sigma=0.0, blur_h=0.375, blur_cutoff_sigmas=4.0, blur_pad=8.0,
                 stream=None):
        lib = _abi.load()
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        desc = _abi.PocketDesc(self.xyz.ctypes.data_as(ctypes.c_void_p), len(self.xyz), grid_h, pad, blur_sigma,
                               blur_h, blur_cutoff_sigmas, blur_pad)
        h = ctypes.c_void_p()
        _abi.check(lib.gd_create_pocket(ctypes.byref(desc), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.grid_h = float(grid_h)

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _abi._lib is not None:
                _abi._lib.gd_destroy_pocket(self._h)
                self._h = None
        except Exception:  # interpreter shutdown
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = _abi.PocketInfo()
        _abi.check(_abi.load().gd_pocket_get_info(self._h, ctypes.byref(inf)))
        return dict(box_lo=tuple(inf.box_lo), box_dim=tuple(inf.box_dim), n_occupied=inf.n_occupied,
                    centroid=tuple(inf.centroid), grid_h=inf.grid_h, blur_lo=tuple(inf.blur_lo),
                    blur_dim=tuple(inf.blur_dim), blur_h=inf.blur_h)

    def read_grid(self) -> np.ndarray:
        """Distance grid D as uint16 array indexed [z, y, x]."""
        inf = self.info()
        nx, ny, nz = inf["box_dim"]
        out = np.zeros((nz, ny, nx), np.uint16)
        _abi.check(_abi.load().gd_pocket_read_grid(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def read_density(self) -> np.ndarray:
        inf = self.info()
        nx, ny, nz = inf["blur_dim"]
        out = np.zeros((nz, ny, nx), np.float32)
        _abi.check(_abi.load().gd_pocket_read_density(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out


class _LigandArrays:
    """Keeps the host arrays of a gd_ligands descriptor alive."""

    def __init__(self, ligs):
        c = np.ascontiguousarray
        self.atom_off = c(ligs.atom_off, dtype=np.int32)
        self.x = c(ligs.x, dtype=np.float32)
        self.y = c(ligs.y, dtype=np.float32)
        self.z = c(ligs.z, dtype=np.float32)
        self.bond_off = c(ligs.bond_off, dtype=np.int32)
        self.bonds = c(np.asarray(ligs.bonds).reshape(-1), dtype=np.int32)
        self.rot_off = c(ligs.rot_off, dtype=np.int32)
        self.rot = c(np.asarray(ligs.rot).reshape(-1), dtype=np.int32)
        if self.bonds.size == 0:
            self.bonds = np.zeros(2, np.int32)
        if self.rot.size == 0:
            self.rot = np.zeros(2, np.int32)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self.desc = _abi.Ligands(len(self.atom_off) - 1, p(self.atom_off), p(self.x), p(self.y), p(self.z),
                                 p(self.bond_off), p(self.bonds), p(self.rot_off), p(self.rot), 0)

    @property
    def n(self):
        return len(self.atom_off) - 1

    def n_atoms(self):
        return np.diff(self.atom_off)


class DeviceLigands(_LigandArrays):
    """A ligand set whose CSR arrays live in device memory (gd_ligands with
    on_device = 1): the library reads them there.  The host copies of the
    offsets stay for the binding's own shape checks."""

    def __init__(self, ligs, stream=None):
        super().__init__(ligs)
        torch = _torch()
        dev = torch.device("cuda")
        self.dev = {k: torch.from_numpy(getattr(self, k).copy()).to(dev)
                    for k in ("atom_off", "x", "y", "z", "bond_off", "bonds", "rot_off", "rot")}
        torch.cuda.synchronize()
        d = lambda k: ctypes.c_void_p(self.dev[k].data_ptr())
        self.desc = _abi.Ligands(self.n, d("atom_off"), d("x"), d("y"), d("z"), d("bond_off"), d("bonds"),
                                 d("rot_off"), d("rot"), 1)


class DockResult:
    """Top-k poses per ligand (device tensors) and the call's counters."""

    def __init__(self, recs, angles, xyz, counters, n_lig, top_k):
        self.recs = recs          # int32 (n_lig*top_k, 6): orient, S, clash, n_atoms, overlap(f64 bits)
        self.angles = angles      # uint16 view held as int16 tensor or None
        self.xyz = xyz            # float32 (n_lig, top_k, max_atoms, 3) or None
        self.counters = counters  # int64 (4,)
        self.n_lig, self.top_k = n_lig, top_k

    def host(self) -> dict:
        r = self.recs.cpu().numpy()
        out = dict(orient=r[:, 0].reshape(self.n_lig, self.top_k).copy(),
                   S=r[:, 1].reshape(self.n_lig, self.top_k).copy(),
                   clash=r[:, 2].reshape(self.n_lig, self.top_k).copy(),
                   n_atoms=r[:, 3].reshape(self.n_lig, self.top_k).copy(),
                   overlap=np.ascontiguousarray(r[:, 4:6]).view(np.float64).reshape(self.n_lig, self.top_k).copy(),
                   counters=self.counters.cpu().numpy().copy())
        if self.angles is not None:
            out["angles"] = self.angles.cpu().numpy().view(np.uint16).copy()
        if self.xyz is not None:
            out["xyz"] = self.xyz.cpu().numpy().copy()
        return out


class Batch:
    """A validated, device-resident ligand batch for one pocket and knob setting."""

    def __init__(self, pocket: Pocket, ligands, quats, hp=10, lp=None, threshold=0.0, repetitions=1, refine=False,
                 top_k=10, clash_dist=2.0, clash_min_bonds=4, stream=None):
        lib = _abi.load()
        self.pocket = pocket
        self.lig = ligands if isinstance(ligands, _LigandArrays) else _LigandArrays(ligands)
        self.quats = np.ascontiguousarray(quats, dtype=np.float64).reshape(-1, 4)
        k = _abi.Knobs(int(hp), int(lp if lp is not None else hp), float(threshold), int(repetitions), int(bool(refine)),
                       len(self.quats), self.quats.ctypes.data_as(ctypes.c_void_p), int(top_k), float(clash_dist),
                       int(clash_min_bonds))
        self.knobs = k
        h = ctypes.c_void_p()
        _abi.check(lib.gd_prepare_batch(pocket.handle, ctypes.byref(self.lig.desc), ctypes.byref(k),
                                        _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        inf = _abi.BatchInfo()
        _abi.check(lib.gd_batch_get_info(self._h, ctypes.byref(inf)))
        self.n_ligands, self.max_atoms, self.max_rot = inf.n_ligands, inf.max_atoms, inf.max_rot
        self.repetitions, self.top_k, self.n_orient = inf.repetitions, inf.top_k, inf.n_orient
        self.poses_expected, self.n_pairs_total = inf.poses_expected, inf.n_pairs_total
        self.n_atoms_total, self.algo_flops, self.algo_bytes = inf.n_atoms_total, inf.algo_flops, inf.algo_bytes

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _abi._lib is not None:
                _abi._lib.gd_destroy_batch(self._h)
                self._h = None
        except Exception:  # interpreter shutdown
            pass

    def enable_timing(self, on=True):
        """Bracket the docking kernel of every later call with HIP events."""
        _abi.check(_abi.load().gd_batch_enable_timing(self._h, int(bool(on))))

    def read_timing(self, max_n=256):
        """Docking-kernel durations (ms) of the calls since the last read, oldest first."""
        buf = (ctypes.c_float * max_n)()
        n = ctypes.c_int32(0)
        _abi.check(_abi.load().gd_batch_read_timing(self._h, buf, int(max_n), ctypes.byref(n)))
        return [buf[i] for i in range(n.value)]

    def set_tiling(self, waves_per_block, angle_block, pairs_per_lane):
        t = _abi.Tiling(waves_per_block, angle_block, pairs_per_lane)
        _abi.check(_abi.load().gd_batch_set_tiling(self._h, ctypes.byref(t)))

    def tiling(self):
        t = _abi.Tiling()
        _abi.check(_abi.load().gd_batch_get_tiling(self._h, ctypes.byref(t)))
        return (t.waves_per_block, t.angle_block, t.pairs_per_lane)

    def autotune(self, reps=2, cache_path=None, stream=None):
        t = _abi.Tiling()
        cp = cache_path.encode() if cache_path else None
        _abi.check(_abi.load().gd_batch_autotune(self.pocket.handle, self._h, _stream_ptr(stream), int(reps), cp,
                                                 ctypes.byref(t)))
        return (t.waves_per_block, t.angle_block, t.pairs_per_lane)

    def alloc_outputs(self, want_angles=True, want_xyz=True):
        torch = _torch()
        dev = torch.device("cuda")
        n, k = self.n_ligands, self.top_k
        recs = torch.empty((n * k, 6), dtype=torch.int32, device=dev)
        ang = torch.empty((n, k, self.repetitions, self.max_rot, 2), dtype=torch.int16, device=dev) \
            if want_angles else None
        xyz = torch.empty((n, k, self.max_atoms, 3), dtype=torch.float32, device=dev) if want_xyz else None
        cnt = torch.zeros(4, dtype=torch.int64, device=dev)
        return DockResult(recs, ang, xyz, cnt, n, k)

    def dock(self, mode=BATCHED, out: DockResult = None, want_angles=True, want_xyz=True, stream=None):
        if out is None:
            out = self.alloc_outputs(want_angles, want_xyz)
        _abi.check(_abi.load().gd_dock_prepared(self.pocket.handle, self._h, int(mode), _stream_ptr(stream),
                                                _dptr(out.recs), _dptr(out.angles), _dptr(out.xyz),
                                                _dptr(out.counters)))
        return out


def dock(pocket: Pocket, ligands, quats, mode=BATCHED, stream=None, **knobs) -> DockResult:
    b = Batch(pocket, ligands, quats, stream=stream, **knobs)
    res = b.dock(mode, stream=stream)
    _torch().cuda.synchronize()
    return res


def dock_batch(pocket: Pocket, ligands, quats, mode=BATCHED, out: DockResult = None, want_angles=True, want_xyz=True,
               stream=None, hp=10, lp=None, threshold=0.0, repetitions=1, refine=False, top_k=10, clash_dist=2.0,
               clash_min_bonds=4) -> DockResult:
    """gd_dock_batch: prepare and dock in one call.  With device outputs (the
    default) the call returns once the work is enqueued on `stream`; the
    results are there when the stream has reached it."""
    lib = _abi.load()
    lg = ligands if isinstance(ligands, _LigandArrays) else _LigandArrays(ligands)
    q = np.ascontiguousarray(quats, dtype=np.float64).reshape(-1, 4)
    k = _abi.Knobs(int(hp), int(lp if lp is not None else hp), float(threshold), int(repetitions), int(bool(refine)),
                   len(q), q.ctypes.data_as(ctypes.c_void_p), int(top_k), float(clash_dist), int(clash_min_bonds))
    if out is None:
        torch = _torch()
        dev = torch.device("cuda")
        n, kk = lg.n, int(top_k)
        lmax = max(int(lg.n_atoms().max()), 1)
        rmax = max(int(np.diff(lg.rot_off).max()), 1)
        recs = torch.empty((n * kk, 6), dtype=torch.int32, device=dev)
        ang = torch.empty((n, kk, int(repetitions), rmax, 2), dtype=torch.int16, device=dev) if want_angles else None
        xyz = torch.empty((n, kk, lmax, 3), dtype=torch.float32, device=dev) if want_xyz else None
        cnt = torch.empty(4, dtype=torch.int64, device=dev)
        out = DockResult(recs, ang, xyz, cnt, n, kk)
    _abi.check(lib.gd_dock_batch(pocket.handle, ctypes.byref(lg.desc), ctypes.byref(k), int(mode), _stream_ptr(stream),
                                 _dptr(out.recs), _dptr(out.angles), _dptr(out.xyz), _dptr(out.counters)))
    out._keep = (lg, q)  # host arrays of the call (already consumed) and device inputs (read by the stream)
    return out


from ._ops import score_poses, score_poses_noalloc, overlap_continuous, OverlapLayout, sweep_profile, refine, surrogate_fwd, surrogate_bwd, SurrogateScore  # noqa: E402,E501
