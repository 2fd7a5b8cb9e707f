"""ctypes declarations of the C ABI in include/gd.h."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgd.so")
_lib = None

P = ctypes.c_void_p
I32 = ctypes.c_int32
F32 = ctypes.c_float


class GdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("gd status %d: %s" % (status, msg))
        self.status = status


class PocketDesc(ctypes.Structure):
    _fields_ = [("xyz", P), ("n_points", I32), ("grid_h", F32), ("pad", F32), ("blur_sigma", F32), ("blur_h", F32),
                ("blur_cutoff_sigmas", F32), ("blur_pad", F32)]


class PocketInfo(ctypes.Structure):
    _fields_ = [("box_lo", I32 * 3), ("box_dim", I32 * 3), ("n_occupied", I32), ("centroid", ctypes.c_double * 3),
                ("grid_h", F32), ("blur_lo", I32 * 3), ("blur_dim", I32 * 3), ("blur_h", F32)]


class Ligands(ctypes.Structure):
    _fields_ = [("n_ligands", I32), ("atom_off", P), ("x", P), ("y", P), ("z", P), ("bond_off", P), ("bonds", P),
                ("rot_off", P), ("rot", P), ("on_device", I32)]


class Knobs(ctypes.Structure):
    _fields_ = [("hp_step_deg", I32), ("lp_step_deg", I32), ("threshold", F32), ("repetitions", I32),
                ("enable_refinement", I32), ("n_orient", I32), ("quats", P), ("top_k", I32), ("clash_dist", F32),
                ("clash_min_bonds", I32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_ligands", I32), ("max_atoms", I32), ("max_rot", I32), ("repetitions", I32), ("top_k", I32),
                ("n_orient", I32), ("poses_expected", ctypes.c_int64), ("n_pairs_total", ctypes.c_int64),
                ("n_atoms_total", ctypes.c_int64), ("algo_flops", ctypes.c_double), ("algo_bytes", ctypes.c_double)]


class Tiling(ctypes.Structure):
    _fields_ = [("waves_per_block", I32), ("angle_block", I32), ("pairs_per_lane", I32)]


class BumpPenalty(ctypes.Structure):
    _fields_ = [("weight", F32), ("clash_dist", F32), ("clash_min_bonds", I32)]


class RefineOpts(ctypes.Structure):
    _fields_ = [("steps", I32), ("lr_t", F32), ("lr_q", F32), ("lr_tau", F32), ("max_dt", F32), ("max_dtau", F32),
                ("kernel_ms", ctypes.POINTER(F32)), ("clash_weight", F32)]


# every exported symbol of include/gd.h: (name, restype, argtypes)
SIGNATURES = [
    ("gd_last_error", ctypes.c_char_p, []),
    ("gd_create_pocket", I32, [P, P, P]),
    ("gd_destroy_pocket", I32, [P]),
    ("gd_pocket_get_info", I32, [P, P]),
    ("gd_pocket_read_grid", I32, [P, P]),
    ("gd_pocket_read_density", I32, [P, P]),
    ("gd_prepare_batch", I32, [P, P, P, P, P]),
    ("gd_destroy_batch", I32, [P]),
    ("gd_batch_get_info", I32, [P, P]),
    ("gd_batch_set_tiling", I32, [P, P]),
    ("gd_batch_enable_timing", I32, [P, I32]),
    ("gd_batch_read_timing", I32, [P, P, I32, P]),
    ("gd_batch_get_tiling", I32, [P, P]),
    ("gd_batch_autotune", I32, [P, P, P, I32, ctypes.c_char_p, P]),
    ("gd_dock_prepared", I32, [P, P, I32, P, P, P, P, P]),
    ("gd_dock_batch", I32, [P, P, P, I32, P, P, P, P, P]),
    ("gd_score_poses", I32, [P, P, I32, P, P, P, P, F32, I32, P, P, P]),
    ("gd_score_poses_noalloc", I32, [P, P, I32, P, P, P, P, F32, I32, P, P, P]),
    ("gd_overlap_continuous", I32, [P, I32, P, ctypes.c_int64, P, P, P, P, P, P, P]),
    ("gd_sweep_profile", I32, [P, P, P, I32, P, P, P, P]),
    ("gd_surrogate_fwd", I32, [P, P, I32, P, P, P, P, P, P, P, I32, P, P, P]),
    ("gd_surrogate_bwd", I32, [P, P, I32, P, P, P, P, P, P, P, I32, P, P, P, P, P, P]),
    ("gd_refine", I32, [P, P, I32, P, P, P, P, P, F32, I32, P, P, P, P, P, P, P, P]),
]


def load():
    """Load libgd.so; raises when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgd.so not built (run __graft_entry__.build()); there is no CPU fallback")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def check(status):
    if status != 0:
        msg = load().gd_last_error()
        raise GdError(status, msg.decode() if msg else "")
