"""Plain FP64 CPU oracle of the docking hot path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never links or
calls it.  ``oracle.c`` holds the arithmetic; this file is a ctypes binding.

Parity status per function (what pins each one is listed in the tests):
  edt / D(c)         pinned: brute force is the definition; one-point closed form
  score / clash      pinned: closed forms, lattice symmetries, hand-built cases
  schedules / tiles  pinned: Eq. 2/3 and the paper's 18-degree example
  dock (Alg. 2)      pinned: pose-count closed form, kinematic invariants,
                     independent brute force over torsion combinations
  sweep profile      pinned: its argmin is the flat 1-degree sweep's choice;
                     subsampling; the rotation by 0 is the pose itself
  continuous Eq. 1   pinned: exact rational brute force, one-point closed form,
                     lattice and permutation invariances
  overlap values     parity unpinned against the paper's own numbers (the paper
                     prints no scores and its figures are missing)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, ERR_ARG, ERR_GRAPH, ERR_ROTAMER, ERR_KNOB = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile liboracle.so: gcc -O2, strict IEEE (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Knobs(ctypes.Structure):
    """The paper's five knobs (Section III-C) plus the clash rule."""
    _fields_ = [("hp_step", ctypes.c_int), ("lp_step", ctypes.c_int), ("threshold", ctypes.c_double),
                ("repetitions", ctypes.c_int), ("refine", ctypes.c_int), ("clash_dist", ctypes.c_double),
                ("clash_min_bonds", ctypes.c_int)]


def knobs(hp=10, lp=None, threshold=0.0, repetitions=1, refine=False, clash_dist=2.0, clash_min_bonds=4):
    # the threshold travels as float32 through the GPU library's ABI; widen the
    # same float32 value here so both sides compare identical numbers
    return Knobs(int(hp), int(lp if lp is not None else hp), float(np.float32(threshold)), int(repetitions),
                 int(bool(refine)), float(np.float32(clash_dist)), int(clash_min_bonds))


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_pocket_new.argtypes = [P, ctypes.c_int, ctypes.c_double]
        lib.orc_pocket_new.restype = P
        lib.orc_pocket_free.argtypes = [P]
        lib.orc_pocket_centroid.argtypes = [P, P]
        lib.orc_pocket_n_occ.argtypes = [P]
        lib.orc_pocket_n_occ.restype = ctypes.c_int
        lib.orc_pocket_occ.argtypes = [P, P]
        lib.orc_D.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        lib.orc_D.restype = ctypes.c_int64
        lib.orc_score_xyz.argtypes = [P, ctypes.c_int, P]
        lib.orc_score_xyz.restype = ctypes.c_int64
        lib.orc_tile_size.argtypes = [ctypes.c_int]
        lib.orc_tile_size.restype = ctypes.c_int
        lib.orc_side_mode.argtypes = [ctypes.POINTER(Knobs), ctypes.c_int, ctypes.c_int]
        lib.orc_side_mode.restype = ctypes.c_int
        lib.orc_dock.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_int, P, ctypes.c_int, P,
                                 ctypes.POINTER(Knobs), ctypes.c_int, P, P, P, P, P, P]
        lib.orc_dock.restype = ctypes.c_int
        lib.orc_topk.argtypes = [ctypes.c_int, P, P, ctypes.c_int, P]
        lib.orc_topk.restype = ctypes.c_int
        lib.orc_overlap.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double]
        lib.orc_overlap.restype = ctypes.c_double
        lib.orc_overlap_continuous.argtypes = [P, ctypes.c_int, P, P]
        lib.orc_sweep_profile.argtypes = [P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, P, P]
        lib.orc_sweep_profile.restype = ctypes.c_int
        lib.orc_overlap_continuous.restype = ctypes.c_double
        lib.orc_score_poses.argtypes = [P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, P, ctypes.c_double,
                                        ctypes.c_int, P, P]
        lib.orc_score_poses.restype = ctypes.c_int
        lib.orc_topology.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, P]
        lib.orc_topology.restype = ctypes.c_int
        lib.orc_place.argtypes = [ctypes.c_int, P, P, P, P, P, P]
        lib.orc_apply_torsions.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int, P]
        lib.orc_apply_torsions.restype = ctypes.c_int
        D = ctypes.c_double
        lib.orc_blur_new.argtypes = [P, D, D, D]
        lib.orc_blur_new.restype = P
        lib.orc_blur_free.argtypes = [P]
        lib.orc_rho_node.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        lib.orc_rho_node.restype = D
        lib.orc_rho_interp.argtypes = [P, P, P, P]
        lib.orc_rho_interp.restype = D
        lib.orc_surrogate.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, P, D, D, ctypes.c_int,
                                      P, P, P]
        lib.orc_surrogate.restype = ctypes.c_int
        lib.orc_refine.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int, D, D, D, D, D,
                                   D, D, ctypes.c_int, P, P, P]
        lib.orc_refine.restype = ctypes.c_int
        lib.orc_torsion_tree.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, P, P, P]
        lib.orc_torsion_tree.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class OraclePocket:
    """Pocket point cloud on the lattice of spacing h (FP64)."""

    def __init__(self, xyz, h=0.5):
        lib = _load()
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        self.h = float(h)
        self._ptr = lib.orc_pocket_new(_p(self.xyz), len(self.xyz), self.h)
        if not self._ptr:
            raise ValueError("oracle: bad pocket")

    def __del__(self):
        if getattr(self, "_ptr", None) and _lib is not None:
            _lib.orc_pocket_free(self._ptr)
            self._ptr = None

    @property
    def centroid(self):
        c = np.zeros(3)
        _load().orc_pocket_centroid(self._ptr, _p(c))
        return c

    def occupied(self):
        lib = _load()
        n = lib.orc_pocket_n_occ(self._ptr)
        out = np.zeros((n, 3), np.int64)
        lib.orc_pocket_occ(self._ptr, _p(out))
        return out

    def D(self, cx, cy, cz) -> int:
        return int(_load().orc_D(self._ptr, int(cx), int(cy), int(cz)))

    def score_xyz(self, X) -> int:
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
        return int(_load().orc_score_xyz(self._ptr, len(X), _p(X)))

    def overlap_continuous(self, X):
        """Eq. 1 over the raw points: (sum over atoms of the smallest squared
        distance, per-atom minima, overlap l / sum)."""
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
        m = np.zeros(len(X))
        s = float(_load().orc_overlap_continuous(self._ptr, len(X), _p(X), _p(m)))
        with np.errstate(divide="ignore", invalid="ignore"):
            o = float(np.float64(len(X)) / np.float64(s))  # IEEE: +inf for 0 sum, NaN for no atoms
        return s, m, o


def tile_size(hp: int) -> int:
    return int(_load().orc_tile_size(int(hp)))


def side_mode(k: Knobs, side_size: int, l: int) -> int:
    return int(_load().orc_side_mode(ctypes.byref(k), int(side_size), int(l)))


def topology(lig: dict):
    """(rc, bond-count distance matrix, left masks (nr x l))."""
    l = len(lig["x"])
    bonds = np.ascontiguousarray(lig["bonds"], np.int32).reshape(-1)
    rot = np.ascontiguousarray(lig["rot"], np.int32).reshape(-1)
    dist = np.zeros((l, l), np.int32)
    left = np.zeros((max(len(rot) // 2, 1), l), np.uint8)
    rc = _load().orc_topology(l, len(bonds) // 2, _p(bonds), len(rot) // 2, _p(rot), _p(dist), _p(left))
    return rc, dist, left[:len(rot) // 2]


def sweep_profile(pocket: OraclePocket, lig: dict, X, r: int, side: int, step: int = 1, clash_dist=2.0,
                  clash_min_bonds=4):
    """Overlap landscape of one rotamer side from pose X (l x 3 FP64):
    (side size, S per angle, feasible per angle) for angles 0, step, ..."""
    X = np.ascontiguousarray(X, np.float64).reshape(-1, 3)
    bonds = np.ascontiguousarray(lig["bonds"], np.int32).reshape(-1)
    rot = np.ascontiguousarray(lig["rot"], np.int32).reshape(-1)
    n = 360 // step
    S = np.zeros(n, np.int64)
    f = np.zeros(n, np.uint8)
    cd = float(np.float32(clash_dist))
    rc = _load().orc_sweep_profile(pocket._ptr, len(X), len(bonds) // 2, _p(bonds), len(rot) // 2, _p(rot), _p(X),
                                   int(r), int(side), int(step), cd, int(clash_min_bonds), _p(S), _p(f))
    if rc < 0:
        raise OracleError(-rc)
    return rc, S, f.astype(bool)


class DockResult:
    def __init__(self, S, clash, angles, xyz, n_cand):
        self.S, self.clash, self.angles, self.xyz, self.n_cand = S, clash, angles, xyz, n_cand


def dock(pocket: OraclePocket, lig: dict, k: Knobs, quats, want_xyz=True) -> DockResult:
    """Alg. 2 for one ligand over every orientation; raises on invalid input."""
    lib = _load()
    x = np.ascontiguousarray(lig["x"], np.float32)
    y = np.ascontiguousarray(lig["y"], np.float32)
    z = np.ascontiguousarray(lig["z"], np.float32)
    bonds = np.ascontiguousarray(lig["bonds"], np.int32).reshape(-1)
    rot = np.ascontiguousarray(lig["rot"], np.int32).reshape(-1)
    q = np.ascontiguousarray(quats, np.float64).reshape(-1, 4)
    l, nr, no = len(x), len(rot) // 2, len(q)
    S = np.zeros(no, np.int64)
    clash = np.zeros(no, np.uint8)
    angles = np.zeros((no, k.repetitions, max(nr, 1), 2), np.int16)
    xyz = np.zeros((no, l, 3), np.float64) if want_xyz else None
    ncand = ctypes.c_int64(0)
    rc = lib.orc_dock(pocket._ptr, l, _p(x), _p(y), _p(z), len(bonds) // 2, _p(bonds), nr, _p(rot), ctypes.byref(k),
                      no, _p(q), _p(S), _p(clash), _p(angles), _p(xyz), ctypes.byref(ncand))
    if rc != OK:
        raise OracleError(rc)
    return DockResult(S, clash, angles[:, :, :nr, :], xyz, int(ncand.value))


class OracleError(RuntimeError):
    def __init__(self, rc):
        super().__init__("oracle error %d" % rc)
        self.rc = rc


def topk(S, clash, k):
    S = np.ascontiguousarray(S, np.int64)
    clash = np.ascontiguousarray(clash, np.uint8)
    out = np.zeros(k, np.int32)
    rc = _load().orc_topk(len(S), _p(S), _p(clash), int(k), _p(out))
    if rc != OK:
        raise OracleError(rc)
    return out


def overlap(l, S, h=0.5):
    return float(_load().orc_overlap(int(l), int(S), float(h)))


def score_poses(pocket: OraclePocket, lig: dict, px, py, pz, clash_dist=2.0, min_bonds=4):
    """Exact S and whole-ligand clash of FP32 poses (n_poses x l arrays)."""
    px = np.ascontiguousarray(px, np.float32)
    py = np.ascontiguousarray(py, np.float32)
    pz = np.ascontiguousarray(pz, np.float32)
    n, l = px.shape
    bonds = np.ascontiguousarray(lig["bonds"], np.int32).reshape(-1)
    S = np.zeros(n, np.int64)
    clash = np.zeros(n, np.uint8)
    rc = _load().orc_score_poses(pocket._ptr, l, len(bonds) // 2, _p(bonds), n, _p(px), _p(py), _p(pz),
                                 float(np.float32(clash_dist)), int(min_bonds), _p(S), _p(clash))
    if rc != OK:
        raise OracleError(rc)
    return S, clash


def place(lig: dict, q, centre) -> np.ndarray:
    """Rigid placement X = R(q)(x - c_L) + c_P (FP64, l x 3)."""
    x = np.ascontiguousarray(lig["x"], np.float32)
    y = np.ascontiguousarray(lig["y"], np.float32)
    z = np.ascontiguousarray(lig["z"], np.float32)
    q = np.ascontiguousarray(q, np.float64)
    c = np.ascontiguousarray(centre, np.float64)
    X = np.zeros((len(x), 3), np.float64)
    _load().orc_place(len(x), _p(x), _p(y), _p(z), _p(q), _p(c), _p(X))
    return X


def apply_torsions(lig: dict, X, moves) -> np.ndarray:
    """Apply (rotamer, side, degrees) fragment rotations in order to a copy of X."""
    X = np.ascontiguousarray(X, np.float64).copy()
    bonds = np.ascontiguousarray(lig["bonds"], np.int32).reshape(-1)
    rot = np.ascontiguousarray(lig["rot"], np.int32).reshape(-1)
    mv = np.ascontiguousarray(moves, np.int32).reshape(-1, 3)
    rc = _load().orc_apply_torsions(len(X), len(bonds) // 2, _p(bonds), len(rot) // 2, _p(rot), _p(X), len(mv),
                                    _p(mv))
    if rc != OK:
        raise OracleError(rc)
    return X


class OracleBlur:
    """Blurred pocket density rho on the lattice bh*(i,j,k) (nodes by definition)."""

    def __init__(self, pocket: OraclePocket, sigma=0.6, cutoff_sigmas=4.0, bh=0.375):
        lib = _load()
        self.pocket = pocket
        # sigma, cutoff and spacing travel as float32 through the GPU ABI
        self.sigma = float(np.float32(sigma))
        self.cutoff = float(np.float32(cutoff_sigmas)) * self.sigma
        self.bh = float(np.float32(bh))
        self._ptr = lib.orc_blur_new(pocket._ptr, self.sigma, self.cutoff, self.bh)

    def __del__(self):
        if getattr(self, "_ptr", None) and _lib is not None:
            _lib.orc_blur_free(self._ptr)
            self._ptr = None

    def node(self, i, j, k) -> float:
        return float(_load().orc_rho_node(self.pocket._ptr, self._ptr, int(i), int(j), int(k)))

    def interp(self, x):
        x = np.ascontiguousarray(x, np.float64)
        g = np.zeros(3)
        v = _load().orc_rho_interp(self.pocket._ptr, self._ptr, _p(x), _p(g))
        return float(v), g

    def surrogate(self, lig: dict, X0, prm, want_grad=True, clash_weight=0.0, clash_dist=2.0, clash_min_bonds=4):
        """(F, dF/dprm, pose) with prm = [t(3), q(4), tau(nr)] (tau in list order);
        with clash_weight > 0 the bump penalty is subtracted from F."""
        bonds = np.ascontiguousarray(lig["bonds"], np.int32).reshape(-1)
        rot = np.ascontiguousarray(lig["rot"], np.int32).reshape(-1)
        X0 = np.ascontiguousarray(X0, np.float64)
        prm = np.ascontiguousarray(prm, np.float64)
        F = ctypes.c_double(0)
        grad = np.zeros(len(prm)) if want_grad else None
        X = np.zeros_like(X0)
        rc = _load().orc_surrogate(self.pocket._ptr, self._ptr, len(X0), len(bonds) // 2, _p(bonds), len(rot) // 2,
                                   _p(rot), _p(X0), _p(prm), float(np.float32(clash_weight)),
                                   float(np.float32(clash_dist)), int(clash_min_bonds), ctypes.byref(F), _p(grad),
                                   _p(X))
        if rc != OK:
            raise OracleError(rc)
        return F.value, grad, X

    def refine(self, lig: dict, X0, steps=50, lr_t=0.002, lr_q=1e-5, lr_tau=5e-4, max_dt=0.1, max_dtau=0.05,
               clash_weight=0.0, clash_dist=2.0, clash_min_bonds=4):
        bonds = np.ascontiguousarray(lig["bonds"], np.int32).reshape(-1)
        rot = np.ascontiguousarray(lig["rot"], np.int32).reshape(-1)
        X0 = np.ascontiguousarray(X0, np.float64)
        nr = len(rot) // 2
        prm = np.zeros(7 + nr)
        X = np.zeros_like(X0)
        F = ctypes.c_double(0)
        f32 = lambda v: float(np.float32(v))
        rc = _load().orc_refine(self.pocket._ptr, self._ptr, len(X0), len(bonds) // 2, _p(bonds), nr, _p(rot), _p(X0),
                                int(steps), f32(lr_t), f32(lr_q), f32(lr_tau), f32(max_dt), f32(max_dtau),
                                f32(clash_weight), f32(clash_dist), int(clash_min_bonds), _p(prm), _p(X),
                                ctypes.byref(F))
        if rc != OK:
            raise OracleError(rc)
        return prm, X, F.value


def torsion_tree(lig: dict):
    """(root-first order, near atoms, far atoms, moving masks nr x l)."""
    bonds = np.ascontiguousarray(lig["bonds"], np.int32).reshape(-1)
    rot = np.ascontiguousarray(lig["rot"], np.int32).reshape(-1)
    l, nr = len(lig["x"]), len(rot) // 2
    order = np.zeros(max(nr, 1), np.int32)
    near = np.zeros(max(nr, 1), np.int32)
    far = np.zeros(max(nr, 1), np.int32)
    mov = np.zeros((max(nr, 1), l), np.uint8)
    rc = _load().orc_torsion_tree(l, len(bonds) // 2, _p(bonds), nr, _p(rot), _p(order), _p(near), _p(far), _p(mov))
    if rc != OK:
        raise OracleError(rc)
    return order[:nr], near[:nr], far[:nr], mov[:nr].astype(bool)
