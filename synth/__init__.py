"""Seeded synthetic ligands, pockets and orientation sets.

Stand-ins for the paper's private ligand library and PASS pockets
(Section IV-A): random-tree heavy-atom ligands with 1.5 A bonds and
109.5 +/- 3 degree bond angles, ellipsoid point-cloud pockets, and uniform
unit quaternions for the rigid orientations.  The generator is plain C
(``synth.c``) behind ctypes; it holds none of the docking arithmetic and is
the only code shared by the oracle tests and the GPU path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libsynth.so`` with gcc (plain C, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.sy_ligands.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_double, P, P, P, P, P, P, P, P]
        lib.sy_ligands.restype = ctypes.c_int
        lib.sy_pocket.argtypes = [ctypes.c_uint64, ctypes.c_int] + [ctypes.c_double] * 6 + [P]
        lib.sy_pocket.restype = ctypes.c_int
        lib.sy_quaternions.argtypes = [ctypes.c_uint64, ctypes.c_int, P]
        lib.sy_quaternions.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class LigandBatch:
    """Ragged batch of ligands in CSR form (ligand-local atom indices).

    atom_off[n+1], x/y/z float32 (structure of arrays), bond_off[n+1],
    bonds int32 (2 per bond), rot_off[n+1], rot int32 ((a,b) pairs, a = left).
    """

    def __init__(self, atom_off, x, y, z, bond_off, bonds, rot_off, rot):
        self.atom_off = np.ascontiguousarray(atom_off, dtype=np.int32)
        self.x = np.ascontiguousarray(x, dtype=np.float32)
        self.y = np.ascontiguousarray(y, dtype=np.float32)
        self.z = np.ascontiguousarray(z, dtype=np.float32)
        self.bond_off = np.ascontiguousarray(bond_off, dtype=np.int32)
        self.bonds = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1)
        self.rot_off = np.ascontiguousarray(rot_off, dtype=np.int32)
        self.rot = np.ascontiguousarray(rot, dtype=np.int32).reshape(-1)

    @property
    def n(self) -> int:
        return len(self.atom_off) - 1

    def n_atoms(self, i: int) -> int:
        return int(self.atom_off[i + 1] - self.atom_off[i])

    def n_rot(self, i: int) -> int:
        return int(self.rot_off[i + 1] - self.rot_off[i])

    def ligand(self, i: int) -> dict:
        a0, a1 = self.atom_off[i], self.atom_off[i + 1]
        b0, b1 = self.bond_off[i], self.bond_off[i + 1]
        r0, r1 = self.rot_off[i], self.rot_off[i + 1]
        return dict(x=self.x[a0:a1].copy(), y=self.y[a0:a1].copy(), z=self.z[a0:a1].copy(),
                    bonds=self.bonds[2 * b0:2 * b1].reshape(-1, 2).copy(),
                    rot=self.rot[2 * r0:2 * r1].reshape(-1, 2).copy())

    def subset(self, idx) -> "LigandBatch":
        ligs = [self.ligand(int(i)) for i in idx]
        return LigandBatch.from_list(ligs)

    @staticmethod
    def from_list(ligs) -> "LigandBatch":
        ao, bo, ro = [0], [0], [0]
        xs, ys, zs, bs, rs = [], [], [], [], []
        for L in ligs:
            xs.append(np.asarray(L["x"], np.float32)); ys.append(np.asarray(L["y"], np.float32))
            zs.append(np.asarray(L["z"], np.float32))
            b = np.asarray(L["bonds"], np.int32).reshape(-1, 2)
            r = np.asarray(L["rot"], np.int32).reshape(-1, 2)
            bs.append(b.reshape(-1)); rs.append(r.reshape(-1))
            ao.append(ao[-1] + len(L["x"])); bo.append(bo[-1] + len(b)); ro.append(ro[-1] + len(r))
        cat = lambda v, dt: np.concatenate(v).astype(dt) if v else np.zeros(0, dt)
        return LigandBatch(np.array(ao), cat(xs, np.float32), cat(ys, np.float32), cat(zs, np.float32),
                           np.array(bo), cat(bs, np.int32), np.array(ro), cat(rs, np.int32))


def ligands(seed: int, first: int, count: int, lmin: int, lmax: int, bmin: int, bmax: int,
            ring_frac: float = 0.0) -> LigandBatch:
    """Ligands [first, first+count) of the stream ``seed``.  Every ligand has
    its own generator stream, so large requests are split over threads (the
    C generator runs without the interpreter lock) with the same result."""
    parts = min(os.cpu_count() or 1, 16, count // 4096)
    if parts <= 1:
        return _ligands_serial(seed, first, count, lmin, lmax, bmin, bmax, ring_frac)
    from concurrent.futures import ThreadPoolExecutor
    cut = np.linspace(0, count, parts + 1).astype(np.int64)
    with ThreadPoolExecutor(parts) as ex:
        bs = list(ex.map(lambda k: _ligands_serial(seed, first + int(cut[k]), int(cut[k + 1] - cut[k]), lmin, lmax,
                                                   bmin, bmax, ring_frac), range(parts)))
    return _concat(bs)


def _concat(bs) -> LigandBatch:
    def offs(name):
        out, base = [np.zeros(1, np.int32)], 0
        for b in bs:
            o = getattr(b, name)
            out.append((o[1:] + base).astype(np.int32))
            base += int(o[-1])
        return np.concatenate(out)
    cat = lambda name: np.concatenate([getattr(b, name) for b in bs])
    return LigandBatch(offs("atom_off"), cat("x"), cat("y"), cat("z"), offs("bond_off"), cat("bonds"),
                       offs("rot_off"), cat("rot"))


def _ligands_serial(seed: int, first: int, count: int, lmin: int, lmax: int, bmin: int, bmax: int,
                    ring_frac: float = 0.0) -> LigandBatch:
    lib = _load()
    atom_off = np.zeros(count + 1, np.int32)
    bond_off = np.zeros(count + 1, np.int32)
    rot_off = np.zeros(count + 1, np.int32)
    cap = max(count * lmax, 1)
    x = np.zeros(cap, np.float32); y = np.zeros(cap, np.float32); z = np.zeros(cap, np.float32)
    bonds = np.zeros(2 * count * (lmax + 1) + 2, np.int32)
    rot = np.zeros(2 * count * lmax + 2, np.int32)
    rc = lib.sy_ligands(seed, first, count, lmin, lmax, bmin, bmax, ring_frac, _ptr(atom_off), _ptr(x), _ptr(y),
                        _ptr(z), _ptr(bond_off), _ptr(bonds), _ptr(rot_off), _ptr(rot))
    if rc != 0:
        raise ValueError("synth.ligands: invalid parameters")
    na, nb, nr = atom_off[-1], bond_off[-1], rot_off[-1]
    return LigandBatch(atom_off, x[:na], y[:na], z[:na], bond_off, bonds[:2 * nb], rot_off, rot[:2 * nr])


def pocket(seed: int, n: int, axes, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """n points uniform in an ellipsoid, float32 (n, 3)."""
    lib = _load()
    out = np.zeros((n, 3), np.float32)
    rc = lib.sy_pocket(seed, n, float(axes[0]), float(axes[1]), float(axes[2]), float(center[0]),
                       float(center[1]), float(center[2]), _ptr(out))
    if rc != 0:
        raise ValueError("synth.pocket: invalid parameters")
    return out


def quaternions(seed: int, n: int) -> np.ndarray:
    """n uniform unit quaternions (w, x, y, z), float64 (n, 4), w >= 0."""
    lib = _load()
    out = np.zeros((n, 4), np.float64)
    if lib.sy_quaternions(seed, n, _ptr(out)) != 0:
        raise ValueError("synth.quaternions: invalid parameters")
    return out
