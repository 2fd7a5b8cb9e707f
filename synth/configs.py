"""Seeded workload recipes (synthetic stand-ins for the paper's data sets).

Each recipe fixes the generator streams, sizes and knobs of one workload:

  single     1 ligand (32 atoms, 4 rotatable bonds, seed 0) x 1 pocket
             (1,000 points, ellipsoid 8/6/5 A); 256 orientations, 10-degree
             steps, 1 repetition, top-10.
  screen     10,000 ligands (atoms U[20,80], rotatable bonds U[2,12]) x 1
             pocket (4,000 points, 12/9/7 A); 512 orientations, 15-degree
             steps; the per-ligand and the batched forms.
  grid       the screen ligands plus 90,000 more of the same stream x 4
             pockets (1,000/2,000/4,000/8,000 points, major semi-axis
             6/8.67/11.33/14 A, axis ratios 1 : 0.75 : 0.625); knob grid
             orientations {64,256,1024} x step {30,15,10}.
  refine     4,096 ligands (20-80 atoms, 2-12 rotatable bonds) x top-64 poses
             docked with the 'single' knobs in the 'single' pocket; Gaussian
             blur sigma 0.6 A on a 0.375 A lattice; 50 ascent steps; the
             clash-penalised variant with weight 1,000.
  large      1,000,000 ligands (atoms U[15,120], rotatable bonds U[0,16], 5 %
             with a rigid 3-6 ring) x 1 pocket (10,000 points, 16/12/9 A);
             1024 orientations, 10-degree steps, chunks of 65,536, top-8
             refined.
  dse        20,000 ligands (atoms U[28,120], rotatable bonds U[2,16]: the
             paper's library spans 28-153 atoms and 2-53 rotamers, capped here
             at the library's 128-atom limit and a moderate rotamer count) x
             the screen pocket; 32 orientations, top-1 pose per ligand; the
             knob configurations of the flat and full design spaces.
  tts        time-to-solution campaign: the grid workload's 4 pockets x 5
             ligand mixes of 5,000 ligands (atoms/rotatable bonds U[20,40]/
             U[2,5], U[28,70]/U[2,8], U[28,120]/U[2,16], U[70,110]/U[2,5],
             U[40,70]/U[9,14]) for training; validation databases of 1,000,
             2,000, 5,000 and 10,000 ligands drawn from the dse distribution
             with another seed; 32 orientations.

Pocket centres sit off the lattice origin so that no symmetry of the grid is
accidentally exploited.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import ligands, pocket, quaternions

GRID_H = 0.5
POCKET_CENTRE = (3.2109375, -1.3671875, 2.0546875)


@dataclass
class Workload:
    name: str
    lig_seed: int
    n_ligands: int
    lmin: int
    lmax: int
    bmin: int
    bmax: int
    ring_frac: float
    pockets: list  # (seed, n_points, axes)
    n_orient: int
    hp: int
    lp: int = 0
    threshold: float = 0.0
    repetitions: int = 1
    refine: bool = False
    top_k: int = 10
    quat_seed: int = 77
    chunk: int = 0
    pad: float = 12.0  # distance-grid margin (A): a speed setting, results do not depend on it
    extra: dict = field(default_factory=dict)

    def ligands(self, first=0, count=None):
        count = self.n_ligands - first if count is None else count
        return ligands(self.lig_seed, first, count, self.lmin, self.lmax, self.bmin, self.bmax, self.ring_frac)

    def pocket_points(self, k=0):
        seed, n, axes = self.pockets[k]
        return pocket(seed, n, axes, POCKET_CENTRE)

    def quaternions(self, n=None):
        return quaternions(self.quat_seed, self.n_orient if n is None else n)

    def knob_dict(self):
        return dict(hp=self.hp, lp=self.lp or self.hp, threshold=self.threshold, repetitions=self.repetitions,
                    refine=self.refine)


SINGLE = Workload("single", lig_seed=0, n_ligands=1, lmin=32, lmax=32, bmin=4, bmax=4, ring_frac=0.0,
                  pockets=[(1000, 1000, (8.0, 6.0, 5.0))], n_orient=256, hp=10, top_k=10)

SCREEN = Workload("screen", lig_seed=2, n_ligands=10_000, lmin=20, lmax=80, bmin=2, bmax=12, ring_frac=0.0,
                  pockets=[(1001, 4000, (12.0, 9.0, 7.0))], n_orient=512, hp=15, top_k=8, pad=20.0)

_GRID_MAJOR = (6.0, 8.0 + 2.0 / 3.0, 11.0 + 1.0 / 3.0, 14.0)
GRID = Workload("grid", lig_seed=2, n_ligands=100_000, lmin=20, lmax=80, bmin=2, bmax=12, ring_frac=0.0,
                pockets=[(1002 + k, n, (a, 0.75 * a, 0.625 * a))
                         for k, (n, a) in enumerate(zip((1000, 2000, 4000, 8000), _GRID_MAJOR))],
                n_orient=256, hp=15, top_k=8, extra=dict(orient_grid=(64, 256, 1024), step_grid=(30, 15, 10)))

REFINE = Workload("refine", lig_seed=4, n_ligands=4096, lmin=20, lmax=80, bmin=2, bmax=12, ring_frac=0.0,
                  pockets=[(1000, 1000, (8.0, 6.0, 5.0))], n_orient=256, hp=10, top_k=64,
                  extra=dict(blur_sigma=0.6, blur_h=0.375, steps=50, lr_t=0.002, lr_q=1e-5, lr_tau=5e-4, max_dt=0.1,
                             max_dtau=0.05, clash_weight=1000.0))

LARGE = Workload("large", lig_seed=5, n_ligands=1_000_000, lmin=15, lmax=120, bmin=0, bmax=16, ring_frac=0.05,
                 pockets=[(1010, 10_000, (16.0, 12.0, 9.0))], n_orient=1024, hp=10, top_k=8, chunk=65_536, pad=20.0)

DSE = Workload("dse", lig_seed=6, n_ligands=20_000, lmin=28, lmax=120, bmin=2, bmax=16, ring_frac=0.0,
               pockets=[(1001, 4000, (12.0, 9.0, 7.0))], n_orient=32, hp=1, repetitions=3, top_k=1, pad=20.0)

TTS = Workload("tts", lig_seed=8, n_ligands=5000, lmin=28, lmax=120, bmin=2, bmax=16, ring_frac=0.0,
               pockets=GRID.pockets, n_orient=32, hp=1, repetitions=3, top_k=1, pad=20.0,
               extra=dict(mixes=((20, 40, 2, 5), (28, 70, 2, 8), (28, 120, 2, 16), (70, 110, 2, 5), (40, 70, 9, 14)),
                          val_seed=9, val_sizes=(1000, 2000, 5000, 10000)))


def tts_training_sets(w=None):
    """The campaign's ligand mixes (one LigandBatch per mix)."""
    w = w or TTS
    return [ligands(w.lig_seed + 10 * i, 0, w.n_ligands, lo, hi, bl, bh, 0.0)
            for i, (lo, hi, bl, bh) in enumerate(w.extra["mixes"])]


def tts_validation_set(n, fold, w=None):
    """A validation database of n ligands for one held-out pocket."""
    w = w or TTS
    return ligands(w.extra["val_seed"] + 100 * fold, 0, n, DSE.lmin, DSE.lmax, DSE.bmin, DSE.bmax, 0.0)


ALL = {w.name: w for w in (SINGLE, SCREEN, GRID, REFINE, LARGE, DSE, TTS)}


def tiny_ligand(seed: int, l: int, nrot: int):
    """A small ligand for brute-force checks (one item of a dedicated stream)."""
    return ligands(9000 + seed, 0, 1, l, l, nrot, nrot).ligand(0)


def stack_poses(xyz_list):
    return np.stack(xyz_list)
