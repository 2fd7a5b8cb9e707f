"""Independent numpy/scipy re-derivations used to pin the oracle.

Nothing here calls the oracle's arithmetic: fragments come from scipy's graph
routines, rotations from scipy's Rotation (rotation-vector form), the
distance field from scipy's exact Euclidean distance transform, and cell
indices from numpy.  The oracle is then checked against these by value.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components, shortest_path
from scipy.spatial.transform import Rotation


def adjacency(l, bonds, drop=None):
    rows, cols = [], []
    for a, c in np.asarray(bonds).reshape(-1, 2):
        if drop is not None and {int(a), int(c)} == set(drop):
            continue
        rows += [a, c]
        cols += [c, a]
    return csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(l, l))


def bond_distances(l, bonds):
    return shortest_path(adjacency(l, bonds), unweighted=True, directed=False)


def left_mask(l, bonds, a, c):
    """Atoms on a's side once the bond (a, c) is removed."""
    _, lab = connected_components(adjacency(l, bonds, drop=(a, c)), directed=False)
    return lab == lab[a]


def rotate_fragment(X, mask, a, c, side, deg):
    """Rotate the atoms in `mask` about the a->c axis through the moving side's bond atom."""
    X = X.copy()
    k = X[c] - X[a]
    k = k / np.linalg.norm(k)
    p = X[a] if side == 0 else X[c]
    R = Rotation.from_rotvec(np.deg2rad(float(deg)) * k)
    X[mask] = p + R.apply(X[mask] - p)
    return X


class EdtTable:
    """D(c) on a box around the occupied cells via scipy's exact EDT."""

    def __init__(self, pts, h=0.5, margin=40):
        cells = np.floor(np.asarray(pts, np.float64) / h).astype(np.int64)
        self.h = h
        self.lo = cells.min(0) - margin
        dims = cells.max(0) - self.lo + 1 + margin
        free = np.ones(tuple(dims), bool)
        ci = cells - self.lo
        free[ci[:, 0], ci[:, 1], ci[:, 2]] = False
        d = ndimage.distance_transform_edt(free)
        self.D = np.rint(d * d).astype(np.int64)
        self.occ = np.unique(cells, axis=0)

    def lookup(self, cells):
        ci = np.asarray(cells) - self.lo
        return self.D[ci[..., 0], ci[..., 1], ci[..., 2]]

    def score(self, X):
        c = np.floor(np.asarray(X) / self.h).astype(np.int64)
        return int(self.lookup(c).sum())

    def face_margin(self, X):
        """Smallest distance (in A) of any coordinate to a cell face."""
        t = np.asarray(X) / self.h
        f = t - np.floor(t)
        return float(np.min(np.minimum(f, 1 - f)) * self.h)


def clash_flag(X, dist, min_bonds=4, cd=2.0):
    l = len(X)
    d2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    far = dist >= min_bonds
    iu = np.triu_indices(l, 1)
    return bool(np.any((d2[iu] < cd * cd) & far[iu]))


def cross_feasible(X, mask, dist, min_bonds=4, cd=2.0):
    mv = np.where(mask)[0]
    fx = np.where(~mask)[0]
    if len(mv) == 0 or len(fx) == 0:
        return True
    d2 = ((X[mv][:, None, :] - X[fx][None, :, :]) ** 2).sum(-1)
    far = dist[np.ix_(mv, fx)] >= min_bonds
    return not np.any((d2 < cd * cd) & far)


# Tile size for the peel/tile refinement: Eq. 2, y = 360/x + x/hp, minimised
# by hand over the divisors of 360 that are multiples of hp (ties -> smaller).
# hp = 1 gives the paper's 18-degree tile.
TILE_TABLE = {1: (18, 38), 2: (24, 27), 3: (30, 22), 5: (40, 17), 10: (60, 12), 15: (60, 10), 30: (90, 7),
              45: (90, 6), 60: (120, 5), 90: (180, 4)}
