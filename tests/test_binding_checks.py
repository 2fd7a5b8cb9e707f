"""The Python binding rejects malformed pose and parameter arrays before any
call into the library (CPU only: the checks run before the pocket is used)."""
import numpy as np
import pytest
import torch

import paper_1901_06363_amd as g
from paper_1901_06363_amd import _ops
from synth import configs


def _ligs():
    return configs.SCREEN.ligands(0, 3)


def _coords(n, dtype=torch.float32):
    return [torch.zeros(n, dtype=dtype) for _ in range(3)]


def test_pose_ligand_index_out_of_range():
    L = _ligs()
    for bad in ([3], [-1], [0, 1, 7]):
        with pytest.raises(ValueError, match="pose_lig"):
            g.score_poses(None, L, np.array(bad), *_coords(1000))


@pytest.mark.parametrize("fn", ["score_poses", "refine"])
def test_coordinate_arrays_rejected(fn):
    L = _ligs()
    pl = np.array([0, 2, 1, 2])
    need = int(np.diff(L.atom_off)[pl].sum())
    call = getattr(g, fn)
    x, y, z = _coords(need)
    # float64 instead of float32
    with pytest.raises(TypeError, match="float32"):
        call(None, L, pl, x.double(), y, z)
    # a strided view (every other element of a longer array)
    with pytest.raises(ValueError, match="contiguous"):
        call(None, L, pl, x, torch.zeros(2 * need)[::2], z)
    # one value short of the poses' atom count
    with pytest.raises(ValueError, match="poses need"):
        call(None, L, pl, x, y, z[:need - 1])
    # not a tensor
    with pytest.raises(TypeError, match="torch tensor"):
        call(None, L, pl, x, y, np.zeros(need, np.float32))
    # everything right but on the host: the device check comes last
    with pytest.raises(TypeError, match="CUDA"):
        call(None, L, pl, x, y, z)


def test_surrogate_coordinates_rejected_before_parameters():
    L = _ligs()
    pl = np.array([0, 1])
    need = int(np.diff(L.atom_off)[pl].sum())
    x, y, z = _coords(need)
    t, q, tau = torch.zeros(2, 3), torch.zeros(2, 4), torch.zeros(2, 12)
    with pytest.raises(ValueError, match="poses need"):
        g.surrogate_fwd(None, L, pl, x[:5], y, z, t, q, tau)
    with pytest.raises(ValueError, match="contiguous"):
        g.surrogate_bwd(None, L, pl, x, torch.zeros(2 * need)[::2], z, t, q, tau, torch.ones(2))


def test_parameter_shapes_rejected():
    n, rmax = 4, 5
    ok = dict(t=torch.zeros(n, 3), q=torch.zeros(n, 4), tau=torch.zeros(n, rmax))
    cases = [
        dict(t=torch.zeros(3)),              # one translation for all poses
        dict(t=torch.zeros(n, 4)),
        dict(q=torch.zeros(n - 1, 4)),
        dict(q=torch.zeros(n, 3)),
        dict(tau=torch.zeros(n, rmax - 1)),  # fewer columns than rotamers
        dict(tau=torch.zeros(n + 1, rmax)),
        dict(tau=None),                      # rotamers but no torsions
        dict(t=torch.zeros(n, 3, dtype=torch.int32)),
    ]
    for c in cases:
        a = dict(ok, **c)
        with pytest.raises((ValueError, TypeError)):
            _ops._prm(a["t"], a["q"], a["tau"], n, rmax)
    # well-formed host tensors pass the shape checks and stop at the device check
    with pytest.raises(TypeError, match="CUDA"):
        _ops._prm(ok["t"], ok["q"], ok["tau"], n, rmax)
    # dF: one value per pose
    for bad in (torch.zeros(n + 1), torch.zeros(n, 1)):
        with pytest.raises(ValueError, match="dF"):
            _ops._check_param("dF", bad, n, None)
