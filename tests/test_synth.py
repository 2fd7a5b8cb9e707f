"""The seeded input generators: a large request split over threads returns
exactly the serial stream."""
import numpy as np

import synth


def test_parallel_generation_equals_serial():
    a = synth.ligands(5, 1000, 9000, 15, 120, 0, 16, 0.05)
    b = synth._ligands_serial(5, 1000, 9000, 15, 120, 0, 16, 0.05)
    for k in ("atom_off", "x", "y", "z", "bond_off", "bonds", "rot_off", "rot"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    # and any ligand is the same whichever request draws it
    c = synth.ligands(5, 1000 + 4321, 1, 15, 120, 0, 16, 0.05)
    assert np.array_equal(c.ligand(0)["x"], a.ligand(4321)["x"])
