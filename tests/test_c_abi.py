"""The C ABI used from C alone: tests/c_abi/dock_file.c compiles and links
against include/gd.h and libgd.so (CPU); on the GPU its ranked poses equal the
Python binding's on the same input file, and docking the same ligands from
device-resident arrays (on_device = 1, asynchronous on a stream of its own)
gives the same poses."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import synth
from synth import configs
from tests import gpuutil
from tests.gpuutil import gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_abi", "dock_file.c")
LIBDIR = os.path.join(ROOT, "paper_1901_06363_amd")


def _build(tmp):
    exe = os.path.join(tmp, "dock_file")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                           "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include", SRC, "-o", exe,
                           "-L" + LIBDIR, "-lgd", "-L/opt/rocm/lib", "-lamdhip64",
                           "-Wl,-rpath," + LIBDIR + ":/opt/rocm/lib"])
    return exe


def _write_input(path, pts, ligs, quats, hp, top_k):
    with open(path, "wb") as f:
        f.write(struct.pack("<i", len(pts)))
        f.write(np.asarray(pts, "<f4").tobytes())
        f.write(struct.pack("<i", ligs.n))
        for arr, dt in ((ligs.atom_off, "<i4"), (ligs.x, "<f4"), (ligs.y, "<f4"), (ligs.z, "<f4"),
                        (ligs.bond_off, "<i4"), (ligs.bonds, "<i4"), (ligs.rot_off, "<i4"), (ligs.rot, "<i4")):
            f.write(np.asarray(arr, dt).tobytes())
        f.write(struct.pack("<i", len(quats)))
        f.write(np.asarray(quats, "<f8").tobytes())
        f.write(struct.pack("<ii", hp, top_k))


@pytest.mark.skipif(shutil.which("gcc") is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"),
                    reason="needs gcc and the HIP headers")
def test_c_program_compiles_and_links(tmp_path):
    assert os.path.exists(os.path.join(LIBDIR, "libgd.so")), "build the library first"
    exe = _build(str(tmp_path))
    assert os.access(exe, os.X_OK)


@gpu
def test_c_program_matches_binding(tmp_path):
    g = gpuutil.gd()
    pts = configs.SINGLE.pocket_points()
    ligs = synth.ligands(61, 0, 5, 16, 40, 1, 5, 0.0)
    q = synth.quaternions(12, 24)
    inp = os.path.join(str(tmp_path), "in.bin")
    _write_input(inp, pts, ligs, q, 10, 3)
    exe = _build(str(tmp_path))
    out = subprocess.run([exe, inp], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.strip().splitlines()
    assert lines[-1].startswith("poses ")
    assert lines[-2] == "device-resident inputs identical 1", lines[-2]
    rows = np.array([[float(v) for v in ln.split()] for ln in lines[:-2]])
    P = g.Pocket(pts, 0.5, 12.0)
    b = g.Batch(P, ligs, q, hp=10, top_k=3)
    h = b.dock(g.BATCHED).host()
    assert int(lines[-1].split()[1]) == b.poses_expected == int(h["counters"][0])
    for row in rows:
        i, k = int(row[0]), int(row[1])
        assert int(row[2]) == h["orient"][i, k] and int(row[3]) == h["S"][i, k] and int(row[4]) == h["clash"][i, k]
        assert row[5] == h["overlap"][i, k]
    assert len(rows) == ligs.n * 3
