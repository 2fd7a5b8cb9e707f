"""Build libgd.so (HIP kernels + host runtime) for gfx950 with hipcc.

Flags: strict IEEE arithmetic (no fast-math, no automatic contraction: the
FP32 fast path writes its fused multiply-adds explicitly) and the packed-FP32
instruction forms disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgd.so")
PROBE_LIB = os.path.join(HERE, "libgdprobe.so")
SOURCES = ["dock.hip", "score.hip", "refine.hip", "overlap.hip", "runtime.cpp", "api_extra.cpp", "refine_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
         "-I" + os.path.join(os.path.dirname(HERE), "include")]


def build(verbose: bool = False, jobs: int = 4) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    procs = []
    objs = []
    for s in srcs:
        obj = os.path.join(objdir, s + ".o")
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        # compiler output goes to a file: a pipe nobody reads while waiting
        # would block a compiler that prints more than the pipe holds
        log = open(obj + ".log", "w+b")
        procs.append((s, subprocess.Popen(cmd, stdout=log, stderr=subprocess.STDOUT), log))
        while sum(p.poll() is None for _, p, _ in procs) >= jobs:
            procs[[p.poll() is None for _, p, _ in procs].index(True)][1].wait()
    failed = []
    for s, p, log in procs:
        p.wait()
        log.seek(0)
        txt = log.read().decode(errors="replace")
        log.close()
        lines = [ln for ln in txt.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed.append((s, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        for s, txt in failed:
            print("=== %s ===\n%s" % (s, txt), file=sys.stderr)
        raise RuntimeError("hipcc failed for: " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # the measurement-only gather probe (bench.py's L2 reference), a library of its own
    tmp = PROBE_LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC] + FLAGS + ["-shared", "-o", tmp, os.path.join(CSRC, "probe.hip")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    os.replace(tmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
