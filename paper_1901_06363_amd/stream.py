"""Streaming screen of a large ligand library through the persistent kernel.

A library too large for one batch is docked chunk by chunk.  While chunk i
docks on the GPU, a host thread prepares chunk i+1 (validation, topology,
straddling pairs, work queue, upload on a side stream), so host preparation
overlaps device work.  The top-k poses of each chunk can then be refined on
the density surrogate and re-scored exactly (``refine_poses=dict(...)``, the
options of ``refine``).

Ligand sources are callables ``source(first, count) -> LigandBatch`` so that a
chunk is generated (or read) only when it is about to be prepared.
"""
from __future__ import annotations

import threading

import numpy as np

from . import BATCHED, Batch, _torch, refine as _refine


def poses_from_topk(res, ligands):
    """CSR pose arrays (pose_lig, px, py, pz) of every top-k pose of a docking
    result, gathered on the device from its (n, k, max_atoms, 3) coordinates."""
    torch = _torch()
    n, k, lmax = res.xyz.shape[0], res.xyz.shape[1], res.xyz.shape[2]
    nat = np.diff(np.asarray(ligands.atom_off)).astype(np.int64)
    pose_lig = np.repeat(np.arange(n), k)
    pa = nat[pose_lig]
    first = np.concatenate([[0], np.cumsum(pa)[:-1]])
    idx = np.repeat(np.arange(len(pose_lig)) * lmax - first, pa) + np.arange(pa.sum())
    X = res.xyz.reshape(-1, 3).index_select(0, torch.from_numpy(idx).to(res.xyz.device))
    return pose_lig, X[:, 0].contiguous(), X[:, 1].contiguous(), X[:, 2].contiguous()


class _Prepared:
    def __init__(self):
        self.batch = None
        self.ligands = None
        self.error = None


def _prepare(slot, pocket, source, first, count, quats, knobs, stream, tiling):
    try:
        ligs = source(first, count)
        slot.ligands = ligs
        slot.batch = Batch(pocket, ligs, quats, stream=stream, **knobs)
        if tiling:
            slot.batch.set_tiling(*tiling)
    except BaseException as e:  # re-raised in the consumer
        slot.error = e


def screen(pocket, source, n_ligands, quats, chunk=65536, mode=BATCHED, refine_poses=None, want_xyz=True, tiling=None,
           **knobs):
    """Dock ligands [0, n_ligands) of ``source`` in chunks; yields one dict per
    chunk: first, count, ligands, poses, dock_ms (docking kernel time, HIP
    events), result (host arrays of the top-k poses), and with ``refine_poses``
    the refined poses' surrogate, exact S, clash, acceptance and coordinates.
    ``knobs`` are the Batch knobs (hp, lp, threshold, repetitions, refine (tile
    peeling), top_k, clash_dist, clash_min_bonds); the pocket needs a density
    grid for ``refine_poses``.  ``tiling`` (waves per block, angle block,
    pairs per lane) is applied to every chunk's batch.

    The chunks are pipelined: while chunk i docks on the GPU, a host thread
    prepares chunk i+1, and chunk i-1 is refined on its own stream (after its
    docking, concurrently with chunk i's) and copied to the host on a third
    stream that waits for chunk i-1's work only.
    """
    torch = _torch()
    if refine_poses is not None and not want_xyz:
        raise ValueError("refinement needs the pose coordinates (want_xyz=True)")
    side = torch.cuda.Stream()
    rstream = torch.cuda.Stream()
    copy = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    starts = list(range(0, n_ligands, chunk))

    def launch(i):
        slot = _Prepared()
        first = starts[i]
        th = threading.Thread(target=_prepare, args=(slot, pocket, source, first, min(chunk, n_ligands - first),
                                                     quats, knobs, side, tiling))
        th.start()
        return slot, th

    def finish(p):
        # refinement of one chunk on its stream after its docking, then the
        # host copies on the copy stream after both
        item = p["item"]
        refined = None
        if refine_poses is not None:
            rstream.wait_event(p["event"])
            with torch.cuda.stream(rstream):
                pose_lig, px, py, pz = poses_from_topk(p["out"], item["ligands"])
                r = _refine(pocket, item["ligands"], pose_lig, px, py, pz, stream=rstream, **refine_poses)
            refined = (pose_lig, px, py, pz, r)
            copy.wait_stream(rstream)
        copy.wait_event(p["event"])
        with torch.cuda.stream(copy):
            if refined is not None:
                pose_lig, px, py, pz, r = refined
                item["refine"] = dict(pose_lig=pose_lig, F=r["F"].cpu().numpy(), S=r["S"].cpu().numpy(),
                                      clash=r["clash"].cpu().numpy(), accepted=r["accepted"].cpu().numpy(),
                                      xyz=torch.stack([px, py, pz], 1).cpu().numpy())
            item["result"] = p["out"].host()
        copy.synchronize()
        item["dock_ms"] = float(sum(p["batch"].read_timing()))
        return item

    nxt = launch(0) if starts else None
    pending = None
    for i, first in enumerate(starts):
        slot, th = nxt
        th.join()
        if slot.error is not None:
            raise slot.error
        B = slot.batch
        out = B.alloc_outputs(want_angles=True, want_xyz=want_xyz)
        B.enable_timing(True)
        B.dock(mode, out)
        ev = torch.cuda.Event()
        ev.record(main)
        # prepare the next chunk while this one docks
        nxt = launch(i + 1) if i + 1 < len(starts) else None
        if pending is not None:
            yield finish(pending)
        pending = dict(item=dict(first=first, count=B.n_ligands, ligands=slot.ligands, poses=B.poses_expected),
                       batch=B, out=out, event=ev)
        del slot
    if pending is not None:
        yield finish(pending)
