#!/usr/bin/env python
"""Benchmark of the docking hot path on one MI355X.

Headline workload (the large library): 1,000,000 synthetic ligands (15-120
heavy atoms, 0-16 rotatable bonds, 5 % with a rigid 3-6 ring) against one
10,000-point ellipsoid pocket (16/12/9 A, 0.5 A grid), 1024 rigid
orientations, 10-degree torsion steps, one repetition, top-8 poses per
ligand, streamed in chunks of 65,536 ligands.  One step = one chunk: queue
reset, the persistent docking kernel (placement, greedy sweeps, scoring, bump
tests, FP64 commits, endpoint), top-k reduction, replay of the selected poses,
then 50 ascent steps of the density-surrogate refinement of the chunk's top-8
poses with exact rescoring and acceptance, on the same stream right behind
the docking (their host-side set-up overlaps the docking: uploads go through
pinned staging).  Step s docks chunk s mod 16, so warm-up plus timed
steps cover the whole library.  Chunks are generated and prepared (validated,
topology and work queue built, copied to HBM) on a host thread while earlier
chunks dock; the timed steps start only once every chunk is resident in HBM.

Prints one JSON line: poses scored per second (the knob-determined candidate
count; every candidate is scored and bump-tested), ligands and atoms per
second, the per-ligand-launch form on one chunk with a check that both forms
return identical results, the docking kernel's roofline, a wall-clock rate of
a true stream (generation, preparation, upload, docking, refinement and host
copies of chunks), the CPU oracle baseline (one core and all cores), and the
screening workload (10,000 ligands x 4,000-point pocket) as secondary context.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak
# the FP32 vector rate without the packed two-wide FP32 instructions, which this
# build does not emit: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP32_NONPACKED_TFLOPS = 78.6
FP64_PEAK_TFLOPS = 78.6          # MI355X published FP64 peak (vector and matrix)
# sources of the docking kernel; the HBM traffic measured with rocprofv3 counters
# is reported only while they are unchanged since the measurement
KERNEL_SOURCES = ["dock.hip", "device_common.h", "gd_internal.h"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "dock_persistent_kernel.screen.traffic.md")
OVERLAP_SOURCES = ["overlap.hip", "gd_internal.h"]
OVERLAP_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "overlap_min_kernel.screen_top8.traffic.md")
LARGE_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "dock_persistent_kernel.large.traffic.md")


def kernel_fingerprint(sources=None):
    import hashlib
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1901_06363_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(profile=TRAFFIC_PROFILE, sources=None):
    """HBM bytes per launch of a kernel from its committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy kernel's
    reading), or None when the kernel sources changed since it was taken."""
    try:
        vals = {}
        with open(profile) as fh:
            for ln in fh:
                if ":" in ln and ln.startswith("- "):
                    k, v = ln[2:].split(":", 1)
                    vals[k.strip()] = v.strip().strip("`")
        if vals.get("kernel source fingerprint") != kernel_fingerprint(sources):
            return None
        return dict(fetch=float(vals["HBM bytes read per launch"]), write=float(vals["HBM bytes written per launch"]))
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_share():
    """Host cores this process may use, capped at the 16 a one-GPU machine grants."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def oracle_shard(task):
    """Dock ligands [first, first + count) of a workload with the FP64 oracle
    (one process, one core); returns (candidate poses, seconds)."""
    name, first, count = task
    import oracle
    from synth import configs
    w = configs.ALL[name]
    O = oracle.OraclePocket(w.pocket_points(), 0.5)
    kn = oracle.knobs(**w.knob_dict())
    q = w.quaternions()
    ligs = w.ligands(first, count)
    t0 = time.perf_counter()
    poses = 0
    for i in range(count):
        poses += oracle.dock(O, ligs.ligand(i), kn, q, want_xyz=False).n_cand
    return poses, time.perf_counter() - t0


def cpu_baseline(pool, workers, name, first, n_single, n_per_worker):
    """The FP64 oracle as it stands on the host cores: one process on the
    ligands [first, first + n_single), then `workers` processes at once on
    disjoint shards of n_per_worker ligands each (the paper's master/slave
    data parallelism over ligands).  The pool is forked before the GPU is
    touched; its processes only run the CPU oracle."""
    poses1, dt1 = pool.apply(oracle_shard, ((name, first, n_single),))
    shards = [(name, first + n_single + k * n_per_worker, n_per_worker) for k in range(workers)]
    t0 = time.perf_counter()
    res = pool.map(oracle_shard, shards, chunksize=1)
    wall = time.perf_counter() - t0
    poses_all = sum(p for p, _ in res)
    return dict(value=poses_all / wall, unit="poses/s", cores=workers, kind="oracle",
                sample="%s workload: %d oracle processes at once, each on its own %d ligands (ligands %d-%d), all "
                       "orientations, %d candidate poses in %.1f s of wall clock" % (
                           name, workers, n_per_worker, first + n_single, first + n_single + workers * n_per_worker - 1,
                           poses_all, wall),
                per_core=dict(value=poses1 / dt1, unit="poses/s", cores=1,
                              sample="ligands %d-%d of the %s workload, %d candidate poses in %.1f s" % (
                                  first, first + n_single - 1, name, poses1, dt1)),
                cpu_model=cpu_model(), nproc=os.cpu_count(), host_cores_usable=cpu_share())


def l2_gather_peak(torch):
    """Reference peak of random gathers from an L2-resident table (the
    measurement-only probe library): GB/s gathered for 2-byte and 4-byte
    elements, tables of 2 and 4 MB, the best of each."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1901_06363_amd", "libgdprobe.so"))
    lib.gd_probe_gather.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]
    lib.gd_probe_gather.restype = ctypes.c_int
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    blocks, iters, reps = 256 * 16, 256, 5
    out = {}
    for eb, name in ((2, "u16"), (4, "f32")):
        best = 0.0
        for mb in (2, 4):
            log2 = {2: 20, 4: 19}[eb] + (mb // 4)
            ms = ctypes.c_float(0.0)
            rc = lib.gd_probe_gather(eb, log2, blocks, iters, reps, stream, ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError("gather probe failed (HIP error %d)" % rc)
            gbps = blocks * 256.0 * iters * 8 * eb / (ms.value * 1e-3) / 1e9
            out["%s_%dMB_GBps" % (name, mb)] = gbps
            best = max(best, gbps)
        out["%s_GBps" % name] = best
    out["note"] = ("random gathers, 8 independent index chains per lane, %d blocks of 256 lanes: the reference peak "
                   "for grid lookups that hit in L2" % blocks)
    return out


def torsion_subtree_atoms(np, ligs):
    """Per ligand, the atoms each rotamer's forward kinematics moves (the side
    without atom 0), summed over its rotamers."""
    out = np.zeros(ligs.n, np.int64)
    for i in range(ligs.n):
        lig = ligs.ligand(i)
        l = len(lig["x"])
        adj = [[] for _ in range(l)]
        for a, b in lig["bonds"]:
            adj[a].append(b)
            adj[b].append(a)
        tot = 0
        for a, b in lig["rot"]:
            seen = {0}
            stack = [0]
            while stack:
                u = stack.pop()
                for v in adj[u]:
                    if v not in seen and {u, v} != {int(a), int(b)}:
                        seen.add(v)
                        stack.append(v)
            tot += l - len(seen)
        out[i] = tot
    return out


def refine_leg(gd, torch, np, n_lig, l2=None):
    """The refinement workload: top-64 docked poses of n_lig ligands, 50 ascent
    steps on the blurred-density surrogate, exact rescoring and acceptance."""
    from synth import configs
    from paper_1901_06363_amd.stream import poses_from_topk
    w = configs.REFINE
    e = w.extra
    ligs = w.ligands(0, n_lig)
    P = gd.Pocket(w.pocket_points(), 0.5, w.pad, blur_sigma=e["blur_sigma"], blur_h=e["blur_h"])
    B = gd.Batch(P, ligs, w.quaternions(), hp=w.hp, top_k=w.top_k)
    r = B.dock(gd.BATCHED)
    k = w.top_k
    pose_lig, px, py, pz = poses_from_topk(r, ligs)
    pa = np.diff(ligs.atom_off)[pose_lig]
    kw = dict(steps=e["steps"], lr_t=e["lr_t"], lr_q=e["lr_q"], lr_tau=e["lr_tau"], max_dt=e["max_dt"],
              max_dtau=e["max_dtau"])
    # warm-up on a slice, then the timed call over every pose
    m = min(len(pose_lig), 4096)
    n_warm = int(pa[:m].sum())
    gd.refine(P, ligs, pose_lig[:m], px[:n_warm].clone(), py[:n_warm].clone(), pz[:n_warm].clone(), **kw)
    inputs = (px.clone(), py.clone(), pz.clone())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = gd.refine(P, ligs, pose_lig, px, py, pz, time_kernel=True, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = out["kernel_ms"]
    # the clash-penalised surrogate on the same inputs
    cw = e["clash_weight"]
    outp = gd.refine(P, ligs, pose_lig, *inputs, time_kernel=True, clash_weight=cw, **kw)
    atoms = int(pa.sum())
    passes = e["steps"] + 1
    # algorithmic work per pass (e["steps"] forward + backward passes, one final forward):
    #   bytes: 8 trilinear corners of 4 B per atom
    #   flops: forward kinematics 21 per moved atom of every rotamer's subtree and 32 per rotamer (axis and
    #          matrix), rigid motion 21 per atom, trilinear value and gradient 40 per atom; backward: 15 per atom
    #          (x x g and sums) and 10 per moved atom of every subtree (torsion terms)
    sub = torsion_subtree_atoms(np, ligs)[pose_lig]
    nrot = np.diff(np.asarray(ligs.rot_off))[pose_lig]
    fwd = 21.0 * sub.sum() + 32.0 * nrot.sum() + 61.0 * atoms
    bwd = 15.0 * atoms + 10.0 * sub.sum()
    flops = e["steps"] * (fwd + bwd) + fwd
    gather_bytes = atoms * passes * 8 * 4
    gbps = gather_bytes / (kms * 1e-3) / 1e9
    peak = l2["f32_GBps"] if l2 else None
    return dict(workload="refine: %d ligands x top-%d poses (%d poses, %d atoms), %d ascent steps, sigma %.2f A on a "
                         "%.3f A lattice" % (n_lig, k, len(pose_lig), atoms, e["steps"], e["blur_sigma"], e["blur_h"]),
                poses=len(pose_lig), steps=e["steps"], kernel="refine_kernel", kernel_ms=kms,
                pose_steps_per_s=len(pose_lig) * e["steps"] / (kms * 1e-3),
                refined_poses_per_s_end_to_end=len(pose_lig) / wall,
                accepted=int(out["accepted"].sum().item()),
                gather_GBps=gbps,
                roofline=dict(bound="l2", achieved=gbps, peak=peak, unit="GB/s", frac=(gbps / peak) if peak else None,
                              algo_gather_bytes_per_launch=gather_bytes, algo_flops_per_launch=flops,
                              flops_TFLOPs=flops / (kms * 1e-3) / 1e12,
                              flops_frac_of_fp32_peak=flops / (kms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                              peak_source="l2_gather_peak.f32_GBps (random 4-byte gathers from an L2-resident table)",
                              note="the 8 density nodes of 4 B per atom and pass are read as two 16-byte corner-packed "
                                   "nodes, a quarter of the probe's requests per byte, so a fraction near 1 does not "
                                   "make the kernel gather-bound: its counters show it bound by instruction issue"),
                penalised=dict(clash_weight=cw, kernel_ms=outp["kernel_ms"],
                               accepted=int(outp["accepted"].sum().item())))


def continuous_leg(gd, torch, np, P, out, ligs, n_points, reps=10):
    """Continuous Eq. 1 (no lattice) over the raw pocket points for every
    top-k pose of the screen: per atom the smallest squared distance to any of
    the points in FP64, per pose the in-order sum and l / sum."""
    from paper_1901_06363_amd.stream import poses_from_topk
    pose_lig, px, py, pz = poses_from_topk(out, ligs)
    lay = gd.OverlapLayout(np.diff(np.asarray(ligs.atom_off))[pose_lig])
    for _ in range(2):
        gd.overlap_continuous(P, lay, px, py, pz)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        gd.overlap_continuous(P, lay, px, py, pz)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    pairs = lay.n_atoms * n_points
    achieved = 8.0 * pairs / (ms * 1e-3) / 1e12  # 3 differences, 3 squares, 2 additions per pair
    full = out.xyz.shape[0] == 10_000
    tr = measured_traffic(OVERLAP_TRAFFIC_PROFILE, OVERLAP_SOURCES) if full else None
    return dict(workload="continuous Eq. 1 rescoring of the screen's top-%d poses: %d poses, %d atoms x %d pocket "
                         "points, FP64" % (out.xyz.shape[1], lay.n_poses, lay.n_atoms, n_points),
                poses=lay.n_poses, atoms=lay.n_atoms, points=n_points, ms=ms, pairs_per_s=pairs / (ms * 1e-3),
                poses_per_s=lay.n_poses / (ms * 1e-3),
                roofline=dict(bound="alu", kernel="overlap_min_kernel (+ overlap_sum_kernel)", achieved=achieved,
                              peak=FP64_PEAK_TFLOPS, unit="TFLOP/s", frac=achieved / FP64_PEAK_TFLOPS,
                              algo_flops_per_launch=8.0 * pairs,
                              traffic=(tr["fetch"] + tr["write"]) if tr else None,
                              traffic_unit="HBM bytes per launch of overlap_min_kernel (rocprofv3 FETCH_SIZE + "
                                           "WRITE_SIZE, copy-calibrated)"))


def dse_leg(gd, torch, np, spaces, n_lig):
    """Knob exploration (flat and/or full design space) on the exploration
    workload: per configuration the docking and continuous re-scoring time,
    atoms/s, the top-1 % mean continuous overlap, its Eq. 5 degradation
    against the baseline and the Pareto front."""
    from synth import configs
    from paper_1901_06363_amd import dse
    w = configs.DSE
    n_lig = n_lig or w.n_ligands
    ligs = w.ligands(0, n_lig)
    P = gd.Pocket(w.pocket_points(), 0.5, w.pad)
    q = w.quaternions()
    res = {}
    for sp in spaces:
        t0 = time.perf_counter()

        def prog(i, n, rec):
            log("dse %s %d/%d: hp %d lp %d thr %.1f reps %d peel %d: %.1f ms, top mean %.5f (%.0f s)" % (
                sp, i + 1, n, rec["hp"], rec["lp"], rec["threshold"], rec["repetitions"], rec["refine"],
                rec["time_ms"], rec["top_mean"], time.perf_counter() - t0))
        recs = dse.explore(P, ligs, q, space=sp, top_k=w.top_k, progress=prog)
        base = [r for r in recs if dse.is_baseline(r)][0]
        front = sorted((r for r in recs if r["pareto"]), key=lambda r: -r["atoms_per_s"])
        res[sp] = dict(configs=recs, baseline_ms=base["time_ms"],
                       front=[dict(hp=r["hp"], lp=r["lp"], threshold=r["threshold"], repetitions=r["repetitions"],
                                   refine=r["refine"], speedup=base["time_ms"] / r["time_ms"],
                                   degradation=r["degradation"]) for r in front],
                       wall_s=time.perf_counter() - t0)
    return dict(workload="dse: %d ligands (28-120 atoms, 2-16 rotatable bonds) x 4,000-point pocket, %d "
                         "orientations, top-1 pose re-scored with continuous Eq. 1; degradation over the top 1 %% "
                         "ligands (Eq. 5)" % (n_lig, len(q)), spaces=res)


def tts_leg(gd, torch, np, dse_ligands=5000, records_path=None):
    """Time-to-solution model (Eq. 4): a profiling campaign of every full-space
    configuration on 4 pockets x 5 ligand mixes (5,000 ligands each), the
    per-configuration regressions, their leave-one-pocket-out validation on
    fresh databases of 1,000-10,000 ligands, and the budget-driven knob choice
    of the two use-case scenarios with the degradations of a 5,000-ligand
    exploration."""
    import synth
    from synth import configs
    from paper_1901_06363_amd import dse, tts
    w = configs.TTS
    q = w.quaternions()
    cfgs = dse.configurations("full")
    pockets = []
    for k in range(len(w.pockets)):
        pts = w.pocket_points(k)
        pockets.append((gd.Pocket(pts, 0.5, w.pad), len(pts)))
    t0 = time.perf_counter()

    def prog(tag):
        def f(i, n, rec):
            if i % 64 == 0 or i == n:
                log("tts %s %d/%d (%.0f s)" % (tag, i, n, time.perf_counter() - t0))
        return f
    train_sets = configs.tts_training_sets()
    recs = tts.campaign(pockets, train_sets, q, cfgs, warm=False, progress=prog("train"), top_k=1)
    # floors: 1,000 ligands of the exploration's distribution (mix 2) on pockets 1 and 2
    mix = 2
    lo, hi, bl, bh = w.extra["mixes"][mix]
    small = synth.ligands(w.lig_seed + 10 * mix, 0, 1000, lo, hi, bl, bh, 0.0)
    fl = {pk: tts.floors(tts.campaign([pockets[pk]], [small], q, cfgs, warm=False, progress=prog("floor p%d" % pk),
                                      top_k=1)) for pk in (1, 2)}
    models = tts.fit_models(recs, fl[2])
    r2 = np.array([m.r2_adj for m in models.values()])
    errs = {v: {n: [] for n in w.extra["val_sizes"]} for v in ("eq4", "eq4_floor")}
    vrecs = []
    for f, (P, npts) in enumerate(pockets):
        tr = [r for r in recs if r["pocket"] != f]
        mf = {"eq4": tts.fit_models(tr), "eq4_floor": tts.fit_models(tr, fl[1 if f == 2 else 2])}
        for n in w.extra["val_sizes"]:
            L = configs.tts_validation_set(n, f)
            a, r = tts.ligand_features(L)
            for vr in tts.campaign([(P, npts)], [L], q, cfgs, warm=False, progress=prog("val p%d n%d" % (f, n)),
                                   top_k=1):
                vrecs.append(dict(vr, fold=f))
                for v, m in mf.items():
                    pred = m[tts.key(vr)].predict(npts, a, r, n)
                    errs[v][n].append(100.0 * (pred - vr["ms"]) / vr["ms"])

    def summ(e):
        e = np.asarray(e)
        return dict(runs=len(e), mean_abs_pct=float(np.mean(np.abs(e))), median_abs_pct=float(np.median(np.abs(e))),
                    p95_abs_pct=float(np.percentile(np.abs(e), 95)), max_abs_pct=float(np.max(np.abs(e))),
                    mean_signed_pct=float(np.mean(e)))
    val = {v: {str(n): summ(e) for n, e in ev.items()} for v, ev in errs.items()}
    if records_path:
        with open(records_path, "w") as fh:
            json.dump(dict(train=recs, val=vrecs, floors={str(k): {str(kk): vv for kk, vv in o.items()}
                                                          for k, o in fl.items()}), fh)
    # accuracy of every configuration (platform-independent): a 5,000-ligand exploration
    d = configs.DSE
    dl = d.ligands(0, dse_ligands)
    drecs = dse.explore(gd.Pocket(d.pocket_points(), 0.5, d.pad), dl, d.quaternions(), space="full", top_k=1)
    deg = {tts.key(r): r["degradation"] for r in drecs}
    bkey = tts.key(dse.BASE_KNOBS | dict(lp=45))
    p_d, (a_d, r_d) = len(d.pocket_points()), tts.ligand_features(dl)
    tb = models[bkey].per_ligand(p_d, a_d, r_d)

    def point(nu, budget_ms):
        c = tts.choose(models, deg, p_d, a_d, r_d, nu, budget_ms)
        k = c["key"]
        return dict(ligands=nu, budget_h=budget_ms / 3.6e6, hp=k[0], lp=k[1], threshold=k[2], repetitions=k[3],
                    refine=k[4], completion=c["completion"], degradation=c["degradation"],
                    baseline_completion=min(1.0, budget_ms / (nu * tb)))
    s1 = [point(nu, 3.6e6) for nu in (1e7, 2e7, 5e7, 1e8, 2e8, 5e8, 1e9, 2e9)]
    s2 = [point(5e8, h * 3.6e6) for h in (0.25, 0.5, 1, 2, 4, 8, 24, 48)]
    return dict(workload="tts: %d full-space configurations x 4 pockets (1,000-8,000 points) x 5 ligand mixes of 5,000 "
                         "ligands, 32 orientations; leave-one-pocket-out validation on 1,000-10,000-ligand databases"
                         % len(cfgs),
                train_runs=len(recs), r2_adj_mean=float(np.mean(r2)), r2_adj_min=float(np.min(r2)),
                validation_error=val, baseline_ms_per_ligand=tb,
                scenario1_budget_1h=s1, scenario2_500M_ligands=s2, wall_s=time.perf_counter() - t0)


def grid_leg(gd, torch, np, n_lig=2000):
    """The knob grid: for each of the 4 pockets x orientations {64, 256, 1024}
    x steps {30, 15, 10} degrees, the same n_lig ligands spread over the
    100,000-ligand stream docked in one batched call (persistent kernel) and
    with one launch per ligand; wall clock of each call between
    synchronisations, and whether both forms return identical results."""
    import synth
    from synth import configs
    w = configs.GRID
    idx = np.linspace(0, w.n_ligands - 1, n_lig).astype(int)
    ligs = synth.LigandBatch.from_list([w.ligands(int(i), 1).ligand(0) for i in idx])
    rows = []
    t_all = time.perf_counter()
    for pk in range(len(w.pockets)):
        P = gd.Pocket(w.pocket_points(pk), 0.5, 20.0)
        for n_o in w.extra["orient_grid"]:
            q = synth.quaternions(w.quat_seed, n_o)
            for hp in w.extra["step_grid"]:
                B = gd.Batch(P, ligs, q, hp=hp, top_k=w.top_k)
                times = {}
                res = {}
                for mode, name in ((gd.BATCHED, "batched"), (gd.PER_LIGAND, "per_ligand")):
                    out = B.dock(mode)  # warm-up (and graph capture for the batched form)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    B.dock(mode, out)
                    torch.cuda.synchronize()
                    times[name] = time.perf_counter() - t0
                    res[name] = out.host()
                same = all(np.array_equal(res["batched"][k], res["per_ligand"][k])
                           for k in ("orient", "S", "clash", "angles", "xyz"))
                rows.append(dict(pocket=pk, points=len(P.xyz), orientations=n_o, step=hp, poses=B.poses_expected,
                                 batched_s=times["batched"], per_ligand_s=times["per_ligand"],
                                 batched_poses_per_s=B.poses_expected / times["batched"],
                                 per_ligand_poses_per_s=B.poses_expected / times["per_ligand"],
                                 ratio=times["per_ligand"] / times["batched"], results_identical=bool(same)))
                log("grid pocket %d, %4d orientations, %2d deg: batched %.1f ms, per-ligand %.1f ms, %.2fx, same %s"
                    % (pk, n_o, hp, 1e3 * times["batched"], 1e3 * times["per_ligand"], rows[-1]["ratio"], same))
                del B
    r = np.array([x["ratio"] for x in rows])
    return dict(workload="grid: %d ligands spread over the 100,000-ligand stream x 4 pockets (1,000-8,000 points) x "
                         "orientations {64, 256, 1024} x steps {30, 15, 10} degrees, top-8" % n_lig,
                rows=rows, ratio_min=float(r.min()), ratio_median=float(np.median(r)), ratio_max=float(r.max()),
                all_identical=all(x["results_identical"] for x in rows), wall_s=time.perf_counter() - t_all)


def tiling_sweep(gd, torch, np, workload, n_lig=0, tilings=None):
    """Docking-kernel time of one full batch (a 65,536-ligand chunk of the
    large library, or the screening workload) under every tiling the library
    offers (waves per block x angle block x pairs per lane), HIP events."""
    from synth import configs
    w = configs.LARGE if workload == "large" else configs.SCREEN
    n_lig = n_lig or (w.chunk if workload == "large" else w.n_ligands)
    P = gd.Pocket(w.pocket_points(), 0.5, w.pad)
    B = gd.Batch(P, w.ligands(0, n_lig), w.quaternions(), hp=w.hp, top_k=w.top_k)
    out = B.alloc_outputs(want_angles=True, want_xyz=True)
    rows = []
    tilings = tilings or [(w_, nb, ppl) for w_ in (2, 4, 8) for nb in (8, 16, 32) for ppl in (2, 4, 8)]
    for wpb, nb, ppl in tilings:
        B.set_tiling(wpb, nb, ppl)
        B.dock(gd.BATCHED, out)
        torch.cuda.synchronize()
        B.read_timing()
        B.enable_timing(True)
        B.dock(gd.BATCHED, out)
        ms = float(B.read_timing()[0])
        B.enable_timing(False)
        rows.append(dict(waves_per_block=wpb, angle_block=nb, pairs_per_lane=ppl, kernel_ms=ms))
        log("tiling %d,%d,%d: %.1f ms" % (wpb, nb, ppl, ms))
    best = min(rows, key=lambda r: r["kernel_ms"])
    auto = B.autotune(reps=1)
    hit = [r["kernel_ms"] for r in rows
           if (r["waves_per_block"], r["angle_block"], r["pairs_per_lane"]) == tuple(auto)]
    return dict(workload="%s: %d ligands" % (workload, n_lig), rows=rows, best=best, autotuned=list(auto),
                autotuned_ms=hit[0] if hit else None)


def peaks_leg(gd, torch, np, n_lig=2000, step=1):
    """Peak analysis (Sec. III-B) on synthetic ligands: the exploration
    workload's first n_lig ligands docked at the baseline knobs (hp 1, 3
    repetitions), then the overlap landscape of every rotamer side at each
    best pose in 1-degree steps, summarised by relative fragment size."""
    from synth import configs
    from paper_1901_06363_amd import dse, peaks
    w = configs.DSE
    ligs = w.ligands(0, n_lig)
    P = gd.Pocket(w.pocket_points(), 0.5, w.pad)
    b = dse.BASE_KNOBS
    B = gd.Batch(P, ligs, w.quaternions(), hp=b["hp"], lp=b["lp"], threshold=b["threshold"],
                 repetitions=b["repetitions"], refine=b["refine"], top_k=1)
    res = B.dock(gd.BATCHED)
    gd.sweep_profile(P, B, res, step=step)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    S, f, sz = gd.sweep_profile(P, B, res, step=step)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    h = res.host()
    nat = np.diff(np.asarray(ligs.atom_off))
    nrt = np.diff(np.asarray(ligs.rot_off))
    evals = int(nrt.sum()) * 2 * (360 // step)
    t0 = time.perf_counter()
    recs = peaks.analyse(S.cpu().numpy(), f.cpu().numpy(), sz.cpu().numpy(), nat, nrt, h["S"], step=step)
    summ = peaks.summarize(recs)
    return dict(workload="peaks: %d ligands (28-120 atoms, 2-16 rotatable bonds) docked at the baseline knobs, "
                         "landscapes of every rotamer side at the best pose in %d-degree steps" % (n_lig, step),
                kernel="profile_kernel", kernel_ms=ms, evaluations=evals, evaluations_per_s=evals / (ms * 1e-3),
                host_analysis_s=time.perf_counter() - t0, summary=summ)


def large_leg(gd, torch, n_chunks, tiling=None):
    """The large library streamed through the persistent kernel in chunks of
    65,536 ligands (host preparation of the next chunk overlaps docking), with
    the top-8 poses of every chunk refined and re-scored."""
    from synth import configs
    from paper_1901_06363_amd.stream import screen
    w = configs.LARGE
    r = configs.REFINE.extra
    P = gd.Pocket(w.pocket_points(), 0.5, w.pad, blur_sigma=r["blur_sigma"], blur_h=r["blur_h"])
    ropt = dict(steps=r["steps"], lr_t=r["lr_t"], lr_q=r["lr_q"], lr_tau=r["lr_tau"], max_dt=r["max_dt"],
                max_dtau=r["max_dtau"])
    n = n_chunks * w.chunk
    poses = atoms = 0
    dock_ms = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for item in screen(P, w.ligands, n, w.quaternions(), chunk=w.chunk, refine_poses=ropt, tiling=tiling, hp=w.hp,
                       top_k=w.top_k):
        poses += item["poses"]
        atoms += int(item["ligands"].atom_off[-1])
        dock_ms += item["dock_ms"]
        log("large: chunk at %d done (%.1f s)" % (item["first"], time.perf_counter() - t0))
    dt = time.perf_counter() - t0
    return dict(workload="large: %d ligands (15-120 atoms, 0-16 rotatable bonds, 5%% with a ring) x 10,000-point "
                         "pocket, 1024 orientations, 10-degree steps, chunks of %d, top-8 refined" % (n, w.chunk),
                ligands=n, poses=poses, seconds=dt, poses_per_s=poses / dt, ligands_per_s=n / dt,
                atoms_per_s=atoms / dt, dock_kernel_s=dock_ms * 1e-3,
                kernel_poses_per_s=poses / (dock_ms * 1e-3),
                note="wall clock over the whole stream: generation, preparation, docking, top-k, refinement and host "
                     "copies; dock_kernel_s is the docking kernels' share (HIP events)")


def screen_leg(gd, torch, np, args, steps, warmup, n_lig=0, tiling=""):
    """The screening workload: 10,000 ligands x 4,000-point pocket, 512
    orientations, 15-degree steps, top-8; warm-up, then `steps` timed batched
    docking calls of the resident batch, the per-ligand form on the same
    ligands and the continuous Eq. 1 rescoring of the top-8 poses."""
    from synth import configs
    w = configs.SCREEN
    n_lig = n_lig or w.n_ligands
    t = time.perf_counter()
    ligs = w.ligands(0, n_lig)
    pts = w.pocket_points()
    q = w.quaternions()
    log("screen: inputs generated in %.1f s" % (time.perf_counter() - t))
    P = gd.Pocket(pts, 0.5, w.pad)
    t = time.perf_counter()
    B = gd.Batch(P, ligs, q, hp=w.hp, top_k=w.top_k)
    prep_s = time.perf_counter() - t
    log("screen: batch prepared in %.2f s: %d ligands, %d poses per call" % (prep_s, B.n_ligands, B.poses_expected))
    if tiling:
        B.set_tiling(*[int(v) for v in tiling.split(",")])
    if args.autotune:
        log("screen: autotuned tiling", B.autotune(reps=1))
    tiling = B.tiling()
    out = B.alloc_outputs(want_angles=True, want_xyz=True)
    for _ in range(warmup):
        B.dock(gd.BATCHED, out)
    torch.cuda.synchronize()
    B.enable_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        B.dock(gd.BATCHED, out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kernel_ms = B.read_timing()
    B.enable_timing(False)
    host = out.host()
    counters = host["counters"]
    assert counters[0] == B.poses_expected, (counters[0], B.poses_expected)
    k_ms = float(np.mean(kernel_ms))
    log("screen: %d steps, %.1f ms/step, docking kernel %.1f ms" % (steps, dt * 1e3 / steps, k_ms))
    per_lig = None
    if not args.no_per_ligand:
        rp = B.dock(gd.PER_LIGAND)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        rp = B.dock(gd.PER_LIGAND, rp)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        hp_ = rp.host()
        same = all(np.array_equal(host[k], hp_[k]) for k in ("orient", "S", "clash", "angles", "xyz"))
        per_lig = dict(ligands=n_lig, per_ligand_poses_per_s=B.poses_expected / tp, per_ligand_ligands_per_s=n_lig / tp,
                       batched_poses_per_s=B.poses_expected * steps / dt, batched_over_per_ligand=tp / (dt / steps),
                       results_identical=bool(same))
        log("screen: per-ligand launches:", per_lig)
    cont = None
    if not args.no_continuous:
        cont = continuous_leg(gd, torch, np, P, out, ligs, len(pts))
        log("screen: continuous rescoring:", cont)
    achieved = B.algo_flops / (k_ms * 1e-3) / 1e12
    tr = measured_traffic() if n_lig == w.n_ligands else None
    return dict(
        workload="screen: %d ligands (20-80 atoms, 2-12 rotatable bonds) x 4,000-point pocket, 512 orientations, "
                 "15-degree steps, 1 repetition, top-8" % n_lig,
        ligands=n_lig, orientations=len(q), hp_step_deg=w.hp, poses_per_step=B.poses_expected, tiling=list(tiling),
        grid_pad_A=w.pad, steps=steps, warmup=warmup, ms_per_step=dt * 1e3 / steps,
        poses_per_s=B.poses_expected * steps / dt, ligands_per_s=n_lig * steps / dt,
        atoms_per_s=B.n_atoms_total * steps / dt,
        fallback_per_pose=float(counters[1]) / float(counters[0]), oob_lookups=int(counters[2]), prep_s=prep_s,
        per_ligand=per_lig, continuous=cont,
        roofline=dict(bound="alu", achieved=achieved, peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                      frac_of_nonpacked_fp32=achieved / FP32_NONPACKED_TFLOPS,
                      frac=achieved / FP32_VECTOR_PEAK_TFLOPS,
                      traffic=(tr["fetch"] + tr["write"]) if tr else None,
                      traffic_unit="HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                      kernel="dock_persistent_kernel", kernel_ms=k_ms, algo_flops_per_launch=B.algo_flops,
                      algo_gather_bytes_per_launch=B.algo_bytes,
                      gather_GBps=B.algo_bytes / (k_ms * 1e-3) / 1e9))


class ChunkOutputs:
    """Sets of docking outputs sized for the largest chunk, viewed per chunk
    (a chunk always uses the same set, so its captured graph keeps its output
    pointers)."""

    def __init__(self, gd, torch, n_max, k, reps, rmax, lmax, n_sets=2):
        dev = torch.device("cuda")
        self.gd, self.k = gd, k
        self.sets = [dict(recs=torch.empty(n_max * k * 6, dtype=torch.int32, device=dev),
                          ang=torch.empty(n_max * k * reps * rmax * 2, dtype=torch.int16, device=dev),
                          xyz=torch.empty(n_max * k * lmax * 3, dtype=torch.float32, device=dev),
                          cnt=torch.zeros(4, dtype=torch.int64, device=dev)) for _ in range(n_sets)]

    def view(self, i, B):
        s = self.sets[i]
        n, k = B.n_ligands, B.top_k
        recs = s["recs"][:n * k * 6].view(n * k, 6)
        ang = s["ang"][:n * k * B.repetitions * B.max_rot * 2].view(n, k, B.repetitions, B.max_rot, 2)
        xyz = s["xyz"][:n * k * B.max_atoms * 3].view(n, k, B.max_atoms, 3)
        return self.gd.DockResult(recs, ang, xyz, s["cnt"], n, k)


def large_headline(gd, torch, np, args):
    """Headline: the large library, one chunk of 65,536 ligands per step (see
    the module docstring)."""
    import threading
    from synth import configs
    w = configs.LARGE
    rx = configs.REFINE.extra
    n_lib = args.large_ligands or w.n_ligands
    chunk = args.chunk or w.chunk
    starts = list(range(0, n_lib, chunk))
    nch = len(starts)
    ropt = dict(steps=rx["steps"], lr_t=rx["lr_t"], lr_q=rx["lr_q"], lr_tau=rx["lr_tau"], max_dt=rx["max_dt"],
                max_dtau=rx["max_dtau"])
    P = gd.Pocket(w.pocket_points(), 0.5, w.pad, blur_sigma=rx["blur_sigma"], blur_h=rx["blur_h"])
    q = w.quaternions()
    side = torch.cuda.Stream()

    # host thread: generate and prepare every chunk once, in order; they stay resident in HBM
    slots = [None] * nch
    gidx = [None] * nch  # per chunk: the rows of its top-k poses in CSR order (device), and their ligands
    plig = [None] * nch
    ready = [threading.Event() for _ in range(nch)]
    prep_s = [0.0] * nch
    err = []

    def producer():
        try:
            for i, first in enumerate(starts):
                t = time.perf_counter()
                ligs = w.ligands(first, min(chunk, n_lib - first))
                B_ = gd.Batch(P, ligs, q, stream=side, hp=w.hp, top_k=w.top_k)
                # gather index of the chunk's top-k poses from the (n, k, max_atoms, 3) outputs into CSR
                # rows (fixed by the atom counts), uploaded once with the chunk
                nat = np.diff(np.asarray(ligs.atom_off)).astype(np.int64)
                pl = np.repeat(np.arange(B_.n_ligands), w.top_k)
                pa = nat[pl]
                first_row = np.concatenate([[0], np.cumsum(pa)[:-1]])
                idx = np.repeat(np.arange(len(pl)) * B_.max_atoms - first_row, pa) + np.arange(pa.sum())
                with torch.cuda.stream(side):
                    gidx[i] = torch.from_numpy(idx.astype(np.int32)).to("cuda")
                plig[i] = pl
                slots[i] = B_
                prep_s[i] = time.perf_counter() - t
                ready[i].set()
        except BaseException as e:  # re-raised by the consumer
            err.append(e)
            for ev in ready:
                ev.set()

    t_setup = time.perf_counter()
    th = threading.Thread(target=producer, daemon=True)
    th.start()

    def batch(i):
        ready[i].wait()
        if err:
            raise err[0]
        return slots[i]

    B0 = batch(0)
    if args.tiling:
        tiling = tuple(int(v) for v in args.tiling.split(","))
    else:
        tiling = B0.autotune(reps=1)
    log("large: chunk 0 prepared in %.1f s, tiling %s (%s)" % (prep_s[0], tiling,
                                                                "given" if args.tiling else "autotuned"))
    lmax = max(w.lmax, B0.max_atoms)
    # one output set: a chunk's refinement runs on the same stream right behind its docking
    outs = ChunkOutputs(gd, torch, chunk, w.top_k, B0.repetitions, 16 if w.bmax <= 16 else w.bmax, lmax, 1)
    n_steps = args.warmup + args.steps
    cnt_hist = torch.zeros((n_steps, 4), dtype=torch.int64, device="cuda")
    acc_hist = torch.zeros(n_steps, dtype=torch.int64, device="cuda")
    configured = set()
    timed_batches = []
    t0 = None
    # Each step enqueues, on one stream: the chunk's docking (graph: queue reset, persistent kernel, top-k,
    # replay), the gather of its top-8 poses into CSR rows, and their refinement and exact rescoring.  The
    # refinement's host-side preparation and uploads (pinned staging) run while the chunk docks, so the device
    # goes from one chunk's refinement straight to the next chunk's docking.
    for s in range(n_steps):
        if s == args.warmup:
            th.join()  # every chunk resident before the timed region
            if err:
                raise err[0]
            torch.cuda.synchronize()
            for i in range(nch):
                slots[i].read_timing()  # drop the warm-up durations
            t0 = time.perf_counter()
            log("large: %d warm-up steps done, all %d chunks resident (setup %.1f s)" % (
                args.warmup, nch, t0 - t_setup))
        c = s % nch
        B = batch(c)
        if c not in configured:
            B.set_tiling(*tiling)
            B.enable_timing(True)
            configured.add(c)
        if B.max_atoms > lmax or B.max_rot > 16:
            raise RuntimeError("chunk %d exceeds the output buffers" % c)
        o = outs.view(0, B)
        B.dock(gd.BATCHED, o)
        cnt_hist[s].copy_(o.counters)
        X = o.xyz.reshape(-1, 3).index_select(0, gidx[c])
        r = gd.refine(P, B.lig, plig[c], X[:, 0].contiguous(), X[:, 1].contiguous(), X[:, 2].contiguous(), **ropt)
        acc_hist[s] = r["accepted"].sum()
        if t0 is not None:
            timed_batches.append(B)
        if s < args.warmup or (s - args.warmup) % 4 == 3:
            log("large: step %d (chunk %d) enqueued, %.1f s" % (s, c, time.perf_counter() - t_setup))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms = {}
    for i in range(nch):
        kms[i] = slots[i].read_timing()
    cnt = cnt_hist.cpu().numpy()
    acc = acc_hist.cpu().numpy()
    poses = lig_n = atoms = 0
    flops = gbytes = 0.0
    kernel_ms = []
    for j, B in enumerate(timed_batches):
        s = args.warmup + j
        assert cnt[s][0] == B.poses_expected, (s, cnt[s][0], B.poses_expected)
        poses += B.poses_expected
        lig_n += B.n_ligands
        atoms += B.n_atoms_total
        flops += B.algo_flops
        gbytes += B.algo_bytes
    for i, v in kms.items():
        kernel_ms.extend(v)
    k_s = sum(kernel_ms) * 1e-3
    fallbacks = int(cnt[args.warmup:, 1].sum())
    log("large: %d timed steps in %.1f s (%.0f ms/step), docking kernels %.1f s" % (
        args.steps, dt, dt * 1e3 / args.steps, k_s))

    # per-ligand launches against the batched form on one chunk (or a sample of it)
    per_lig = None
    if not args.no_per_ligand:
        ns = min(args.per_ligand_sample or B0.n_ligands, B0.n_ligands)
        Bs = B0 if ns == B0.n_ligands else gd.Batch(P, w.ligands(0, ns), q, hp=w.hp, top_k=w.top_k)
        Bs.set_tiling(*tiling)
        rb = Bs.dock(gd.BATCHED)
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        rb = Bs.dock(gd.BATCHED, rb)
        torch.cuda.synchronize()
        tb = time.perf_counter() - tb0
        hb = rb.host()
        del rb
        tp0 = time.perf_counter()
        rp = Bs.dock(gd.PER_LIGAND)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        hp_ = rp.host()
        del rp
        same = all(np.array_equal(hb[k], hp_[k]) for k in ("orient", "S", "clash", "angles", "xyz"))
        per_lig = dict(ligands=ns, chunk=0, per_ligand_poses_per_s=Bs.poses_expected / tp,
                       per_ligand_ligands_per_s=ns / tp, batched_poses_per_s=Bs.poses_expected / tb,
                       batched_over_per_ligand=tp / tb, results_identical=bool(same),
                       note="one docking call each (batched: persistent kernel, top-k and replay; per-ligand: one "
                            "launch per ligand, then top-k and replay), wall clock between synchronisations")
        log("large: per-ligand launches:", per_lig)
        del Bs
    lib_poses = sum(slots[i].poses_expected for i in range(nch))
    lib_flops = sum(slots[i].algo_flops for i in range(nch))
    n_launch = len(kernel_ms)
    n_timed = len(timed_batches)
    torch.cuda.synchronize()
    del slots, outs, timed_batches, B0, B, o, X, r, gidx
    torch.cuda.empty_cache()

    achieved = flops / k_s / 1e12
    tr = measured_traffic(LARGE_TRAFFIC_PROFILE) if n_lib == w.n_ligands and chunk == w.chunk else None
    return dict(
        value=poses / dt, ms_per_step=dt * 1e3 / args.steps,
        config=dict(workload="large: %d ligands (15-120 atoms, 0-16 rotatable bonds, 5%% with a rigid 3-6 ring) x "
                             "10,000-point pocket (16/12/9 A), 1024 orientations, 10-degree steps, 1 repetition, "
                             "chunks of %d ligands, top-8 poses refined (50 ascent steps) and re-scored" % (n_lib, chunk),
                    ligands=n_lib, chunk=chunk, chunks=nch, orientations=len(q), hp_step_deg=w.hp, top_k=w.top_k,
                    poses_per_library=lib_poses, tiling=list(tiling), grid_pad_A=w.pad,
                    step="one chunk: dock + top-k + replay + top-8 refinement and exact rescoring"),
        ligands_per_s=lig_n / dt, atoms_per_s=atoms / dt, poses_timed=poses,
        kernel=dict(docking_kernel_s=k_s, poses_per_s=poses / k_s, ligands_per_s=lig_n / k_s,
                    note="docking-kernel time only (HIP events on its stream), summed over the timed steps"),
        refined_poses_accepted_timed=int(acc[args.warmup:].sum()),
        fallback_per_pose=fallbacks / max(poses, 1),
        prep=dict(per_chunk_s=prep_s, setup_s=(t0 - t_setup),
                  note="generation + validation + topology + upload of each chunk on a host thread, overlapping the "
                       "warm-up steps"),
        per_ligand=per_lig,
        roofline=dict(bound="alu", achieved=achieved, peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                      frac_of_nonpacked_fp32=achieved / FP32_NONPACKED_TFLOPS,
                      frac=achieved / FP32_VECTOR_PEAK_TFLOPS,
                      traffic=(tr["fetch"] + tr["write"]) if tr else None,
                      traffic_unit="HBM bytes per launch of one full chunk (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                   "copy-calibrated)",
                      kernel="dock_persistent_kernel", kernel_ms=1e3 * k_s / n_launch,
                      algo_flops_per_launch=flops / n_timed, library_algo_flops=lib_flops,
                      algo_gather_bytes_per_launch=gbytes / n_timed, gather_GBps=gbytes / k_s / 1e9))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps (large: chunks)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=("large", "screen"), default="large", help="headline workload")
    ap.add_argument("--large-ligands", type=int, default=0, help="library size of the large workload (testing only)")
    ap.add_argument("--chunk", type=int, default=0, help="chunk size of the large workload (testing only)")
    ap.add_argument("--per-ligand-sample", type=int, default=0,
                    help="ligands of the per-ligand comparison (default: a whole chunk / the whole screen)")
    ap.add_argument("--cpu-single", type=int, default=12, help="ligands of the one-core oracle run")
    ap.add_argument("--cpu-per-worker", type=int, default=6, help="ligands per oracle process of the all-core run")
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle processes (default: usable cores, <= 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-ligand", action="store_true")
    ap.add_argument("--no-refine", action="store_true")
    ap.add_argument("--no-screen", action="store_true", help="skip the secondary screening leg")
    ap.add_argument("--screen-steps", type=int, default=3)
    ap.add_argument("--refine-only", action="store_true", help="run only the refinement leg (profiling)")
    ap.add_argument("--refine-ligands", type=int, default=4096)
    ap.add_argument("--stream-chunks", type=int, default=2,
                    help="chunks of the wall-clock stream leg (generation to host copies), 0 = none")
    ap.add_argument("--dse", type=str, default="", help="run only the knob exploration: flat, full or both")
    ap.add_argument("--dse-ligands", type=int, default=0)
    ap.add_argument("--peaks", action="store_true", help="run only the peak analysis of overlap landscapes")
    ap.add_argument("--grid", action="store_true", help="run only the knob-grid leg (batched vs per-ligand)")
    ap.add_argument("--tiling-sweep", type=str, default="", help="time every tiling on one batch: large or screen")
    ap.add_argument("--sweep-tilings", type=str, default="", help="tilings of the sweep, e.g. 2,8,4;8,32,4")
    ap.add_argument("--grid-ligands", type=int, default=2000)
    ap.add_argument("--tts-records", type=str, default="", help="also write the campaign's raw records (JSON)")
    ap.add_argument("--tts", action="store_true", help="run only the time-to-solution campaign, validation and "
                                                          "budget scenarios")
    ap.add_argument("--no-continuous", action="store_true")
    ap.add_argument("--tiling", type=str, default="")
    ap.add_argument("--autotune", action="store_true", help="screen workload: autotune the tiling")
    ap.add_argument("--n-ligands", type=int, default=0, help="screen ligand count (testing only)")
    ap.add_argument("--fingerprint", action="store_true", help="print the docking kernel's source fingerprint")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (the reference kernel for HBM byte counters)")
    args = ap.parse_args()

    if args.fingerprint:
        print(kernel_fingerprint(), kernel_fingerprint(OVERLAP_SOURCES))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (ligand batches shard trivially "
              "across GPUs); got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)
    only = (args.copy_calibration or args.refine_only or args.peaks or args.tts or args.dse or args.grid
            or args.tiling_sweep)
    pool = None
    workers = args.cpu_workers or cpu_share()
    if not only and not args.no_cpu_baseline:
        # forked before anything touches the GPU; the processes run the CPU oracle only
        import multiprocessing
        pool = multiprocessing.get_context("fork").Pool(workers)

    import numpy as np
    import torch

    import paper_1901_06363_amd as gd

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # One elementwise kernel that reads and writes exactly n bytes each; the
        # counters it produces convert FETCH_SIZE / WRITE_SIZE readings into bytes.
        n = args.copy_calibration << 20
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        log("copy calibration: read %d B, wrote %d B" % (n, n))
        return
    if args.refine_only:
        print(json.dumps(refine_leg(gd, torch, np, args.refine_ligands, l2_gather_peak(torch))), flush=True)
        return
    if args.peaks:
        print(json.dumps(peaks_leg(gd, torch, np)), flush=True)
        return
    if args.grid:
        print(json.dumps(grid_leg(gd, torch, np, args.grid_ligands)), flush=True)
        return
    if args.tiling_sweep:
        til = [tuple(int(v) for v in t.split(",")) for t in args.sweep_tilings.split(";") if t]
        print(json.dumps(tiling_sweep(gd, torch, np, args.tiling_sweep, tilings=til or None)), flush=True)
        return
    if args.tts:
        print(json.dumps(tts_leg(gd, torch, np, records_path=args.tts_records or None)), flush=True)
        return
    if args.dse:
        spaces = ["flat", "full"] if args.dse == "both" else [args.dse]
        print(json.dumps(dse_leg(gd, torch, np, spaces, args.dse_ligands)), flush=True)
        return

    metric = "poses scored/s and ligands docked/s, batched vs per-ligand, same GPU, exact"
    l2 = l2_gather_peak(torch)
    log("l2 gather peak:", l2)
    if args.workload == "screen":
        sc = screen_leg(gd, torch, np, args, args.steps, args.warmup, args.n_ligands, args.tiling)
        head = dict(value=sc["poses_per_s"], ms_per_step=sc["ms_per_step"],
                    config=dict(workload=sc["workload"], ligands=sc["ligands"], orientations=sc["orientations"],
                                hp_step_deg=sc["hp_step_deg"], poses_per_step=sc["poses_per_step"],
                                tiling=sc["tiling"], grid_pad_A=sc["grid_pad_A"]),
                    ligands_per_s=sc["ligands_per_s"], atoms_per_s=sc["atoms_per_s"],
                    fallback_per_pose=sc["fallback_per_pose"], prep_s=sc["prep_s"], per_ligand=sc["per_ligand"],
                    continuous=sc["continuous"], roofline=sc["roofline"])
        cpu_name, cpu_first = "screen", 0
    else:
        head = large_headline(gd, torch, np, args)
        log("large headline:", json.dumps(head))
        if not args.no_screen:
            head["screen"] = screen_leg(gd, torch, np, args, args.screen_steps, 1, args.n_ligands)
        cpu_name, cpu_first = "large", 0
    if args.stream_chunks > 0 and args.workload == "large":
        head["stream"] = large_leg(gd, torch, args.stream_chunks, head["config"]["tiling"])
        log("stream:", head["stream"])
    if not args.no_refine and args.refine_ligands > 0:
        head["refine"] = refine_leg(gd, torch, np, args.refine_ligands, l2)
        log("refinement:", head["refine"])
    head["l2_gather_peak"] = l2
    rf = head["roofline"]
    if rf.get("gather_GBps"):
        rf["gather_frac_of_l2_peak"] = rf["gather_GBps"] / l2["u16_GBps"]
    cpu = None
    if pool is not None:
        cpu = cpu_baseline(pool, workers, cpu_name, cpu_first, args.cpu_single, args.cpu_per_worker)
        pool.close()
        pool.join()
        log("cpu baseline:", cpu)
    line = {
        "metric": metric,
        "value": head.pop("value"),
        "unit": "poses/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": head.pop("config"),
    }
    line.update(head)
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
