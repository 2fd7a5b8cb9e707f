"""GPU parity of the density-surrogate refinement against the FP64 oracle.

Bar: density nodes within FP32 rounding of the FP64 definition; surrogate
values within 1e-4 and every gradient component within 1e-3 of its
parameter group's norm (translation, quaternion, torsions) against the
oracle's analytic gradient at the same parameters; 50-step trajectories
within 1e-3 A (RMSD) of the FP64 oracle's; the refined pose is re-scored with
the exact score, which must match the oracle's score of the returned FP32
pose bit for bit, and the acceptance rule is checked pose by pose.

The trilinear density's gradient jumps across lattice faces, and the ascent
map can amplify rounding-size differences.  The gradient check excludes only
poses whose FP32 and FP64 positions may sit in different trilinear cells, i.e.
(as decided on the oracle's FP64 positions) an atom within the FP32
coordinate bound (1e-4 A) of a face of the density lattice.  A trajectory may
part from the FP64 one only for a reason certified on the oracle where the
paths first separate: a face crossing, or the map's own sensitivity (oracle
runs of as many steps from inputs moved by a few FP32 ulps part as far).
Excluded cases are counted and printed.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import configs
from tests import gpuutil
from tests.gpuutil import gpu

SIG, CUTS, BH = 0.6, 4.0, 0.375


@pytest.fixture(scope="module")
def g():
    return gpuutil.gd()


@pytest.fixture(scope="module")
def setup(g):
    import torch
    w = configs.REFINE
    pts = w.pocket_points()
    P = g.Pocket(pts, 0.5, 12.0, blur_sigma=SIG, blur_h=BH, blur_cutoff_sigmas=CUTS, blur_pad=8.0)
    O = oracle.OraclePocket(pts, 0.5)
    B = oracle.OracleBlur(O, SIG, CUTS, BH)
    # a ragged sample that includes ligands of more than 64 atoms (two atoms
    # per lane) with 12 or more rotatable bonds (deep torsion trees)
    pool = w.ligands(0, 200)
    ligs = pool.subset(list(range(8)) + [37, 39, 85, 128])
    # docked poses as refinement inputs: top-4 of 64 orientations
    q = synth.quaternions(w.quat_seed, 64)
    b = g.Batch(P, ligs, q, hp=w.hp, top_k=4)
    res = b.dock(1).host()
    pose_lig, rows = [], []
    for i in range(ligs.n):
        l = ligs.n_atoms(i)
        for k in range(4):
            pose_lig.append(i)
            rows.append(res["xyz"][i, k, :l].astype(np.float32))
    allx = np.concatenate(rows)
    dev = lambda a: torch.tensor(a.copy(), device="cuda")
    return dict(P=P, O=O, B=B, ligs=ligs, pose_lig=np.array(pose_lig), rows=rows,
                px=dev(allx[:, 0]), py=dev(allx[:, 1]), pz=dev(allx[:, 2]))


@gpu
def test_density_grid_matches_definition(g, setup):
    P, B = setup["P"], setup["B"]
    inf = P.info()
    rho = P.read_density()
    lo = np.array(inf["blur_lo"])
    nx, ny, nz = inf["blur_dim"]
    rng = np.random.default_rng(0)
    # nodes near the pocket carry weight; sample there and anywhere
    c = (np.array(setup["P"].xyz.mean(0)) / float(np.float32(BH))).astype(int) - lo
    idx = np.concatenate([c + rng.integers(-12, 13, (3000, 3)),
                          np.stack([rng.integers(0, nx, 500), rng.integers(0, ny, 500), rng.integers(0, nz, 500)], 1)])
    idx = idx[(idx >= 0).all(1) & (idx < [nx, ny, nz]).all(1)]
    for ix, iy, iz in idx:
        want = B.node(ix + lo[0], iy + lo[1], iz + lo[2])
        assert rho[iz, iy, ix] == np.float32(want)


FP32_XYZ = gpuutil.FP32_XYZ


def _face_dist(X):
    return gpuutil.face_dist(X, float(np.float32(BH)))


def _params(n, nrmax, seed):
    rng = np.random.default_rng(seed)
    t = rng.normal(0, 0.3, (n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[:, 0] += 3.0  # mostly small rotations
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    tau = rng.normal(0, 0.4, (n, nrmax))
    return t.astype(np.float32), q.astype(np.float32), tau.astype(np.float32)


@gpu
@pytest.mark.parametrize("pen", [{}, dict(clash_weight=0.25, clash_dist=4.5, clash_min_bonds=4)])
def test_surrogate_value_and_gradient(g, setup, pen):
    """pen: the clash-penalised surrogate (a wide bump distance puts many far
    pairs in the penalty band)."""
    import torch
    S = setup
    ligs, pl = S["ligs"], S["pose_lig"]
    n = len(pl)
    nrmax = max(ligs.n_rot(i) for i in range(ligs.n))
    t, q, tau = _params(n, nrmax, 1)
    T = lambda a: torch.tensor(a, device="cuda")
    F = g.surrogate_fwd(S["P"], ligs, pl, S["px"], S["py"], S["pz"], T(t), T(q), T(tau), **pen).cpu().numpy()
    dF = np.linspace(0.5, 1.5, n).astype(np.float32)
    dt, dq, dtau = (x.cpu().numpy() for x in
                    g.surrogate_bwd(S["P"], ligs, pl, S["px"], S["py"], S["pz"], T(t), T(q), T(tau), T(dF), **pen))
    excused = 0
    for p in range(n):
        lig = ligs.ligand(pl[p])
        nr = ligs.n_rot(pl[p])
        X0 = S["rows"][p].astype(np.float64)
        prm = np.concatenate([t[p], q[p], tau[p, :nr]]).astype(np.float64)
        Fo, go, Xo = S["B"].surrogate(lig, X0, prm, **pen)
        assert abs(F[p] - Fo) <= 1e-4 * max(abs(Fo), 1.0), (p, F[p], Fo)
        gg = np.concatenate([dt[p], dq[p], dtau[p, :nr]]) / dF[p]
        ok = True
        for sl in (slice(0, 3), slice(3, 7), slice(7, 7 + nr)):
            a, b = gg[sl], go[sl]
            if len(a) and np.max(np.abs(a - b)) > 1e-3 * max(np.linalg.norm(b), 1e-3):
                ok = False
        if not ok:
            # certified only if the FP32 and FP64 positions may lie in different trilinear cells
            assert _face_dist(Xo) < FP32_XYZ, (p, _face_dist(Xo))
            excused += 1
        assert np.all(dtau[p, nr:] == 0)
    print("surrogate gradient%s: %d of %d poses excused (an atom within %.0e A of a trilinear face)"
          % (" (penalised)" if pen else "", excused, n, FP32_XYZ))
    assert sum(ligs.n_atoms(i) > 64 and ligs.n_rot(i) >= 12 for i in set(pl.tolist())) >= 2


@gpu
def test_autograd_function(g, setup):
    import torch
    S = setup
    ligs, pl = S["ligs"], S["pose_lig"]
    n = len(pl)
    nrmax = max(ligs.n_rot(i) for i in range(ligs.n))
    t, q, tau = (torch.tensor(a, device="cuda", requires_grad=True) for a in _params(n, nrmax, 2))
    spec = (S["P"], ligs, pl, S["px"], S["py"], S["pz"])
    F = g.SurrogateScore.apply(t, q, tau, spec)
    F.sum().backward()
    dt, dq, dtau = g.surrogate_bwd(S["P"], ligs, pl, S["px"], S["py"], S["pz"], t.detach(), q.detach(), tau.detach(),
                                   torch.ones(n, device="cuda"))
    assert torch.equal(t.grad, dt) and torch.equal(q.grad, dq) and torch.equal(tau.grad, dtau)
    # the penalised surrogate through the same autograd function
    pen = dict(clash_weight=0.25, clash_dist=4.5, clash_min_bonds=4)
    for v in (t, q, tau):
        v.grad = None
    Fp = g.SurrogateScore.apply(t, q, tau, spec + (pen,))
    Fp.sum().backward()
    dt, dq, dtau = g.surrogate_bwd(S["P"], ligs, pl, S["px"], S["py"], S["pz"], t.detach(), q.detach(), tau.detach(),
                                   torch.ones(n, device="cuda"), **pen)
    assert torch.equal(t.grad, dt) and torch.equal(q.grad, dq) and torch.equal(tau.grad, dtau)
    assert bool((Fp <= F).all())  # the penalty only subtracts


def _gpu_iterates(g, S, steps, cw):
    """The GPU's iterate after every step count 1..steps (one call each)."""
    ligs, pl = S["ligs"], S["pose_lig"]
    out = []
    for k in range(1, steps + 1):
        px, py, pz = S["px"].clone(), S["py"].clone(), S["pz"].clone()
        r = g.refine(S["P"], ligs, pl, px, py, pz, steps=k, want_iterate=True, clash_weight=cw)
        out.append(np.stack([v.cpu().numpy() for v in r["iterate"]], 1))
    return out


@gpu
@pytest.mark.parametrize("cw", [0.0, 10.0, 1000.0])
def test_refine_rescoring_and_acceptance(g, setup, cw):
    """cw > 0: the clash-penalised surrogate, against the oracle's penalised
    ascent.  Every 50-step trajectory must stay within 1e-3 A (RMSD) of the
    FP64 one unless the paths part at a certified face crossing."""
    import torch
    S = setup
    ligs, pl = S["ligs"], S["pose_lig"]
    px, py, pz = S["px"].clone(), S["py"].clone(), S["pz"].clone()
    steps = 50
    out = g.refine(S["P"], ligs, pl, px, py, pz, steps=steps, want_iterate=True, clash_weight=cw)
    F, Sg, cg, acc = (out[k].cpu().numpy() for k in ("F", "S", "clash", "accepted"))
    X = np.stack([px.cpu().numpy(), py.cpu().numpy(), pz.cpu().numpy()], 1)
    It = np.stack([v.cpu().numpy() for v in out["iterate"]], 1)
    off = 0
    rms, fdiff, split = [], [], []
    for p in range(len(pl)):
        lig = ligs.ligand(pl[p])
        l = len(lig["x"])
        Xp, X0, Xi = X[off:off + l], S["rows"][p], It[off:off + l]
        s_in, c_in = oracle.score_poses(S["O"], lig, X0[None, :, 0], X0[None, :, 1], X0[None, :, 2])
        s_out, c_out = oracle.score_poses(S["O"], lig, Xp[None, :, 0], Xp[None, :, 1], Xp[None, :, 2])
        assert Sg[p] == s_out[0] and cg[p] == c_out[0]
        if acc[p]:
            assert not c_out[0] and s_out[0] < s_in[0]
        else:
            assert np.array_equal(Xp, X0) and Sg[p] == s_in[0]
        # trajectory against the FP64 oracle
        prm, Xo, Fo = S["B"].refine(lig, X0.astype(np.float64), steps=steps, clash_weight=cw)
        r = np.sqrt(((Xi - Xo) ** 2).sum(1).mean())
        rms.append(r)
        if r > 1e-3:
            split.append((p, off, l))
        else:
            fdiff.append(abs(F[p] - Fo) / max(abs(Fo), 1.0))
        if acc[p]:
            assert np.array_equal(Xp, Xi)
        off += l
    certified = []
    if split:
        its = _gpu_iterates(g, S, steps, cw)
        for p, o, l in split:
            why, info = gpuutil.certify_split(S["B"], ligs.ligand(pl[p]), S["rows"][p],
                                              lambda k: its[k - 1][o:o + l], steps, float(np.float32(BH)),
                                              clash_weight=cw)
            assert why, ("uncertified split", p, info)
            certified.append((p, why, info["step"]))
    rms = np.array(rms)
    print("refine (clash weight %g): accepted %d/%d; final-iterate RMSD vs the FP64 trajectory: median %.2e, "
          "max over unsplit %.2e; %d certified split(s) (pose, reason, step): %s; median |dF|/F %.2e"
          % (cw, acc.sum(), len(pl), np.median(rms), max([v for v in rms if v <= 1e-3] or [0.0]), len(certified),
             certified, np.median(fdiff)))
    assert acc.sum() > 0
    assert np.median(fdiff) < 1e-4


@gpu
def test_refine_penalty_single_step(g, setup):
    """One ascent step on the heavily penalised surrogate: every pose's iterate
    within 1e-4 A of the FP64 oracle's (no room for paths to part)."""
    S = setup
    ligs, pl = S["ligs"], S["pose_lig"]
    px, py, pz = S["px"].clone(), S["py"].clone(), S["pz"].clone()
    out = g.refine(S["P"], ligs, pl, px, py, pz, steps=1, want_iterate=True, clash_weight=1000.0)
    It = np.stack([v.cpu().numpy() for v in out["iterate"]], 1)
    off = 0
    worst = 0.0
    for p in range(len(pl)):
        lig = ligs.ligand(pl[p])
        l = len(lig["x"])
        _, Xo, _ = S["B"].refine(lig, S["rows"][p].astype(np.float64), steps=1, clash_weight=1000.0)
        worst = max(worst, float(np.sqrt(((It[off:off + l] - Xo) ** 2).sum(1).mean())))
        off += l
    assert worst <= 1e-4, worst


@gpu
def test_surrogate_gradient_far_from_origin(g, setup):
    """The same pocket and poses moved by (100, -80, 60) A: lever arms are
    taken from the rotation centre, so the torque and torsion gradients keep
    the same bar (every component within 1e-3 of its group norm, faces
    excused as above) although coordinates are ~140 A from the origin."""
    import torch
    S = setup
    shift = np.array([100.0, -80.0, 60.0], np.float32)
    pts = configs.REFINE.pocket_points().astype(np.float32) + shift
    P = g.Pocket(pts, 0.5, 12.0, blur_sigma=SIG, blur_h=BH, blur_cutoff_sigmas=CUTS, blur_pad=8.0)
    B = oracle.OracleBlur(oracle.OraclePocket(pts, 0.5), SIG, CUTS, BH)
    ligs, pl = S["ligs"], S["pose_lig"]
    rows = [(r + shift).astype(np.float32) for r in S["rows"]]
    allx = np.concatenate(rows)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda")
    px, py, pz = dev(allx[:, 0]), dev(allx[:, 1]), dev(allx[:, 2])
    n = len(pl)
    nrmax = max(ligs.n_rot(i) for i in range(ligs.n))
    t, q, tau = _params(n, nrmax, 3)
    T = lambda a: torch.tensor(a, device="cuda")
    dF = np.ones(n, np.float32)
    dt, dq, dtau = (x.cpu().numpy() for x in g.surrogate_bwd(P, ligs, pl, px, py, pz, T(t), T(q), T(tau), T(dF)))
    excused, worst = 0, 0.0
    for p in range(n):
        lig = ligs.ligand(pl[p])
        nr = ligs.n_rot(pl[p])
        prm = np.concatenate([t[p], q[p], tau[p, :nr]]).astype(np.float64)
        Fo, go, Xo = B.surrogate(lig, rows[p].astype(np.float64), prm)
        gg = np.concatenate([dt[p], dq[p], dtau[p, :nr]])
        rel = max(np.max(np.abs(gg[sl] - go[sl])) / max(np.linalg.norm(go[sl]), 1e-3)
                  for sl in (slice(0, 3), slice(3, 7), slice(7, 7 + nr)) if sl.stop > sl.start)
        if rel > 1e-3:
            assert _face_dist(Xo) < FP32_XYZ, (p, rel, _face_dist(Xo))
            excused += 1
        else:
            worst = max(worst, rel)
    print("surrogate gradient 140 A from the origin: worst relative component error %.2e, %d of %d poses excused"
          % (worst, excused, n))
    assert excused <= n // 4
