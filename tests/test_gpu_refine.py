"""GPU parity of the density-surrogate refinement against the FP64 oracle.

Bar: density nodes within FP32 rounding of the FP64 definition; surrogate
values within 1e-4 and gradients within 1e-3 (relative, per parameter
group) of the oracle's analytic gradient at the same parameters; the
refined pose is re-scored with the exact score, which must match the oracle's
score of the returned FP32 pose bit for bit, and the acceptance rule is
checked pose by pose.
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
    ligs = w.ligands(0, 12)
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
    bad = 0
    for p in range(n):
        lig = ligs.ligand(pl[p])
        nr = ligs.n_rot(pl[p])
        X0 = S["rows"][p].astype(np.float64)
        prm = np.concatenate([t[p], q[p], tau[p, :nr]]).astype(np.float64)
        Fo, go, _ = S["B"].surrogate(lig, X0, prm, **pen)
        assert abs(F[p] - Fo) <= 1e-4 * max(abs(Fo), 1.0), (p, F[p], Fo)
        gg = np.concatenate([dt[p], dq[p], dtau[p, :nr]]) / dF[p]
        for sl in (slice(0, 3), slice(3, 7), slice(7, 7 + nr)):
            a, b = gg[sl], go[sl]
            if len(a) and np.linalg.norm(a - b) > 1e-3 * max(np.linalg.norm(b), 1e-3):
                bad += 1
        assert np.all(dtau[p, nr:] == 0)
    # FP32 vs FP64 positions can straddle a trilinear face, where the gradient jumps
    assert bad <= max(1, n // 50), bad


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


@gpu
@pytest.mark.parametrize("cw,split_ok", [(0.0, 0.9), (10.0, 0.9), (1000.0, 0.8)])
def test_refine_rescoring_and_acceptance(g, setup, cw, split_ok):
    """cw > 0: the clash-penalised surrogate, against the oracle's penalised
    ascent.  A heavy penalty makes clipped ascent steps flip more often between
    FP32 and FP64 paths, so at weight 1,000 up to a fifth of the 50-step
    trajectories may part ways (the single-step test below bounds every pose)."""
    import torch
    S = setup
    ligs, pl = S["ligs"], S["pose_lig"]
    px, py, pz = S["px"].clone(), S["py"].clone(), S["pz"].clone()
    out = g.refine(S["P"], ligs, pl, px, py, pz, steps=50, want_iterate=True, clash_weight=cw)
    F, Sg, cg, acc = (out[k].cpu().numpy() for k in ("F", "S", "clash", "accepted"))
    X = np.stack([px.cpu().numpy(), py.cpu().numpy(), pz.cpu().numpy()], 1)
    It = np.stack([v.cpu().numpy() for v in out["iterate"]], 1)
    off = 0
    rms, fdiff = [], []
    for p in range(len(pl)):
        lig = ligs.ligand(pl[p])
        l = len(lig["x"])
        Xp, X0, Xi = X[off:off + l], S["rows"][p], It[off:off + l]
        off += l
        s_in, c_in = oracle.score_poses(S["O"], lig, X0[None, :, 0], X0[None, :, 1], X0[None, :, 2])
        s_out, c_out = oracle.score_poses(S["O"], lig, Xp[None, :, 0], Xp[None, :, 1], Xp[None, :, 2])
        assert Sg[p] == s_out[0] and cg[p] == c_out[0]
        if acc[p]:
            assert not c_out[0] and s_out[0] < s_in[0]
        else:
            assert np.array_equal(Xp, X0) and Sg[p] == s_in[0]
        # trajectory against the FP64 oracle (FP32 arithmetic; kinks can split paths)
        prm, Xo, Fo = S["B"].refine(lig, X0.astype(np.float64), steps=50, clash_weight=cw)
        fdiff.append(abs(F[p] - Fo) / max(abs(Fo), 1.0))
        rms.append(np.sqrt(((Xi - Xo) ** 2).sum(1).mean()))
        if acc[p]:
            assert np.array_equal(Xp, Xi)
    rms = np.array(rms)
    print("refine (clash weight %g): accepted %d/%d; final-iterate RMSD vs the FP64 trajectory: median %.2e, "
          "fraction <= 1e-3 A %.2f, max %.2e; median |dF|/F %.2e"
          % (cw, acc.sum(), len(pl), np.median(rms), np.mean(rms <= 1e-3), rms.max(), np.median(fdiff)))
    assert acc.sum() > 0
    assert np.median(fdiff) < 1e-4
    # the trilinear gradient jumps at lattice faces: an FP32 and an FP64 path
    # that straddle a face part ways, so a few trajectories are allowed to split
    assert np.median(rms) < 1e-5
    assert np.mean(rms <= 1e-3) >= split_ok


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
