"""Parity of the HIP chain step with the FP64 oracle on identical seeded inputs.

Tolerances follow from FP32 arithmetic on the device against FP64 on the
host.  Every value of a smooth quantity (f, log p, p, f/p, the holding
weight, each score coordinate, x') is held to 1e-4 relative, except where
the oracle itself shows that the sample is ill-conditioned for FP32: its
value moves by more than 1e-4 / (16 L) when every coordinate of the point is
perturbed by one FP32 ulp (`_sens`).  Such a sample may err by up to 16 L
times that sensitivity (the roundings along its path, `_cond`), and by no
more.  Decisions (kill, pixel) are
identical except where the FP64 value lies within the FP32 rounding band of
the threshold.  Paths whose discrete choices (hit triangle, light,
visibility, lobe) differ between the two precisions are excluded from value
checks, and their share is bounded.
"""
import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2605_08916_amd import dr, inputs  # noqa: E402

LUMW = np.array([0.2126, 0.7152, 0.0722])


def say(*a):
    """Progress and error statistics: to stderr, and appended to the file
    named by DR_PARITY_LOG when that is set."""
    print(*a, file=sys.stderr, flush=True)
    path = os.environ.get("DR_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            print(*a, file=f)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dr.lib()
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def scenes():
    out = {}
    out["tiny"] = inputs.cornell_tiny()
    out["spheres_small"] = inputs.procedural_spheres(n_spheres=3, subdiv=3, width=128, height=128)
    out["specular"] = inputs.specular_box()
    return out


def _rel(a, b, floor):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


# First-order FP32 error bound used by every parity check: the device's path
# evaluation rounds at about 16 stages per vertex (ray direction, hit point,
# light vector, r^2 and its root, cosines, BSDF value, throughput), over the
# camera ray and at most L - 1 vertices, and each rounding moves the result
# by about what a one-ulp perturbation of the point does (`_sens`); so a value
# may err by 16 L times that sensitivity (and the score additionally by 16 L
# unit roundoffs of its condition measure, `_score_within`).
def _cond(L):
    return 16.0 * L


TOL = 1e-4
ULP = 2.0 ** -24


def _vec_rel(a, b, floor):
    """Relative error of each row vector: max |a - b| over the row / max(max |b|, floor)."""
    return np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), floor)


def _coord_rel(g, go):
    """Relative error of each score coordinate, against its own size or 1e-2
    of the sample's largest coordinate, whichever is larger.  Quantities the
    adjoint shares between coordinates (the path's throughput, distances and
    cosines, computed once) carry the FP32 rounding of the largest terms into
    every coordinate: a few ulps of the largest coordinate whatever a
    coordinate's own size (1e-4 of the floor is 1e-6 of the largest, 17
    ulps)."""
    fl = np.maximum(1e-2 * np.abs(go).max(axis=1, keepdims=True), 1e-6)
    return np.abs(g - go) / np.maximum(np.abs(go), fl)


def _fop(f, p):
    return np.where(p[:, None] > 0, f / np.where(p > 0, p, 1.0)[:, None], 0.0)


def _round_allow(L):
    """Multiple of the unit roundoff times the score's condition measure that
    the reverse sweep may err by (the roundings along a dependency path from
    a coordinate to p, as in `_cond`)."""
    return _cond(L) * 2.0 ** -24


def _sens(O, L, u, K=6, seed=12345):
    """Conditioning of each point for FP32: the largest relative change of the
    oracle's f, p, f/p and score (max over coordinates) when every coordinate
    of the point moves by one FP32 ulp at 1 (2^-24, random signs), over K
    draws that keep the discrete path; measured with the same error norms the
    tests use.  Returns (sensitivities, oracle values at u)."""
    u = np.ascontiguousarray(u, np.float64)
    f0, p0, g0, r0 = O.path_eval(L, u)
    fscale = max(1e-6, float(np.abs(f0).mean()))
    pscale = max(1e-6, float(p0.mean()))
    fop0 = _fop(f0, p0)
    n = u.shape[0]
    s = {k: np.zeros(n) for k in ("f", "p", "fop", "g")}
    rng = np.random.default_rng(seed)
    for _ in range(K):
        u1 = np.clip(u + rng.choice([-1.0, 1.0], size=u.shape) * ULP, 0.0, 1.0 - ULP)
        f1, p1, g1, r1 = O.path_eval(L, u1)
        same = np.all(r1 == r0, axis=1)
        s["f"] = np.maximum(s["f"], np.where(same, _vec_rel(f1, f0, 1e-3 * fscale), 0.0))
        s["p"] = np.maximum(s["p"], np.where(same, np.abs(p1 - p0) / np.maximum(p0, 1e-3 * pscale), 0.0))
        s["fop"] = np.maximum(s["fop"], np.where(same, (np.abs(_fop(f1, p1) - fop0) /
                                                         np.maximum(1.0, np.abs(fop0))).max(axis=1), 0.0))
        s["g"] = np.maximum(s["g"], np.where(same, _coord_rel(g1, g0).max(axis=1), 0.0))
    # the score's condition measure per coordinate (terms' magnitudes / (p + eps))
    s["kappa"] = O.path_cond(L, u)
    return s, (f0, p0, g0, r0)


def _score_within(name, g, go, sens, L):
    """Every score coordinate within TOL of its size (floored, `_coord_rel`),
    or within _cond(L) times the point's sensitivity; plus the reverse sweep's
    rounding, `_round_allow(L)` times the coordinate's condition measure
    (where terms cancel, FP32 keeps fewer digits of the sum)."""
    fl = np.maximum(1e-2 * np.abs(go).max(axis=1, keepdims=True), 1e-6)
    scale = np.maximum(np.abs(go), fl)
    err = np.abs(g - go) / scale
    allow = np.maximum(TOL, _cond(L) * sens["g"])[:, None] + _round_allow(L) * sens["kappa"] / scale
    bad = ~(err <= allow)
    beyond = err > TOL
    say(f"  {name}: max err {err.max():.2e}, beyond {TOL:g} {int(beyond.sum())} (within the conditioning "
        f"allowance: {int((beyond & ~bad).sum())}), failing {int(bad.sum())}")
    if bad.any():
        i = np.argsort(-(err - allow).ravel())[:5]
        r, c = np.unravel_index(i, err.shape)
        detail = [f"(sample {a}, coord {b}: oracle {go[a, b]:.6e} device {g[a, b]:.6e} max|score| "
                  f"{np.abs(go[a]).max():.3e} kappa {sens['kappa'][a, b]:.3e} sens {sens['g'][a]:.2e})"
                  for a, b in zip(r, c)]
        raise AssertionError(f"{name}: {int(bad.sum())} coordinates beyond the allowance; worst err "
                             f"{err.ravel()[i]} allowance {allow.ravel()[i]} " + " ".join(detail))


def _within(name, err, sens, L):
    """Every sample within TOL, or within _cond(L) times its sensitivity."""
    err, sens = np.asarray(err, np.float64), np.asarray(sens, np.float64)
    if err.size == 0:
        return
    allow = np.maximum(TOL, _cond(L) * sens)
    bad = ~(err <= allow)
    cond = (err > TOL) & ~bad
    say(f"  {name}: max err {err.max():.2e}, beyond {TOL:g} {int((err > TOL).sum())} "
        f"(within the conditioning allowance: {int(cond.sum())}), failing {int(bad.sum())}")
    if bad.any():
        i = np.argsort(-(err - allow).ravel())[:5]
        raise AssertionError(f"{name}: {int(bad.sum())} beyond the allowance; worst err {err.ravel()[i]} "
                             f"allowance {allow.ravel()[i]}")


def _eval_both(orc, sc, L, n, seed):
    d = 4 * (L - 1)
    u = inputs.random_points(d, n, seed)
    S = dr.Scene(sc)
    ut = torch.from_numpy(u).cuda()
    f, logp, g, rec = S.eval_logp_grad(L, ut, rec=True)
    torch.cuda.synchronize()
    f, logp, g = f.cpu().numpy(), logp.cpu().numpy(), g.cpu().numpy()
    rec = rec.cpu().numpy().view(np.uint32)
    O = orc.Scene(sc)
    fo, po, go, ro = O.path_eval(L, u.astype(np.float64))
    # oracle record -> (prim << 8 | light << 1 | contrib) like the device's
    V = L - 1
    rec_o = np.full((n, V), 0xFFFFFFFF, np.uint64)
    prim = ro[:, 0::2].astype(np.int64)
    nee = ro[:, 1::2].astype(np.uint64)
    has = prim.astype(np.int32) >= 0
    rec_o[has] = (prim[has].astype(np.uint64) << 8) | (nee[has] & 0xFF)
    match = np.all(rec_o.astype(np.uint32) == rec, axis=1)
    return u, (f, logp, g), (fo, po, go), match


def _check_eval(O, L, u, dev, match, name=""):
    """f, log(p + eps) and every score coordinate of the device evaluation
    against the oracle, per sample (conditioning allowance as in `_within`),
    on the samples whose discrete path matches."""
    f, logp, g = dev
    sens, (fo, po, go, _) = _sens(O, L, u)
    m = match
    fscale = max(1e-6, float(np.abs(fo).mean()))
    _within(f"{name}f", _vec_rel(f[m], fo[m], 1e-3 * fscale), sens["f"][m], L)
    pos = m & (po > 1e-3 * po.mean())
    # |d log p| = |dp| / p: the relative error of p
    _within(f"{name}log p", np.abs(logp[pos] - np.log(po[pos] + 1e-8)), sens["p"][pos], L)
    _score_within(f"{name}score", g[pos], go[pos], {k: v[pos] for k, v in sens.items()}, L)
    # p == 0 paths have a zero score on both sides
    zero = m & (po == 0)
    assert np.all(g[zero] == 0)


@pytest.mark.parametrize("which,L,n", [("tiny", 4, 4000), ("spheres_small", 8, 3000), ("specular", 8, 4000)])
def test_eval_matches_oracle(orc, scenes, which, L, n):
    say(f"[eval parity] scene={which} L={L} n={n}")
    u, dev, _, match = _eval_both(orc, scenes[which], L, n, seed=5)
    say(f"  path-signature match {match.mean():.5f}")
    assert match.mean() > 0.995
    _check_eval(orc.Scene(scenes[which]), L, u.astype(np.float64), dev, match)


def test_root_leaf_and_empty_child_slots(orc, scenes):
    """The empty room of the tiny scene (its 10 wall triangles and the 2 of
    its ceiling light) fits one leaf of 16: the root node then holds that
    leaf beside three empty slots (NaN boxes no ray passes).  Its evaluations
    match the oracle and, bit for bit, those of a tree of one-triangle
    leaves."""
    sc = dict(scenes["tiny"])
    keep = np.r_[0:10, 30:32]
    sc["indices"] = sc["indices"][keep].copy()
    sc["tri_material"] = sc["tri_material"][keep].copy()
    L, n = 4, 4000
    u, dev, _, match = _eval_both(orc, sc, L, n, seed=21)
    say(f"[root leaf] path-signature match {match.mean():.5f}")
    assert match.mean() > 0.995
    _check_eval(orc.Scene(sc), L, u.astype(np.float64), dev, match)
    ut = torch.from_numpy(u).cuda()
    outs = []
    for ml in (16, 1):
        S = dr.Scene(sc, max_leaf=ml)
        st = S.stats()
        say(f"  max_leaf={ml} {st}")
        if ml == 16:
            assert st["n_nodes"] == 1
        outs.append(S.eval_logp_grad(L, ut, grad=True, rec=True))
        torch.cuda.synchronize()
        S.close()
    for a, b in zip(*outs):
        assert torch.equal(a, b)


@pytest.mark.parametrize("which,L,n", [("tiny", 4, 3000), ("spheres_small", 8, 20000), ("specular", 8, 20000)])
def test_forward_only_eval_matches_eval_with_score(scenes, which, L, n):
    """Forward-only evaluation (the ray-refill evaluator) returns exactly the
    f, log p and path records of the evaluation that also runs the adjoint."""
    say(f"[eval forward-only vs with score] scene={which} L={L} n={n}")
    S = dr.Scene(scenes[which])
    g = torch.Generator().manual_seed(5)
    u = torch.rand((n, 4 * (L - 1)), generator=g).cuda()
    f0, lp0, _, r0 = S.eval_logp_grad(L, u, grad=False, rec=True)
    f1, lp1, g1, r1 = S.eval_logp_grad(L, u, grad=True, rec=True)
    torch.cuda.synchronize()
    assert torch.equal(f0, f1) and torch.equal(lp0, lp1) and torch.equal(r0, r1)
    assert torch.isfinite(g1).all()


def test_bvh_shape_does_not_change_results(scenes):
    """Closest hits are defined by the geometry (ties to the lower input
    index) and box tests are conservative, so trees built with different leaf
    sizes (leaf batches of 2 and 4 triangles) give bit-identical f, log p,
    scores and path records."""
    sc = scenes["spheres_small"]
    L, n = 8, 20000
    g = torch.Generator().manual_seed(9)
    u = torch.rand((n, 4 * (L - 1)), generator=g).cuda()
    ref = None
    for ml in (1, 2, 4, 8):
        S = dr.Scene(sc, max_leaf=ml)
        say(f"[bvh shape] max_leaf={ml} {S.stats()}")
        out = S.eval_logp_grad(L, u, grad=True, rec=True)
        torch.cuda.synchronize()
        if ref is None:
            ref = out
        else:
            for a, b in zip(ref, out):
                assert torch.equal(a, b)


def test_autograd_matches_finite_differences_and_oracle(orc, scenes):
    from paper_2605_08916_amd.autograd import LogContribution
    sc = scenes["spheres_small"]
    L, n, h = 8, 512, 1e-3
    d = 4 * (L - 1)
    say(f"[autograd] L={L} n={n} h={h}")
    S = dr.Scene(sc)
    u = torch.from_numpy(inputs.random_points(d, n, 9)).cuda().requires_grad_(True)
    lp = LogContribution.apply(S, L, u)
    w = torch.randn(n, device="cuda")
    (lp * w).sum().backward()
    grad = (u.grad / w[:, None]).detach().cpu().numpy()
    _, _, g_eval, rec0 = S.eval_logp_grad(L, u.detach(), rec=True)
    assert np.allclose(grad, g_eval.cpu().numpy(), rtol=1e-5, atol=1e-6)
    O = orc.Scene(sc)
    _, po, go, _ = O.path_eval(L, u.detach().cpu().numpy().astype(np.float64))
    # central differences on the device in FP32 (h = 1e-3) where the path keeps its choices
    un = u.detach()
    checked = bad = 0
    rec0 = rec0.cpu().numpy()
    lp0 = lp.detach().cpu().numpy()
    for i in range(d):
        e = torch.zeros_like(un)
        e[:, i] = h
        _, lpp, _, rp = S.eval_logp_grad(L, (un + e).clamp(0, 1 - 2 ** -24), grad=False, rec=True)
        _, lpm, _, rm = S.eval_logp_grad(L, (un - e).clamp(0, 1 - 2 ** -24), grad=False, rec=True)
        same = np.all(rp.cpu().numpy() == rec0, 1) & np.all(rm.cpu().numpy() == rec0, 1)
        same &= (po > 1e-2 * po.mean()) & (un[:, i].cpu().numpy() > h) & (un[:, i].cpu().numpy() < 1 - h)
        fd = (lpp - lpm).cpu().numpy() / (2 * h)
        # FD truncation error is O(h^2 f'''); allow 5% + FP32 noise of log p / h
        tol = 0.05 * np.abs(go[:, i]) + 0.05 * np.abs(fd) + 2e-4 / h * np.maximum(1.0, np.abs(lp0))
        ok = np.abs(fd - grad[:, i]) <= tol
        checked += same.sum()
        bad += (same & ~ok).sum()
    say(f"  FD checked {checked}, outside tolerance {bad}")
    assert checked > 2000
    assert bad <= 0.01 * checked


def _onestep(orc, sc, L, N, mode, seed, k0, gamma=0.5, sigma=None, sample=None, state_seed=3, rao_blackwell=1):
    """Write one generated state to the device and the oracle, take one step,
    return both states (device state restricted to `sample`)."""
    d = 4 * (L - 1)
    st = inputs.random_state(d, N, seed=state_seed, killed_frac=0.15, score_scale=40.0)
    S = dr.Scene(sc)
    sig_t = None if sigma is None else torch.from_numpy(sigma).cuda()
    ch = dr.Chains(S, N, L, seed, k0=k0, gamma=gamma, mode=mode, sigma=sig_t, rao_blackwell=rao_blackwell)
    ch.set_record(True)
    step0 = (7 << 32) + 11
    # the frame buffer starts empty, so after the step it holds that step's splats only
    npx = int(sc["width"]) * int(sc["height"])
    ch.write_state(x=st["x"], score=st["score"], killed=st["killed"], accum=np.zeros((3, npx), np.float32),
                   step=step0, k0=k0)
    ch.step(1)
    gs = ch.read_state()
    idx = np.arange(N) if sample is None else np.asarray(sample)
    O = orc.Scene(sc)
    oc = orc.Chains.scene(O, L, len(idx), seed=seed, k0=k0, gamma=gamma,
                          sigma=None if sigma is None else sigma[:, idx], rao_blackwell=rao_blackwell)
    oc.set_ids(idx.astype(np.uint32))
    score_in = st["score"][:, idx]
    aux = {}
    if mode == dr.DR_MODE_PLAIN:
        # the plain form recomputes the score of the current state at the start
        # of its step (Alg. 5.1 starts from it): give the oracle its own score
        # at x, and keep that score's FP32 conditioning for the x' check
        sens_x, (_, _, sc_o, _) = _sens(O, L, st["x"][:, idx].T.astype(np.float64))
        score_in = sc_o.T.astype(np.float32)
        aux = {"score_x": sc_o, "score_x_sens": sens_x["g"], "score_x_kappa": sens_x["kappa"].max(axis=1)}
    oc.set_state(st["x"][:, idx], score_in, st["killed"][idx], step0, k0=k0)
    oc.step(1, nthreads=16)
    os_ = oc.state()
    os_.update(aux)
    os_["accum"] = oc.accum()["accum"].T  # 3 x W*H, sum of w f/p
    gsel = {k: (v[..., idx] if isinstance(v, np.ndarray) and v.shape[-1] == N and k != "accum" else v)
            for k, v in gs.items()}
    return st, gsel, os_, idx, step0


def _compare_step(orc, sc, L, st, gs, os_, idx, seed, step0, k0, dt=1e-5, eps=1e-8, check_score=True,
                  plain=False, stddev=5e-3, gamma=0.5):
    W, H = sc["width"], sc["height"]
    prim = os_["rec"][0::2].astype(np.int64)
    nee = os_["rec"][1::2].astype(np.uint64)
    rec_o = np.where(prim.astype(np.int32) >= 0, (prim.astype(np.uint64) << 8) | (nee & 0xFF), 0xFFFFFFFF)
    match = np.all(rec_o.astype(np.uint32) == gs["path_rec"], axis=0)
    say(f"  path-signature match {match.mean():.5f}")
    assert match.mean() > 0.99
    # FP32 conditioning of the new state (the oracle at its own x')
    O = orc.Scene(sc)
    sens, _ = _sens(O, L, os_["x"].T)
    # x' on the torus: error relative to the step
    dx = gs["x"].astype(np.float64) - os_["x"]
    dx = np.abs(dx - np.round(dx))
    step = np.abs(os_["x"] - st["x"][:, idx].astype(np.float64))
    step = np.minimum(step, 1 - step)
    xerr = dx / np.maximum(step, 5e-3)
    say(f"  x' step-relative err max {xerr.max():.2e}")
    if plain:
        # the plain form computes its own FP32 score at x; its error moves x'
        # by the drift's factor (stddev^2/2 + gamma~) times the score error,
        # which the conditioning of that score bounds
        gx = np.abs(os_["score_x"]).max(axis=1)
        allow_dx = (stddev ** 2 / 2 + dt * gamma / 2) * (_cond(L) * os_["score_x_sens"] * gx +
                                                         _round_allow(L) * os_["score_x_kappa"])
        live = st["killed"][idx] == 0
        allow = TOL + np.where(live, allow_dx, 0.0)[None, :] / np.maximum(step, 5e-3)
        bad = xerr > allow
        say(f"  x' beyond {TOL:g}: {int((xerr > TOL).sum())}, beyond the score-conditioning allowance: "
            f"{int(bad.sum())}")
        assert not bad.any(), (xerr[bad][:5], allow[bad][:5])
    else:
        assert xerr.max() < TOL
    # pixel: identical except within 1e-3 pixel of an edge
    fx = os_["x"][0] * W
    fy = os_["x"][1] * H
    near = (np.abs(fx - np.round(fx)) < 1e-3) | (np.abs(fy - np.round(fy)) < 1e-3)
    pix_bad = (gs["pixel"] != os_["pixel"]) & ~near
    assert pix_bad.sum() == 0, pix_bad.sum()
    # kill decisions: identical except inside the band set by the p difference
    Ea = np.array([-math.log(1 - orc.uniform(seed, int(c), step0, orc.TAG_HOLD, 0)) for c in idx])
    Eb = np.array([-math.log(1 - orc.uniform(seed, int(c), step0, orc.TAG_HOLD, 1)) for c in idx])
    k = k0 / (os_["p"] + eps)
    gap = np.abs(k * dt * Ea - Eb) / np.maximum(Eb, 1e-30)
    prel = np.abs(gs["p"] - os_["p"]) / np.maximum(os_["p"], 1e-30)
    band = 1e-6 + 4 * np.where(match, prel, np.inf)
    kill_bad = (gs["killed"] != os_["killed"]) & (gap > band)
    say(f"  kill agreement {(gs['killed'] == os_['killed']).mean():.5f}, outside band {kill_bad.sum()}")
    assert kill_bad.sum() == 0
    m = match
    pscale = max(1e-6, float(os_["p"].mean()))
    _within("p", _rel(gs["p"][m], os_["p"][m], 1e-3 * pscale), sens["p"][m], L)
    fop_err = (np.abs(gs["f_over_p"][:, m] - os_["f_over_p"][:, m]) / np.maximum(1, np.abs(os_["f_over_p"][:, m]))).max(0)
    _within("f/p", fop_err, sens["fop"][m], L)
    # w = dt/(1 + k dt) with k = k0/(p + eps): its error follows p's
    praw = np.abs(gs["p"][m] - os_["p"][m]) / np.maximum(os_["p"][m] + eps, 1e-30)
    werr = _rel(gs["weight"][m], os_["w"][m], 1e-30)
    assert np.all(werr <= 2 * praw + 1e-5), np.max(werr - 2 * praw)
    if len(idx) == gs["x"].shape[1] and np.array_equal(idx, np.arange(len(idx))):
        _check_accum(gs, os_, sens, match, dt, L)
    if check_score:
        live = m & (os_["killed"] == 0) & (gs["killed"] == 0) & (os_["p"] > 1e-3 * pscale)
        if not live.any():  # e.g. a single chain that was killed: no score to compare
            return
        go, gg = os_["score"][:, live].T, gs["score"][:, live].T.astype(np.float64)
        _score_within("score", gg, go, {k: v[live] for k, v in sens.items()}, L)


def _check_accum(gs, os_, sens, match, dt, L):
    """The frame buffer after one step from an empty one, pixel by pixel: the
    device's sum of (w/dt) f/p times dt against the oracle's sum of w f/p.
    Each chain's splat may err by its allowances for f/p and for the weight
    (twice p's), the atomics' summation order adds a rounding of the pixel's
    sum per contribution; pixels that a chain with a different discrete path
    or pixel reaches are left out."""
    dev = gs["accum"].astype(np.float64) * dt
    orc_acc = os_["accum"]
    npx = orc_acc.shape[1]
    pix = os_["pixel"].astype(np.int64)
    live = os_["p"] > 0
    fop = np.abs(os_["f_over_p"])  # 3 x n
    w = os_["w"]
    a_fop = np.maximum(TOL, _cond(L) * sens["fop"])
    a_w = 2 * np.maximum(TOL, _cond(L) * sens["p"])
    err_c = w * (a_fop * np.maximum(1.0, fop.max(axis=0)) + a_w * fop.max(axis=0) + 1e-6)
    bound = np.bincount(pix[live], weights=err_c[live], minlength=npx)
    count = np.bincount(pix[live], minlength=npx)
    off = ~match | (gs["pixel"] != os_["pixel"])
    skip = np.zeros(npx, bool)
    skip[pix[off & live]] = True
    skip[gs["pixel"][off].astype(np.int64)] = True
    bound = bound[None, :] + count[None, :] * 2.0 ** -22 * orc_acc
    diff = np.abs(dev - orc_acc)
    bad = (diff > bound) & ~skip[None, :]
    say(f"  accum: {int(live.sum())} splats over {int((count > 0).sum())} pixels, left out {int(skip.sum())}, "
        f"max rel {float((diff / np.maximum(orc_acc, 1e-30))[:, ~skip].max()):.2e}, failing {int(bad.sum())}")
    assert skip.mean() < 0.01
    assert not bad.any(), (diff[bad][:5], bound[bad][:5])


@pytest.mark.parametrize("mode", [dr.DR_MODE_FUSED, dr.DR_MODE_PLAIN])
@pytest.mark.parametrize("which,L,N", [("tiny", 4, 1000), ("spheres_small", 8, 1500), ("specular", 8, 1500),
                                       # degenerate shapes: one chain, the shortest path (d = 4), ragged counts
                                       ("tiny", 2, 1), ("tiny", 2, 129), ("spheres_small", 3, 77)])
def test_one_step_matches_oracle(orc, scenes, which, L, N, mode):
    say(f"[one step] scene={which} L={L} N={N} mode={mode}")
    k0 = 300.0
    st, gs, os_, idx, step0 = _onestep(orc, scenes[which], L, N, mode, seed=21, k0=k0)
    # the plain form computes the score at the start of the next step
    _compare_step(orc, scenes[which], L, st, gs, os_, idx, 21, step0, k0, check_score=(mode == dr.DR_MODE_FUSED),
                  plain=(mode == dr.DR_MODE_PLAIN))


@pytest.mark.parametrize("mode", [dr.DR_MODE_FUSED, dr.DR_MODE_PLAIN])
def test_one_step_sampled_holding_weight(orc, scenes, mode):
    """The literal Alg. 4.1 weight (rao_blackwell = 0: the sampled holding
    time min(dt E_a, E_b / k)) against the oracle's, with the same clocks."""
    say(f"[one step, sampled weight] scene=specular L=8 N=1500 mode={mode}")
    k0 = 300.0
    st, gs, os_, idx, step0 = _onestep(orc, scenes["specular"], 8, 1500, mode, seed=23, k0=k0, rao_blackwell=0)
    _compare_step(orc, scenes["specular"], 8, st, gs, os_, idx, 23, step0, k0, check_score=(mode == dr.DR_MODE_FUSED),
                  plain=(mode == dr.DR_MODE_PLAIN))
    # the sampled weights differ from chain to chain (the RB weight depends on p only)
    live = os_["p"] > 0
    assert np.unique(np.round(os_["w"][live] / 1e-12)).size > 10


@pytest.mark.parametrize("mode", [dr.DR_MODE_FUSED, dr.DR_MODE_PLAIN])
def test_full_size_sampled_parity(orc, mode):
    """The benchmark configuration itself (53k triangles, 512x512, L = 8,
    65,536 chains, default launch): one step on every chain, 1,024 sampled
    chains checked against the oracle evaluating just those chain ids."""
    sc = inputs.procedural_spheres(seed=1)
    L, N = 8, 65536
    sample = np.random.default_rng(0).choice(N, 1024, replace=False)
    sample.sort()
    say(f"[full size] scene=spheres 53k L={L} N={N} mode={mode} sampled={len(sample)}")
    st, gs, os_, idx, step0 = _onestep(orc, sc, L, N, mode, seed=77, k0=300.0, sample=sample)
    _compare_step(orc, sc, L, st, gs, os_, idx, 77, step0, 300.0, check_score=(mode == dr.DR_MODE_FUSED),
                  plain=(mode == dr.DR_MODE_PLAIN))


def test_one_step_per_chain_sigma_and_rotation(orc, scenes):
    """Nonreversible drift (gamma = 0.5) with per-chain diagonal Sigma."""
    sc = scenes["spheres_small"]
    L, N = 8, 800
    sigma = inputs.per_chain_sigma(4 * (L - 1), N, seed=4)
    say(f"[one step sigma] L={L} N={N}")
    st, gs, os_, idx, step0 = _onestep(orc, sc, L, N, dr.DR_MODE_FUSED, seed=5, k0=200.0, gamma=0.5, sigma=sigma)
    _compare_step(orc, sc, L, st, gs, os_, idx, 5, step0, 200.0)


def test_init_matches_oracle(orc, scenes):
    sc = scenes["tiny"]
    L, N, seed = 4, 2048, 13
    say(f"[init] L={L} N={N}")
    S = dr.Scene(sc)
    ch = dr.Chains(S, N, L, seed, k0=0.0)
    ch.set_record(True)
    ch.reinit(3)
    gs = ch.read_state()
    O = orc.Scene(sc)
    oc = orc.Chains.scene(O, L, N, seed=seed)
    oc.init(frame=3, nthreads=16)
    os_ = oc.state()
    oa = oc.accum()
    assert np.array_equal(gs["x"].astype(np.float64), os_["x"])   # regeneration draws are exact in FP32
    assert gs["step"] == oa["step"] == (3 << 32) + 1
    assert abs(gs["p_lambda_hat"] / oa["p_lambda_hat"] - 1) < 1e-5
    assert abs(gs["k0"] / oa["k0"] - 1) < 1e-5
    agree = (gs["killed"] == os_["killed"]).mean()
    say(f"  init kill agreement {agree:.5f}")
    assert agree > 0.999
    assert (gs["pixel"] == os_["pixel"]).all()


def test_fused_and_plain_agree(scenes):
    """The fused persistent form and the plain multi-kernel form draw the same
    streams and compile the same arithmetic, so 20 steps from the same
    initial state leave bit-identical chains (the plain form's score at the
    start of a step is the one the fused form computed after the previous
    one); the frame buffers differ only by the atomics' summation order."""
    sc = scenes["tiny"]
    L, N, seed = 4, 1024, 17
    say(f"[fused vs plain] L={L} N={N}")
    S = dr.Scene(sc)
    out = []
    for mode in (dr.DR_MODE_FUSED, dr.DR_MODE_PLAIN):
        ch = dr.Chains(S, N, L, seed, k0=400.0, mode=mode)
        ch.step(20)
        s = ch.read_state()
        out.append(s)
    a, b = out
    say(f"  kill agreement {(a['killed'] == b['killed']).mean():.5f}, max |dx| {np.abs(a['x'] - b['x']).max():.2e}, "
        f"tours {a['tour_count']} {b['tour_count']}")
    assert np.array_equal(a["x"], b["x"])
    assert np.array_equal(a["killed"], b["killed"])
    assert a["tour_count"] == b["tour_count"]
    assert np.allclose(a["accum"], b["accum"], rtol=1e-5, atol=0)


def test_pt_render_matches_oracle(orc, scenes):
    sc = scenes["tiny"]
    L, spp, seed = 4, 64, 3
    say(f"[pt] L={L} spp={spp}")
    S = dr.Scene(sc)
    img = S.pt_render(L, seed, spp).cpu().numpy()
    ref = orc.Scene(sc).pt_render(L, seed, spp)
    err = np.abs(img - ref) / np.maximum(np.abs(ref), 1e-2)
    say(f"  pt per-pixel rel err median {np.median(err):.2e} p99.9 {np.quantile(err, 0.999):.2e}")
    assert np.median(err) < 1e-5
    assert (err > 1e-3).mean() < 0.01


def test_image_statistics_match_oracle(orc, scenes):
    """The tiny configuration (256 chains x 1000 steps): device and oracle
    images over 32 seeds each (the same seeds on both sides); their MRSE
    against a path-traced reference must lie in each other's 95% band, and
    their means agree within the seed-to-seed spread."""
    sc = scenes["tiny"]
    L, N, steps, R = 4, 256, 1000, 32
    say(f"[image stats] L={L} N={N} steps={steps} R={R}")
    S = dr.Scene(sc)
    O = orc.Scene(sc)
    ref = O.pt_render(L, 12345, 1024, nthreads=16)

    def mrse(img):
        return float(((img - ref) ** 2 / (ref ** 2 + 1e-2)).mean())

    g_m, o_m, g_means, o_means = [], [], [], []
    for r in range(R):
        ch = dr.Chains(S, N, L, 1000 + r)
        ch.step(steps)
        img, _ = ch.image_read()
        ch.close()
        g_m.append(mrse(img.astype(np.float64)))
        g_means.append(img.mean())
        oc = orc.Chains.scene(O, L, N, seed=1000 + r)
        oc.init(nthreads=16)
        oc.step(steps, nthreads=16)
        oi = oc.resolve()
        o_m.append(mrse(oi))
        o_means.append(oi.mean())
        say(f"  seed {r}: MRSE device {g_m[-1]:.4f} oracle {o_m[-1]:.4f}")
    g_m, o_m = np.array(g_m), np.array(o_m)
    say(f"  MRSE device {g_m.mean():.4f}+-{g_m.std():.4f}  oracle {o_m.mean():.4f}+-{o_m.std():.4f}")
    se = math.sqrt(g_m.var(ddof=1) / R + o_m.var(ddof=1) / R)
    assert abs(g_m.mean() - o_m.mean()) < 1.96 * se + 1e-4
    sm = math.sqrt(np.var(g_means, ddof=1) / R + np.var(o_means, ddof=1) / R)
    assert abs(np.mean(g_means) - np.mean(o_means)) < 1.96 * sm + 1e-5


def test_resume_is_bit_identical(scenes):
    sc = scenes["spheres_small"]
    L, N, seed = 8, 2048, 23
    say(f"[resume] L={L} N={N}")
    S = dr.Scene(sc)
    a = dr.Chains(S, N, L, seed)
    a.step(5)
    snap = a.read_state()
    a.step(7)
    ra = a.read_state()
    b = dr.Chains(S, N, L, seed + 99)   # different seed: state must fully come from the snapshot
    b.close()
    b = dr.Chains(S, N, L, seed)
    b.write_state(x=snap["x"], score=snap["score"], killed=snap["killed"], accum=snap["accum"], step=snap["step"],
                  tour_count=snap["tour_count"], k0=snap["k0"])
    b.step(7)
    rb = b.read_state()
    assert np.array_equal(ra["x"], rb["x"]) and np.array_equal(ra["killed"], rb["killed"])
    assert ra["tour_count"] == rb["tour_count"]


def test_counters_and_scene_change(scenes):
    sc = scenes["tiny"]
    L, N = 4, 512
    S = dr.Scene(sc)
    ch = dr.Chains(S, N, L, 1)
    ch.set_counters(True)
    ch.reinit(0)
    ch.step(10)
    st = ch.stats()
    say(f"[counters] {st}")
    assert st["chain_steps"] == N * 11
    assert st["rays"] > N * 11 and st["node_visits"] >= st["rays"]
    assert st["tours"] > 0 and st["adjoints"] > 0
    cam = sc["camera"].copy()
    cam[0] += 0.05
    S.set_camera(cam)
    with pytest.raises(dr.DrError) as e:
        ch.step(1)
    assert e.value.status == dr.DR_ERR_BAD_STATE
    ch.reinit(1)
    ch.step(1)


@pytest.mark.parametrize("lanes", [1, 2])
def test_non_finite_state_is_killed_and_regenerated(scenes, lanes):
    """A chain whose position or score holds NaN or Inf evaluates to p = 0 at
    its next step (nothing traced), is killed, and regenerates at the step
    after; the frame buffer stays finite and every other chain is exactly what
    it is in a clean run."""
    S = dr.Scene(scenes["spheres_small"])
    N, L = 2000, 8
    bad = [5, 9, 11, 700]
    runs = []
    for inject in (False, True):
        ch = dr.Chains(S, N, L, 23, k0=250.0)
        ch.set_launch(lanes_per_chain=lanes)
        ch.step(2)
        st = ch.read_state()
        x, sc, killed = st["x"].copy(), st["score"].copy(), st["killed"].copy()
        if inject:
            x[:, 5] = np.nan        # the whole position
            x[7, 9] = np.inf        # one coordinate
            sc[3, 11] = np.nan      # the score: the move carries it into x
            x[2, 700] = np.nan      # the light block of the first vertex only
            killed[bad] = 0
        ch.write_state(x=x, score=sc, killed=killed, accum=st["accum"], step=st["step"],
                       tour_count=st["tour_count"], k0=st["k0"])
        ch.set_record(True)
        ch.step(1)
        a = ch.read_state()
        ch.step(1)
        b = ch.read_state()
        runs.append((a, b))
    (a0, b0), (a1, b1) = runs
    say(f"[non-finite] lanes={lanes} killed {a1['killed'][bad]} p {a1['p'][bad]}")
    assert a1["killed"][bad].all() and np.all(a1["p"][bad] == 0)
    assert np.all(np.isfinite(b1["x"])) and np.all((b1["x"] >= 0) & (b1["x"] < 1))
    assert np.all(np.isfinite(a1["accum"])) and np.all(np.isfinite(b1["accum"]))
    good = np.setdiff1d(np.arange(N), bad)
    for u, v in ((a0, a1), (b0, b1)):
        assert np.array_equal(u["x"][:, good], v["x"][:, good])
        assert np.array_equal(u["killed"][good], v["killed"][good])


def test_all_black_initialisation(scenes):
    """With every emitter off, p_lambda = 0 at initialisation: k0 falls back to
    eps/(m dt), tours end, and the resolved image is exactly zero."""
    sc = dict(scenes["tiny"])
    sc["materials"] = sc["materials"].copy()
    sc["materials"][:, 8:11] = 0.0
    sc["lights"] = sc["lights"].copy()
    sc["lights"][:, 9:12] = 0.0
    S = dr.Scene(sc)
    ch = dr.Chains(S, 1000, 4, 3)
    ch.step(3)
    st = ch.read_state()
    say(f"[all black] k0 {st['k0']} p_lambda {st['p_lambda_hat']} tours {st['tour_count']}")
    assert st["p_lambda_hat"] == 0.0
    assert st["k0"] == pytest.approx(1e-8 / (64 * 1e-5), rel=1e-6)
    assert st["tour_count"] > 0
    img, _ = ch.image_read()
    assert np.all(img == 0)


def test_scene_stats(scenes):
    """The device scene reports its size and the exact traversal stack bound
    its kernels reserve in LDS."""
    for which in ("tiny", "spheres_small"):
        sc = scenes[which]
        st = dr.Scene(sc).stats()
        say(f"[scene stats] {which}: {st}")
        assert st["n_triangles"] == sc["indices"].shape[0]
        assert st["n_nodes"] >= 1
        assert 1 <= st["stack_entries"] <= 64
        assert st["stack_bytes_per_lane"] == 4 * st["stack_entries"]


@pytest.mark.parametrize("which,L,N", [("tiny", 4, 1000), ("spheres_small", 8, 3000), ("specular", 8, 3000)])
def test_paired_lanes_match_single_lane(scenes, which, L, N):
    """Two lanes per chain (continuation and shadow rays traced concurrently)
    must give exactly the chains one lane per chain gives."""
    say(f"[pair vs single] scene={which} L={L} N={N}")
    S = dr.Scene(scenes[which])
    out = []
    for lanes in (1, 2):
        ch = dr.Chains(S, N, L, 31, k0=250.0)
        ch.set_launch(lanes_per_chain=lanes)
        ch.step(6)
        out.append(ch.read_state())
    a, b = out
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["killed"], b["killed"])
    assert np.array_equal(a["score"][:, a["killed"] == 0], b["score"][:, b["killed"] == 0])
    assert a["tour_count"] == b["tour_count"]
    assert np.allclose(a["accum"], b["accum"], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("lanes,order", [(1, "length"), (2, "length"), (1, "tile"), (2, "tile")])
def test_length_ordering_matches_identity_order(scenes, lanes, order):
    """Processing chains grouped by their last path length, or by the screen
    tile of their film coordinates (a counting sort and a move of the state
    rows before each launch), gives exactly the chains of the identity order;
    only the order of the splat additions differs."""
    N, L = 5000, 8
    say(f"[sorted vs identity] scene=spheres_small L={L} N={N} lanes={lanes} order={order}")
    S = dr.Scene(scenes["spheres_small"])
    out = []
    for sort in (2, 1):
        ch = dr.Chains(S, N, L, 57, k0=250.0)
        key = "sort_by_length" if order == "length" else "sort_by_tile"
        ch.set_launch(lanes_per_chain=lanes, **{key: sort})
        assert ch.get_launch()[key] == (1 if sort == 1 else 0)
        for _ in range(3):
            ch.step(1)
        ch.step(4)
        out.append(ch.read_state())
    a, b = out
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["killed"], b["killed"])
    assert np.array_equal(a["score"][:, a["killed"] == 0], b["score"][:, b["killed"] == 0])
    assert np.array_equal(a["path_rec"], b["path_rec"])
    assert a["tour_count"] == b["tour_count"]
    assert np.allclose(a["accum"], b["accum"], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("which,L,N", [("tiny", 4, 1500), ("spheres_small", 8, 5000), ("specular", 8, 5000)])
def test_refill_form_matches_straight_line(scenes, which, L, N):
    """The ray-refill form of the fused kernel (lanes refill with their next
    ray or step while others traverse) gives exactly the chains of the
    straight-line forms (one and two lanes per chain), over several launches
    and with path-length ordering."""
    say(f"[refill vs straight] scene={which} L={L} N={N}")
    S = dr.Scene(scenes[which])
    out = []
    for refill, sort, lanes in ((2, 2, 1), (1, 2, 1), (1, 1, 1), (2, 2, 2)):
        ch = dr.Chains(S, N, L, 91, k0=250.0)
        ch.set_launch(refill=refill, sort_by_length=sort, lanes_per_chain=lanes)
        assert ch.get_launch()["refill"] == (1 if refill == 1 else 0)
        ch.step(1)
        ch.step(5)
        ch.step(3)
        out.append(ch.read_state())
    a = out[0]
    for b in out[1:]:
        assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["killed"], b["killed"])
        assert np.array_equal(a["score"][:, a["killed"] == 0], b["score"][:, b["killed"] == 0])
        assert np.array_equal(a["path_rec"], b["path_rec"])
        assert a["tour_count"] == b["tour_count"]
        assert np.allclose(a["accum"], b["accum"], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("which,L,N", [("tiny", 4, 3000), ("spheres_small", 8, 20000), ("specular", 8, 20000),
                                       ("interior", 8, 65536)])
def test_wavefront_init_matches_straight_line(scenes, which, L, N):
    """The initialise pass evaluated as ray waves (traversal and event
    kernels alternating) or with the ray-refill state machine leaves exactly
    the state the one-lane kernel does:
    positions, kill decisions, p, f/p, pixels, path records, scores, k0 and
    the tour count; the frame buffers differ only by the atomics' order."""
    say(f"[wavefront and refill init] scene={which} L={L} N={N}")
    # the interior: the 2M-triangle tree, whose traversals run deepest
    S = dr.Scene(inputs.procedural_interior() if which == "interior" else scenes[which])
    out = []
    for wf, rf in ((2, 2), (1, 2), (2, 1)):
        ch = dr.Chains(S, N, L, 31, frame=2)
        ch.set_launch(wavefront=wf, init_refill=rf)
        ch.set_record(True)
        ch.reinit(5)
        out.append(ch.read_state())
        ch.close()
    a = out[0]
    for b in out[1:]:
        for k in ("x", "killed", "p", "pixel", "f_over_p", "path_rec", "score", "weight"):
            assert np.array_equal(a[k], b[k]), k
        assert a["k0"] == b["k0"] and a["tour_count"] == b["tour_count"]
        assert np.allclose(a["accum"], b["accum"], rtol=1e-5, atol=0)


@pytest.mark.parametrize("N", [1, 63, 65, 257])
def test_init_forms_with_ragged_chain_counts(scenes, N):
    """Chain counts below, just under and just over one wavefront (and a
    ragged multiple of a block): the persistent straight-line, ray-refill and
    ray-wave initialise passes give the same state, and every chain holds a
    finite p and a pixel inside the image."""
    say(f"[ragged init] N={N}")
    S = dr.Scene(scenes["spheres_small"])
    out = []
    for wf, rf in ((2, 2), (2, 1), (1, 2)):
        ch = dr.Chains(S, N, 8, 77, frame=1)
        ch.set_launch(wavefront=wf, init_refill=rf)
        ch.set_record(True)
        ch.reinit(3)
        out.append(ch.read_state())
        ch.close()
    a = out[0]
    assert np.all(np.isfinite(a["p"])) and np.all(a["pixel"] < 128 * 128)
    for b in out[1:]:
        for k in ("x", "killed", "p", "pixel", "f_over_p", "path_rec", "score", "weight"):
            assert np.array_equal(a[k], b[k]), k
        assert a["k0"] == b["k0"] and a["tour_count"] == b["tour_count"]


@pytest.mark.parametrize("order", ["none", "length", "tile"])
def test_captured_frames_replay_like_eager(scenes, order):
    """A captured frame (re-init + n steps + resolve) replayed several times,
    with a camera change between replays and eager work in between, gives the
    chains and image the same calls give eagerly.  With chain ordering on, the
    frame's steps move chains between slots: host reads and writes of the
    state between replays must still see every chain in its own slot."""
    sc = scenes["spheres_small"]
    L, N, n = 8, 4096, 5
    say(f"[frame graph] L={L} N={N} steps/frame={n} order={order}")
    S1, S2 = dr.Scene(sc), dr.Scene(sc)
    a = dr.Chains(S1, N, L, 41, frame=3)
    b = dr.Chains(S2, N, L, 41, frame=3)
    if order != "none":
        cfg = {"sort_by_length": 1} if order == "length" else {"sort_by_tile": 1}
        a.set_launch(**cfg)
        b.set_launch(**cfg)
    stream = torch.cuda.Stream()
    img_a = torch.zeros((3, S1.W * S1.H), device="cuda")
    with torch.cuda.stream(stream):
        frame = a.capture_frame(n, True, img_a, stream)
    for k in range(3):
        cam = sc["camera"].copy()
        cam[0] += 0.03 * k
        S1.set_camera(cam)
        S2.set_camera(cam)
        frame.launch(stream)
        stream.synchronize()
        b.reinit(4 + k)
        b.step(n)
        img_b = b.resolve()
        torch.cuda.synchronize()
        sa, sb = a.read_state(), b.read_state()
        assert sa["step"] == sb["step"] == ((4 + k) << 32) + 1 + n
        assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["killed"], sb["killed"])
        assert np.array_equal(sa["score"], sb["score"])
        assert sa["tour_count"] == sb["tour_count"]
        ia, ib = img_a.cpu().numpy(), img_b.cpu().numpy()
        assert np.allclose(ia, ib, rtol=1e-4, atol=1e-6), np.abs(ia - ib).max()
        # a host write between replays (the state read back unchanged) must
        # land every chain in its own slot, then eager work continues
        a.write_state(x=sa["x"], score=sa["score"], killed=sa["killed"])
        b.write_state(x=sb["x"], score=sb["score"], killed=sb["killed"])
        a.step(1)
        b.step(1)
        torch.cuda.synchronize()
        sa, sb = a.read_state(), b.read_state()
        assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["killed"], sb["killed"])
    frame.close()


@pytest.mark.parametrize("name", ["instances", "spheres_1080p_L16", "interior", "spheres_specular"])
def test_large_configs_sampled_parity(orc, name):
    """The larger configurations at their real shapes: ~1M triangles with
    path length 12 and 1M chains; path length 16 with per-chain diagonal
    Sigma at 1920x1080 and 2M chains; ~2M triangles at 1920x1080 with 4M
    chains; the 53k-triangle spheres with glass and mirror spheres.  One
    fused step on every chain, 512 sampled chains against the oracle."""
    factory, L, N = inputs.CONFIGS[name]
    sc = factory()
    d = 4 * (L - 1)
    sigma = inputs.per_chain_sigma(d, N, seed=4) if name == "spheres_1080p_L16" else None
    sample = np.sort(np.random.default_rng(1).choice(N, 512, replace=False))
    say(f"[large] {name}: {sc['indices'].shape[0]} triangles, {sc['width']}x{sc['height']}, L={L}, N={N}")
    st, gs, os_, idx, step0 = _onestep(orc, sc, L, N, dr.DR_MODE_FUSED, seed=91, k0=100.0, sigma=sigma,
                                      sample=sample)
    _compare_step(orc, sc, L, st, gs, os_, idx, 91, step0, 100.0)


@pytest.mark.parametrize("which", ["interior", "specular", "c4"])
def test_adjoint_long_paths_with_segment_recompute(orc, which):
    """Path length 16 (d = 60): the adjoint keeps one checkpoint per 8-vertex
    segment and recomputes each segment in the reverse sweep (through delta
    vertices too, in the specular box).  Checked against the oracle's
    forward-mode score and central differences (h = 1e-3) on the device, for
    every coordinate.  "c4" is the differentiation-stress configuration
    itself: the 53k-triangle spheres at 1920x1080 with 4,096 sampled chain
    states (initialised chains are uniform points of the torus)."""
    n = 1024
    if which == "interior":
        sc = inputs.procedural_interior(n_inst=40, subdiv=3, width=320, height=180)
    elif which == "c4":
        sc = inputs.CONFIGS["spheres_1080p_L16"][0]()
        n = 4096
    else:
        sc = inputs.specular_box(width=128, height=128)
    L, h = 16, 1e-3
    d = 4 * (L - 1)
    say(f"[adjoint L16] {sc['indices'].shape[0]} triangles, n={n}")
    u, (f, logp, g), (fo, po, go), match = _eval_both(orc, sc, L, n, seed=12)
    say(f"  path-signature match {match.mean():.5f}")
    assert match.mean() > 0.99
    live = match & (po > 1e-3 * po.mean())
    _check_eval(orc.Scene(sc), L, u.astype(np.float64), (f, logp, g), match)
    S = dr.Scene(sc)
    ut = torch.from_numpy(u).cuda()
    _, lp0, _, r0 = S.eval_logp_grad(L, ut, grad=False, rec=True)
    # long paths: some samples reach the second 8-vertex segment
    nverts = (r0 != -1).sum(1).cpu().numpy()
    say(f"  samples with more than 8 vertices: {(nverts > 8).sum()}")
    # the open spheres scene lets most paths escape early; the closed scenes exercise the recompute more
    assert (nverts > 8).sum() > (10 if which == "c4" else 20)
    checked = bad = 0
    for i in range(d):
        e = torch.zeros_like(ut)
        e[:, i] = h
        _, lpp, _, rp = S.eval_logp_grad(L, (ut + e).clamp(0, 1 - 2 ** -24), grad=False, rec=True)
        _, lpm, _, rm = S.eval_logp_grad(L, (ut - e).clamp(0, 1 - 2 ** -24), grad=False, rec=True)
        same = (rp == r0).all(1).cpu().numpy() & (rm == r0).all(1).cpu().numpy() & live
        same &= (u[:, i] > h) & (u[:, i] < 1 - h)
        fd = (lpp - lpm).cpu().numpy() / (2 * h)
        tol = 0.05 * np.abs(go[:, i]) + 0.05 * np.abs(fd) + 2e-4 / h * np.maximum(1.0, np.abs(lp0.cpu().numpy()))
        checked += same.sum()
        bad += (same & (np.abs(fd - g[:, i]) > tol)).sum()
    say(f"  FD checked {checked}, outside tolerance {bad}")
    assert checked > 5000 * n // 1024 and bad <= 0.01 * checked


def test_delta_closed_forms_on_device():
    """The closed forms that pin the oracle's delta lobes, on the device: a
    light seen in a smooth-conductor plane at normal incidence is f0 Le; a
    glass slab's branch values (through-through Le, reflection first 0, two
    internal reflections then out Le); the n^2 radiance law from inside."""
    Le = np.array([4.0, 3.0, 2.0])
    say("[delta closed forms] mirror plane, glass slab, camera inside the slab")

    def f_at(sc, L, rows):
        S = dr.Scene(sc)
        u = torch.tensor(np.asarray(rows, np.float32)).cuda()
        f, _, _, _ = S.eval_logp_grad(L, u, grad=True, rec=True)
        torch.cuda.synchronize()
        return f.cpu().numpy().astype(np.float64)

    sc = inputs.mirror_plane(f0=(0.9, 0.6, 0.3), Le=tuple(Le))
    f0 = sc["materials"][0, 5:8].astype(np.float64)
    u = np.full((1, 8), 0.3)
    u[0, :2] = 0.5
    assert np.allclose(f_at(sc, 3, u)[0], f0 * Le, rtol=1e-6)

    L = 6
    rows = []
    for ch in ([0.9, 0.9], [0.01], [0.9, 0.01, 0.01, 0.9], [0.9, 0.01, 0.9]):
        r = np.full(4 * (L - 1), 0.5)
        for j, c in enumerate(ch):
            r[4 * (j + 1)] = c
        rows.append(r)
    f = f_at(inputs.glass_slab(eta=1.5, Le=tuple(Le)), L, rows)
    assert np.allclose(f[0], Le, rtol=1e-5) and np.all(f[1] == 0)
    assert np.allclose(f[2], Le, rtol=1e-5) and np.all(f[3] == 0)

    r = np.full(12, 0.5)
    r[4] = 0.9
    f = f_at(inputs.glass_slab(eta=1.5, Le=tuple(Le), eye_z=-1.25), 4, [r])
    assert np.allclose(f[0], 1.5 ** 2 * Le, rtol=1e-5)


def test_device_matches_stored_oracle_values(orc):
    """The device against the oracle values stored in tests/golden (written by
    the oracle from seeded points on the tiny box, the specular box and the
    mirror plane): path records equal, f and the score within the FP32
    tolerances of the live parity tests."""
    import json
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_paths.json")) as fh:
        gold = json.load(fh)
    for case in gold["cases"]:
        say(f"[golden] {case['name']}: scene={case['scene']} L={case['L']} n={case['n']}")
        L = case["L"]
        S = dr.Scene(getattr(inputs, case["scene"])())
        u = torch.tensor(np.asarray(case["u"], np.float32)).cuda()
        f, logp, g, rec = S.eval_logp_grad(L, u, rec=True)
        torch.cuda.synchronize()
        f, g = f.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
        rec = rec.cpu().numpy().view(np.uint32)
        ro = np.asarray(case["rec"], np.int64)
        prim, nee = ro[:, 0::2], ro[:, 1::2]
        rec_o = np.where(prim >= 0, (prim << 8) | (nee & 0xFF), 0xFFFFFFFF).astype(np.uint32)
        assert np.array_equal(rec_o, rec), case["name"]
        fo, po, go = np.asarray(case["f"]), np.asarray(case["p"]), np.asarray(case["score"])
        u64 = np.asarray(case["u"], np.float32).astype(np.float64)
        sens, (fl, pl, gl, _) = _sens(orc.Scene(getattr(inputs, case["scene"])()), L, u64)
        # the stored values are the oracle's own at these points
        assert np.allclose(fl, fo, rtol=1e-12, atol=0) and np.allclose(gl, go, rtol=1e-9, atol=1e-12)
        _within(f"{case['name']} f", _vec_rel(f, fo, 1e-3 * max(1e-6, np.abs(fo).mean())), sens["f"], L)
        live = po > 1e-3 * po.mean()
        _score_within(f"{case['name']} score", g[live], go[live], {k: v[live] for k, v in sens.items()}, L)


def test_torch_allocator_serves_library_buffers(scenes):
    """With torch's caching allocator installed as the library's allocator,
    chain buffers and evaluation scratch come from torch, the results are the
    same as with hipMalloc, and destroying the chains returns the memory."""
    S = dr.Scene(scenes["tiny"])
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    dr.use_torch_allocator(True)
    try:
        a = dr.Chains(S, 2000, 4, 3, k0=250.0)
        grown = torch.cuda.memory_allocated() - base
        a.step(3)
        u = torch.rand((500, 12), device="cuda")
        fa = S.eval_logp_grad(4, u, grad=True)[0]
        sa = a.read_state()
    finally:
        dr.use_torch_allocator(False)
    say(f"[torch allocator] chain buffers {grown} bytes from torch")
    assert grown > 0
    b = dr.Chains(S, 2000, 4, 3, k0=250.0)
    b.step(3)
    fb = S.eval_logp_grad(4, u, grad=True)[0]
    sb = b.read_state()
    assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["killed"], sb["killed"])
    assert sa["tour_count"] == sb["tour_count"]
    assert torch.equal(fa, fb)
    a.close()
    del fa, u
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - base <= grown - 1  # the chain set's buffers went back to torch


def test_autotune_restores_chains(scenes, tmp_path, monkeypatch):
    """The launch autotuner sweeps configurations on the live chain set, then
    puts the chains back: tuning followed by n steps gives the chains n steps
    give without tuning."""
    from paper_2605_08916_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(autotune, "BLOCKS", (128, 256))
    monkeypatch.setattr(autotune, "BLOCKS_PER_CU", (2, 3))
    say("[autotune] scene=spheres_small L=8 N=3000")
    S = dr.Scene(scenes["spheres_small"])
    a = dr.Chains(S, 3000, 8, 77, k0=250.0)
    b = dr.Chains(S, 3000, 8, 77, k0=250.0)
    a.step(2)
    b.step(2)
    entry = autotune.tune(a, reps=1, use_cache=True, per_launch=2)
    flags = ("sort_by_length", "sort_by_tile", "refill", "wavefront", "init_refill")  # 1 on, 2 off; 1/0 read back
    applied = {k: (int(v == 1) if k in flags else v) for k, v in entry["cfg"].items()}
    got = a.get_launch()
    assert {k: got[k] for k in applied} == applied
    # staged search: block x blocks per CU, then lanes, orderings, queue batch
    # depth (grab) and the refill form, each from the best so far
    assert len(entry["sweep"]) == 2 * 2 + len(autotune.LANES) + (len(autotune.ORDERS) - 1) + (
        len(autotune.GRABS) - 1) + len(autotune.REFILL_PCTS)
    assert entry["ms"] == min([ms for ms, _ in entry["sweep"]] + [entry["current_ms"]])
    a.step(3)
    b.step(3)
    sa, sb = a.read_state(), b.read_state()
    assert sa["step"] == sb["step"]
    assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["killed"], sb["killed"])
    assert sa["tour_count"] == sb["tour_count"]
    assert np.allclose(sa["accum"], sb["accum"], rtol=1e-5, atol=1e-6)
    # a second chain set with the same key takes the cached configuration
    c = dr.Chains(S, 3000, 8, 78, k0=250.0)
    assert autotune.tune(c, reps=1, per_launch=2)["cfg"] == entry["cfg"]
    assert c.get_launch() == a.get_launch()
