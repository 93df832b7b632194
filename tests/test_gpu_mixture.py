"""The chain step on the analytic target (a wrapped Gaussian mixture on T^d,
f = p g with g = 1, cos 2 pi x_i, sin 2 pi x_i) on the device: one step
against the oracle from identical states, the Restore estimator against the
closed form lambda(p g) and against the oracle's estimate (each within the
other's confidence interval), and the move's one-step law against the kernel
the bias quadrature of oracle/bias.py integrates."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2605_08916_amd import dr, inputs  # noqa: E402

TOL = 1e-4


def say(*a):
    import sys
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dr.lib()
    torch.cuda.set_device(0)


def _closed_form(w, m, s, c0):
    """lambda(p g) for the wrapped mixture: the mean of cos / sin 2 pi x under
    a wrapped normal N(mu, s^2) is exp(-2 pi^2 s^2) cos / sin 2 pi mu."""
    d = m.shape[1]
    damp = np.exp(-2 * np.pi ** 2 * s ** 2)
    out = [c0 + w.sum()]
    for i in range(d):
        out.append((w * damp * np.cos(2 * np.pi * m[:, i])).sum())
        out.append((w * damp * np.sin(2 * np.pi * m[:, i])).sum())
    return np.array(out)


def _mixture8():
    mix = inputs.mixture_target(d=8, seed=11)
    return mix["weights"], mix["means"], mix["stds"], 0.1


@pytest.mark.parametrize("sigma", [False, True])
def test_mixture_one_step_matches_oracle(orc, sigma):
    """One step from the same seeded state (15% killed, seeded scores) on the
    d = 8 mixture: x', p, the holding weight and the score within 1e-4, kill
    decisions identical outside the band the p difference sets."""
    w, m, s, c0 = _mixture8()
    d, N, seed, k0, step = 8, 8192, 17, 2000.0, (3 << 32) + 5
    say(f"[mixture one step] d={d} N={N} per-chain sigma={sigma}")
    st = inputs.random_state(d, N, seed=9, killed_frac=0.15)
    score0 = st["score"]
    sig = inputs.per_chain_sigma(d, N, seed=4) if sigma else None
    O = orc.Chains.mixture(d, w, m, s, c0, N, seed=seed, k0=k0)
    if sig is not None:
        O.set_sigma(sig)
    O.set_state(st["x"], score0, st["killed"], step, k0=k0)
    O.step(1)
    os_ = O.state()
    M = dr.Mixture(d, w, m, s, c0)
    sig_t = None if sig is None else torch.from_numpy(sig).cuda()
    g = M.step(st["x"], score0, st["killed"], seed=seed, step=step, k0=k0, sigma=sig_t)
    # x' relative to the step on the torus
    dx = g["x"].astype(np.float64) - os_["x"]
    dx = np.abs(dx - np.round(dx))
    stp = np.abs(os_["x"] - st["x"].astype(np.float64))
    stp = np.minimum(stp, 1 - stp)
    xerr = dx / np.maximum(stp, 5e-3)
    say(f"  x' step-relative err max {xerr.max():.2e}")
    assert xerr.max() < TOL
    perr = np.abs(g["p"] - os_["p"]) / np.maximum(os_["p"], 1e-30)
    say(f"  p rel err max {perr.max():.2e}")
    assert perr.max() < TOL
    werr = np.abs(g["w"] - os_["w"]) / os_["w"]
    assert werr.max() < 2 * TOL
    # kills: identical except within the band the p difference sets
    Ea = np.array([-math.log(1 - orc.uniform(seed, c, step, orc.TAG_HOLD, 0)) for c in range(N)])
    Eb = np.array([-math.log(1 - orc.uniform(seed, c, step, orc.TAG_HOLD, 1)) for c in range(N)])
    kk = k0 / (os_["p"] + 1e-8)
    gap = np.abs(kk * 1e-5 * Ea - Eb) / np.maximum(Eb, 1e-30)
    flip = g["killed"] != os_["killed"]
    say(f"  kills {int(os_['killed'].sum())}, flips {int(flip.sum())}")
    assert np.all(~flip | (gap < 1e-6 + 4 * perr))
    live = (os_["killed"] == 0) & (g["killed"] == 0)
    go, gg = os_["score"][:, live].T, g["score"][:, live].T.astype(np.float64)
    fl = np.maximum(1e-2 * np.abs(go).max(axis=1, keepdims=True), 1e-6)
    serr = np.abs(gg - go) / np.maximum(np.abs(go), fl)
    say(f"  score per-coordinate rel err max {serr.max():.2e}")
    assert serr.max() < TOL


def _mixture8_wide():
    """The d = 8 mixture of the oracle's estimator pin: modes wide enough
    (s = 0.2, 0.25) that chains regenerated uniformly find them within a
    tour; the narrow modes of the one-step test hold too little volume for
    uniform regeneration to estimate p_lambda in d = 8."""
    rng = np.random.default_rng(4)
    s = np.array([0.2, 0.25, 0.2, 0.25])
    m = rng.uniform(size=(len(s), 8))
    w = np.array([0.4, 0.3, 0.2, 0.1])
    return w / w.sum(), m, s, 0.2


def test_mixture_restore_estimator_matches_closed_form_and_oracle(orc):
    """d = 8 mixture, m = 4 (short tours).  (1) 65,536 chains x 20,000 steps:
    the estimate k0 accum / tourCount within its batch confidence interval of
    lambda(p g), plus the ratio estimator's finite-run bias, O(1/steps) of
    the density's mass.  (2) 3,000 steps: the device chains 0..2047 against
    the oracle's chains 0..2047 (the same random streams) within 4.5 of their
    batch standard errors."""
    w, m, s, c0 = _mixture8_wide()
    want = _closed_form(w, m, s, c0)
    d, N = 8, 65536
    M = dr.Mixture(d, w, m, s, c0)
    steps = 20000
    say(f"[mixture estimator] d={d} N={N} steps={steps}")
    r = M.run(N, seed=3, n_steps=steps, n_batches=64, m=4.0)
    bt = r["batch_tours"].astype(np.float64)
    best = r["k0"] * r["dt"] * r["batch_accum"] / bt[:, None]
    se = best.std(0, ddof=1) / math.sqrt(best.shape[0])
    est = r["estimate"]
    bias = 10.0 / steps * want[0]
    say(f"  p_lambda {r['p_lambda']:.5f} (closed form {want[0]:.5f}); max |est - want| / se "
        f"{np.max(np.abs(est - want) / se):.2f}, max |est - want| {np.max(np.abs(est - want)):.2e}")
    # p_lambda (it only sets k0) is the mean of p over N uniform draws
    assert abs(r["p_lambda"] / want[0] - 1) < 0.2
    assert np.all(np.abs(est - want) < 4.5 * se + bias), (est - want, se)
    # device chains 0..2047 (the first 8 blocks of 256) against the oracle's
    steps, No = 3000, 2048
    r = M.run(N, seed=3, n_steps=steps, n_batches=N // 256, m=4.0)
    nb = No // 256
    acc, bt = r["batch_accum"][:nb], r["batch_tours"][:nb].astype(np.float64)
    dev = r["k0"] * r["dt"] * acc.sum(0) / bt.sum()
    O = orc.Chains.mixture(d, w, m, s, c0, No, seed=3, m=4.0)
    O.init(nthreads=16)
    O.step(steps, nthreads=16)
    oest = O.resolve()[:, 0]
    ob = r["k0"] * r["dt"] * r["batch_accum"] / r["batch_tours"].astype(np.float64)[:, None]
    se_n = ob.std(0, ddof=1) / math.sqrt(nb)  # batch spread at this chain count
    say(f"  oracle vs device on chains 0..{No - 1}: max |diff| / se {np.max(np.abs(oest - dev) / se_n):.3f}")
    assert np.all(np.abs(oest - dev) < 4.5 * se_n)


def test_device_move_is_the_bias_quadrature_kernel():
    """The kernel oracle/bias.py integrates, P(x, .) = N(x + dt b(x), dt
    sigma2 I) with b = (sigma2/2) s + (gamma/2) J s (Sec. 5.2 bias term), is the
    device's move: from one point with its score, one step of many chains
    with killing off has mean displacement dt b and covariance dt sigma2 I
    within the sampling error."""
    from oracle import bias
    d, N, dt, sigma2, gamma = 2, 1 << 18, 1e-3, 1.0, 0.5
    x0 = np.array([0.53, 0.46])
    dens = bias.wrapped_mixture([1.0], [(0.5, 0.5)], [0.05], images=0)
    p, gx, gy = dens(np.array([x0[0]]), np.array([x0[1]]))
    sc = np.array([gx[0] / p[0], gy[0] / p[0]])
    b = np.array([0.5 * sigma2 * sc[0] + 0.5 * gamma * sc[1], 0.5 * sigma2 * sc[1] - 0.5 * gamma * sc[0]])
    M = dr.Mixture(d, [1.0], [(0.5, 0.5)], [0.05], 0.0)
    x = np.tile(x0[:, None], (1, N)).astype(np.float32)
    score = np.tile(sc[:, None], (1, N)).astype(np.float32)
    g = M.step(x, score, np.zeros(N, np.uint32), seed=5, step=1, k0=1e-12, stddev=math.sqrt(dt * sigma2), dt=dt,
               gamma=gamma)
    assert g["killed"].sum() == 0
    disp = g["x"].astype(np.float64) - x0[:, None]
    disp -= np.round(disp)
    mean = disp.mean(axis=1)
    se = math.sqrt(dt * sigma2 / N)
    say(f"[device move vs bias kernel] mean disp {mean}, dt b {dt * b}, se {se:.2e}")
    assert np.all(np.abs(mean - dt * b) < 5 * se)
    assert abs(dt * b[1] - dt * 0.5 * sigma2 * sc[1]) > 10 * se  # the rotation is resolved
    cov = np.cov(disp)
    var_se = dt * sigma2 * math.sqrt(2.0 / N)
    assert np.all(np.abs(np.diag(cov) - dt * sigma2) < 5 * var_se)
    assert abs(cov[0, 1]) < 5 * var_se
