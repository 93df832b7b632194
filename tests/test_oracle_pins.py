"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against an independent source: another
implementation of a published generator (rocRAND's Philox4x32-10), a closed
form, an invariant, quadrature, finite differences, or a brute-force search.
Sizes are chosen so the whole file runs in about a minute on 8 cores.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2605_08916_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# Generator
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference program")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "rr")
    subprocess.check_call([hipcc, "-std=c++17", "-O1", os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp"),
                           "-o", exe], stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)

    def run(triples):
        inp = "\n".join(f"{a} {b} {c}" for a, b, c in triples) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], np.uint64)

    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_ref):
    """Philox4x32-10 (Sec. 4.3 tour state; Salmon et al. 2011) against
    rocRAND's independent implementation on 300 counters/keys."""
    rng = np.random.default_rng(0)
    cases, triples = [], []
    for k in range(300):
        ctr = rng.integers(0, 2 ** 32, 4, dtype=np.uint64)
        key = rng.integers(0, 2 ** 32, 2, dtype=np.uint64)
        if k < 3:
            ctr[:] = [0, 0xFFFFFFFF, 1][k]
            key[:] = [0, 0xFFFFFFFF, 7][k]
        seed = int(key[0]) | (int(key[1]) << 32)
        sub = int(ctr[2]) | (int(ctr[3]) << 32)
        off = 4 * (int(ctr[0]) | (int(ctr[1]) << 32))
        if off >= 2 ** 64:
            continue
        cases.append((ctr, key))
        triples.append((seed, sub, off))
    ref = rocrand_ref(triples)
    got = np.array([orc.philox(c, k) for c, k in cases], np.uint64)
    assert np.array_equal(got, ref)


def test_uniform_stream_layout(orc, rocrand_ref):
    """U(c, s, tag, i) takes word i&3 of the block at counter
    (c, s_lo, s_hi, tag<<24 | i>>2), keeps its top 24 bits, scales by 2^-24."""
    seed, c, s = 0x1234_5678_9ABC_DEF0, 77, (5 << 32) + 3
    for tag in (0, 1, 2):
        for i in (0, 1, 2, 3, 4, 13, 59):
            w = (tag << 24) | (i >> 2)
            sub = (s >> 32) | (w << 32)
            off = 4 * (c | ((s & 0xFFFFFFFF) << 32))
            block = rocrand_ref([(seed, sub, off)])[0]
            want = int(block[i & 3]) >> 8
            assert orc.uniform(seed, c, s, tag, i) == want / 2.0 ** 24


def test_box_muller_and_exponential_moments(orc):
    """Box-Muller gives independent N(0,1) pairs; -ln(1-U) has unit mean."""
    n = 100_000
    u = np.array([[orc.uniform(3, k, 0, 1, 0), orc.uniform(3, k, 0, 1, 1)] for k in range(n)])
    z = np.array([orc.box_muller(a, b) for a, b in u])
    se = 1 / math.sqrt(n)
    assert abs(z[:, 0].mean()) < 5 * se and abs(z[:, 1].mean()) < 5 * se
    assert abs(z[:, 0].var() - 1) < 5 * math.sqrt(2) * se and abs(z[:, 1].var() - 1) < 5 * math.sqrt(2) * se
    assert abs(np.mean(z[:, 0] * z[:, 1])) < 5 * se
    e = -np.log(1 - u[:, 0])
    assert abs(e.mean() - 1) < 5 * se


# ---------------------------------------------------------------------------
# Geometry and materials
# ---------------------------------------------------------------------------
def _rays(sc, n, seed):
    rng = np.random.default_rng(seed)
    V = sc["vertices"].astype(np.float64)
    lo, hi = V.min(0), V.max(0)
    o = lo + (hi - lo) * rng.uniform(-0.1, 1.1, (n, 3))
    d = rng.normal(size=(n, 3))
    return o, d / np.linalg.norm(d, axis=1, keepdims=True)


@pytest.mark.parametrize("which", ["tiny", "spheres_small"])
def test_bvh_equals_brute_force(orc, which):
    """The oracle's median-split BVH returns the brute-force closest hit
    (triangle and t, ties to the lower index) and the same occlusion."""
    sc = inputs.cornell_tiny() if which == "tiny" else inputs.procedural_spheres(n_spheres=2, subdiv=2)
    S = orc.Scene(sc)
    o, d = _rays(sc, 4000 if which == "tiny" else 1500, 1)
    p1, t1 = S.trace(o, d)
    o2 = o.copy()
    S.set_brute(True)
    p2, t2 = S.trace(o2, d)
    assert np.array_equal(p1, p2)
    assert np.array_equal(t1[p1 >= 0], t2[p2 >= 0])
    tm = np.where(p2 >= 0, t2 * 0.999, 1e3)
    occ_b = S.occluded(o, d, tm)
    S.set_brute(False)
    occ = S.occluded(o, d, tm)
    assert np.array_equal(occ, occ_b)
    assert (p1 >= 0).mean() > 0.15


def test_onb_orthonormal(orc):
    rng = np.random.default_rng(2)
    for _ in range(200):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        t, b = orc.onb(n)
        M = np.stack([t, b, n])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(t, b), n, atol=1e-12)


def _hemisphere_quadrature(n, nth=400, nph=800):
    """Directions and solid-angle weights on the hemisphere around n
    (midpoint rule in cos(theta) and phi)."""
    t = np.cross(n, [0.3, 0.5, 0.8])
    t /= np.linalg.norm(t)
    b = np.cross(n, t)
    ct = (np.arange(nth) + 0.5) / nth
    ph = 2 * np.pi * (np.arange(nph) + 0.5) / nph
    CT, PH = np.meshgrid(ct, ph, indexing="ij")
    ST = np.sqrt(1 - CT ** 2)
    dirs = (ST * np.cos(PH))[..., None] * t + (ST * np.sin(PH))[..., None] * b + CT[..., None] * n
    w = np.full(CT.shape, (1.0 / nth) * (2 * np.pi / nph))
    return dirs.reshape(-1, 3), w.ravel(), CT.ravel()


@pytest.mark.parametrize("mat", [
    inputs.material(inputs.KIND_LAMBERT, albedo=(0.7, 0.4, 0.2)),
    inputs.material(inputs.KIND_GGX, rough=0.5, f0=(0.95, 0.7, 0.5)),
    inputs.material(inputs.KIND_GGX, rough=0.3, f0=(0.9, 0.6, 0.55)),
])
def test_bsdf_sampling_matches_evaluation(orc, mat):
    """E_(u,v)[weight * g(wi)] from the sampler equals the quadrature of
    f_s cos g over the hemisphere from the evaluator, for several g: pins the
    BSDF value, the sampling density and their Jacobian against each other."""
    n = np.array([0.2, -0.3, 0.93])
    n /= np.linalg.norm(n)
    wo = np.array([0.5, 0.4, 0.6])
    wo = wo / np.linalg.norm(wo)
    assert wo @ n > 0
    k = 1024
    g1 = (np.arange(k) + 0.5) / k
    U, V = np.meshgrid(g1, g1, indexing="ij")
    ok, wi, wt = orc.bsdf_sample_n(mat, n, wo, U.ravel(), V.ravel())
    dirs, w, ct = _hemisphere_quadrature(n)
    fs = orc.bsdf_eval_n(mat, n, wo, dirs)
    gs = [lambda x: np.ones(len(x)), lambda x: (x @ n) ** 2, lambda x: x @ np.array([0.6, 0.0, 0.8]) + 1.0,
          lambda x: np.exp(3 * (x @ wo))]
    for g in gs:
        est = (wt * np.where(ok, g(wi), 0.0)[:, None]).mean(0)
        quad = (fs * (ct * w * g(dirs))[:, None]).sum(0)
        assert np.allclose(est, quad, rtol=1.5e-2, atol=1e-4), (est, quad)
    if mat[0] == inputs.KIND_LAMBERT:
        assert np.allclose((fs * (ct * w)[:, None]).sum(0), mat[1:4], rtol=1e-4)


@pytest.mark.parametrize("alpha", [0.1, 0.3, 0.5])
def test_ggx_normalisation_and_weak_white_furnace(orc, alpha):
    """Exact identities of a microfacet model: the projected microfacet area
    integrates to one, int D(h) cos(theta_h) dh = 1, and the weak white
    furnace, int G1(wo) max(0, wo.h) D(h) dh = cos(theta_o), which holds only
    for the Smith G1 that matches D."""
    n = 2000
    ct = (np.arange(n) + 0.5) / n
    D = np.array([orc.ggx_d(c, alpha) for c in ct])
    assert abs((D * ct).sum() / n * 2 * np.pi - 1) < 2e-3
    # weak furnace for a few outgoing angles (quadrature over h on the hemisphere)
    nth, nph = 1500, 400
    cth = (np.arange(nth) + 0.5) / nth
    ph = 2 * np.pi * (np.arange(nph) + 0.5) / nph
    CT, PH = np.meshgrid(cth, ph, indexing="ij")
    ST = np.sqrt(1 - CT ** 2)
    Dh = np.array([orc.ggx_d(c, alpha) for c in cth])[:, None]
    for th_o in (0.2, 0.7, 1.2):
        wo = np.array([math.sin(th_o), 0.0, math.cos(th_o)])
        dot_oh = ST * np.cos(PH) * wo[0] + CT * wo[2]
        integral = (orc.smith_g1(wo[2], alpha) * np.maximum(dot_oh, 0) * Dh).sum() * (1 / nth) * (2 * np.pi / nph)
        assert abs(integral / wo[2] - 1) < 5e-3, (alpha, th_o, integral / wo[2])


def test_bsdf_reciprocity_and_energy(orc):
    rng = np.random.default_rng(4)
    n = np.array([0.0, 0.0, 1.0])
    for rough in (0.1, 0.3, 0.5):
        mat = inputs.material(inputs.KIND_GGX, rough=rough, f0=(1.0, 1.0, 1.0))
        for _ in range(50):
            a, b = rng.normal(size=(2, 3))
            a[2], b[2] = abs(a[2]), abs(b[2])
            a /= np.linalg.norm(a)
            b /= np.linalg.norm(b)
            assert np.allclose(orc.bsdf_eval(mat, n, a, b), orc.bsdf_eval(mat, n, b, a), rtol=1e-12)
        dirs, w, ct = _hemisphere_quadrature(n)
        for wo in ([0, 0, 1], [0.6, 0, 0.8]):
            alb = (orc.bsdf_eval_n(mat, n, np.array(wo, float), dirs)[:, 0] * ct * w).sum()
            assert 0.5 < alb <= 1.0 + 2e-3


# ---------------------------------------------------------------------------
# The path sampler f(u) and its gradient
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [2, 3, 4])
def test_white_furnace_closed_form(orc, L):
    """Closed cube of inward Lambertian emitters: E_u[f] = Le (1-a^L)/(1-a)."""
    a, Le = 0.5, 1.0
    S = orc.Scene(inputs.white_furnace(albedo=a, Le=Le))
    u = inputs.random_points(4 * (L - 1), 120_000, seed=10 + L).astype(np.float64)
    f, p, _, _ = S.path_eval(L, u, grad=False)
    want = Le * (1 - a ** L) / (1 - a)
    se = f[:, 0].std() / math.sqrt(len(f))
    assert abs(f[:, 0].mean() - want) < 5 * se
    assert np.all(f[:, 0] == f[:, 1]) and np.all(f[:, 1] == f[:, 2])
    assert np.all(f[:, 0] >= Le)  # primary emission always seen


def _one_bounce_closed_form(sc, u):
    """f(u) for path length 2 in the one-bounce scene, written from its
    geometry: pinhole ray, intersection with the plane z = 0 (or the light
    quad in front of it), direct light from a point on the quad light."""
    cam = sc["camera"].astype(np.float64)
    eye, at, up, fov = cam[:3], cam[3:6], cam[6:9], cam[9]
    W, H = sc["width"], sc["height"]
    fwd = (at - eye) / np.linalg.norm(at - eye)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    upv = np.cross(right, fwd)
    th = math.tan(math.radians(fov) / 2)
    lt = sc["lights"][0].astype(np.float64)
    p0, e1, e2, Le = lt[:3], lt[3:6], lt[6:9], lt[9:12]
    A = np.linalg.norm(np.cross(e1, e2))
    alb = sc["materials"][0, 1:4].astype(np.float64)
    out = np.zeros((len(u), 3))
    for k, uu in enumerate(u):
        d = fwd + th * (2 * uu[0] - 1) * (W / H) * right + th * (1 - 2 * uu[1]) * upv
        d /= np.linalg.norm(d)
        # does the camera ray meet the light quad (back side: no emission, black)?
        tl = (p0[2] - eye[2]) / d[2]
        q = eye + tl * d - p0
        a_ = q @ e1 / (e1 @ e1)
        b_ = q @ e2 / (e2 @ e2)
        if 0 <= a_ <= 1 and 0 <= b_ <= 1:
            continue
        t = -eye[2] / d[2]
        x = eye + t * d
        if not (abs(x[0]) <= 2 and abs(x[1]) <= 2):
            continue
        y = p0 + uu[2] * e1 + uu[3] * e2
        w = y - x
        r2 = w @ w
        cx = w[2] / math.sqrt(r2)
        cy = w[2] / math.sqrt(r2)
        out[k] = alb / math.pi * Le * cx * cy / r2 * A
    return out


def test_one_bounce_closed_form_value_and_gradient(orc):
    sc = inputs.one_bounce_plane()
    S = orc.Scene(sc)
    u = inputs.random_points(4, 400, seed=3).astype(np.float64)
    f, p, score, _ = S.path_eval(2, u)
    want = _one_bounce_closed_form(sc, u)
    assert np.allclose(f, want, rtol=1e-10, atol=1e-12)
    assert (want[:, 0] > 0).mean() > 0.3
    # gradient of ln(p + eps) against central differences of the closed form
    lum = np.array([0.2126, 0.7152, 0.0722])
    h = 1e-6
    for k in range(60):
        if want[k, 0] == 0:
            continue
        for i in range(4):
            up, um = u[k].copy(), u[k].copy()
            up[i] += h
            um[i] -= h
            fp, fm = _one_bounce_closed_form(sc, [up, um])
            if fp[0] == 0 or fm[0] == 0:
                continue
            fd = (math.log(fp @ lum + 1e-8) - math.log(fm @ lum + 1e-8)) / (2 * h)
            assert abs(fd - score[k, i]) <= 1e-5 * max(1.0, abs(fd)), (k, i, fd, score[k, i])


@pytest.mark.parametrize("which,L", [("tiny", 4), ("spheres_small", 6), ("specular", 8)])
def test_score_matches_finite_differences(orc, which, L):
    """Forward-mode score equals central differences of ln(p + eps) wherever
    both perturbed points keep the same discrete path (readings A13, A14);
    the specular box runs it through mirror chains, refraction and emission
    seen through delta vertices."""
    sc = {"tiny": inputs.cornell_tiny, "specular": inputs.specular_box,
          "spheres_small": lambda: inputs.procedural_spheres(n_spheres=3, subdiv=2)}[which]()
    S = orc.Scene(sc)
    d = 4 * (L - 1)
    u = inputs.random_points(d, 150, seed=21).astype(np.float64)
    f, p, score, rec = S.path_eval(L, u)
    h = 1e-6
    checked = 0
    for k in range(len(u)):
        if p[k] <= 0:
            assert np.all(score[k] == 0)
            continue
        for i in range(d):
            up, um = u[k].copy(), u[k].copy()
            up[i] += h
            um[i] -= h
            fp, pp, _, rp = S.path_eval(L, up[None], grad=False)
            fm, pm, _, rm = S.path_eval(L, um[None], grad=False)
            if not (np.array_equal(rp[0], rec[k]) and np.array_equal(rm[0], rec[k])):
                continue
            fd = (math.log(pp[0] + 1e-8) - math.log(pm[0] + 1e-8)) / (2 * h)
            assert abs(fd - score[k, i]) <= 2e-4 * max(1.0, abs(fd)), (k, i, fd, score[k, i])
            checked += 1
    assert checked > 200


# ---------------------------------------------------------------------------
# Delta materials: smooth conductor and smooth dielectric (Sec. 6 material set)
# ---------------------------------------------------------------------------
def _random_frames(rng, n):
    """n unit normals and unit directions on the normal's side."""
    nn = rng.normal(size=(n, 3))
    nn /= np.linalg.norm(nn, axis=1, keepdims=True)
    wo = rng.normal(size=(n, 3))
    wo /= np.linalg.norm(wo, axis=1, keepdims=True)
    wo *= np.sign(np.sum(wo * nn, axis=1, keepdims=True))
    return nn, wo


def test_mirror_lobe(orc):
    """Smooth conductor: the law of reflection (wi + wo along n, equal angles,
    unit length) and Schlick's F at its three fixed points: f0 at normal
    incidence, 1 at grazing incidence, increasing towards grazing."""
    mat = inputs.material(inputs.KIND_MIRROR, f0=(0.9, 0.6, 0.3))
    f0 = np.asarray(mat[5:8], np.float32).astype(np.float64)  # the material is stored in FP32
    rng = np.random.default_rng(5)
    nn, wo = _random_frames(rng, 200)
    for n, o in zip(nn, wo):
        lobe, wi, wt = orc.delta_sample(mat, n, True, o, 0.5)
        assert lobe == 0
        assert abs(np.linalg.norm(wi) - 1) < 1e-12
        s = wi + o
        assert np.linalg.norm(np.cross(s, n)) < 1e-12 and np.dot(s, n) >= 0
        assert abs(np.dot(wi, n) - np.dot(o, n)) < 1e-12
        assert np.all(wt >= f0 - 1e-12) and np.all(wt <= 1 + 1e-12)
    n = np.array([0.0, 0.0, 1.0])
    _, wi, wt = orc.delta_sample(mat, n, True, n, 0.5)
    assert np.allclose(wi, n) and np.allclose(wt, f0, rtol=0, atol=1e-15)
    _, _, wt = orc.delta_sample(mat, n, True, np.array([1.0, 0.0, 0.0]), 0.5)
    assert np.allclose(wt, 1.0)
    prev = None
    for th in np.linspace(0, 1.5, 16):
        _, _, wt = orc.delta_sample(mat, n, True, np.array([math.sin(th), 0.0, math.cos(th)]), 0.5)
        if prev is not None:
            assert np.all(wt >= prev - 1e-15)
        prev = wt


@pytest.mark.parametrize("eta", [1.33, 1.5, 2.4])
def test_dielectric_fresnel_fixed_points(orc, eta):
    """Fresnel reflectance of a smooth dielectric against values that do not
    come from its formula: ((eta - 1)/(eta + 1))^2 at normal incidence;
    Brewster's angle, where the p-polarised part vanishes and the
    s-polarised amplitude is (1 - eta^2)/(1 + eta^2); 1 at grazing incidence
    and beyond the critical angle inside the denser medium; Stokes
    reciprocity F(theta_i, eta) = F(theta_t, 1/eta) with Snell's theta_t."""
    assert abs(orc.fresnel_dielectric(1.0, eta) - ((eta - 1) / (eta + 1)) ** 2) < 1e-15
    assert abs(orc.fresnel_dielectric(1.0, 1 / eta) - ((eta - 1) / (eta + 1)) ** 2) < 1e-15
    tb = math.atan(eta)
    assert abs(orc.fresnel_dielectric(math.cos(tb), eta) - 0.5 * ((1 - eta ** 2) / (1 + eta ** 2)) ** 2) < 1e-14
    assert abs(orc.fresnel_dielectric(0.0, eta) - 1.0) < 1e-15
    crit = math.asin(1 / eta)
    for th in np.linspace(crit + 1e-6, math.pi / 2, 7):
        assert orc.fresnel_dielectric(math.cos(th), 1 / eta) == 1.0
    for th in np.linspace(0.0, 1.55, 40):
        st = math.sin(th) / eta
        ct = math.sqrt(1 - st * st)
        a, b = orc.fresnel_dielectric(math.cos(th), eta), orc.fresnel_dielectric(ct, 1 / eta)
        assert 0.0 <= a <= 1.0 and abs(a - b) < 1e-13, (th, a, b)


@pytest.mark.parametrize("front", [True, False])
def test_dielectric_lobe(orc, front):
    """Smooth dielectric sample: the coordinate u picks reflection exactly when
    u < F; reflection obeys the law of reflection with weight 1; refraction
    obeys Snell's law (sin_t etap = sin_i, in the plane of n and wo, on the
    far side) with weight 1/etap^2, etap = eta entering, 1/eta leaving."""
    eta = 1.5
    mat = inputs.material(inputs.KIND_GLASS, eta=eta)
    etap = eta if front else 1 / eta
    rng = np.random.default_rng(9)
    nn, wo = _random_frames(rng, 300)
    refracted = 0
    for n, o in zip(nn, wo):
        ci = float(np.dot(n, o))
        F = orc.fresnel_dielectric(ci, etap)
        for u in (0.0, max(F - 1e-4, 0.0), min(F + 1e-4, 0.9999), 0.9999):
            lobe, wi, wt = orc.delta_sample(mat, n, front, o, u)
            assert abs(np.linalg.norm(wi) - 1) < 1e-12
            if u < F:
                assert lobe == 0
                assert np.linalg.norm(np.cross(wi + o, n)) < 1e-12 and np.allclose(wt, 1.0)
            else:
                assert lobe == 1
                refracted += 1
                sin_i = np.linalg.norm(np.cross(n, o))
                sin_t = np.linalg.norm(np.cross(n, wi))
                assert abs(sin_t * etap - sin_i) < 1e-12
                assert np.dot(wi, n) < 0
                assert abs(np.dot(np.cross(n, o), wi)) < 1e-12                       # coplanar
                assert np.dot(wi - np.dot(wi, n) * n, o - ci * n) <= 1e-12             # tangent reversed
                assert np.allclose(wt, 1 / etap ** 2)
    assert refracted > 100  # leaving the medium, total internal reflection takes the rest


def test_mirror_plane_closed_form(orc):
    """A light seen only in a smooth-conductor plane: the camera ray that
    meets the mirror at normal incidence returns f0 Le; a ray returns
    radiance exactly when the mirror image of the eye, through the mirror
    point, lines up with the light (method of images), with F between f0
    and 1; with one vertex the delta surface gives nothing (no next-event
    estimation at a delta vertex)."""
    f0, Le = np.array([0.9, 0.6, 0.3]), np.array([4.0, 3.0, 2.0])
    sc = inputs.mirror_plane(f0=tuple(f0), Le=tuple(Le))
    f0 = sc["materials"][0, 5:8].astype(np.float64)  # as stored (FP32)
    S = orc.Scene(sc)
    L = 3
    u = np.full((1, 4 * (L - 1)), 0.3)
    u[0, :2] = 0.5
    f, _, _, _ = S.path_eval(L, u, grad=False)
    assert np.allclose(f[0], f0 * Le, rtol=1e-14)
    f1, _, _, _ = S.path_eval(2, np.random.default_rng(2).random((500, 4)), grad=False)
    assert np.all(f1 == 0)
    U = np.random.default_rng(4).random((3000, 4 * (L - 1)))
    U[:, :2] = 0.5 + (U[:, :2] - 0.5) * 0.6
    f, _, _, _ = S.path_eval(L, U, grad=False)
    # primary direction of the pinhole model; image of the eye in z = -1 is (0, 0, -2)
    th = math.tan(math.radians(60.0) / 2)
    D = np.stack([(2 * U[:, 0] - 1) * th, (1 - 2 * U[:, 1]) * th, -np.ones(len(U))], 1)
    P = D / -D[:, 2:3] * 1.0                      # meets z = -1
    R = P - np.array([0.0, 0.0, -2.0])            # image ray through P
    Q = P + R * (2.0 / R[:, 2:3])                 # meets z = +1
    inside = (Q[:, 0] > -0.3) & (Q[:, 0] < 0.4) & (Q[:, 1] > -0.2) & (Q[:, 1] < 0.3)
    edge = (np.minimum.reduce([np.abs(Q[:, 0] + 0.3), np.abs(Q[:, 0] - 0.4), np.abs(Q[:, 1] + 0.2),
                               np.abs(Q[:, 1] - 0.3)]) < 1e-9)
    lit = f[:, 0] > 0
    assert np.array_equal(lit[~edge], inside[~edge]) and inside.sum() > 100
    assert np.all(f[lit] >= f0 * Le * (1 - 1e-12)) and np.all(f[lit] <= Le * (1 + 1e-12))


def test_glass_slab_branches(orc):
    """Camera ray through a smooth-dielectric slab at normal incidence to a
    light behind it: each choice sequence of the dielectric coordinates has
    a fixed value.  Through-through returns Le (the 1/eta^2 entering and
    eta^2 leaving cancel); reflection at the first face returns nothing;
    two internal reflections then exit return Le; the decision sits at
    F = ((eta - 1)/(eta + 1))^2."""
    Le = np.array([4.0, 3.0, 2.0])
    sc = inputs.glass_slab(eta=1.5, Le=tuple(Le))
    S = orc.Scene(sc)
    L = 6
    F = 0.04

    def f_of(choices):
        u = np.full((1, 4 * (L - 1)), 0.5)
        for j, c in enumerate(choices):
            u[0, 4 * (j + 1)] = c
        return S.path_eval(L, u, grad=False)[0][0]

    T, R = 0.9, 0.01
    assert np.allclose(f_of([T, T]), Le, rtol=1e-12)
    assert np.all(f_of([R]) == 0)
    assert np.allclose(f_of([T, R, R, T]), Le, rtol=1e-12)
    assert np.all(f_of([T, R, T]) == 0)
    assert np.all(f_of([T, R, R, R]) == 0)
    assert np.all(f_of([F * (1 - 1e-4), T]) == 0) and np.allclose(f_of([F * (1 + 1e-4), T]), Le)


def test_radiance_seen_from_inside_the_dielectric(orc):
    """Radiance divided by the squared index of refraction is conserved
    across a smooth interface, so a camera inside the slab sees a light
    outside, through the lower face at normal incidence, as eta^2 Le (the
    refraction branch; its probability 1 - F cancels its weight's)."""
    eta, Le = 1.5, np.array([4.0, 3.0, 2.0])
    S = orc.Scene(inputs.glass_slab(eta=eta, Le=tuple(Le), eye_z=-1.25))
    L = 4
    u = np.full((1, 4 * (L - 1)), 0.5)
    u[0, 4] = 0.9
    f = S.path_eval(L, u, grad=False)[0][0]
    assert np.allclose(f, eta ** 2 * Le, rtol=1e-12)
    u[0, 4] = 0.01
    assert np.all(S.path_eval(L, u, grad=False)[0][0] == 0)


# ---------------------------------------------------------------------------
# The chain
# ---------------------------------------------------------------------------
def test_constant_target_tours(orc):
    """p constant, k0 = p_lambda/(m dt): each step kills with probability
    k dt/(1 + k dt) = 1/(m+1); the estimator returns lambda(f) = 1."""
    N, steps = 1000, 1500
    C = orc.Chains.mixture(2, [], np.zeros((0, 2)), [], 1.0, N, seed=3, k0=1.0 / (64 * 1e-5))
    C.init()
    C.step(steps)
    a = C.accum()
    n = N * (steps + 1)
    q = 1 / 65
    assert abs(a["tour_count"] / n - q) < 5 * math.sqrt(q * (1 - q) / n)
    img = C.resolve()[:, 0]
    assert abs(img[0] - 1.0) < 0.01
    assert np.all(np.abs(img[1:]) < 0.03)


def test_estimated_killing_constant(orc):
    """k0 left to the initialise pass (Eq. killing-rate-constant, reading A6):
    p_lambda_hat is the mean of p over the N initial states and k0 =
    p_lambda_hat/(m dt).  On a constant target every state has p = c, so
    p_lambda_hat = c exactly and each step kills with probability 1/(m+1);
    on a wrapped Gaussian mixture the mean over uniform states estimates
    lambda(p) = c0 + sum w within its standard error."""
    N, steps, c, m, dt = 2000, 600, 0.37, 64.0, 1e-5
    C = orc.Chains.mixture(2, [], np.zeros((0, 2)), [], c, N, seed=5, m=m, k0=0.0)
    C.init()
    a0 = C.accum()
    assert a0["p_lambda_hat"] == pytest.approx(c, rel=1e-12)
    assert a0["k0"] == pytest.approx(c / (m * dt), rel=1e-12)
    C.step(steps)
    a = C.accum()
    n = N * (steps + 1)
    q = 1 / (m + 1)
    assert abs(a["tour_count"] / n - q) < 5 * math.sqrt(q * (1 - q) / n)
    # a non-constant target: the estimate is the sample mean of p(x), x ~ U(T^d)
    rng = np.random.default_rng(12)
    d, c0 = 2, 0.1
    w = np.array([0.7, 0.3])
    means = rng.uniform(size=(2, d))
    s = np.array([0.08, 0.12])
    Nm = 20000
    Cm = orc.Chains.mixture(d, w, means, s, c0, Nm, seed=6, k0=0.0)
    Cm.init()
    am = Cm.accum()
    # the sample variance of p over uniform states, from the same draws
    p0 = Cm.state()["p"]
    assert am["p_lambda_hat"] == pytest.approx(p0.mean(), rel=1e-12)
    se = p0.std(ddof=1) / math.sqrt(Nm)
    assert abs(am["p_lambda_hat"] - (c0 + w.sum())) < 5 * se
    assert am["k0"] == pytest.approx(am["p_lambda_hat"] / (64 * dt), rel=1e-12)


def test_per_chain_diagonal_sigma_lyapunov(orc):
    """Per-chain diagonal Sigma (reading A16), killing off, no rotation,
    Gaussian target N(c, s^2 I2): coordinate i of a chain is its own AR(1),
    x'_i - c = a_i (x_i - c) + sd_i xi with a_i = 1 - sd_i^2/(2 s^2), whose
    stationary variance is sd_i^2/(1 - a_i^2).  Two groups of chains with
    different stddevs in the two coordinates, both orders.  The steps are
    large against the target (sd_i^2/(2 s^2) = 1/8 and 1/2), so the
    discretised chain's variance 2 s^2/(2 - sd_i^2/(2 s^2)) depends on sd_i:
    a stddev taken from the wrong coordinate changes it by 20%."""
    dt, s, N = 1e-5, 0.1, 400
    sd_a, sd_b = 0.05, 0.1
    sig = np.empty((2, N), np.float32)
    sig[0, : N // 2], sig[1, : N // 2] = sd_a, sd_b
    sig[0, N // 2:], sig[1, N // 2:] = sd_b, sd_a
    C = orc.Chains.mixture(2, [1.0], np.array([[0.5, 0.5]]), [s], 0.0, N, seed=9, stddev=0.02, dt=dt, gamma=0.0,
                           k0=1e-30)
    C.set_sigma(sig)
    C.init()
    C.step(100)
    x = C.step(2000, trace=True) - 0.5
    for grp, (s0, s1) in ((slice(0, N // 2), (sd_a, sd_b)), (slice(N // 2, N), (sd_b, sd_a))):
        for i, sd in ((0, s0), (1, s1)):
            sd = float(np.float32(sd))
            a = 1 - sd ** 2 / (2 * s ** 2)
            q = sd ** 2 / (1 - a ** 2)
            v = x[:, i, grp].var()
            assert abs(v / q - 1) < 0.03, (i, sd, v, q)


def test_sampled_holding_weight_has_the_rao_blackwell_mean(orc):
    """Competing exponential clocks (reading A8): the sampled weight
    min(dt E_a, E_b / k) of a step is the minimum of independent Exp(h) and
    Exp(k) times, itself Exp(h + k) with mean 1/(h + k) = dt/(1 + k dt) and
    standard deviation equal to its mean; the Rao-Blackwellised weight is
    that mean exactly.  p constant, so every chain has the same k."""
    N, dt, eps = 40000, 1e-5, 1e-8
    k0 = 1.0 / (3 * dt)  # k dt = 1/3: both clocks matter
    k = k0 / (1.0 + eps)  # p = 1 everywhere
    want = 1.0 / (1.0 / dt + k)
    Cs = orc.Chains.mixture(2, [], np.zeros((0, 2)), [], 1.0, N, seed=8, k0=k0, rao_blackwell=0)
    Cs.init()
    Cs.step(1)
    ws = Cs.state()["w"]
    Cr = orc.Chains.mixture(2, [], np.zeros((0, 2)), [], 1.0, N, seed=8, k0=k0, rao_blackwell=1)
    Cr.init()
    Cr.step(1)
    wr = Cr.state()["w"]
    assert np.allclose(wr, want, rtol=1e-12, atol=0)
    assert abs(ws.mean() - want) < 5 * want / math.sqrt(N)
    assert abs(ws.std() - want) < 0.05 * want


def test_local_dynamics_lyapunov(orc):
    """Killing off, Gaussian target N(c, s^2 I2): the Euler-Maruyama move with
    rotation is AR(1), x' - c = A (x - c) + stddev xi, A = alpha I - beta U,
    alpha = 1 - stddev^2/(2 s^2), beta = gamma_tilde / s^2.  Stationary
    covariance q I with q = stddev^2/(1 - alpha^2 - beta^2); lag-one cross
    covariance E[x'_1 x_2] = -beta q (Alg. 5.1, rotate)."""
    sd, dt, gam, s = 0.02, 1e-5, 100.0, 0.1
    C = orc.Chains.mixture(2, [1.0], np.array([[0.5, 0.5]]), [s], 0.0, 400, seed=7, stddev=sd, dt=dt, gamma=gam,
                           k0=1e-30)
    C.init()
    C.step(300)
    x = C.step(3000, trace=True) - 0.5
    alpha = 1 - sd ** 2 / (2 * s ** 2)
    beta = dt * gam / 2 / s ** 2
    q = sd ** 2 / (1 - alpha ** 2 - beta ** 2)
    assert abs(x[:, 0].var() / q - 1) < 0.02 and abs(x[:, 1].var() / q - 1) < 0.02
    c12 = (x[1:, 0] * x[:-1, 1]).mean()
    c21 = (x[1:, 1] * x[:-1, 0]).mean()
    assert abs(c12 + beta * q) < 0.15 * beta * q
    assert abs(c21 - beta * q) < 0.15 * beta * q


def _mixture_closed_form(w, m, s, c0):
    d = m.shape[1]
    damp = np.exp(-2 * np.pi ** 2 * s ** 2)
    out = [c0 + w.sum()]
    for i in range(d):
        out.append((w * damp * np.cos(2 * np.pi * m[:, i])).sum())
        out.append((w * damp * np.sin(2 * np.pi * m[:, i])).sum())
    return np.array(out)


@pytest.mark.parametrize("d,s,c0", [(2, [0.15, 0.2], 0.3), (4, [0.2, 0.25, 0.2], 0.2), (8, [0.2, 0.25, 0.2, 0.25], 0.2)])
def test_restore_estimator_closed_forms(orc, d, s, c0):
    """Wrapped Gaussian mixture on T^d, f = p g with g = (1, cos 2 pi x_i,
    sin 2 pi x_i): k0 accum / tourCount -> lambda(p g) =
    (c0 + sum w, sum_j w_j exp(-2 pi^2 s_j^2) cos/sin(2 pi m_ji)).  m = 4 keeps
    tours short so the finite-run renewal bias of the ratio estimator
    (about 2.5/steps relative here) stays below the noise."""
    rng = np.random.default_rng(4)
    s = np.array(s)
    m = rng.uniform(size=(len(s), d))
    w = np.array([0.4, 0.3, 0.2, 0.1][: len(s)])
    w = w / w.sum()
    want = _mixture_closed_form(w, m, s, c0)
    ests = []
    for seed in range(4):
        C = orc.Chains.mixture(d, w, m, s, c0, 1024, seed=seed, m=4)
        C.init()
        C.step(3000)
        ests.append(C.resolve()[:, 0])
    ests = np.array(ests)
    se = ests.std(0, ddof=1) / 2
    tol = 4.5 * se + 2.5 / 3000 * np.abs(want) + 2e-3
    assert np.all(np.abs(ests.mean(0) - want) < tol), (ests.mean(0) - want, tol)


def test_restore_image_tends_to_path_tracing(orc):
    """As m -> 0 tours last about one step and the Diffusion Restore image
    k0 accum W H / tourCount reduces to importance-sampled path tracing: it
    must match brute-force independent path tracing (pins the estimator's
    normalisation, the pixel map and the holding weights)."""
    sc = inputs.cornell_tiny()
    S = orc.Scene(sc)
    ref = S.pt_render(4, seed=99, spp=512)
    ref2 = S.pt_render(4, seed=98, spp=512)
    C = orc.Chains.scene(S, 4, 4096, seed=1, m=2e-4)
    C.init()
    C.step(300)
    img = C.resolve()
    lum = lambda a: 0.2126 * a[0] + 0.7152 * a[1] + 0.0722 * a[2]
    light = lum(ref) > 5
    # per-sample noise of a 512-spp image, from two independent references
    var_ref = ((lum(ref) - lum(ref2)) ** 2).mean() / 2
    for mask in (light, ~light):
        n = mask.sum()
        diff = lum(img)[mask].mean() - lum(ref)[mask].mean()
        # the DR image holds ~300 samples per pixel: allow 6 sigma of both
        se = math.sqrt(var_ref * (512 / 300 + 1) / n)
        assert abs(diff) < 6 * se + 0.01 * lum(ref)[mask].mean(), (mask.sum(), diff, se)


def test_chain_determinism_and_thread_independence(orc):
    sc = inputs.cornell_tiny()
    S = orc.Scene(sc)
    outs = []
    for nt in (1, 4):
        C = orc.Chains.scene(S, 4, 64, seed=5)
        C.init(nthreads=nt)
        C.step(20, nthreads=nt)
        st = C.state()
        outs.append((st["x"], st["killed"], C.accum()["tour_count"]))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


# ---------------------------------------------------------------------------
# Bias term L*p/p of the modified killing rate (Sec. 5.2, Eq. adjoint-bias)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_bias_term_gaussian_closed_form(gamma):
    """For p = N(c, s^2 I) the Euler-Maruyama kernel (with the rotational
    drift) maps p to N(c, (s^2 (a^2 + beta^2) + dt sigma2) I), so L*p/p has a
    closed form; the grid quadrature must reproduce it."""
    from oracle import bias
    c, s, dt, sigma2 = (0.5, 0.5), 0.05, 1e-3, 1.0
    dens = bias.wrapped_mixture([1.0], [c], [s], c0=0.0, images=0)
    X, Y, p, t = bias.em_bias_term(dens, 128, dt, sigma2, gamma)
    ref = bias.gaussian_term_closed_form(X, Y, c, s, dt, sigma2, gamma)
    inner = (X - c[0]) ** 2 + (Y - c[1]) ** 2 < (3 * s) ** 2
    assert np.abs(ref[inner]).max() > 50.0  # the term is far from zero here
    assert np.abs(t - ref)[inner].max() < 1e-8


def test_bias_term_is_order_dt():
    """The bias term is O(dt) (sigma2 fixed): halving dt halves it on a
    smooth four-mode target."""
    from oracle import bias
    mix = inputs.mixture_target(d=2, seed=11)
    dens = bias.wrapped_mixture(mix["weights"], mix["means"], mix["stds"], c0=0.1)
    out = []
    for dt in (1e-3, 5e-4):
        sd = math.sqrt(dt * 0.25)
        _, _, p, t = bias.em_bias_term(dens, int(math.ceil(3.0 / sd)), dt, 0.25, gamma=0.5)
        out.append(((np.abs(t) * p).sum() / p.sum(), np.abs(t).max()))
    for a, b in zip(out[0], out[1]):
        assert 1.8 < a / b < 2.2


def test_bias_drift_is_the_chain_move(orc):
    """The drift b of the bias term is the oracle chain's move: from one point
    with a given score, the mean displacement of one step is dt b."""
    import oracle as O
    from oracle import bias
    d, N, dt, sigma2, gamma = 2, 40000, 1e-3, 1.0, 0.5
    x0 = np.array([0.53, 0.46])
    dens = bias.wrapped_mixture([1.0], [(0.5, 0.5)], [0.05], images=0)
    p, gx, gy = dens(np.array([x0[0]]), np.array([x0[1]]))
    s = np.array([gx[0] / p[0], gy[0] / p[0]])
    b = np.array([0.5 * sigma2 * s[0] + 0.5 * gamma * s[1], 0.5 * sigma2 * s[1] - 0.5 * gamma * s[0]])
    C = O.Chains.mixture(d, [1.0], [(0.5, 0.5)], [0.05], 0.0, N, seed=5, stddev=math.sqrt(dt * sigma2), dt=dt,
                         gamma=gamma, k0=1e-12)
    C.set_state(np.tile(x0[:, None], (1, N)), np.tile(s[:, None], (1, N)), np.zeros(N), step=1, k0=1e-12)
    C.step(1)
    st = C.state()
    assert st["killed"].sum() == 0
    disp = st["x"] - x0[:, None]
    disp -= np.round(disp)
    se = math.sqrt(dt * sigma2 / N)
    assert np.all(np.abs(disp.mean(axis=1) - dt * b) < 5 * se)
    assert abs(dt * b[1] - dt * 0.5 * sigma2 * s[1]) > 10 * se  # the rotation is resolved


def test_non_finite_state_is_killed_and_regenerated(orc):
    """A point with a non-finite coordinate has f = 0 (nothing traced), so a
    chain whose state left the torus is killed at its next step and
    regenerates at the one after; the frame buffer stays finite."""
    sc = inputs.cornell_tiny()
    S = orc.Scene(sc)
    L, d = 4, 12
    u = inputs.random_points(d, 4, seed=2).astype(np.float64)
    u[1, 5] = np.nan
    u[2, 0] = np.inf
    f, p, score, rec = S.path_eval(L, u)
    assert np.all(f[1:3] == 0) and np.all(p[1:3] == 0) and np.all(np.isfinite(score))
    N = 64
    C = orc.Chains.scene(S, L, N, seed=3, k0=250.0)
    C.init(nthreads=2)
    st = C.state()
    x = st["x"].astype(np.float32)
    x[:, 5] = np.nan
    x[7, 9] = np.inf
    sc_ = st["score"].astype(np.float32)
    sc_[3, 11] = np.nan
    killed = np.zeros(N, np.uint32)
    C.set_state(x, sc_, killed, step=(1 << 32) + 1, k0=250.0)
    C.step(1, nthreads=2)
    a = C.state()
    assert a["killed"][[5, 9, 11]].all() and np.all(a["p"][[5, 9, 11]] == 0)
    C.step(1, nthreads=2)
    b = C.state()
    assert np.all(np.isfinite(b["x"])) and np.all((b["x"] >= 0) & (b["x"] < 1))
    assert np.all(np.isfinite(C.accum()["accum"]))


def _black(sc):
    """The scene with every emitter switched off (p = 0 everywhere)."""
    sc = dict(sc)
    sc["materials"] = sc["materials"].copy()
    sc["materials"][:, 8:11] = 0.0
    sc["lights"] = sc["lights"].copy()
    sc["lights"][:, 9:12] = 0.0
    return sc


def test_all_black_initialisation(orc):
    """p_lambda = 0 at initialisation: k0 falls back to eps/(m dt) (reading
    A6), so tours end at rate 1/(m dt), and the image stays exactly zero."""
    S = orc.Scene(_black(inputs.cornell_tiny()))
    C = orc.Chains.scene(S, 4, 128, seed=3)
    C.init(nthreads=2)
    C.step(3, nthreads=2)
    acc = C.accum()
    assert acc["p_lambda_hat"] == 0.0
    assert acc["k0"] == pytest.approx(1e-8 / (64 * 1e-5), rel=1e-12)
    assert acc["tour_count"] > 0
    assert np.all(acc["accum"] == 0) and np.all(C.resolve() == 0)


def test_oracle_reproduces_its_golden_fixture(orc):
    """Regression guard (not a pin): the oracle still returns the values that
    tests/golden/make_golden.py stored from it (f, p, score, path record), so
    a change to its arithmetic cannot pass unnoticed."""
    import json
    with open(os.path.join(HERE, "golden", "oracle_paths.json")) as fh:
        gold = json.load(fh)
    for case in gold["cases"]:
        sc = getattr(inputs, case["scene"])()
        u = np.asarray(case["u"], np.float64)
        f, p, score, rec = orc.Scene(sc).path_eval(case["L"], u, eps=gold["eps"])
        assert np.array_equal(rec.astype(np.int64), np.asarray(case["rec"], np.int64)), case["name"]
        np.testing.assert_allclose(f, np.asarray(case["f"]), rtol=1e-12, atol=0, err_msg=case["name"])
        np.testing.assert_allclose(p, np.asarray(case["p"]), rtol=1e-12, atol=0, err_msg=case["name"])
        np.testing.assert_allclose(score, np.asarray(case["score"]), rtol=1e-9, atol=1e-12, err_msg=case["name"])


def test_score_condition_measure_bounds_the_score(orc):
    """The condition measure the GPU parity tests allow rounding by (the
    running magnitude of the score's terms, Scene.path_cond) is at least the
    score's magnitude in every coordinate, equals it where the score has a
    single term (the film coordinates of a camera ray that hits an emitter
    directly on a Lambertian box: p there does not depend on the film
    coordinates, so both are zero), and exceeds it where terms cancel."""
    for sc, L in ((inputs.cornell_tiny(), 4), (inputs.specular_box(), 8)):
        S = orc.Scene(sc)
        u = inputs.random_points(4 * (L - 1), 1500, 7).astype(np.float64)
        _, p, g, _ = S.path_eval(L, u)
        k = S.path_cond(L, u)
        assert np.all(np.isfinite(k)) and np.all(k >= np.abs(g) * (1 - 1e-12))
        live = p > 1e-6
        ratio = k[live] / np.maximum(np.abs(g[live]), 1e-300)
        assert np.median(ratio[np.abs(g[live]) > 0]) < 10      # most coordinates: few terms
        assert ratio[np.abs(g[live]) > 0].max() > 100          # some cancel strongly
    # a point whose camera ray ends on the light at vertex 1 with no bounce
    # taken: f = Le, independent of every coordinate
    sc = inputs.white_furnace(albedo=0.0, Le=2.0)
    S = orc.Scene(sc)
    u = inputs.random_points(4, 50, 3).astype(np.float64)
    f, p, g, _ = S.path_eval(2, u)
    k = S.path_cond(2, u)
    assert np.allclose(f, 2.0) and np.all(g == 0) and np.all(k == 0)
