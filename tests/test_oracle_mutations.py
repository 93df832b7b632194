"""The oracle pins catch plausible mistakes: each case plants one mistake in a
copy of oracle.cpp (a dropped factor, a flipped sign, a swapped operand),
builds it, and runs the pin meant to catch it against the mutant, which must
fail.  CPU only; marked slow (about two minutes)."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")

MUTANTS = [
    # (id, original text, mistake, pin that must fail)
    ("drift_half", "0.5 * sd * sd * sc[k]", "sd * sd * sc[k]", "test_local_dynamics_lyapunov"),
    ("rotation_sign", "const double rot[2] = {gt * s1, -gt * s0};", "const double rot[2] = {-gt * s1, gt * s0};",
     "test_local_dynamics_lyapunov"),
    ("rb_weight", "w = 1.0 / (1.0 / C.P.dt + k);", "w = C.P.dt;", "test_constant_target_tours"),
    ("kill_rate", "const double k = C.k0 / (pc + C.P.eps);\n", "const double k = C.k0 * pc / (1.0 + C.P.eps);\n",
     "test_restore_estimator_closed_forms"),
    ("light_cosine", "T cy = -dot(lift<T>(lt.n), wl);", "T cy = T(1.0);", "test_one_bounce_closed_form_value_and_gradient"),
    ("light_pdf", "T g = cx * cy / r2 * ((double)nl * lt.area);", "T g = cx * cy / r2 * (lt.area);",
     "test_white_furnace_closed_form"),
    ("ggx_g1_alpha", "return 2.0 / (1.0 + sqrt(1.0 + alpha * alpha * tan2));",
     "return 2.0 / (1.0 + sqrt(1.0 + alpha * tan2));", "test_ggx_normalisation_and_weak_white_furnace"),
    ("lambert_radius", "T r = sqrt(u);\n        T lz = sqrt(1.0 - u);", "T r = u;\n        T lz = sqrt(1.0 - u * u);",
     "test_bsdf_sampling_matches_evaluation"),
    ("philox_mult", "0xD2511F53u * (uint64_t)c[0]", "0xD2511F55u * (uint64_t)c[0]", "test_philox_matches_rocrand"),
    ("box_muller_radius", "std::sqrt(-2.0 * std::log(1.0 - u0))", "std::sqrt(-std::log(1.0 - u0))",
     "test_box_muller_and_exponential_moments"),
    ("dual_sqrt", "r.g[i] = a.g[i] / (2.0 * r.v);", "r.g[i] = a.g[i] / r.v;", "test_score_matches_finite_differences"),
    ("snell_direction", "wi = wo * (-1.0 / etap) + nn * (ci / etap - ct);", "wi = wo * (-1.0 / etap) + nn * (ci - ct);",
     "test_dielectric_lobe"),
    ("fresnel_parallel", "T rp = (etap * ci - ct) / (etap * ci + ct);", "T rp = (ci - etap * ct) / (ci + etap * ct);",
     "test_dielectric_fresnel_fixed_points"),
    ("radiance_eta", "weight[c] = T(1.0 / (etap * etap));", "weight[c] = T(1.0);",
     "test_radiance_seen_from_inside_the_dielectric"),
    ("leaving_index", "const double etap = front ? m.eta : 1.0 / m.eta;", "const double etap = m.eta;",
     "test_glass_slab_branches"),
    ("mirror_schlick", "T one_m = 1.0 - ci;", "T one_m = ci;", "test_mirror_lobe"),
    ("delta_emission", "if (is_delta(m) && dot(nw2, vald(d)) < 0.0) {", "if (false) {", "test_mirror_plane_closed_form"),
    ("sampled_weight_max", "else w = std::min(Ea * C.P.dt, Eb / k);", "else w = std::max(Ea * C.P.dt, Eb / k);",
     "test_sampled_holding_weight_has_the_rao_blackwell_mean"),
    ("p_lambda_mean", "C.p_lambda_hat = sum / C.N;", "C.p_lambda_hat = sum;", "test_estimated_killing_constant"),
    ("sigma_coordinate", "C.sigma.empty() ? C.P.stddev : C.sigma[ii[k]]", "C.sigma.empty() ? C.P.stddev : C.sigma[i0]",
     "test_per_chain_diagonal_sigma_lyapunov"),
    ("estimator_scale", "(double)npx * C->k0 / (double)C->tour_count", "C->k0 / (double)C->tour_count",
     "test_restore_image_tends_to_path_tracing"),
]


@pytest.mark.slow
@pytest.mark.parametrize("mid,orig,bad,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_mutant(mid, orig, bad, pin):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation site for {mid} not found exactly once"
    d = tempfile.mkdtemp()
    cpp = os.path.join(d, "oracle_mut.cpp")
    so = os.path.join(d, "liboracle_mut.so")
    open(cpp, "w").write(src.replace(orig, bad))
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-pthread", cpp, "-o", so])
    env = dict(os.environ, DR_ORACLE_LIB=so, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", pin],
                       env=env, capture_output=True, text=True, timeout=600)
    assert "passed" in r.stdout or "failed" in r.stdout, r.stdout + r.stderr
    assert r.returncode != 0, f"mutant {mid} was not caught by {pin}:\n{r.stdout[-2000:]}"
