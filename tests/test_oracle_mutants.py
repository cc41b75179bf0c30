"""The pins must pin: plant one plausible mistake at a time (a dropped term, a
wrong sign or index, a transposed operand) in a copy of the oracle's source,
build it, and check that at least one of the named pins fails on it.  The
planted mistakes live only in temporary copies, on the CPU."""
import os
import tempfile

import pytest

import oracle
from oracle import build as obuild

import test_oracle_lsmc as TL
import test_oracle_model as TM
import test_oracle_qe as TQ
import test_oracle_rng as TR

# (name, exact source text, its replacement, pins expected to catch it)
MUTANTS = [
    ("philox-swapped-high-words", "uint32_t n0 = hi1 ^ c1 ^ k0;", "uint32_t n0 = hi0 ^ c1 ^ k0;",
     [TR.test_philox_matches_rocrand]),
    ("philox-key-not-bumped", "k1 += PHILOX_W1;", "k1 += 0u;", [TR.test_philox_matches_rocrand]),
    ("uniform-even-grid", "uint32_t odd = 2u * (w >> 9) + 1u;", "uint32_t odd = 2u * (w >> 9);",
     [TR.test_uniform_map_exact]),
    ("box-muller-sin-cos-swapped", "out[0] = R * cos(a);\n    out[1] = R * sin(a);",
     "out[0] = R * sin(a);\n    out[1] = R * cos(a);", [TR.test_box_muller_high_precision]),
    ("box-muller-missing-factor-2", "double R = sqrt(-2.0 * log(u1));",
     "double R = sqrt(-log(u1));", [TR.test_box_muller_high_precision]),
    ("counter-step-block-swapped", "uint32_t ctr[4] = {(uint32_t)((uint64_t)p), (uint32_t)k, (uint32_t)j,",
     "uint32_t ctr[4] = {(uint32_t)((uint64_t)p), (uint32_t)j, (uint32_t)k,",
     [TR.test_normals_counter_layout]),
    ("pair-words-misassigned", "orc_normal_pair(w[2], w[3], z);", "orc_normal_pair(w[1], w[2], z);",
     [TR.test_normals_counter_layout]),
    ("cholesky-transposed-operand", "for (int k = 0; k < j; ++k) s -= L[i * N + k] * L[j * N + k];",
     "for (int k = 0; k < j; ++k) s -= L[i * N + k] * L[k * N + j];",
     [TM.test_cholesky_matches_numpy]),
    ("correlation-transposed-L", "for (int b = 0; b <= a; ++b) z += L[a * N + b] * eps[b];",
     "for (int b = 0; b <= a; ++b) z += L[b * N + a] * eps[b];",
     [TM.test_stulz_pairs_of_correlated_assets]),
    ("variance-noise-without-sqrt(1-rho^2)-term",
     "double Zv = rho * ZS[a] + sqrt(1.0 - rho * rho) * eta[a];", "double Zv = rho * ZS[a];",
     [lambda: TM.test_european_heston_semi_closed_form(0.04, 2.0, 0.04, 0.3, -0.7, (80.0, 100.0, 120.0)),
      lambda: TM.test_european_heston_semi_closed_form(0.06, 3.0, 0.06, 0.5, 0.0, (60.0, 75.0, 100.0))]),
    ("rho-sign-flipped", "double Zv = rho * ZS[a] + sqrt(1.0 - rho * rho) * eta[a];",
     "double Zv = -rho * ZS[a] + sqrt(1.0 - rho * rho) * eta[a];",
     [lambda: TM.test_european_heston_semi_closed_form(0.04, 2.0, 0.04, 0.3, -0.7, (80.0, 100.0, 120.0)),
      lambda: TM.test_european_heston_semi_closed_form(0.06, 3.0, 0.06, 0.5, 0.0, (60.0, 75.0, 100.0))]),
    ("ito-correction-dropped", "X[a] = X[a] + (m->r - 0.5 * vp) * dt + sq * ZS[a];",
     "X[a] = X[a] + (m->r) * dt + sq * ZS[a];", [TM.test_martingale_with_vol_of_vol]),
    ("rate-drift-dropped", "X[a] = X[a] + (m->r - 0.5 * vp) * dt + sq * ZS[a];",
     "X[a] = X[a] + (-0.5 * vp) * dt + sq * ZS[a];", [TM.test_martingale_with_vol_of_vol]),
    ("mean-reversion-sign", "v[a] = v[a] + m->kappa[a] * (m->theta[a] - vp) * dt",
     "v[a] = v[a] + m->kappa[a] * (vp - m->theta[a]) * dt", [TM.test_variance_recurrence_closed_form]),
    ("vol-of-vol-dropped", "+ m->xi[a] * sq * Zv;", "+ 0.0 * sq * Zv;",
     [lambda: TM.test_european_heston_semi_closed_form(0.04, 2.0, 0.04, 0.3, -0.7, (80.0, 100.0, 120.0)),
      lambda: TM.test_european_heston_semi_closed_form(0.06, 3.0, 0.06, 0.5, 0.0, (60.0, 75.0, 100.0))]),
    ("no-truncation-in-diffusion", "double sq = sqrt(vp * dt);", "double sq = sqrt(fabs(v[a]) * dt);",
     [TM.test_martingale_with_vol_of_vol]),
    ("min-instead-of-max", "if (S > U) U = S;", "if (S > U || U == -INFINITY) U = (U == -INFINITY || S < U) ? S : U;",
     [TM.test_stulz_pairs_of_correlated_assets]),
    ("variance-feature-untruncated", "sv += v[a] > 0.0 ? v[a] : 0.0;", "sv += v[a];",
     [TM.test_variance_feature_is_truncated]),
    ("put-call-swapped", "double h = (cp == ORC_PUT) ? K - U : U - K;",
     "double h = (cp == ORC_PUT) ? U - K : K - U;", [TM.test_european_black_scholes_limit]),
    ("regression-includes-zero-payoff", "if (!(payoff(cp, K, U) > 0.0)) continue;\n                    basis(m, U, A, cU, cA, K, theta_bar, phi);\n                    double Y",
     "basis(m, U, A, cU, cA, K, theta_bar, phi);\n                    double Y",
     [lambda: TL.test_sweep_matches_lstsq_reference("put1", 64)]),
    ("exercise-inequality-reversed", "if (h > cont) {", "if (h < cont) {",
     [lambda: TL.test_bermudan_put_vs_crr_tree(36.0, 40.0, 0.06, 50)]),
    ("continuation-discounted-from-0", "double Y = CF[p] * exp(-r * (double)(tau[p] - k) * dt);",
     "double Y = CF[p] * exp(-r * (double)(tau[p]) * dt);",
     [lambda: TL.test_sweep_matches_lstsq_reference("put1", 256)]),
    ("basis-square-term-wrong", "phi[2] = x * x;", "phi[2] = x * x * x;",
     [lambda: TL.test_sweep_matches_lstsq_reference("put1", 256)]),
    ("basis-cross-term-wrong", "phi[4] = x * w;", "phi[4] = x * x * w;",
     [lambda: TL.test_sweep_matches_lstsq_reference("bestof3", 256)]),
    ("price-not-discounted", "for (int64_t p = c * ORC_CHUNK; p < pend; ++p) a1 += CF[p] * exp(-r * (double)tau[p] * dt);",
     "for (int64_t p = c * ORC_CHUNK; p < pend; ++p) a1 += CF[p];",
     [TM.test_european_black_scholes_limit]),
    ("se-wrong-denominator", "out[1] = sqrt(s2 / (double)(P - 1) / (double)P);\n    if (tau_out)",
     "out[1] = sqrt(s2 / (double)(P - 1));\n    if (tau_out)",
     [lambda: TL.test_sweep_matches_lstsq_reference("put1", 64)]),
    ("delta-half-width", "delta[i] = (up - dn) / (2.0 * hs);", "delta[i] = (up - dn) / hs;",
     [TL.test_greeks_black_scholes_limit]),
    ("gamma-wrong-scale", "gamma[i] = (up - 2.0 * V + dn) / (hs * hs);",
     "gamma[i] = (up - 2.0 * V + dn) / (2.0 * hs * hs);", [TL.test_greeks_black_scholes_limit]),
    ("vega-absolute-bump", "vega[i] = (prices[s + i] - V) / (v0_rel * v0[i]);",
     "vega[i] = (prices[s + i] - V) / v0_rel;", [TL.test_greeks_black_scholes_limit]),
    ("theta-sign", "*theta = (prices[s] - V) / T_abs;", "*theta = (V - prices[s]) / T_abs;",
     [TL.test_greeks_black_scholes_limit]),
    ("spot-down-bumped-up", "S0[idx - N] = q->S0[idx - N] * (1.0 - q->spot_rel);",
     "S0[idx - N] = q->S0[idx - N] * (1.0 + q->spot_rel);",
     [TL.test_greeks_black_scholes_limit, TL.test_scenario_count_and_order]),
    ("corr-bump-one-sided", "C[i * N + j] += q->corr_abs;\n                            C[j * N + i] += q->corr_abs;",
     "C[i * N + j] += q->corr_abs;", [TL.test_correlation_greek_vs_stulz]),
    ("rate-bump-ignored", "if (idx == 0) { r = q->r + q->r_abs; done = 1; }",
     "if (idx == 0) { r = q->r; done = 1; }", [TL.test_greeks_black_scholes_limit]),
    # Andersen QE step
    ("qe-b2-sign", "const double b2 = t - 1.0 + sqrt(t) * sqrt(t - 1.0);",
     "const double b2 = t - 1.0 - sqrt(t) * sqrt(t - 1.0);",
     [lambda: TQ.test_variance_step_matches_cir_moments(0.09)]),
    ("qe-a-without-b2", "const double a = m / (1.0 + b2);", "const double a = m / b2;",
     [lambda: TQ.test_variance_step_matches_cir_moments(0.09)]),
    ("qe-p-inverted", "const double p = (psi - 1.0) / (psi + 1.0);",
     "const double p = (psi + 1.0) / (psi - 1.0) - 1.0;",
     [lambda: TQ.test_variance_step_matches_cir_moments(0.0005)]),
    ("qe-beta-upside-down", "const double beta = (1.0 - p) / m;", "const double beta = m / (1.0 - p);",
     [lambda: TQ.test_variance_step_matches_cir_moments(0.0005)]),
    ("qe-s2-second-term-dropped", "q->c2 = 0.5 * theta * xi * xi * (1.0 - E) * f;", "q->c2 = 0.0;",
     [lambda: TQ.test_variance_step_matches_cir_moments(0.0)]),
    ("qe-mean-reverts-to-zero", "q->mth = theta * (1.0 - E);", "q->mth = 0.0;",
     [TQ.test_zero_vol_of_vol_is_deterministic]),
    ("qe-trapezoid-one-sided", "q->K3 = g1 * dt * (1.0 - rho * rho);", "q->K3 = 2.0 * g1 * dt * (1.0 - rho * rho);",
     [TQ.test_time_dependent_variance]),
    ("qe-rho-sign", "const double rx = xi > 0.0 ? rho / xi : 0.0;", "const double rx = xi > 0.0 ? -rho / xi : 0.0;",
     [lambda: TQ.test_heston_semi_closed_form(0.04, 2.0, 0.04, 0.3, -0.7, (80.0, 100.0, 120.0))]),
    ("qe-kappa-term-in-K2-dropped", "q->K2 = g2 * dt * (kappa * rx - 0.5) + rx;",
     "q->K2 = g2 * dt * (-0.5) + rx;",
     [lambda: TQ.test_heston_semi_closed_form(0.04, 1.0, 0.04, 1.0, -0.5, (70.0, 100.0, 130.0))]),
    ("qe-independent-variance-shocks",
     "const double Zv = rho * ZS[a] + rhobar * eta[a];\n            const double Zx = rhobar * ZS[a] - rho * eta[a];",
     "const double Zv = eta[a];\n            const double Zx = ZS[a];",
     [lambda: TQ.test_joint_law_of_one_step("qe")]),
    ("qe-orthogonal-part-sign", "const double Zx = rhobar * ZS[a] - rho * eta[a];",
     "const double Zx = rhobar * ZS[a] + rho * eta[a];",
     [lambda: TQ.test_joint_law_of_one_step("qe")]),
    ("qe-uniform-from-wrong-tail", "const double u = 0.5 * erfc(-zv / sqrt(2.0));",
     "const double u = 0.5 * erfc(zv / sqrt(2.0));",
     [lambda: TQ.test_variance_step_matches_cir_moments(0.0005), TQ.test_variance_step_branches]),
]


@pytest.fixture(scope="module")
def source():
    with open(obuild.SRC) as f:
        return f.read()


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(source, name, old, new, pins):
    assert source.count(old) == 1, "mutation anchor not unique for " + name
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "mutant.c")
        with open(src, "w") as f:
            f.write(source.replace(old, new))
        lib = obuild.build(src=src, out=os.path.join(d, "libmutant.so"))
        caught = []
        with oracle.use_library(lib):
            for pin in pins:
                try:
                    pin()
                except (AssertionError, ValueError, FloatingPointError) as e:
                    caught.append(repr(e)[:80])
    assert caught, "no pin caught mutant " + name
