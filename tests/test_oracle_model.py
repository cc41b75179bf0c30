"""Pins of the oracle's path generator and path reduction against closed forms
and invariants: Cholesky, the deterministic variance recurrence, the
martingale property, Black-Scholes and Heston (1993) European prices, the
Stulz two-asset max-call, pathwise put-call parity, common random numbers and
thread-count invariance."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from _refs import bs_price, heston_price, stulz_max_call


def _model(S0, v0, kappa, theta, xi, rho, r):
    f = lambda x: np.atleast_1d(np.asarray(x, dtype=np.float64))
    return {"S0": f(S0), "v0": f(v0), "kappa": f(kappa), "theta": f(theta), "xi": f(xi),
            "rho": f(rho), "r": float(r)}


def _euro(feat, K, r, T, cp):
    opt = {"cp": cp, "style": "european", "K": K, "T": T}
    out = oracle.lsmc(feat, opt, r, 1.0, 3)
    return out["price"], out["se"]


def test_cholesky_matches_numpy():
    rng = np.random.default_rng(0)
    for N in (1, 2, 5, 10, 20):
        _, C = W.draw_assets(N, rng)
        L = oracle.cholesky(C)
        assert np.allclose(L, np.linalg.cholesky(C), rtol=0, atol=1e-14)
        assert np.abs(L @ L.T - C).max() <= 1e-14
        assert np.all(np.triu(L, 1) == 0.0)


def test_cholesky_rejects_non_spd():
    C = np.array([[1.0, 0.9, 0.9], [0.9, 1.0, -0.9], [0.9, -0.9, 1.0]])
    with pytest.raises(ValueError):
        oracle.cholesky(C)
    with pytest.raises(ValueError):
        oracle.features(_model([100] * 3, [0.04] * 3, [1] * 3, [0.04] * 3, [0.3] * 3, [0] * 3,
                               0.02), C, 1.0, 4, 8, 1)


def test_variance_recurrence_closed_form():
    # vol-of-vol 0: v_k = theta + (v0 - theta)(1 - kappa dt)^k (deterministic,
    # never truncated); A is the mean over assets of v_k
    n, T = 50, 2.0
    dt = T / n
    kap = np.array([1.5, 3.0, 0.7])
    th = np.array([0.04, 0.09, 0.02])
    v0 = np.array([0.09, 0.01, 0.05])
    m = _model([100, 90, 110], v0, kap, th, [0, 0, 0], [-0.5, 0.2, 0.0], 0.03)
    f = oracle.features(m, np.eye(3), T, n, 16, 3)
    k = np.arange(1, n + 1)[:, None]
    vk = th[None, :] + (v0 - th)[None, :] * (1.0 - kap[None, :] * dt) ** k
    ref = vk.mean(axis=1)
    assert np.allclose(f[:, :, 1], ref[:, None], rtol=1e-13, atol=0)


def test_variance_fixed_point_bitwise():
    m = _model(100, 0.04, 2.0, 0.04, 0.0, -0.7, 0.02)
    f = oracle.features(m, np.eye(1), 1.0, 64, 32, 42)
    assert np.all(f[:, :, 1] == 0.04)


def test_variance_feature_is_truncated():
    # vol-of-vol far beyond the Feller bound drives v negative often; the
    # feature is the mean of max(v, 0), so it is never negative, and it is
    # exactly 0 at dates where every asset's variance is at or below 0
    m = _model([100, 100], [0.02, 0.02], [0.5, 0.5], [0.02, 0.02], [1.5, 1.5], [-0.5, -0.5],
               0.02)
    f = oracle.features(m, np.eye(2), 1.0, 100, 2000, 9)
    A = f[:, :, 1]
    assert np.all(A >= 0.0)
    assert np.mean(A == 0.0) > 0.05


def test_martingale_with_vol_of_vol():
    # E[exp(-r t_k) S_k] = S0 at every date (the scheme is an exact discrete
    # martingale: v+ at step k is independent of that step's normals)
    m = _model(100, 0.04, 2.0, 0.04, 0.6, -0.7, 0.05)
    T, n, P = 1.0, 32, 200000
    f = oracle.features(m, np.eye(1), T, n, P, 11)
    for k in (1, 8, 32):
        d = f[k - 1, :, 0] * math.exp(-0.05 * k * T / n)
        se = d.std(ddof=1) / math.sqrt(P)
        assert abs(d.mean() - 100.0) < 4.0 * se, (k, d.mean(), se)


def test_european_black_scholes_limit():
    # vol-of-vol 0, v0 = theta: lognormal with sigma^2 = theta
    for K in (85.0, 100.0, 115.0):
        m = _model(100, 0.04, 2.0, 0.04, 0.0, 0.0, 0.02)
        f = oracle.features(m, np.eye(1), 1.0, 16, 100000, 5)
        for cp in ("put", "call"):
            v, se = _euro(f, K, 0.02, 1.0, cp)
            assert abs(v - bs_price(100, K, 0.02, 0.2, 1.0, cp)) < 4 * se


def test_european_time_dependent_variance():
    # vol-of-vol 0, v0 != theta: log-Euler is exact for the deterministic
    # variance path, so S_T is lognormal with sigma_eff^2 T = sum_k v_k dt
    n, T, kap, th, v0 = 20, 1.5, 2.5, 0.03, 0.10
    dt = T / n
    vk = th + (v0 - th) * (1 - kap * dt) ** np.arange(n)
    sig = math.sqrt(vk.sum() * dt / T)
    m = _model(100, v0, kap, th, 0.0, 0.3, 0.01)
    f = oracle.features(m, np.eye(1), T, n, 100000, 8)
    v, se = _euro(f, 105.0, 0.01, T, "call")
    assert abs(v - bs_price(100, 105.0, 0.01, sig, T, "call")) < 4 * se


@pytest.mark.slow
@pytest.mark.parametrize("v0,kappa,theta,xi,rho,strikes", [
    # the single-asset put's model: the skew pins rho's sign
    (0.04, 2.0, 0.04, 0.3, -0.7, (80.0, 100.0, 120.0)),
    # rho = 0: all variance noise comes from the independent sqrt(1 - rho^2) term
    (0.06, 3.0, 0.06, 0.5, 0.0, (60.0, 75.0, 100.0)),
])
def test_european_heston_semi_closed_form(v0, kappa, theta, xi, rho, strikes):
    m = _model(100, v0, kappa, theta, xi, rho, 0.02)
    P = 200000
    f64 = oracle.features(m, np.eye(1), 1.0, 64, P, 21)
    f128 = oracle.features(m, np.eye(1), 1.0, 128, P, 21)
    for K in strikes:
        ref = heston_price(100, K, v0, kappa, theta, xi, rho, 0.02, 1.0, "put")
        v64, _ = _euro(f64, K, 0.02, 1.0, "put")
        v128, se = _euro(f128, K, 0.02, 1.0, "put")
        bias = abs(v64 - v128)
        assert abs(v128 - ref) < 4 * se + 2 * bias, (K, v128, ref, se, bias)
    # the wing is far from the Black-Scholes price at the same variance
    K = strikes[0]
    vw, sew = _euro(f128, K, 0.02, 1.0, "put")
    assert abs(vw - bs_price(100, K, 0.02, math.sqrt(theta), 1.0, "put")) > 20 * sew


def test_stulz_pairs_of_correlated_assets():
    # vol-of-vol 0: for each pair (i, j) of a 4-asset model, make the other two
    # assets negligible; the best-of call is then Stulz's two-asset max-call
    # with correlation C_ij, pinning every pair of the Cholesky construction
    C = np.array([[1.0, 0.6, -0.3, 0.2], [0.6, 1.0, 0.1, 0.5], [-0.3, 0.1, 1.0, -0.4],
                  [0.2, 0.5, -0.4, 1.0]])
    sig2 = np.array([0.04, 0.09, 0.0625, 0.0225])
    T, r, K = 1.0, 0.03, 100.0
    for i, j in [(0, 1), (0, 2), (1, 3), (2, 3)]:
        S0 = np.full(4, 1e-3)
        S0[i], S0[j] = 100.0, 95.0
        m = _model(S0, sig2, [1.0] * 4, sig2, [0.0] * 4, [0.0] * 4, r)
        f = oracle.features(m, C, T, 4, 100000, 13)
        v, se = _euro(f, K, r, T, "call")
        ref = stulz_max_call(100.0, 95.0, K, r, math.sqrt(sig2[i]), math.sqrt(sig2[j]), C[i, j], T)
        assert abs(v - ref) < 4 * se, (i, j, v, ref, se)


def test_put_call_parity_pathwise():
    m = _model([100, 105, 95], [0.05, 0.03, 0.08], [2, 1, 3], [0.05, 0.04, 0.06],
               [0.5, 0.3, 0.4], [-0.7, -0.4, -0.6], 0.02)
    C = W.one_factor_corr([0.5, 0.6, 0.55])
    f = oracle.features(m, C, 1.0, 12, 5000, 3)
    K, r, T = 102.0, 0.02, 1.0
    c, _ = _euro(f, K, r, T, "call")
    p, _ = _euro(f, K, r, T, "put")
    ref = math.exp(-r * T) * (f[-1, :, 0].mean() - K)
    assert abs((c - p) - ref) <= 1e-12 * max(abs(ref), c)


def test_common_random_numbers_spot_bump():
    # X is accumulated from 0 and does not depend on S0: a spot-bumped
    # scenario's underlying is the base one times (1 + h), to rounding
    m = _model(100, 0.04, 2.0, 0.04, 0.3, -0.7, 0.02)
    mb = dict(m, S0=np.array([101.0]))
    f = oracle.features(m, np.eye(1), 1.0, 64, 256, 42)
    fb = oracle.features(mb, np.eye(1), 1.0, 64, 256, 42)
    assert np.allclose(fb[:, :, 0] / f[:, :, 0], 1.01, rtol=4e-16, atol=0)
    assert np.array_equal(fb[:, :, 1], f[:, :, 1])


def test_thread_count_invariance():
    w = W.best_of_call(n_assets=3, n_paths=9000, n_steps=10)
    f1 = oracle.features(w["model"], w["corr"], 1.0, 10, 9000, 42, nthreads=1)
    f8 = oracle.features(w["model"], w["corr"], 1.0, 10, 9000, 42, nthreads=8)
    assert np.array_equal(f1, f8)
    tb = float(np.mean(w["model"]["theta"]))
    a = oracle.lsmc(f1, w["option"], 0.02, tb, 5, nthreads=1)
    b = oracle.lsmc(f1, w["option"], 0.02, tb, 5, nthreads=8)
    assert a["price"] == b["price"] and a["se"] == b["se"]
    assert np.array_equal(a["tau"], b["tau"])


def test_features_at_equals_features():
    # single paths of a run (used to check sampled paths of full-size GPU runs)
    w = W.best_of_call(n_assets=4, n_paths=700, n_steps=9)
    f = oracle.features(w["model"], w["corr"], 1.0, 9, 700, 42)
    idx = [0, 1, 63, 64, 350, 699]
    g = oracle.features_at(w["model"], w["corr"], 1.0, 9, idx, 42)
    for i, p in enumerate(idx):
        assert np.array_equal(g[i], f[:, p])
