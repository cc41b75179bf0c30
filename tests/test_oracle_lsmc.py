"""Pins of the oracle's Longstaff-Schwartz sweep, pricing and Greeks: an
independent numpy sweep whose regressions use numpy.linalg.lstsq, the
Bermudan CRR tree in the Black-Scholes limit, the never-early-exercised
call, Black-Scholes and Stulz Greeks, decision replay and degenerate cases."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from _refs import (bs_delta, bs_gamma, bs_price, crr_bermudan_put, numpy_lsmc,
                   stulz_max_call)


def _model(S0, v0, kappa, theta, xi, rho, r):
    f = lambda x: np.atleast_1d(np.asarray(x, dtype=np.float64))
    return {"S0": f(S0), "v0": f(v0), "kappa": f(kappa), "theta": f(theta), "xi": f(xi),
            "rho": f(rho), "r": float(r)}


@pytest.mark.parametrize("case", ["put1", "bestof3", "bestof5_quad"])
@pytest.mark.parametrize("P", [16, 64, 256])
def test_sweep_matches_lstsq_reference(case, P):
    if case == "put1":
        w = W.single_asset_put(n_paths=P, n_steps=24)
        m = 3
    elif case == "bestof3":
        w = W.best_of_call(n_assets=3, n_paths=P, n_steps=24)
        m = 5
    else:
        w = W.best_of_call(n_assets=5, n_paths=P, n_steps=24)
        w["option"]["basis"] = "quad"
        m = 3
    f = oracle.features(w["model"], w["corr"], 1.0, 24, P, 42)
    tb = float(np.mean(w["model"]["theta"]))
    o = oracle.lsmc(f, w["option"], w["model"]["r"], tb, m)
    ref = numpy_lsmc(f, w["option"]["K"], w["model"]["r"], 1.0, w["option"]["cp"], m, tb)
    assert np.array_equal(o["tau"], ref["tau"])
    assert o["skipped"] == ref["skipped"]
    assert abs(o["price"] - ref["price"]) <= 1e-13 * abs(ref["price"])
    assert abs(o["se"] - ref["se"]) <= 1e-10 * ref["se"]


@pytest.mark.parametrize("S0,K,r,n", [(36.0, 40.0, 0.06, 50), (100.0, 100.0, 0.06, 25)])
def test_bermudan_put_vs_crr_tree(S0, K, r, n):
    # Black-Scholes limit (vol-of-vol 0, v0 = theta): LSMC with the quadratic
    # basis recovers most of the early-exercise premium of the tree price with
    # exercise at the same dates, and never exceeds it beyond the MC error
    P = 200000
    w = W.gbm_limit_put(S0=S0, K=K, r=r, n_paths=P, n_steps=n, seed=3)
    f = oracle.features(w["model"], w["corr"], 1.0, n, P, 3)
    o = oracle.lsmc(f, w["option"], r, 0.04, 3)
    tree = crr_bermudan_put(S0, K, r, 0.2, 1.0, n)
    eu = bs_price(S0, K, r, 0.2, 1.0, "put")
    assert o["price"] < tree + 4 * o["se"]
    assert o["price"] - eu > 0.85 * (tree - eu) - 4 * o["se"]
    assert o["skipped"] == 0


def test_american_call_not_exercised_early():
    # no dividends: early exercise of a call never pays, so the LSMC price on
    # the same paths equals the European one up to the MC error
    P = 100000
    m = _model(100, 0.04, 2.0, 0.04, 0.3, -0.7, 0.03)
    f = oracle.features(m, np.eye(1), 1.0, 32, P, 17)
    am = oracle.lsmc(f, {"cp": "call", "style": "american", "K": 100.0, "T": 1.0}, 0.03, 0.04, 3)
    eu = oracle.lsmc(f, {"cp": "call", "style": "european", "K": 100.0, "T": 1.0}, 0.03, 0.04, 3)
    assert abs(am["price"] - eu["price"]) < 2 * eu["se"]


def test_best_of_two_american_call_vs_stulz():
    P = 100000
    C = np.array([[1.0, 0.4], [0.4, 1.0]])
    m = _model([100.0, 95.0], [0.04, 0.09], [1.0, 1.0], [0.04, 0.09], [0.0, 0.0], [0.0, 0.0],
               0.02)
    f = oracle.features(m, C, 1.0, 20, P, 19)
    am = oracle.lsmc(f, {"cp": "call", "style": "american", "K": 100.0, "T": 1.0}, 0.02, 0.065, 3)
    ref = stulz_max_call(100.0, 95.0, 100.0, 0.02, 0.2, 0.3, 0.4, 1.0)
    assert abs(am["price"] - ref) < 4 * am["se"]


def test_replay_reproduces_price():
    w = W.best_of_call(n_assets=4, n_paths=3000, n_steps=30)
    f = oracle.features(w["model"], w["corr"], 1.0, 30, 3000, 42)
    tb = float(np.mean(w["model"]["theta"]))
    o = oracle.lsmc(f, w["option"], 0.02, tb, 5)
    v, se = oracle.replay(f, w["option"], 0.02, o["tau"])
    assert abs(v - o["price"]) <= 1e-14 * o["price"]
    assert abs(se - o["se"]) <= 1e-12 * o["se"]
    # replaying "always hold to maturity" gives the European price
    eu = oracle.lsmc(f, dict(w["option"], style="european"), 0.02, tb, 5)
    v, _ = oracle.replay(f, w["option"], 0.02, np.full(3000, 30, dtype=np.int32))
    assert abs(v - eu["price"]) <= 1e-14 * eu["price"]


def test_all_out_of_the_money():
    w = W.single_asset_put(n_paths=512, n_steps=16)
    w["option"]["K"] = 1.0
    f = oracle.features(w["model"], w["corr"], 1.0, 16, 512, 42)
    o = oracle.lsmc(f, w["option"], 0.02, 0.04, 3)
    assert o["price"] == 0.0 and o["se"] == 0.0
    assert o["skipped"] == 15
    assert np.all(o["tau"] == 16)


def test_too_few_regression_paths_skip():
    # P = 2 < m: every date is skipped, the price is the European one
    w = W.single_asset_put(n_paths=2, n_steps=8)
    f = oracle.features(w["model"], w["corr"], 1.0, 8, 2, 42)
    o = oracle.lsmc(f, w["option"], 0.02, 0.04, 3)
    eu = oracle.lsmc(f, dict(w["option"], style="european"), 0.02, 0.04, 3)
    assert o["skipped"] == 7 and o["price"] == eu["price"]


def test_single_date():
    w = W.single_asset_put(n_paths=1000, n_steps=1)
    f = oracle.features(w["model"], w["corr"], 1.0, 1, 1000, 42)
    o = oracle.lsmc(f, w["option"], 0.02, 0.04, 3)
    ref = np.maximum(100.0 - f[0, :, 0], 0.0).mean() * math.exp(-0.02)
    assert abs(o["price"] - ref) <= 1e-14 * ref and o["skipped"] == 0


def test_greeks_black_scholes_limit():
    # European put, vol-of-vol 0, v0 = theta: every Greek against Black-Scholes
    P, n, kap = 200000, 16, 1.5
    w = W.gbm_limit_put(n_paths=P, n_steps=n, seed=4, style="european")
    b = W.default_bumps(W.MASK_ALL)
    g = oracle.price_greeks(w["model"], w["corr"], w["option"], P, n, b, 4)
    bs = lambda **kw: bs_price(kw.get("S", 100.0), 100.0, kw.get("r", 0.02), kw.get("s", 0.2),
                               kw.get("T", 1.0), "put")
    assert abs(g["price"] - bs()) < 4 * g["price_se"]
    assert abs(g["delta"][0] - bs_delta(100, 100, 0.02, 0.2, 1.0, "put")) < 0.004
    assert abs(g["gamma"][0] / bs_gamma(100, 100, 0.02, 0.2, 1.0) - 1.0) < 0.06
    dT = b["T_abs"]
    assert abs(g["theta"] / ((bs(T=1.0 - dT) - bs()) / dT) - 1.0) < 0.02
    assert abs(g["rho"] / ((bs(r=0.021) - bs()) / 1e-3) - 1.0) < 0.02
    # vega w.r.t. v0: sigma_eff^2 T = sum_k v_k dt with v_k = theta + (v0 - theta)(1 - kappa dt)^k
    v0b = 0.04 * 1.01
    vk = 0.04 + (v0b - 0.04) * (1 - kap / n) ** np.arange(n)
    seff = math.sqrt(vk.sum() / n)
    assert abs(g["vega"][0] / ((bs(s=seff) - bs()) / (0.01 * 0.04)) - 1.0) < 0.03
    assert np.all(g["skipped"] == 0)


def test_correlation_greek_vs_stulz():
    P = 200000
    C = np.array([[1.0, 0.4], [0.4, 1.0]])
    m = _model([100.0, 95.0], [0.04, 0.09], [1.0, 1.0], [0.04, 0.09], [0.0, 0.0], [0.0, 0.0],
               0.02)
    opt = {"cp": "call", "style": "european", "underlying": "max_of", "basis": "quad",
           "K": 100.0, "T": 1.0}
    b = W.default_bumps(W.MASK_CORR)
    g = oracle.price_greeks(m, C, opt, P, 4, b, 23)
    ref = (stulz_max_call(100.0, 95.0, 100.0, 0.02, 0.2, 0.3, 0.41, 1.0)
           - stulz_max_call(100.0, 95.0, 100.0, 0.02, 0.2, 0.3, 0.40, 1.0)) / 0.01
    assert g["n_scenarios"] == 2
    assert abs(g["corr"][0] / ref - 1.0) < 0.05


def test_scenario_count_and_order():
    for N, mask, S in [(1, 1, 3), (5, 31, 28), (10, 31, 78), (20, 31, 253), (1, 31, 6),
                       (3, 16, 4), (4, 2 | 8, 6)]:
        assert oracle.num_scenarios(N, mask) == S
    # order: base, spot+, spot-, v0, T, r, corr -- a call's price rises with spot
    w = W.best_of_call(n_assets=3, n_paths=4000, n_steps=12)
    w["option"]["style"] = "european"
    g = oracle.price_greeks(w["model"], w["corr"], w["option"], 4000, 12, w["bumps"], 42)
    p = g["scenario_price"]
    assert np.all(p[1:4] > p[0]) and np.all(p[4:7] < p[0])
    assert p[10] < p[0]            # shorter maturity
    assert p[11] > p[0]            # higher rate, call


def test_bumped_correlation_not_spd_rejected():
    w = W.best_of_call(n_assets=2, n_paths=64, n_steps=4)
    w["corr"] = np.array([[1.0, 0.995], [0.995, 1.0]])
    with pytest.raises(ValueError):
        oracle.price_greeks(w["model"], w["corr"], w["option"], 64, 4, w["bumps"], 42)
