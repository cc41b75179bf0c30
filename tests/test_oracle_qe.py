"""Pins of the oracle's Andersen quadratic-exponential (QE) step.

- One variance step has the exact conditional mean and variance of the CIR
  process (the textbook moments, integrated over the normal input with
  quadrature, split at the exponential branch's mass point), in both
  branches and across the switch.
- Vol of vol 0: the variance path is the deterministic CIR mean, and the
  trapezoid-variance log step makes S_T lognormal: Black-Scholes prices.
- Vol of vol > 0: the Heston (1993) semi-closed form within 4 SE plus the
  time-step bias; the discounted spot is a martingale within the same bar.
- The variance never goes negative, so the path reduction's A is the plain mean."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from _refs import bs_price, heston_price


def _model(S0, v0, kappa, theta, xi, rho, r):
    f = lambda x: np.atleast_1d(np.asarray(x, dtype=np.float64))
    return {"S0": f(S0), "v0": f(v0), "kappa": f(kappa), "theta": f(theta), "xi": f(xi),
            "rho": f(rho), "r": float(r)}


def _euro(feat, K, r, T, cp):
    opt = {"cp": cp, "style": "european", "K": K, "T": T}
    out = oracle.lsmc(feat, opt, r, 1.0, 3)
    return out["price"], out["se"]


def cir_moments(v, kappa, theta, xi, dt):
    """Exact conditional mean and variance of the CIR variance after dt."""
    e = math.exp(-kappa * dt)
    mean = theta + (v - theta) * e
    var = v * xi ** 2 * e * (1 - e) / kappa + theta * xi ** 2 * (1 - e) ** 2 / (2 * kappa)
    return mean, var


def step_moments(kappa, theta, xi, dt, v):
    """E[v'] and Var[v'] of the oracle's step over Z ~ N(0, 1), by quadrature."""
    f = lambda z: oracle.qe_variance_step(kappa, theta, xi, 0.0, dt, v, z)
    # the exponential branch is flat (v' = 0) below Phi^-1(p): split there
    mean, var = cir_moments(v, kappa, theta, xi, dt)
    psi = var / mean ** 2
    pts = [stats.norm.ppf((psi - 1) / (psi + 1))] if psi > 1.5 else [0.0]
    out = []
    for k in (1, 2):
        g = lambda z: f(z) ** k * stats.norm.pdf(z)
        acc = 0.0
        edges = [-8.0] + pts + [8.0]  # the inputs are Box-Muller normals, |z| < 5.8
        for a, b in zip(edges[:-1], edges[1:]):
            acc += integrate.quad(g, a, b, limit=400, epsabs=0, epsrel=1e-12)[0]
        out.append(acc)
    return out[0], out[1] - out[0] ** 2


@pytest.mark.parametrize("v", [0.09, 0.04, 0.012, 0.004, 0.0005, 0.0])
def test_variance_step_matches_cir_moments(v):
    # xi = 0.6 and dt = 1/52: psi spans both branches as v shrinks
    kappa, theta, xi, dt = 1.5, 0.04, 0.6, 1.0 / 52
    m_ref, s2_ref = cir_moments(v, kappa, theta, xi, dt)
    m, s2 = step_moments(kappa, theta, xi, dt, v)
    assert abs(m - m_ref) <= 1e-9 * m_ref
    assert abs(s2 - s2_ref) <= 1e-7 * s2_ref


def test_variance_step_branches():
    kappa, theta, xi, dt = 1.5, 0.04, 0.6, 1.0 / 52
    # quadratic branch: v' = a (b + z)^2 >= 0 with its minimum 0 at z = -b
    vals = [oracle.qe_variance_step(kappa, theta, xi, 0.0, dt, 0.09, z)
            for z in np.linspace(-6, 6, 121)]
    assert min(vals) >= 0.0
    # exponential branch: exactly 0 below the mass point, increasing above
    m, s2 = cir_moments(0.0005, kappa, theta, xi, dt)
    psi = s2 / m ** 2
    assert psi > 1.5
    zp = stats.norm.ppf((psi - 1) / (psi + 1))
    assert oracle.qe_variance_step(kappa, theta, xi, 0.0, dt, 0.0005, zp - 0.01) == 0.0
    hi = [oracle.qe_variance_step(kappa, theta, xi, 0.0, dt, 0.0005, z)
          for z in np.linspace(zp + 0.01, 5, 50)]
    assert all(b > a for a, b in zip(hi, hi[1:]))


def test_zero_vol_of_vol_is_deterministic():
    kappa, theta, dt = 2.0, 0.04, 0.1
    for v in (0.0, 0.02, 0.04, 0.1):
        for z in (-3.0, 0.0, 2.0):
            got = oracle.qe_variance_step(kappa, theta, 0.0, 0.0, dt, v, z)
            assert got == pytest.approx(theta + (v - theta) * math.exp(-kappa * dt), rel=1e-15)


def test_black_scholes_limit():
    # xi = 0, rho = 0, v0 = theta: X' = X + (r - theta/2) dt + sqrt(theta dt) Z
    for K in (85.0, 100.0, 115.0):
        m = _model(100, 0.04, 2.0, 0.04, 0.0, 0.0, 0.02)
        f = oracle.features(m, np.eye(1), 1.0, 16, 100000, 5, scheme="qe")
        for cp in ("put", "call"):
            v, se = _euro(f, K, 0.02, 1.0, cp)
            assert abs(v - bs_price(100, K, 0.02, 0.2, 1.0, cp)) < 4 * se


def test_time_dependent_variance():
    # xi = 0, v0 != theta: v_k = theta + (v0 - theta) e^{-kappa k dt} exactly and
    # the log step uses the trapezoid of v, so sigma_eff^2 T = sum of
    # (v_k + v_{k+1}) dt / 2
    n, T, kap, th, v0 = 20, 1.5, 2.5, 0.03, 0.10
    dt = T / n
    vk = th + (v0 - th) * np.exp(-kap * dt * np.arange(n + 1))
    sig = math.sqrt(0.5 * (vk[:-1] + vk[1:]).sum() * dt / T)
    m = _model(100, v0, kap, th, 0.0, 0.0, 0.01)
    f = oracle.features(m, np.eye(1), T, n, 100000, 8, scheme="qe")
    v, se = _euro(f, 105.0, 0.01, T, "call")
    assert abs(v - bs_price(100, 105.0, 0.01, sig, T, "call")) < 4 * se
    # the variance feature is the deterministic path itself
    assert np.allclose(f[:, 0, 1], vk[1:], rtol=1e-14, atol=0)


@pytest.mark.slow
@pytest.mark.parametrize("v0,kappa,theta,xi,rho,strikes", [
    (0.04, 2.0, 0.04, 0.3, -0.7, (80.0, 100.0, 120.0)),
    # high vol of vol: the exponential branch carries much of the mass
    (0.04, 1.0, 0.04, 1.0, -0.5, (70.0, 100.0, 130.0)),
])
def test_heston_semi_closed_form(v0, kappa, theta, xi, rho, strikes):
    m = _model(100, v0, kappa, theta, xi, rho, 0.02)
    P = 200000
    f32 = oracle.features(m, np.eye(1), 1.0, 32, P, 21, scheme="qe")
    f64 = oracle.features(m, np.eye(1), 1.0, 64, P, 21, scheme="qe")
    for K in strikes:
        ref = heston_price(100, K, v0, kappa, theta, xi, rho, 0.02, 1.0, "put")
        v32, _ = _euro(f32, K, 0.02, 1.0, "put")
        v64, se = _euro(f64, K, 0.02, 1.0, "put")
        bias = abs(v32 - v64)
        assert abs(v64 - ref) < 4 * se + 2 * bias, (K, v64, ref, se, bias)
    # martingale: E[e^{-rT} S_T] = S0
    ST = f64[-1, :, 0]
    disc = math.exp(-0.02)
    mean = disc * ST.mean()
    se = disc * ST.std(ddof=1) / math.sqrt(P)
    assert abs(mean - 100.0) < 4 * se + 2 * abs(disc * (f32[-1, :, 0].mean() - ST.mean()))
    # QE variance never goes negative
    assert f64[:, :, 1].min() >= 0.0


def _three_assets():
    beta = np.array([0.75, 0.6, 0.5])
    C = np.outer(beta, beta)
    np.fill_diagonal(C, 1.0)
    m = _model([100.0, 95.0, 110.0], [0.04, 0.06, 0.05], [2.0, 1.5, 3.0], [0.04, 0.06, 0.05],
               [0.5, 0.4, 0.3], [-0.7, -0.5, -0.3], 0.02)
    return m, C


@pytest.mark.parametrize("scheme", ["euler", "qe"])
def test_joint_law_of_one_step(scheme):
    """One daily step from fixed (X, v) = (0, v0): the assets' log-price shocks
    correlate as C_ij, the variance shocks as rho_i rho_j C_ij, and the spot of
    asset i with the variance of asset j as rho_j C_ij (the continuous model's
    instantaneous correlations).  Bar: 4 standard errors of a sample
    correlation, (1 - c^2)/sqrt(P), plus 0.003 for the step's own departure
    from the instantaneous law (measured well below that: halving dt twice
    moves the estimates by < 5e-4)."""
    m, C = _three_assets()
    rho = m["rho"]
    P = 200000
    st = oracle.states(m, C, 1.0 / 252, 1, P, 11, scheme=scheme)
    Z = np.concatenate([st[:, :, 0], st[:, :, 1]], axis=1)  # X_0..2, v_0..2
    c = np.corrcoef(Z.T)
    N = 3
    for i in range(N):
        for j in range(N):
            vv = 1.0 if i == j else rho[i] * rho[j] * C[i, j]
            want = {"XX": C[i, j], "vv": vv, "Xv": rho[j] * C[i, j]}
            got = {"XX": c[i, j], "vv": c[N + i, N + j], "Xv": c[i, N + j]}
            for k in want:
                bar = 4 * (1 - want[k] ** 2) / math.sqrt(P) + 0.003
                assert abs(got[k] - want[k]) <= bar, (scheme, k, i, j, got[k], want[k])


@pytest.mark.slow
def test_multi_asset_qe_matches_euler_european():
    """Under the same joint law both schemes converge to one price as dt -> 0:
    a 5-asset European best-of call (the workload's draws) under QE and
    full-truncation Euler agree within 4 standard errors of their pathwise
    difference plus twice each scheme's time-step bias, estimated by halving
    dt."""
    import workloads as W
    w = W.best_of_call(5, 200000, 64)
    mod, C, K, T, r = w["model"], w["corr"], w["option"]["K"], 1.0, w["model"]["r"]
    P = 200000
    pay = {}
    for scheme in ("euler", "qe"):
        for n in (32, 64):
            f = oracle.features(mod, C, T, n, P, 5, scheme=scheme)
            pay[scheme, n] = math.exp(-r * T) * np.maximum(f[-1, :, 0] - K, 0.0)
    d = pay["qe", 64] - pay["euler", 64]
    se = d.std(ddof=1) / math.sqrt(P)
    bias = sum(abs(pay[s, 64].mean() - pay[s, 32].mean()) for s in ("euler", "qe"))
    assert abs(d.mean()) <= 4 * se + 2 * bias, (d.mean(), se, bias)
