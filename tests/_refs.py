"""Independent mathematics the oracle is pinned to (closed forms, trees, a
vectorised numpy LSMC that solves its regressions with numpy.linalg.lstsq).

Nothing here calls the oracle or the HIP library.
"""
import math

import numpy as np
from scipy import integrate, stats


# ---------------------------------------------------------------------------
# Black-Scholes (no dividends)

def bs_price(S, K, r, sigma, T, cp="put"):
    d1 = (math.log(S / K) + (r + 0.5 * sigma * sigma) * T) / (sigma * math.sqrt(T))
    d2 = d1 - sigma * math.sqrt(T)
    N = stats.norm.cdf
    if cp == "call":
        return S * N(d1) - K * math.exp(-r * T) * N(d2)
    return K * math.exp(-r * T) * N(-d2) - S * N(-d1)


def bs_delta(S, K, r, sigma, T, cp="put"):
    d1 = (math.log(S / K) + (r + 0.5 * sigma * sigma) * T) / (sigma * math.sqrt(T))
    return stats.norm.cdf(d1) - (1.0 if cp == "put" else 0.0)


def bs_gamma(S, K, r, sigma, T):
    d1 = (math.log(S / K) + (r + 0.5 * sigma * sigma) * T) / (sigma * math.sqrt(T))
    return stats.norm.pdf(d1) / (S * sigma * math.sqrt(T))


# ---------------------------------------------------------------------------
# Bermudan put on a Cox-Ross-Rubinstein (1979) tree: exercise only at the
# dates k*T/n, k = 1..n (not at 0); `refine` tree steps per date.

def crr_bermudan_put(S0, K, r, sigma, T, n_dates, refine=50):
    M = n_dates * refine
    dt = T / M
    u = math.exp(sigma * math.sqrt(dt))
    d = 1.0 / u
    p = (math.exp(r * dt) - d) / (u - d)
    disc = math.exp(-r * dt)
    j = np.arange(M + 1)
    S = S0 * u ** (M - j) * d ** j
    V = np.maximum(K - S, 0.0)
    for step in range(M - 1, -1, -1):
        V = disc * (p * V[:-1] + (1.0 - p) * V[1:])
        if step > 0 and step % refine == 0:
            jj = np.arange(step + 1)
            S = S0 * u ** (step - jj) * d ** jj
            V = np.maximum(V, K - S)
    return float(V[0])


# ---------------------------------------------------------------------------
# Heston (1993) European prices via the characteristic function of ln S_T in
# the numerically stable form of Albrecher, Mayer, Schoutens & Tistaert (2007).

def heston_cf(u, S0, v0, kappa, theta, xi, rho, r, T):
    iu = 1j * u
    b = kappa - rho * xi * iu
    d = np.sqrt(b * b + xi * xi * (iu + u * u))
    g = (b - d) / (b + d)
    e = np.exp(-d * T)
    C = r * iu * T + kappa * theta / (xi * xi) * ((b - d) * T - 2.0 * np.log((1.0 - g * e) / (1.0 - g)))
    D = (b - d) / (xi * xi) * (1.0 - e) / (1.0 - g * e)
    return np.exp(C + D * v0 + iu * math.log(S0))


def heston_price(S0, K, v0, kappa, theta, xi, rho, r, T, cp="call"):
    lnK = math.log(K)
    fwd = S0 * math.exp(r * T)

    def f1(u):
        return (np.exp(-1j * u * lnK) * heston_cf(u - 1j, S0, v0, kappa, theta, xi, rho, r, T)
                / (1j * u * fwd)).real

    def f2(u):
        return (np.exp(-1j * u * lnK) * heston_cf(u, S0, v0, kappa, theta, xi, rho, r, T)
                / (1j * u)).real

    P1 = 0.5 + integrate.quad(f1, 1e-10, 400.0, limit=800, epsabs=1e-12, epsrel=1e-10)[0] / math.pi
    P2 = 0.5 + integrate.quad(f2, 1e-10, 400.0, limit=800, epsabs=1e-12, epsrel=1e-10)[0] / math.pi
    call = S0 * P1 - K * math.exp(-r * T) * P2
    if cp == "call":
        return call
    return call - S0 + K * math.exp(-r * T)


# ---------------------------------------------------------------------------
# Stulz (1982): European call on the maximum of two lognormal assets (no
# dividends).

def _bvn(a, b, rho):
    return stats.multivariate_normal(mean=[0.0, 0.0], cov=[[1.0, rho], [rho, 1.0]]).cdf([a, b])


def stulz_max_call(S1, S2, K, r, s1, s2, rho, T):
    sq = math.sqrt(T)
    s = math.sqrt(s1 * s1 + s2 * s2 - 2.0 * rho * s1 * s2)
    d = (math.log(S1 / S2) + 0.5 * s * s * T) / (s * sq)
    y1 = (math.log(S1 / K) + (r + 0.5 * s1 * s1) * T) / (s1 * sq)
    y2 = (math.log(S2 / K) + (r + 0.5 * s2 * s2) * T) / (s2 * sq)
    r1 = (s1 - rho * s2) / s
    r2 = (s2 - rho * s1) / s
    return (S1 * _bvn(y1, d, r1) + S2 * _bvn(y2, -d + s * sq, r2)
            - K * math.exp(-r * T) * (1.0 - _bvn(-y1 + s1 * sq, -y2 + s2 * sq, rho)))


def max_call_by_quadrature(S1, S2, K, r, s1, s2, rho, T):
    """The same price by direct 2-D integration over the Gaussian drivers
    (used only to check stulz_max_call)."""
    sq = math.sqrt(T)
    a = math.sqrt(1.0 - rho * rho)

    def f(z2, z1):
        x1 = S1 * math.exp((r - 0.5 * s1 * s1) * T + s1 * sq * z1)
        x2 = S2 * math.exp((r - 0.5 * s2 * s2) * T + s2 * sq * (rho * z1 + a * z2))
        return max(max(x1, x2) - K, 0.0) * math.exp(-0.5 * (z1 * z1 + z2 * z2)) / (2.0 * math.pi)

    v = integrate.dblquad(f, -9.0, 9.0, -9.0, 9.0, epsabs=1e-9, epsrel=1e-9)[0]
    return math.exp(-r * T) * v


# ---------------------------------------------------------------------------
# Independent vectorised Longstaff-Schwartz sweep on given features, with the
# regression solved by numpy.linalg.lstsq (SVD) instead of normal equations.

def numpy_lsmc(feat, K, r, T, cp, m, theta_bar, american=True):
    n, P, _ = feat.shape
    dt = T / n
    U = feat[:, :, 0]
    A = feat[:, :, 1]
    h = np.maximum(K - U, 0.0) if cp == "put" else np.maximum(U - K, 0.0)
    CF = h[n - 1].copy()
    tau = np.full(P, n, dtype=np.int64)
    skipped = 0
    if american:
        for k in range(n - 1, 0, -1):
            hk = h[k - 1]
            I = np.nonzero(hk > 0.0)[0]
            if I.size < m:
                skipped += 1
                continue
            x = (U[k - 1, I] - U[k - 1, I].mean()) / K
            cols = [np.ones_like(x), x, x * x]
            if m == 5:
                w = (A[k - 1, I] - A[k - 1, I].mean()) / theta_bar
                cols += [w, x * w]
            Phi = np.stack(cols, axis=1)
            Y = CF[I] * np.exp(-r * (tau[I] - k) * dt)
            beta, _, rank, _ = np.linalg.lstsq(Phi, Y, rcond=None)
            if rank < m:
                skipped += 1
                continue
            cont = Phi @ beta
            ex = hk[I] > cont
            CF[I[ex]] = hk[I[ex]]
            tau[I[ex]] = k
    disc = CF * np.exp(-r * tau * dt)
    return {"price": disc.mean(), "se": disc.std(ddof=1) / math.sqrt(P), "tau": tau,
            "skipped": skipped}
