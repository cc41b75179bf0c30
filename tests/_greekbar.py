"""The FP32 Greek bar: every Greek of a GPU Greek set within 1e-3 relative of
the FP64 oracle's on the same Philox streams.

Relative to what (the near-zero rule): the error of Greek G is divided by
max(|G_ref|, floor_G, SE_G), where
- floor_G = 1e-8 V_base / unit_G guards a Greek that is zero to rounding
  (unit_G: S0_i for delta, S0_i^2 for gamma, v0_i for vega, 1 for theta, rho
  and the correlation Greeks);
- SE_G is the Greek's own Monte Carlo standard error: the finite-difference
  stencil applied path by path to the oracle's discounted cash flows (common
  random numbers: the same paths in every scenario), sd / sqrt(P).  A Greek
  with |G_ref| < SE_G is "noise-level": its FP32 error must then stay within
  1e-3 of its Monte Carlo error instead of 1e-3 of a value that the sampling
  does not resolve.

The stencils restate the finite differences of the Greek set (central spot
differences for delta and gamma, one-sided v0, maturity, rate and correlation
differences, in the fixed scenario order); check_stencils confirms that they
reproduce the oracle's own Greeks from its scenario prices."""
import math

import numpy as np

BAR = 1e-3


def stencils(N, mask, S0, v0, bumps):
    """name -> (list of (scenario index, coefficient), unit) in the scenario
    order [base, spot+ 0..N-1, spot- 0..N-1, v0 0..N-1, T, r, corr (i<j)]."""
    out = {}
    s = 1
    h = bumps["spot_rel"]
    if mask & 1:
        for i in range(N):
            hs = h * S0[i]
            up, dn = 1 + i, 1 + N + i
            out["delta_%d" % i] = ([(up, 1 / (2 * hs)), (dn, -1 / (2 * hs))], S0[i])
            out["gamma_%d" % i] = ([(up, 1 / hs ** 2), (0, -2 / hs ** 2), (dn, 1 / hs ** 2)],
                                   S0[i] ** 2)
        s += 2 * N
    if mask & 2:
        for i in range(N):
            d = bumps["v0_rel"] * v0[i]
            out["vega_%d" % i] = ([(s + i, 1 / d), (0, -1 / d)], v0[i])
        s += N
    if mask & 4:
        out["theta"] = ([(s, 1 / bumps["T_abs"]), (0, -1 / bumps["T_abs"])], 1.0)
        s += 1
    if mask & 8:
        out["rho"] = ([(s, 1 / bumps["r_abs"]), (0, -1 / bumps["r_abs"])], 1.0)
        s += 1
    if mask & 16:
        t = 0
        for i in range(N):
            for j in range(i + 1, N):
                out["corr_%d_%d" % (i, j)] = ([(s + t, 1 / bumps["corr_abs"]),
                                               (0, -1 / bumps["corr_abs"])], 1.0)
                t += 1
    return out


def greek_value(g, name):
    """The named Greek from a result dict (GPU or oracle)."""
    if name in ("theta", "rho"):
        return float(g[name])
    kind, rest = name.split("_", 1)
    if kind == "corr":
        i, j = map(int, rest.split("_"))
        N = len(g["delta"]) if len(g["delta"]) else len(g["vega"])
        return float(g["corr"][i * N - i * (i + 1) // 2 + (j - i - 1)])
    return float(g[kind][int(rest)])


def check_stencils(o, st):
    """The stencils give the oracle's own Greeks from its scenario prices."""
    V = o["scenario_price"]
    for name, (terms, _) in st.items():
        val = sum(c * V[s] for s, c in terms)
        ref = greek_value(o, name)
        scale = sum(abs(c * V[s]) for s, c in terms)
        assert abs(val - ref) <= 1e-12 * scale, (name, val, ref)


def greek_se(dcf_rows, terms):
    """Monte Carlo standard error of sum_s c_s V_s from per-path discounted cash
    flows (dcf_rows[s] is the row of scenario s)."""
    x = sum(c * dcf_rows[s] for s, c in terms)
    return float(np.std(x, ddof=1) / math.sqrt(len(x)))


def compare(gval, oval, terms, unit, V_base, dcf_rows):
    se = greek_se(dcf_rows, terms) if dcf_rows is not None else 0.0
    floor = 1e-8 * abs(V_base) / unit
    den = max(abs(oval), floor, se)
    return {"gpu": float(gval), "oracle": float(oval), "se": se,
            "noise_level": bool(abs(oval) < se), "rel_err": float(abs(gval - oval) / den)}
