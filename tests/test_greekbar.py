"""CPU checks of the FP32 Greek bar's ingredients: the finite-difference
stencils reproduce the oracle's Greeks from its scenario prices, the per-path
discounted cash flows average to the scenario prices and give their standard
errors, and common random numbers make a spot Greek's Monte Carlo error far
smaller than the bound that ignores them."""
import math

import numpy as np

import oracle
import workloads as W
from _greekbar import check_stencils, compare, greek_se, greek_value, stencils


def test_stencils_and_cash_flows():
    w = W.best_of_call(n_assets=4, n_paths=3000, n_steps=24)
    o = oracle.price_greeks(w["model"], w["corr"], w["option"], 3000, 24, w["bumps"], w["seed"],
                            export_dcf=True)
    st = stencils(4, w["bumps"]["mask"], w["model"]["S0"], w["model"]["v0"], w["bumps"])
    assert len(st) == 4 * 3 + 2 + 6
    check_stencils(o, st)
    P = 3000
    assert np.allclose(o["dcf"].mean(axis=1), o["scenario_price"], rtol=1e-13, atol=0)
    assert np.allclose(o["dcf"].std(axis=1, ddof=1) / math.sqrt(P), o["scenario_se"], rtol=1e-12)
    for i in range(4):
        terms = st["delta_%d" % i][0]
        crn = greek_se(o["dcf"], terms)
        bound = sum(abs(c) * o["scenario_se"][s] for s, c in terms)
        assert crn < 0.5 * bound
    # the comparison's denominator: |ref| when resolved, else the Monte Carlo error
    r = compare(1.001, 1.0, st["rho"][0], 1.0, o["price"], o["dcf"])
    assert abs(r["rel_err"] - 1e-3 / max(1.0, r["se"])) < 1e-12
    assert greek_value(o, "corr_1_3") == o["corr"][4]
