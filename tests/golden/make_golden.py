"""Write tests/golden/single_asset_put_oracle.json from the FP64 oracle alone.

The paper prints no option values, Greeks or per-path values, so the stored
expected values here are the oracle's own for the single-asset Heston American
put (S0 = K = 100, r = 0.02, T = 1, kappa = 2, theta = v0 = 0.04, xi = 0.3,
rho = -0.7; 1024 paths x 64 steps, Philox seed 42, +-1% spot bumps).  They
guard the oracle against unintended change; the oracle itself is pinned by
the closed-form and invariant tests.  Usage: python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    w = W.single_asset_put()
    g = oracle.price_greeks(w["model"], w["corr"], w["option"], w["n_paths"], w["n_steps"],
                            w["bumps"], w["seed"], export_tau=True)
    out = {"workload": w["name"], "seed": w["seed"],
           "scenario_price": [float(x) for x in g["scenario_price"]],
           "scenario_se": [float(x) for x in g["scenario_se"]],
           "delta": float(g["delta"][0]), "gamma": float(g["gamma"][0]),
           "skipped": [int(x) for x in g["skipped"]],
           "tau_base_head": [int(x) for x in g["tau"][0][:64]]}
    with open(os.path.join(HERE, "single_asset_put_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
