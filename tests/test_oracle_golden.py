"""The oracle still reproduces its stored single-asset put outputs (written by
tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np

import oracle
import workloads as W


def test_single_asset_put_golden():
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "single_asset_put_oracle.json")) as f:
        gold = json.load(f)
    w = W.single_asset_put()
    g = oracle.price_greeks(w["model"], w["corr"], w["option"], w["n_paths"], w["n_steps"],
                            w["bumps"], w["seed"], export_tau=True)
    assert np.array_equal(g["scenario_price"], np.array(gold["scenario_price"]))
    assert np.array_equal(g["scenario_se"], np.array(gold["scenario_se"]))
    assert g["delta"][0] == gold["delta"] and g["gamma"][0] == gold["gamma"]
    assert list(g["tau"][0][:64]) == gold["tau_base_head"]
