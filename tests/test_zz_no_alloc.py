"""hs_price_greeks_noalloc (through the C ABI) against hs_price_greeks: the
same Greek set, bit for bit, from the library's static scratch, on two calls
in a row -- the second with a smaller request, which must not see the first
one's contents -- and the rejection of a request whose minimum workspace
exceeds the scratch."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("scenario_price", "scenario_se", "delta", "gamma", "vega", "corr")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    for k in ("price", "price_se", "theta", "rho", "skipped_regressions"):
        assert a[k] == b[k] or (np.isnan(a[k]) and np.isnan(b[k])), k


def test_noalloc_matches_workspace_call_twice():
    import paper_2206_03719_amd as hs
    cases = [("5-asset best-of, 6000 x 40, fp32",
              W.best_of_call(n_assets=5, n_paths=6000, n_steps=40), "fp32"),
             ("single-asset put, 1024 x 64, fp64", W.single_asset_put(), "fp64")]
    for name, w, prec in cases:
        _say("noalloc vs workspace call: " + name)
        ref = hs.price_greeks(w["model"], w["corr"], w["option"], w["n_paths"], w["n_steps"],
                              w["bumps"], seed=w["seed"], precision=prec)
        got = hs.price_greeks(w["model"], w["corr"], w["option"], w["n_paths"], w["n_steps"],
                              w["bumps"], seed=w["seed"], precision=prec, noalloc=True)
        _same(got, ref)


def test_noalloc_windows_and_limit():
    import paper_2206_03719_amd as hs
    # larger than the scratch at once: runs in windows of dates, same bits
    w = W.best_of_call(n_assets=5, n_paths=25000, n_steps=252)
    full = hs.workspace_bytes(w["model"], w["option"], 25000, 252, w["bumps"])
    assert full > hs.NOALLOC_SCRATCH_BYTES
    _say("noalloc 5-asset 25k x 252 in windows (needs %.0f MB at once)" % (full / 1e6))
    ref = hs.price_greeks(w["model"], w["corr"], w["option"], 25000, 252, w["bumps"],
                          seed=w["seed"], precision="fp32")
    got = hs.price_greeks(w["model"], w["corr"], w["option"], 25000, 252, w["bumps"],
                          seed=w["seed"], precision="fp32", noalloc=True)
    _same(got, ref)
    big = W.best_of_call(n_assets=10, n_paths=1_000_000, n_steps=252)
    with pytest.raises(hs.HSError) as e:
        hs.price_greeks(big["model"], big["corr"], big["option"], 1_000_000, 252, big["bumps"],
                        seed=big["seed"], precision="fp64", noalloc=True)
    assert e.value.status == hs.ENOMEM
