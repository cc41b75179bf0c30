"""Checkpoint-recompute (windows of dates) on the GPU.

A Greek set whose features do not fit its workspace runs the backward sweep in
windows of dates, from the last window back, and recomputes each earlier
window's path features from a checkpoint of the path state.  The random
numbers are counter-based and the state is kept exactly, so every scenario
price, standard error, skipped-date count and exercise date must equal the
run over all dates at once, bit for bit; the windowed FP64 run is also
checked against the oracle."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

hs = None


def setup_module(module):
    global hs
    import paper_2206_03719_amd as _hs
    hs = _hs
    hs.lib()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(w, precision, **kw):
    return hs.price_greeks(w["model"], w["corr"], w["option"], w["n_paths"], w["n_steps"],
                           w["bumps"], seed=w["seed"], precision=precision, export_tau=True, **kw)


def same(a, b):
    assert np.array_equal(a["scenario_price"], b["scenario_price"])
    assert np.array_equal(a["scenario_se"], b["scenario_se"])
    assert a["skipped_regressions"] == b["skipped_regressions"]
    assert np.array_equal(a["tau"], b["tau"])
    assert np.array_equal(a["delta"], b["delta"])


@pytest.mark.parametrize("window", [1, 7, 16, 63, 64])
def test_windows_equal_one_pass_fp32(window):
    _say("windows fp32 5 assets 4000 x 64, %d dates per window" % window)
    w = W.best_of_call(n_assets=5, n_paths=4000, n_steps=64)
    same(run(w, "fp32", window_dates=window), run(w, "fp32"))


@pytest.mark.parametrize("scheme,N,P,n,window", [("qe", 3, 2000, 50, 9), ("euler", 10, 1500, 40, 6),
                                                 ("qe", 5, 1000, 30, 4)])
def test_windows_equal_one_pass_fp64(scheme, N, P, n, window):
    _say("windows fp64 %s N=%d P=%d n=%d, %d dates per window" % (scheme, N, P, n, window))
    w = W.best_of_call(n_assets=N, n_paths=P, n_steps=n)
    same(run(w, "fp64", scheme=scheme, window_dates=window), run(w, "fp64", scheme=scheme))


def test_windows_fp32_qe():
    w = W.best_of_call(n_assets=5, n_paths=3000, n_steps=48)
    same(run(w, "fp32", scheme="qe", window_dates=5), run(w, "fp32", scheme="qe"))


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_windows_in_each_sweep(mode):
    # windows keep the state in the workspace, so the register sweep (mode 1)
    # runs as the workspace-state sweep (mode 2) there
    _say("windows, sweep mode %d" % mode)
    w = W.best_of_call(n_assets=3, n_paths=3000, n_steps=40)
    ref = run(w, "fp64", sweep_mode=2 if mode == 1 else mode)
    same(run(w, "fp64", sweep_mode=mode, window_dates=11), ref)


def test_single_asset_put_windows_and_oracle():
    w = W.single_asset_put()
    g = run(w, "fp64", window_dates=10)
    same(g, run(w, "fp64"))
    o = oracle.price_greeks(w["model"], w["corr"], w["option"], w["n_paths"], w["n_steps"],
                            w["bumps"], w["seed"], export_tau=True)
    assert np.array_equal(g["tau"], o["tau"])
    rel = np.abs(g["scenario_price"] - o["scenario_price"]) / np.abs(o["scenario_price"])
    assert rel.max() <= 1e-12


def test_european_ignores_windows():
    w = W.best_of_call(n_assets=4, n_paths=2000, n_steps=30)
    w["option"] = dict(w["option"], style="european")
    same(run(w, "fp64", window_dates=5), run(w, "fp64"))


def test_workspace_below_one_unit_runs_in_windows():
    import torch
    _say("5-asset 25,000 x 252 Greek set in the minimum workspace")
    w = W.best_of_call(n_assets=5, n_paths=25000, n_steps=252)
    full = run(w, "fp32")
    mn = hs.workspace_bytes(w["model"], w["option"], 25000, 252, w["bumps"], "fp32",
                            minimum=True)
    unit = 11 * 252 * 25000 * 8  # base and spot scenarios' features alone
    assert mn < unit / 8
    for nbytes in (mn, 3 * mn):
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        same(run(w, "fp32", workspace=ws), full)
        del ws
    with pytest.raises(hs.HSError):
        ws = torch.empty(mn - 4096, dtype=torch.uint8, device="cuda")
        run(w, "fp32", workspace=ws)


def test_graph_replay_of_windowed_pass():
    import torch
    w = W.best_of_call(n_assets=5, n_paths=4000, n_steps=64)
    ref = run(w, "fp32")
    ws = torch.empty(hs.workspace_bytes(w["model"], w["option"], 4000, 64, w["bumps"], "fp32",
                                        window_dates=8), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    for _ in range(3):
        same(run(w, "fp32", window_dates=8, workspace=ws, stream=stream, graph=True), ref)
        torch.cuda.synchronize()
