"""GPU tests of the HIP-graph path (HS_FLAG_GRAPH) and the autotuner.

Graph replays are checked bit-for-bit against the eager launch sequence over
several replays, with other eager work and synchronizations in between, on
the cluster sweep, the single-workgroup sweeps and a multi-pass workspace.
The autotuner only changes launch shapes of the path kernel, so a Greek set
after tuning must equal the untuned one bit-for-bit."""
import sys

import numpy as np
import pytest

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


def gpu(w, precision="fp32", **kw):
    return hs.price_greeks(w["model"], w["corr"], w["option"], w["n_paths"], w["n_steps"],
                           w["bumps"], seed=w["seed"], precision=precision, **kw)


def _same(a, b):
    for k in ("scenario_price", "scenario_se"):
        assert np.array_equal(a[k], b[k]), k
    assert a["skipped_regressions"] == b["skipped_regressions"]


@pytest.mark.parametrize("P,n,sweep_mode,precision", [
    (3000, 40, 0, "fp32"),     # cluster sweep, one workgroup per scenario
    (25000, 64, 0, "fp32"),    # cluster sweep, several workgroups per scenario
    (5000, 30, 1, "fp64"),     # single workgroup, state in registers
    (5000, 30, 2, "fp32"),     # single workgroup, state in the workspace
])
def test_graph_replays_match_eager(P, n, sweep_mode, precision):
    import torch
    _say("graph replay P=%d n=%d sweep_mode=%d %s" % (P, n, sweep_mode, precision))
    w = W.best_of_call(n_assets=5, n_paths=P, n_steps=n)
    stream = torch.cuda.Stream()
    nbytes = hs.workspace_bytes(w["model"], w["option"], P, n, w["bumps"], precision)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    eager = gpu(w, precision, workspace=ws, stream=stream, sweep_mode=sweep_mode)
    x = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        g = gpu(w, precision, workspace=ws, stream=stream, sweep_mode=sweep_mode, graph=True)
        _same(g, eager)
        # unrelated eager work on the same workspace and device between replays
        ws.fill_(rep + 1)
        y = (x * 2.0).sum().item()
        assert np.isfinite(y)
        torch.cuda.synchronize()
    # an eager run after the replays still agrees
    _same(gpu(w, precision, workspace=ws, stream=stream, sweep_mode=sweep_mode), eager)


def test_graph_multi_pass_workspace():
    import torch
    _say("graph replay with the minimum workspace (several passes)")
    w = W.best_of_call(n_assets=5, n_paths=3000, n_steps=40)
    mn = hs.workspace_bytes(w["model"], w["option"], 3000, 40, w["bumps"], minimum=True)
    ws = torch.empty(mn, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    ref = gpu(w, workspace=ws, stream=stream)
    for _ in range(3):
        _same(gpu(w, workspace=ws, stream=stream, graph=True), ref)
        torch.cuda.synchronize()


def test_graph_two_requests_interleaved():
    # two request shapes alternate on one stream: each replay must pick its own graph
    import torch
    _say("graph replay, two requests interleaved")
    a = W.best_of_call(n_assets=5, n_paths=4000, n_steps=32)
    b = W.best_of_call(n_assets=3, n_paths=6000, n_steps=20, seed=7)
    stream = torch.cuda.Stream()
    ra = gpu(a, stream=stream)
    rb = gpu(b, stream=stream)
    for _ in range(3):
        _same(gpu(a, stream=stream, graph=True), ra)
        _same(gpu(b, stream=stream, graph=True), rb)


def test_autotune_keeps_results():
    _say("autotune: tuned shape gives identical results")
    w = W.best_of_call(n_assets=5, n_paths=8000, n_steps=64)
    ref = gpu(w)
    best = hs.autotune(w["model"], w["corr"], w["option"], w["n_paths"], w["n_steps"],
                       w["bumps"], seed=w["seed"], repeats=2)
    assert best > 0
    _same(gpu(w), ref)
    _same(gpu(w, graph=True), ref)
