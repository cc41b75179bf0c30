"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs and the same Philox streams.

Bars: bit-exact Philox words; FP64 paths within 1e-13 relative of the oracle's
features and every FP64 scenario price within 1e-12 relative with identical
exercise dates; FP32 paths within 1e-4 relative on prices and 1e-3 on every
Greek (relative to max(|ref|, rounding floor, the Greek's own Monte Carlo
error), tests/_greekbar.py), with the decision flips counted (and, as a reported diagnostic only, the FP64
reprice of the GPU's own exercise dates); bit-for-bit invariance across launch
shapes, sweep modes and workspace passes."""
import json
import math
import os
import sys

import numpy as np
import pytest

import _greekbar as GB
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


def gpu(w, precision, **kw):
    return hs.price_greeks(w["model"], w["corr"], w["option"], w["n_paths"], w["n_steps"],
                           w["bumps"], seed=w["seed"], precision=precision, **kw)


def orc(w, **kw):
    return oracle.price_greeks(w["model"], w["corr"], w["option"], w["n_paths"], w["n_steps"],
                               w["bumps"], w["seed"], **kw)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


# ---------------------------------------------------------------------------
# random numbers

def test_philox_words_bit_exact():
    _say("philox words: seed 42, 300 paths x 7 steps x 3 blocks")
    words = hs.philox_words(42, 300, 7, 3)
    for p in range(300):
        for k in range(7):
            for j in range(3):
                assert list(words[p, k, j]) == oracle.philox([p, k, j, 0], [42, 0]), (p, k, j)
    words = hs.philox_words((7 << 32) | 99, 50, 2, 2)
    for p in range(50):
        for k in range(2):
            for j in range(2):
                assert list(words[p, k, j]) == oracle.philox([p, k, j, 0], [99, 7])


@pytest.mark.parametrize("N", [1, 5, 20])
def test_normals(N):
    _say("normals N=%d" % N)
    P, n = 200, 5
    e64, h64 = hs.normals(42, N, P, n, "fp64")
    e32, h32 = hs.normals(42, N, P, n, "fp32")
    for p in range(P):
        for k in range(n):
            re, rh = oracle.normals(N, 42, p, k)
            assert np.abs(e64[p, k] - re).max() <= 4e-15
            assert np.abs(h64[p, k] - rh).max() <= 4e-15
            assert np.abs(e32[p, k] - re).max() <= 2e-6
            assert np.abs(h32[p, k] - rh).max() <= 2e-6


# ---------------------------------------------------------------------------
# paths + path reduction (the paper's measured kernel)

@pytest.mark.parametrize("kernel", ["base", "greek_set"])
@pytest.mark.parametrize("N", [1, 3, 5, 12, 13, 16, 20])
def test_path_features_fp64(N, kernel):
    _say("path features fp64 N=%d %s kernel" % (N, kernel))
    w = W.best_of_call(n_assets=N, n_paths=1000, n_steps=40)
    ref = oracle.features(w["model"], w["corr"], 1.0, 40, 1000, 42)
    got = hs.path_features(w["model"], w["corr"], 1.0, 1000, 40, seed=42, precision="fp64",
                           greek_set_kernel=kernel == "greek_set").cpu().numpy()
    assert got.shape == ref.shape
    assert rel(got[..., 0], ref[..., 0]).max() <= 1e-13
    assert np.abs(got[..., 1] - ref[..., 1]).max() <= 1e-15 + 1e-13 * np.abs(ref[..., 1]).max()


@pytest.mark.parametrize("kernel", ["base", "greek_set"])
@pytest.mark.parametrize("N", [1, 5, 10])
def test_path_features_fp32(N, kernel):
    _say("path features fp32 N=%d %s kernel" % (N, kernel))
    w = W.best_of_call(n_assets=N, n_paths=777, n_steps=252)
    ref = oracle.features(w["model"], w["corr"], 1.0, 252, 777, 42)
    got = hs.path_features(w["model"], w["corr"], 1.0, 777, 252, seed=42, precision="fp32",
                           greek_set_kernel=kernel == "greek_set").cpu().numpy().astype(np.float64)
    assert rel(got[..., 0], ref[..., 0]).max() <= 5e-5
    assert np.abs(got[..., 1] - ref[..., 1]).max() <= 5e-6


# ---------------------------------------------------------------------------
# Greek sets, FP64: the oracle's numbers to 1e-12

def _fp64_parity(w, **kw):
    g = gpu(w, "fp64", export_tau=True, **kw)
    o = orc(w, export_tau=True)
    worst = rel(g["scenario_price"], o["scenario_price"]).max()
    flips = int((g["tau"] != o["tau"]).sum())
    _say("  fp64 worst scenario rel err %.3e, tau mismatches %d" % (worst, flips))
    assert flips == 0
    assert worst <= 1e-12
    assert np.allclose(g["scenario_se"], o["scenario_se"], rtol=1e-9, atol=0)
    assert g["skipped_regressions"] == int(o["skipped"].sum())
    # each Greek against the bound propagated from 1e-12 on every scenario price
    V = np.abs(o["scenario_price"])
    N = len(w["model"]["S0"])
    if w["bumps"]["mask"] & 1:
        hsv = w["bumps"]["spot_rel"] * np.asarray(w["model"]["S0"])
        for a in range(N):
            up, dn = V[1 + a], V[1 + N + a]
            assert abs(g["delta"][a] - o["delta"][a]) <= 4e-12 * (up + dn) / (2 * hsv[a])
            assert abs(g["gamma"][a] - o["gamma"][a]) <= 4e-12 * (up + 2 * V[0] + dn) / hsv[a] ** 2
    return g, o


def test_single_asset_put_fp64():
    _say("single-asset Heston American put, 1024 x 64, fp64")
    w = W.single_asset_put()
    g, o = _fp64_parity(w)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "single_asset_put_oracle.json")))
    assert np.allclose(g["scenario_price"], gold["scenario_price"], rtol=1e-12, atol=0)


@pytest.mark.parametrize("N,P,n,style,basis", [
    (5, 3000, 50, "american", "auto"),
    (3, 777, 30, "american", "quad"),
    (10, 1500, 20, "american", "auto"),
    (4, 2000, 25, "european", "auto"),
    (1, 1000, 12, "american", "auto"),
])
def test_greek_set_fp64(N, P, n, style, basis):
    _say("greek set fp64 N=%d P=%d n=%d %s %s" % (N, P, n, style, basis))
    w = W.best_of_call(n_assets=N, n_paths=P, n_steps=n)
    w["option"]["style"] = style
    w["option"]["basis"] = basis
    _fp64_parity(w)


def test_put_on_max_fp64():
    _say("american put on the max of 3, fp64")
    w = W.best_of_call(n_assets=3, n_paths=2000, n_steps=30)
    w["option"]["cp"] = "put"
    w["option"]["K"] = 125.0
    _fp64_parity(w)


# ---------------------------------------------------------------------------
# Greek sets, FP32 paths (FP64 regression): 1e-4 on prices, decisions replayed

def _fp32_parity(w, scheme="euler"):
    g = gpu(w, "fp32", export_tau=True, scheme=scheme)
    o = orc(w, export_tau=True, export_dcf=True, scheme=scheme)
    rep = orc(w, replay_tau=g["tau"], scheme=scheme)  # FP64 prices of the GPU's own decisions
    price_err = rel(g["scenario_price"], o["scenario_price"])
    arith_err = rel(g["scenario_price"], rep["scenario_price"])
    flips = (g["tau"] != o["tau"]).sum(axis=1)
    report = {"workload": w["name"], "scheme": scheme, "max_price_rel_err": float(price_err.max()),
              "max_arith_rel_err": float(arith_err.max()),
              "flip_fraction": float(flips.sum() / g["tau"].size)}
    # every Greek against the FP32 Greek bar (tests/_greekbar.py: relative to
    # max(|ref|, rounding floor, its own Monte Carlo standard error))
    N = len(w["model"]["S0"])
    st = GB.stencils(N, w["bumps"]["mask"], w["model"]["S0"], w["model"]["v0"], w["bumps"])
    GB.check_stencils(o, st)
    greeks = {name: GB.compare(GB.greek_value(g, name), GB.greek_value(o, name), terms, unit,
                               o["price"], o["dcf"])
              for name, (terms, unit) in st.items()}
    worst = max(greeks, key=lambda k: greeks[k]["rel_err"])
    report["max_greek_rel_err"] = greeks[worst]["rel_err"]
    report["worst_greek"] = worst
    report["noise_level_greeks"] = [k for k, v in greeks.items() if v["noise_level"]]
    report["greeks"] = greeks
    _say("  fp32 " + json.dumps({k: v for k, v in report.items() if k != "greeks"}))
    for k, v in greeks.items():
        _say("  %-9s gpu %.8e oracle %.8e se %.2e rel err %.2e%s"
             % (k, v["gpu"], v["oracle"], v["se"], v["rel_err"],
                " (noise level)" if v["noise_level"] else ""))
    os.makedirs("gpurun_out", exist_ok=True)
    with open(os.path.join("gpurun_out", "fp32_parity_%s_%s.json" % (w["name"], scheme)), "w") as f:
        json.dump(report, f, indent=1)
    # the replay figure uses the GPU's exercise dates as oracle input: a
    # diagnostic in the report, not a parity assertion
    assert price_err.max() <= 1e-4
    bad = {k: v["rel_err"] for k, v in greeks.items() if v["rel_err"] > GB.BAR}
    assert not bad, bad
    return g, o, report


def test_greek_set_fp32_small():
    _say("greek set fp32 N=5 P=4000 n=64")
    _fp32_parity(W.best_of_call(n_assets=5, n_paths=4000, n_steps=64))


def test_greek_set_fp32_bestof5_full_size():
    # the 5-asset best-of workload at its full size, in the launch shape the
    # benchmark times (the oracle runs the same 25k paths: the regression
    # couples every path)
    _say("greek set fp32 N=5 P=25000 n=252 (full size)")
    _fp32_parity(W.best_of_call(n_assets=5, n_paths=25000, n_steps=252))


# ---------------------------------------------------------------------------
# invariances: results are a function of the request alone

def test_bitwise_invariance_launch_shape_and_passes():
    _say("bitwise invariance: waves per block, workspace passes")
    w = W.best_of_call(n_assets=5, n_paths=3000, n_steps=40)
    ref = gpu(w, "fp32")
    for kw in (dict(waves_per_block=1), dict(waves_per_block=8), dict(sweep_mode=3)):
        g = gpu(w, "fp32", **kw)
        assert np.array_equal(g["scenario_price"], ref["scenario_price"]), kw
        assert np.array_equal(g["scenario_se"], ref["scenario_se"]), kw
    import torch
    mn = hs.workspace_bytes(w["model"], w["option"], 3000, 40, w["bumps"], minimum=True)
    ws = torch.empty(mn, dtype=torch.uint8, device="cuda")
    g = gpu(w, "fp32", workspace=ws)
    assert np.array_equal(g["scenario_price"], ref["scenario_price"])
    # the single-workgroup sweeps sum the same FP64 terms in another order
    for sm in (1, 2):
        g = gpu(w, "fp32", sweep_mode=sm)
        assert rel(g["scenario_price"], ref["scenario_price"]).max() <= 1e-13


@pytest.mark.parametrize("P", [20000, 25000])
def test_cluster_sweep_fp64_five_and_six_paths(P):
    # FP64 features, 28 scenarios, 8 or 9 workgroups per scenario: 5 paths per
    # thread (two workgroups per CU) and 6 (one per CU: FP64 pairs need the
    # larger register budget there); exercise dates identical to the oracle's
    w = W.best_of_call(n_assets=5, n_paths=P, n_steps=16)
    _say("cluster sweep FP64 P=%d" % P)
    o = orc(w, export_tau=True)
    g = gpu(w, "fp64", export_tau=True)
    assert rel(g["scenario_price"], o["scenario_price"]).max() <= 1e-12
    assert rel(g["scenario_se"], o["scenario_se"]).max() <= 1e-9
    assert np.array_equal(g["tau"], o["tau"])


@pytest.mark.parametrize("P", [140000, 157000, 175000])
def test_cluster_sweep_wide_threads(P):
    # FP32 features with 15 scenarios: the cluster sweep holds 18, 20 and 22
    # paths per thread (16 workgroups per scenario, ragged last one); against
    # the single-workgroup sweep with the state in the workspace on the same
    # features, which adds the same FP64 terms in another order
    _say("cluster sweep, wide threads, P=%d" % P)
    w = W.best_of_call(n_assets=3, n_paths=P, n_steps=8)
    g = gpu(w, "fp32")
    b = gpu(w, "fp32", sweep_mode=2)
    assert rel(g["scenario_price"], b["scenario_price"]).max() <= 1e-13
    assert rel(g["scenario_se"], b["scenario_se"]).max() <= 1e-11


def test_bitwise_invariance_fp64_16_asset_wave_cap():
    # FP64 at 13-16 assets runs at most 4 waves per block: asking for 8, or
    # fewer, gives the same features and so the same prices bit for bit
    _say("bitwise invariance: FP64 N=16 waves per block 0, 2, 8")
    w = W.best_of_call(n_assets=16, n_paths=700, n_steps=12, precision="fp64")
    ref = gpu(w, "fp64")
    for wpb in (2, 8):
        g = gpu(w, "fp64", waves_per_block=wpb)
        assert np.array_equal(g["scenario_price"], ref["scenario_price"]), wpb
        assert np.array_equal(g["scenario_se"], ref["scenario_se"]), wpb


@pytest.mark.parametrize("P", [16384, 16385, 25000, 70001])
def test_sweep_variants_vs_oracle(P):
    # cluster sweep (G workgroups per scenario, ragged last workgroup), and the
    # single-workgroup sweeps with the state in registers or the workspace
    _say("sweep variants at P=%d" % P)
    w = W.best_of_call(n_assets=5, n_paths=P, n_steps=40, mask=0)
    o = orc(w, export_tau=True)
    modes = [0, 2, 3] + ([1] if P <= 16384 else [])
    for sm in modes:
        g = gpu(w, "fp64", sweep_mode=sm, export_tau=True)
        assert rel(g["price"], o["price"]) <= 1e-12, sm
        assert rel(g["price_se"], o["price_se"]) <= 1e-9, sm
        assert np.array_equal(g["tau"], o["tau"]), sm


@pytest.mark.parametrize("N,mask,P", [(3, 1, 25000), (2, 2, 7001), (5, 31, 3000)])
def test_cluster_sweep_scenarios_vs_oracle(N, mask, P):
    # the cluster sweep over several scenarios per launch (7, 3 and 28), the
    # last workgroup of each scenario ragged; FP64 paths, so the exercise
    # dates are the oracle's
    w = W.best_of_call(n_assets=N, n_paths=P, n_steps=40, mask=mask)
    S = oracle.num_scenarios(N, mask)
    _say("cluster sweep N=%d mask=%d P=%d (%d scenarios)" % (N, mask, P, S))
    o = orc(w, export_tau=True)
    g = gpu(w, "fp64", export_tau=True)
    assert rel(g["scenario_price"], o["scenario_price"]).max() <= 1e-12
    assert rel(g["scenario_se"], o["scenario_se"]).max() <= 1e-9
    assert g["skipped_regressions"] == int(o["skipped"].sum())
    assert np.array_equal(g["tau"], o["tau"])


def test_repeat_runs_identical():
    w = W.best_of_call(n_assets=4, n_paths=5000, n_steps=30)
    a = gpu(w, "fp32")
    b = gpu(w, "fp32")
    assert np.array_equal(a["scenario_price"], b["scenario_price"])


def test_all_out_of_the_money_gpu():
    w = W.single_asset_put(n_paths=512, n_steps=16)
    w["option"]["K"] = 1.0
    g = gpu(w, "fp64")
    assert g["price"] == 0.0 and g["price_se"] == 0.0
    assert g["skipped_regressions"] == 3 * 15


def test_timing_fields():
    w = W.best_of_call(n_assets=5, n_paths=4096, n_steps=32)
    g = gpu(w, "fp32", timing=True)
    assert g["t_paths_ms"] > 0 and g["t_sweep_ms"] > 0
    assert abs(g["t_total_ms"] - g["t_paths_ms"] - g["t_gram_ms"] - g["t_sweep_ms"]) < 1e-6
