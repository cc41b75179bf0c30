"""GPU parity of the quadratic-exponential (QE) scheme against the oracle's QE.

FP64: path features within 1e-13 relative (both branches of the variance step
exercised: moderate and high vol of vol), Greek sets within 1e-12 with
identical exercise dates.  FP32: the branch test runs in FP64 on the FP32
state, which differs from the oracle's FP64 state by rounding, so a path whose
psi passes within rounding of 1.5 may take the other branch from there on;
features are checked on all but a tiny fraction of paths, and prices within
1e-4 and every Greek within the FP32 Greek bar at the full 5-asset 25k x 252
size.  Several assets: QE and Euler price the same joint law (a European
best-of call agrees within the time-step bias)."""
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


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def high_volvol(w):
    m = {k: (np.array(v, copy=True) if k != "r" else v) for k, v in w["model"].items()}
    m["xi"] = m["xi"] * 2.0  # xi in [0.4, 1.2]: psi > 1.5 on a large share of steps
    return dict(w, model=m)


@pytest.mark.parametrize("N,volvol", [(1, "base"), (5, "base"), (5, "high"), (10, "high")])
def test_qe_path_features_fp64(N, volvol):
    _say("QE path features fp64 N=%d %s vol of vol" % (N, volvol))
    w = W.best_of_call(n_assets=N, n_paths=1000, n_steps=40)
    if volvol == "high":
        w = high_volvol(w)
    ref = oracle.features(w["model"], w["corr"], 1.0, 40, 1000, 42, scheme="qe")
    got = hs.path_features(w["model"], w["corr"], 1.0, 1000, 40, seed=42, precision="fp64",
                           scheme="qe").cpu().numpy()
    assert rel(got[..., 0], ref[..., 0]).max() <= 1e-13
    assert np.abs(got[..., 1] - ref[..., 1]).max() <= 1e-15 + 1e-13 * np.abs(ref[..., 1]).max()


@pytest.mark.parametrize("N", [5, 16])
def test_qe_path_features_fp64_greek_set_kernel(N):
    # the Greek-set path kernel under QE (at 16 assets the variant that runs
    # at most 4 waves per block)
    _say("QE path features fp64 N=%d Greek-set kernel" % N)
    w = high_volvol(W.best_of_call(n_assets=N, n_paths=1000, n_steps=40))
    ref = oracle.features(w["model"], w["corr"], 1.0, 40, 1000, 42, scheme="qe")
    got = hs.path_features(w["model"], w["corr"], 1.0, 1000, 40, seed=42, precision="fp64",
                           scheme="qe", greek_set_kernel=True).cpu().numpy()
    assert rel(got[..., 0], ref[..., 0]).max() <= 1e-13
    assert np.abs(got[..., 1] - ref[..., 1]).max() <= 1e-15 + 1e-13 * np.abs(ref[..., 1]).max()


@pytest.mark.parametrize("N", [1, 5])
def test_qe_path_features_fp32(N):
    _say("QE path features fp32 N=%d" % N)
    w = high_volvol(W.best_of_call(n_assets=N, n_paths=2000, n_steps=252))
    ref = oracle.features(w["model"], w["corr"], 1.0, 252, 2000, 42, scheme="qe")
    got = hs.path_features(w["model"], w["corr"], 1.0, 2000, 252, seed=42, precision="fp32",
                           scheme="qe").cpu().numpy().astype(np.float64)
    eu = rel(got[..., 0], ref[..., 0]).max(axis=0)  # worst date per path
    bad = int((eu > 5e-5).sum())
    _say("  paths off the FP64 branch sequence: %d of 2000; median worst err %.2e"
         % (bad, float(np.median(eu))))
    assert bad <= 4
    assert np.median(eu) <= 5e-6


@pytest.mark.parametrize("N,P,n,volvol", [(5, 3000, 50, "base"), (3, 2000, 30, "high"),
                                          (1, 1024, 64, "base")])
def test_qe_greek_set_fp64(N, P, n, volvol):
    _say("QE greek set fp64 N=%d P=%d n=%d %s" % (N, P, n, volvol))
    w = W.best_of_call(n_assets=N, n_paths=P, n_steps=n)
    if volvol == "high":
        w = high_volvol(w)
    g = hs.price_greeks(w["model"], w["corr"], w["option"], P, n, w["bumps"], seed=w["seed"],
                        precision="fp64", export_tau=True, scheme="qe")
    o = oracle.price_greeks(w["model"], w["corr"], w["option"], P, n, w["bumps"], w["seed"],
                            export_tau=True, scheme="qe")
    assert int((g["tau"] != o["tau"]).sum()) == 0
    assert rel(g["scenario_price"], o["scenario_price"]).max() <= 1e-12


def test_qe_greek_set_fp32_full_size():
    # prices within 1e-4 and every Greek within the FP32 Greek bar
    _say("QE greek set fp32 N=5 P=25000 n=252 (full size)")
    import test_gpu_parity as TP
    TP.hs = hs
    TP._fp32_parity(W.best_of_call(n_assets=5, n_paths=25000, n_steps=252), scheme="qe")


def test_qe_multi_asset_matches_euler_on_gpu():
    # both schemes price the same joint law: a 5-asset European best-of call
    # agrees within 4 SE of the pathwise difference plus twice the schemes'
    # time-step biases (halved dt), here on the GPU's FP64 paths
    _say("QE vs Euler European best-of call N=5 P=100000 n=32/64, fp64")
    P = 100000
    price = {}
    for scheme in ("euler", "qe"):
        for n in (32, 64):
            w = W.best_of_call(n_assets=5, n_paths=P, n_steps=n, mask=0)
            w["option"]["style"] = "european"
            f = hs.path_features(w["model"], w["corr"], 1.0, P, n, seed=w["seed"],
                                 precision="fp64", scheme=scheme).cpu().numpy()
            price[scheme, n] = np.exp(-w["model"]["r"]) * np.maximum(f[-1, :, 0] - 100.0, 0.0)
    d = price["qe", 64] - price["euler", 64]
    se = d.std(ddof=1) / np.sqrt(P)
    bias = sum(abs(price[s, 64].mean() - price[s, 32].mean()) for s in ("euler", "qe"))
    _say("  QE - Euler %.4f, SE %.4f, bias %.4f" % (d.mean(), se, bias))
    assert abs(d.mean()) <= 4 * se + 2 * bias
