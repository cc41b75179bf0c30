"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Python access (ctypes) to ``hs_oracle.c``, the plain definition of the Heston
paths + Longstaff-Schwartz Greek set that the HIP library must reproduce.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the product never does, and this
package imports nothing from the product.

Parity notes: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, library routines or brute force; none is
"parity unpinned".
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))

# integer codes of the public interface (option, exercise style, bumps)
PUT, CALL = 0, 1
EUROPEAN, AMERICAN = 0, 1
DELTA_GAMMA, VEGA, THETA, RHO, CORR = 1, 2, 4, 8, 16
ALL_BUMPS = 31
OK, EINVAL, ENOTSPD, ENOMEM = 0, -1, -2, -3

_CP = {"put": PUT, "call": CALL}
_STYLE = {"european": EUROPEAN, "american": AMERICAN}

_lib = None


def lib(path=None):
    """Load (building on first use if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        if path is None:
            path = _build.LIB
            if not os.path.exists(path):
                _build.build()
        L = ctypes.CDLL(path)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_uniform.argtypes = [ctypes.c_uint32]
        L.orc_uniform.restype = ctypes.c_double
        L.orc_normal_pair.argtypes = [ctypes.c_uint32, ctypes.c_uint32, dp]
        L.orc_normals.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                  dp, dp]
        L.orc_cholesky.argtypes = [ctypes.c_int32, dp, dp]
        L.orc_cholesky.restype = ctypes.c_int
        L.orc_features.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_int32,
                                   ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, dp]
        L.orc_features.restype = ctypes.c_int
        L.orc_qe_variance_step.argtypes = [ctypes.c_double] * 7
        L.orc_qe_variance_step.restype = ctypes.c_double
        L.orc_features_at.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_int32,
                                      ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_uint64, dp]
        L.orc_features_at.restype = ctypes.c_int
        L.orc_states.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_int32,
                                 ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, dp]
        L.orc_states.restype = ctypes.c_int
        L.orc_lsmc.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_double, ctypes.c_int32, dp,
                               ctypes.POINTER(ctypes.c_int32), dp,
                               ctypes.POINTER(ctypes.c_int64)]
        L.orc_lsmc.restype = ctypes.c_int
        L.orc_replay.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_int32), dp]
        L.orc_replay.restype = ctypes.c_int
        L.orc_num_scenarios.argtypes = [ctypes.c_int32, ctypes.c_uint32]
        L.orc_num_scenarios.restype = ctypes.c_int64
        L.orc_price_scenarios.argtypes = [ctypes.c_void_p, dp, dp, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int32)]
        L.orc_price_scenarios.restype = ctypes.c_int
        L.orc_price_scenarios_replay.argtypes = [ctypes.c_void_p, dp, dp,
                                                 ctypes.POINTER(ctypes.c_int64),
                                                 ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_int32)]
        L.orc_price_scenarios_replay.restype = ctypes.c_int
        L.orc_price_scenarios_dcf.argtypes = [ctypes.c_void_p, dp, dp,
                                              ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_int32), dp]
        L.orc_price_scenarios_dcf.restype = ctypes.c_int
        L.orc_greeks.argtypes = [ctypes.c_int32, ctypes.c_uint32, dp, dp, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, dp, dp, dp, dp, dp, dp, dp]
        L.orc_greeks.restype = ctypes.c_int
        _lib = L
    return _lib


class use_library:
    """Context manager: route every oracle call through another build of
    hs_oracle.c (the mutation tests load deliberately broken copies)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = None
        lib(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


SCHEMES = {"euler": 0, "qe": 1}


class _Model(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32),
                ("S0", ctypes.c_void_p), ("v0", ctypes.c_void_p), ("kappa", ctypes.c_void_p),
                ("theta", ctypes.c_void_p), ("xi", ctypes.c_void_p), ("rho", ctypes.c_void_p),
                ("r", ctypes.c_double), ("scheme", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32),
                ("S0", ctypes.c_void_p), ("v0", ctypes.c_void_p), ("kappa", ctypes.c_void_p),
                ("theta", ctypes.c_void_p), ("xi", ctypes.c_void_p), ("rho", ctypes.c_void_p),
                ("r", ctypes.c_double), ("C", ctypes.c_void_p),
                ("cp", ctypes.c_int32), ("style", ctypes.c_int32), ("m", ctypes.c_int32),
                ("K", ctypes.c_double), ("T", ctypes.c_double),
                ("P", ctypes.c_int64), ("n", ctypes.c_int32), ("mask", ctypes.c_uint32),
                ("spot_rel", ctypes.c_double), ("v0_rel", ctypes.c_double),
                ("T_abs", ctypes.c_double), ("r_abs", ctypes.c_double),
                ("corr_abs", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("nthreads", ctypes.c_int32), ("scheme", ctypes.c_int32)]


# ---------------------------------------------------------------------------
# primitives

def philox(ctr, key):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def uniform(w):
    return lib().orc_uniform(int(w) & 0xFFFFFFFF)


def normal_pair(w1, w2):
    o = np.zeros(2)
    lib().orc_normal_pair(int(w1) & 0xFFFFFFFF, int(w2) & 0xFFFFFFFF, _dp(o))
    return float(o[0]), float(o[1])


def normals(n_assets, seed, path, step):
    eps = np.zeros(n_assets)
    eta = np.zeros(n_assets)
    lib().orc_normals(n_assets, seed, path, step, _dp(eps), _dp(eta))
    return eps, eta


def cholesky(C):
    C = _f64(C)
    N = C.shape[0]
    L = np.zeros((N, N))
    st = lib().orc_cholesky(N, _dp(C), _dp(L))
    if st != OK:
        raise ValueError("correlation matrix is not SPD")
    return L


def _model_struct(model, keep, scheme="euler"):
    arrs = [_f64(model[k]) for k in ("S0", "v0", "kappa", "theta", "xi", "rho")]
    keep.extend(arrs)
    m = _Model(len(arrs[0]), *[a.ctypes.data for a in arrs], float(model["r"]), SCHEMES[scheme])
    return m


def features(model, corr, T, n_steps, n_paths, seed, nthreads=0, scheme="euler"):
    """(n_steps, n_paths, 2) array of (U, A) at dates 1..n for one scenario."""
    keep = []
    m = _model_struct(model, keep, scheme)
    C = _f64(corr)
    out = np.empty((n_steps, n_paths, 2))
    st = lib().orc_features(ctypes.byref(m), _dp(C), float(T), int(n_steps), int(n_paths),
                            int(seed), int(nthreads), _dp(out))
    if st != OK:
        raise ValueError("orc_features failed with status %d" % st)
    return out


def features_at(model, corr, T, n_steps, paths, seed, scheme="euler"):
    """(len(paths), n_steps, 2) array of (U, A) at dates 1..n for the given path
    indices of one scenario (the same paths as features() produces)."""
    keep = []
    m = _model_struct(model, keep, scheme)
    C = _f64(corr)
    idx = np.ascontiguousarray(np.asarray(paths, dtype=np.int64))
    out = np.empty((len(idx), n_steps, 2))
    st = lib().orc_features_at(ctypes.byref(m), _dp(C), float(T), int(n_steps), len(idx),
                               idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(seed),
                               _dp(out))
    if st != OK:
        raise ValueError("orc_features_at failed with status %d" % st)
    return out


def states(model, corr, T, n_steps, n_paths, seed, nthreads=0, scheme="euler"):
    """(n_paths, n_assets, 2) array of each asset's (X, v) after n_steps, X
    from 0 (the per-asset joint law behind the features)."""
    keep = []
    m = _model_struct(model, keep, scheme)
    C = _f64(corr)
    out = np.empty((n_paths, m.N, 2))
    st = lib().orc_states(ctypes.byref(m), _dp(C), float(T), int(n_steps), int(n_paths),
                          int(seed), int(nthreads), _dp(out))
    if st != OK:
        raise ValueError("orc_states failed with status %d" % st)
    return out


def basis_size(n_assets, basis="auto"):
    if basis == "auto":
        return 3 if n_assets == 1 else 5
    return {"quad": 3, "quad_vol": 5}[basis]


def lsmc(feat, option, r, theta_bar, m, nthreads=0):
    """Price one scenario from its features; returns dict(price, se, tau, cf, skipped)."""
    feat = np.ascontiguousarray(feat, dtype=np.float64)
    n, P, _ = feat.shape
    out = np.zeros(2)
    tau = np.zeros(P, dtype=np.int32)
    cf = np.zeros(P)
    sk = ctypes.c_int64(0)
    st = lib().orc_lsmc(_dp(feat), P, n, float(option["T"]), float(r), float(option["K"]),
                        _CP[option["cp"]], _STYLE[option["style"]], int(m), float(theta_bar),
                        int(nthreads), _dp(out),
                        tau.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(cf),
                        ctypes.byref(sk))
    if st != OK:
        raise ValueError("orc_lsmc failed with status %d" % st)
    return {"price": out[0], "se": out[1], "tau": tau, "cf": cf, "skipped": sk.value}


def replay(feat, option, r, tau):
    """FP64 price of a given exercise-date vector on these features."""
    feat = np.ascontiguousarray(feat, dtype=np.float64)
    n, P, _ = feat.shape
    tau = np.ascontiguousarray(tau, dtype=np.int32)
    out = np.zeros(2)
    st = lib().orc_replay(_dp(feat), P, n, float(option["T"]), float(r), float(option["K"]),
                          _CP[option["cp"]], tau.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          _dp(out))
    if st != OK:
        raise ValueError("orc_replay failed with status %d" % st)
    return out[0], out[1]


def num_scenarios(n_assets, mask):
    return int(lib().orc_num_scenarios(int(n_assets), int(mask)))


def qe_variance_step(kappa, theta, xi, rho, dt, v, zv):
    """One quadratic-exponential variance step from v with normal zv."""
    return lib().orc_qe_variance_step(float(kappa), float(theta), float(xi), float(rho),
                                      float(dt), float(v), float(zv))


def price_greeks(model, corr, option, n_paths, n_steps, bumps, seed, nthreads=0,
                 export_tau=False, replay_tau=None, scheme="euler", export_dcf=False):
    """The full Greek set: scenario prices, SEs, skipped counts and the Greeks.

    replay_tau (scenarios x paths int32): price each scenario with these
    exercise dates instead of regressing (decision replay).  export_dcf: also
    return "dcf" (scenarios x paths), each path's discounted cash flow."""
    keep = []
    arrs = [_f64(model[k]) for k in ("S0", "v0", "kappa", "theta", "xi", "rho")]
    C = _f64(corr)
    keep.extend(arrs)
    N = len(arrs[0])
    m = basis_size(N, option.get("basis", "auto"))
    mask = int(bumps["mask"])
    q = _Request(N, *[a.ctypes.data for a in arrs], float(model["r"]), C.ctypes.data,
                 _CP[option["cp"]], _STYLE[option["style"]], m, float(option["K"]),
                 float(option["T"]), int(n_paths), int(n_steps), mask,
                 float(bumps["spot_rel"]), float(bumps["v0_rel"]), float(bumps["T_abs"]),
                 float(bumps["r_abs"]), float(bumps["corr_abs"]), int(seed), int(nthreads),
                 SCHEMES[scheme])
    S = num_scenarios(N, mask)
    prices = np.zeros(S)
    ses = np.zeros(S)
    skipped = np.zeros(S, dtype=np.int64)
    tau = np.zeros((S, n_paths), dtype=np.int32) if export_tau else None
    rt = None
    if replay_tau is not None:
        rt = np.ascontiguousarray(replay_tau, dtype=np.int32)
        assert rt.shape == (S, n_paths)
    taup = tau.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if tau is not None else None
    dcf = None
    if export_dcf:
        assert rt is None
        dcf = np.zeros((S, n_paths))
        st = lib().orc_price_scenarios_dcf(
            ctypes.byref(q), _dp(prices), _dp(ses),
            skipped.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), taup, _dp(dcf))
    else:
        st = lib().orc_price_scenarios_replay(
            ctypes.byref(q), _dp(prices), _dp(ses),
            skipped.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), taup,
            rt.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if rt is not None else None)
    if st != OK:
        raise ValueError("orc_price_scenarios failed with status %d" % st)
    g = greeks_from_prices(N, mask, arrs[0], arrs[1], bumps, prices)
    g.update({"scenario_price": prices, "scenario_se": ses, "skipped": skipped,
              "price": prices[0], "price_se": ses[0], "n_scenarios": S})
    if tau is not None:
        g["tau"] = tau
    if dcf is not None:
        g["dcf"] = dcf
    return g


def greeks_from_prices(N, mask, S0, v0, bumps, prices):
    S0 = _f64(S0)
    v0 = _f64(v0)
    prices = _f64(prices)
    delta = np.full(N, np.nan)
    gamma = np.full(N, np.nan)
    vega = np.full(N, np.nan)
    th = np.full(1, np.nan)
    rh = np.full(1, np.nan)
    corr = np.full(max(N * (N - 1) // 2, 1), np.nan)
    lib().orc_greeks(N, int(mask), _dp(S0), _dp(v0), float(bumps["spot_rel"]),
                     float(bumps["v0_rel"]), float(bumps["T_abs"]), float(bumps["r_abs"]),
                     float(bumps["corr_abs"]), _dp(prices), _dp(delta), _dp(gamma), _dp(vega),
                     _dp(th), _dp(rh), _dp(corr))
    return {"delta": delta, "gamma": gamma, "vega": vega, "theta": float(th[0]),
            "rho": float(rh[0]), "corr": corr[: N * (N - 1) // 2]}
