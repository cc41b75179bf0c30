"""Python binding of libhs.so, the MI355X (gfx950) Heston / Longstaff-Schwartz
Greek engine.  Argument marshalling only: every step of the computation runs
in the library's HIP kernels; torch provides device memory and the stream.

The C ABI is ``include/hs_api.h``; the functions here keep its names without
the ``hs_`` prefix.  Importing this package never falls back to another
implementation: if the built library is missing, :func:`lib` raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libhs.so")

OK, EINVAL, ENOTSPD, ENOMEM, EDEVICE, EBUSY, ECANCELLED, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7
PUT, CALL = 0, 1
EUROPEAN, AMERICAN = 0, 1
SINGLE, MAX_OF = 0, 1
BASIS_AUTO, BASIS_QUAD, BASIS_QUAD_VOL = 0, 1, 2
BUMP_DELTA_GAMMA, BUMP_VEGA, BUMP_THETA, BUMP_RHO, BUMP_CORR, BUMP_ALL = 1, 2, 4, 8, 16, 31
FP64, FP32_PATHS = 0, 1
FLAG_EXPORT_TAU, FLAG_TIMING, FLAG_GRAPH, FLAG_GREEK_SET_KERNEL = 1, 2, 4, 8
MAX_ASSETS, MAX_PATH_ASSETS = 20, 64
NOALLOC_SCRATCH_BYTES = 64 << 20  # HS_NOALLOC_SCRATCH_BYTES
SCHEME_EULER_FT, SCHEME_QE = 0, 1
SCHEMES = {"euler": SCHEME_EULER_FT, "qe": SCHEME_QE}
FEATURES_NATIVE, FEATURES_FP16, FEATURES_BF16 = 0, 1, 2
FEATURES = {"native": FEATURES_NATIVE, "fp16": FEATURES_FP16, "bf16": FEATURES_BF16}
MAX_ASSETS = 20

_CP = {"put": PUT, "call": CALL}
_STYLE = {"european": EUROPEAN, "american": AMERICAN}
_UND = {"single": SINGLE, "max_of": MAX_OF}
_BASIS = {"auto": BASIS_AUTO, "quad": BASIS_QUAD, "quad_vol": BASIS_QUAD_VOL}
_PREC = {"fp64": FP64, "fp32": FP32_PATHS}

_STATUS = {0: "HS_OK", -1: "HS_EINVAL", -2: "HS_ENOTSPD", -3: "HS_ENOMEM", -4: "HS_EDEVICE",
           -5: "HS_EBUSY", -6: "HS_ECANCELLED", -7: "HS_ENOTFOUND"}


class HSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


_dp = ctypes.POINTER(ctypes.c_double)


class Model(ctypes.Structure):
    _fields_ = [("n_assets", ctypes.c_int32), ("S0", _dp), ("v0", _dp), ("kappa", _dp),
                ("theta_lr", _dp), ("xi", _dp), ("rho_sv", _dp), ("r", ctypes.c_double)]


class Option(ctypes.Structure):
    _fields_ = [("cp", ctypes.c_int32), ("style", ctypes.c_int32), ("underlying", ctypes.c_int32),
                ("basis", ctypes.c_int32), ("K", ctypes.c_double), ("T", ctypes.c_double)]


class Bumps(ctypes.Structure):
    _fields_ = [("mask", ctypes.c_uint32), ("spot_rel", ctypes.c_double),
                ("v0_rel", ctypes.c_double), ("T_abs", ctypes.c_double),
                ("r_abs", ctypes.c_double), ("corr_abs", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("sweep_mode", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("feature_format", ctypes.c_int32), ("window_dates", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Greeks(ctypes.Structure):
    _fields_ = [("price", ctypes.c_double), ("price_se", ctypes.c_double),
                ("delta", _dp), ("gamma", _dp), ("vega", _dp),
                ("theta", ctypes.c_double), ("rho", ctypes.c_double), ("corr", _dp),
                ("scenario_price", _dp), ("scenario_se", _dp),
                ("tau", ctypes.POINTER(ctypes.c_int32)), ("n_scenarios", ctypes.c_int64),
                ("skipped_regressions", ctypes.c_int64),
                ("t_paths_ms", ctypes.c_double), ("t_gram_ms", ctypes.c_double),
                ("t_sweep_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("model", Model), ("corr", _dp), ("option", Option), ("n_paths", ctypes.c_int64),
                ("n_steps", ctypes.c_int32), ("bumps", Bumps), ("opts", Opts)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("cancelled", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("running", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("pool_bytes", ctypes.c_size_t), ("pool_in_use", ctypes.c_size_t),
                ("pool_peak", ctypes.c_size_t), ("path_steps_done", ctypes.c_double),
                ("device_max_concurrent", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("device_overlap_s", ctypes.c_double)]


# every symbol include/hs_api.h declares, with its ctypes signature
_SIGS = {
    "hs_num_scenarios": (ctypes.c_int64, [ctypes.c_int32, ctypes.POINTER(Bumps)]),
    "hs_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Model), ctypes.POINTER(Option),
                                             ctypes.c_int64, ctypes.c_int32,
                                             ctypes.POINTER(Bumps), ctypes.POINTER(Opts)]),
    "hs_workspace_min_bytes": (ctypes.c_size_t, [ctypes.POINTER(Model), ctypes.POINTER(Option),
                                                 ctypes.c_int64, ctypes.c_int32,
                                                 ctypes.POINTER(Bumps), ctypes.POINTER(Opts)]),
    "hs_price_greeks": (ctypes.c_int32, [ctypes.POINTER(Model), _dp, ctypes.POINTER(Option),
                                         ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(Bumps),
                                         ctypes.POINTER(Opts), ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_void_p, ctypes.POINTER(Greeks)]),
    "hs_price_greeks_noalloc": (ctypes.c_int32, [ctypes.POINTER(Model), _dp,
                                                 ctypes.POINTER(Option), ctypes.c_int64,
                                                 ctypes.c_int32, ctypes.POINTER(Bumps),
                                                 ctypes.POINTER(Opts), ctypes.c_void_p,
                                                 ctypes.POINTER(Greeks)]),
    "hs_autotune": (ctypes.c_int32, [ctypes.POINTER(Model), _dp, ctypes.POINTER(Option),
                                     ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(Bumps),
                                     ctypes.POINTER(Opts), ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_double)]),
    "hs_path_features_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "hs_path_features": (ctypes.c_int32, [ctypes.POINTER(Model), _dp, ctypes.c_int64,
                                          ctypes.c_int32, ctypes.c_double, ctypes.POINTER(Opts),
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]),
    "hs_philox_words": (ctypes.c_int32, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "hs_normals": (ctypes.c_int32, [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]),
    "hs_server_create": (ctypes.c_int32, [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "hs_submit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Request),
                                   ctypes.POINTER(ctypes.c_uint64)]),
    "hs_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Greeks),
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "hs_cancel": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64]),
    "hs_server_get_stats": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "hs_server_destroy": (None, [ctypes.c_void_p]),
    "hs_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """The loaded libhs.so.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhs.so is not built (%s); run `python -m "
                               "paper_2206_03719_amd._build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st != OK:
        raise HSError(st, lib().hs_last_error().decode())


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class _Marshal:
    """Holds the numpy arrays the ctypes structs point into."""

    def __init__(self, model, corr, option, bumps=None, seed=42, precision="fp32", flags=0,
                 waves_per_block=0, sweep_mode=0, scheme="euler", features="native",
                 window_dates=0):
        self.arrs = [_f64(model[k]) for k in ("S0", "v0", "kappa", "theta", "xi", "rho")]
        N = len(self.arrs[0])
        self.N = N
        self.C = _f64(corr).reshape(N, N)
        ptr = [a.ctypes.data_as(_dp) for a in self.arrs]
        self.model = Model(N, *ptr, float(model["r"]))
        self.option = Option(_CP[option["cp"]], _STYLE[option["style"]],
                             _UND[option.get("underlying", "single" if N == 1 else "max_of")],
                             _BASIS[option.get("basis", "auto")], float(option["K"]),
                             float(option["T"]))
        b = bumps or {"mask": 0, "spot_rel": 0.01, "v0_rel": 0.01, "T_abs": 1 / 252,
                      "r_abs": 1e-3, "corr_abs": 0.01}
        self.bumps = Bumps(int(b["mask"]), float(b["spot_rel"]), float(b["v0_rel"]),
                           float(b["T_abs"]), float(b["r_abs"]), float(b["corr_abs"]))
        prec = _PREC[precision] if isinstance(precision, str) else int(precision)
        self.opts = Opts(prec, int(waves_per_block), int(seed), int(flags), int(sweep_mode),
                         SCHEMES[scheme] if isinstance(scheme, str) else int(scheme),
                         FEATURES[features] if isinstance(features, str) else int(features),
                         int(window_dates), 0)

    @property
    def corr_ptr(self):
        return self.C.ctypes.data_as(_dp)


def num_scenarios(n_assets, mask):
    b = Bumps(int(mask), 0.01, 0.01, 1 / 252, 1e-3, 0.01)
    return int(lib().hs_num_scenarios(int(n_assets), ctypes.byref(b)))


def workspace_bytes(model, option, n_paths, n_steps, bumps, precision="fp32", minimum=False,
                    flags=0, sweep_mode=0, scheme="euler", features="native", window_dates=0):
    m = _Marshal(model, np.eye(len(model["S0"])), option, bumps, precision=precision,
                 flags=flags, sweep_mode=sweep_mode, scheme=scheme, features=features,
                 window_dates=window_dates)
    f = lib().hs_workspace_min_bytes if minimum else lib().hs_workspace_bytes
    n = f(ctypes.byref(m.model), ctypes.byref(m.option), int(n_paths), int(n_steps),
          ctypes.byref(m.bumps), ctypes.byref(m.opts))
    if n == 0:
        raise HSError(EINVAL, lib().hs_last_error().decode())
    return int(n)


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def price_greeks(model, corr, option, n_paths, n_steps, bumps, seed=42, precision="fp32",
                 workspace=None, stream=None, export_tau=False, timing=False,
                 waves_per_block=0, sweep_mode=0, graph=False, scheme="euler",
                 features="native", window_dates=0, noalloc=False):
    """Price + bump-and-revalue Greeks of one option (hs_price_greeks).

    ``workspace``: a CUDA uint8 tensor (allocated here when None).  ``graph``:
    replay the pass's kernels from a cached HIP graph.  ``window_dates``: run
    the backward sweep in windows of that many dates with checkpoint-recompute
    of the paths (0: only if the workspace needs it).  ``noalloc``: call
    hs_price_greeks_noalloc instead, which runs in the library's static
    scratch (no workspace).  Returns a dict of numpy arrays / floats."""
    torch = _torch()
    flags = ((FLAG_EXPORT_TAU if export_tau else 0) | (FLAG_TIMING if timing else 0) |
             (FLAG_GRAPH if graph else 0))
    m = _Marshal(model, corr, option, bumps, seed, precision, flags, waves_per_block, sweep_mode,
                 scheme, features, window_dates)
    N = m.N
    if workspace is None and not noalloc:
        nbytes = workspace_bytes(model, option, n_paths, n_steps, bumps, precision, flags=flags,
                                 sweep_mode=sweep_mode, scheme=scheme, features=features,
                                 window_dates=window_dates)
        workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    S = num_scenarios(N, m.bumps.mask)
    out_arrays = {"delta": np.zeros(N), "gamma": np.zeros(N), "vega": np.zeros(N),
                  "corr": np.zeros(max(N * (N - 1) // 2, 1)), "scenario_price": np.zeros(S),
                  "scenario_se": np.zeros(S)}
    tau = np.zeros((S, n_paths), dtype=np.int32) if export_tau else None
    g = Greeks()
    for k, a in out_arrays.items():
        setattr(g, k, a.ctypes.data_as(_dp))
    if tau is not None:
        g.tau = tau.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    if noalloc:
        st = lib().hs_price_greeks_noalloc(ctypes.byref(m.model), m.corr_ptr,
                                           ctypes.byref(m.option), int(n_paths), int(n_steps),
                                           ctypes.byref(m.bumps), ctypes.byref(m.opts),
                                           _stream_handle(stream), ctypes.byref(g))
    else:
        st = lib().hs_price_greeks(ctypes.byref(m.model), m.corr_ptr, ctypes.byref(m.option),
                                   int(n_paths), int(n_steps), ctypes.byref(m.bumps),
                                   ctypes.byref(m.opts), ctypes.c_void_p(workspace.data_ptr()),
                                   workspace.numel() * workspace.element_size(),
                                   _stream_handle(stream), ctypes.byref(g))
    _check(st)
    res = {"price": g.price, "price_se": g.price_se, "theta": g.theta, "rho": g.rho,
           "n_scenarios": g.n_scenarios, "skipped_regressions": g.skipped_regressions,
           "t_paths_ms": g.t_paths_ms, "t_gram_ms": g.t_gram_ms, "t_sweep_ms": g.t_sweep_ms,
           "t_total_ms": g.t_total_ms}
    res.update(out_arrays)
    res["corr"] = out_arrays["corr"][: N * (N - 1) // 2]
    if tau is not None:
        res["tau"] = tau
    return res


def autotune(model, corr, option, n_paths, n_steps, bumps, seed=42, precision="fp32",
             workspace=None, stream=None, repeats=3, scheme="euler", graph=False):
    """Times the path kernel's launch shapes on this request class and stores
    the fastest for later calls (hs_autotune); ``graph``: time them as graph
    replays, the way the calls will run.  Returns the best ms per set."""
    torch = _torch()
    m = _Marshal(model, corr, option, bumps, seed, precision, FLAG_GRAPH if graph else 0,
                 scheme=scheme)
    if workspace is None:
        nbytes = workspace_bytes(model, option, n_paths, n_steps, bumps, precision)
        workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    best = ctypes.c_double(0.0)
    _check(lib().hs_autotune(ctypes.byref(m.model), m.corr_ptr, ctypes.byref(m.option),
                             int(n_paths), int(n_steps), ctypes.byref(m.bumps),
                             ctypes.byref(m.opts), ctypes.c_void_p(workspace.data_ptr()),
                             workspace.numel() * workspace.element_size(),
                             _stream_handle(stream), int(repeats), ctypes.byref(best)))
    return best.value


def path_features(model, corr, T, n_paths, n_steps, seed=42, precision="fp64", stream=None,
                  scheme="euler", features="native", greek_set_kernel=False, waves_per_block=0,
                  out=None):
    """Heston paths + per-date path reduction of the base model
    (hs_path_features): a CUDA tensor [n_steps, n_paths, 2] of (U, A).
    greek_set_kernel: compute them with the Greek-set path kernel instead of
    the base-model kernel (same result).  out: an existing tensor of that
    shape and dtype to write into."""
    torch = _torch()
    m = _Marshal(model, corr, {"cp": "call", "style": "american", "K": 1.0, "T": T},
                 None, seed, precision, scheme=scheme, features=features,
                 flags=FLAG_GREEK_SET_KERNEL if greek_set_kernel else 0,
                 waves_per_block=waves_per_block)
    dtype = {FEATURES_FP16: torch.float16, FEATURES_BF16: torch.bfloat16}.get(
        m.opts.feature_format, torch.float64 if m.opts.precision == FP64 else torch.float32)
    if out is None:
        out = torch.empty((n_steps, n_paths, 2), dtype=dtype, device="cuda")
    elif out.dtype != dtype or tuple(out.shape) != (n_steps, n_paths, 2) or not out.is_contiguous():
        raise ValueError("out must be a contiguous %s tensor of shape %s"
                         % (dtype, (n_steps, n_paths, 2)))
    wsb = int(lib().hs_path_features_workspace_bytes(m.N))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    st = lib().hs_path_features(ctypes.byref(m.model), m.corr_ptr, int(n_paths), int(n_steps),
                                float(T), ctypes.byref(m.opts), ctypes.c_void_p(out.data_ptr()),
                                out.numel() * out.element_size(), ctypes.c_void_p(ws.data_ptr()),
                                wsb, _stream_handle(stream))
    _check(st)
    return out


def philox_words(seed, n_paths, n_steps, n_blocks, stream=None):
    """Device Philox4x32-10 words as a numpy uint32 array [P, n, blocks, 4]."""
    torch = _torch()
    out = torch.empty(n_paths * n_steps * n_blocks * 4, dtype=torch.int32, device="cuda")
    _check(lib().hs_philox_words(int(seed), int(n_paths), int(n_steps), int(n_blocks),
                                 ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out.cpu().numpy().view(np.uint32).reshape(n_paths, n_steps, n_blocks, 4)


def normals(seed, n_assets, n_paths, n_steps, precision="fp64", stream=None):
    """Device Box-Muller normals: (eps, eta) numpy arrays [P, n, N]."""
    torch = _torch()
    prec = _PREC[precision]
    dtype = torch.float64 if prec == FP64 else torch.float32
    eps = torch.empty((n_paths, n_steps, n_assets), dtype=dtype, device="cuda")
    eta = torch.empty_like(eps)
    _check(lib().hs_normals(int(seed), int(n_assets), int(n_paths), int(n_steps), prec,
                            ctypes.c_void_p(eps.data_ptr()), ctypes.c_void_p(eta.data_ptr()),
                            _stream_handle(stream)))
    return eps.cpu().numpy(), eta.cpu().numpy()


class Server:
    """Continuous-batching request loop over a device pool (hs_server_*)."""

    def __init__(self, pool_bytes, max_slots=4, device=0):
        torch = _torch()
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda:%d" % device)
        h = ctypes.c_void_p()
        _check(lib().hs_server_create(int(device), ctypes.c_void_p(self.pool.data_ptr()),
                                      int(pool_bytes), int(max_slots), ctypes.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, w, precision=None):
        m = _Marshal(w["model"], w["corr"], w["option"], w["bumps"], w.get("seed", 42),
                     precision or w.get("precision", "fp32"), scheme=w.get("scheme", "euler"),
                     features=w.get("features", "native"),
                     window_dates=w.get("window_dates", 0))
        req = Request(m.model, m.corr_ptr, m.option, int(w["n_paths"]), int(w["n_steps"]),
                      m.bumps, m.opts)
        t = ctypes.c_uint64()
        _check(lib().hs_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (m.N, num_scenarios(m.N, m.bumps.mask))
        return t.value

    def poll(self, ticket):
        """None while running; else (result dict, latency seconds)."""
        N, S = self._keep.get(ticket, (1, 1))
        arrs = {"delta": np.zeros(N), "gamma": np.zeros(N), "vega": np.zeros(N),
                "corr": np.zeros(max(N * (N - 1) // 2, 1)), "scenario_price": np.zeros(S),
                "scenario_se": np.zeros(S)}
        g = Greeks()
        for k, a in arrs.items():
            setattr(g, k, a.ctypes.data_as(_dp))
        done = ctypes.c_int32(0)
        lat = ctypes.c_double(0.0)
        st = lib().hs_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(g), ctypes.byref(done),
                           ctypes.byref(lat))
        if st == OK and not done.value:
            return None
        self._keep.pop(ticket, None)
        _check(st)
        res = {"price": g.price, "price_se": g.price_se, "theta": g.theta, "rho": g.rho,
               "n_scenarios": g.n_scenarios, "skipped_regressions": g.skipped_regressions}
        res.update(arrs)
        res["corr"] = arrs["corr"][: N * (N - 1) // 2]
        return res, lat.value

    def cancel(self, ticket):
        _check(lib().hs_cancel(self.h, ctypes.c_uint64(ticket)))

    def stats(self):
        s = ServerStats()
        _check(lib().hs_server_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self.h:
            lib().hs_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
