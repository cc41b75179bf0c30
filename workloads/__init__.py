"""Seeded synthetic inputs for the Heston LSMC Greek engine.

This module holds input *recipes* only -- parameter draws and shapes -- and
none of the method's arithmetic.  Both the FP64 oracle (``oracle/``) and the
HIP library's Python binding take these dictionaries, each mapping the plain
strings below to its own integer codes.

The paper benchmarks STAC-A2, whose specification and data are not available
here; these recipes stand in for it with the shapes the paper uses (5-50
assets, 126-1260 daily timesteps, 25k paths; Table 1) and the parameter ranges
of the workload definitions below.

Model dict: ``S0, v0, kappa, theta, xi, rho`` (arrays of length N) and ``r``.
Option dict: ``cp`` ('put'|'call'), ``style`` ('american'|'european'),
``underlying`` ('single'|'max_of'), ``basis`` ('auto'|'quad'|'quad_vol'),
``K``, ``T``.  Bumps dict: ``mask`` (1 delta/gamma, 2 vega, 4 theta, 8 rho,
16 corr) and the sizes ``spot_rel, v0_rel, T_abs, r_abs, corr_abs``.
"""
import numpy as np

MASK_DELTA_GAMMA, MASK_VEGA, MASK_THETA, MASK_RHO, MASK_CORR = 1, 2, 4, 8, 16
MASK_ALL = 31


def default_bumps(mask=MASK_ALL):
    """Bump sizes: +-1% spot, +1% v0 (relative), T - 1/252, r + 1e-3, C_ij + 0.01."""
    return {"mask": int(mask), "spot_rel": 0.01, "v0_rel": 0.01, "T_abs": 1.0 / 252.0,
            "r_abs": 1e-3, "corr_abs": 0.01}


def single_asset_put(n_paths=1024, n_steps=64, seed=42):
    """Single-asset Heston American put, FP64: S0=K=100, r=0.02, T=1, kappa=2,
    theta=0.04, xi=0.3, rho=-0.7, v0=0.04; price + delta/gamma by +-1% spot."""
    model = {"S0": np.array([100.0]), "v0": np.array([0.04]), "kappa": np.array([2.0]),
             "theta": np.array([0.04]), "xi": np.array([0.3]), "rho": np.array([-0.7]),
             "r": 0.02}
    option = {"cp": "put", "style": "american", "underlying": "single", "basis": "auto",
              "K": 100.0, "T": 1.0}
    return {"name": "heston-american-put-1x%dx%d" % (n_paths, n_steps), "model": model,
            "corr": np.eye(1), "option": option, "n_paths": n_paths, "n_steps": n_steps,
            "bumps": default_bumps(MASK_DELTA_GAMMA), "seed": seed, "precision": "fp64"}


def one_factor_corr(beta):
    """SPD correlation C_ij = beta_i beta_j (i != j), C_ii = 1."""
    beta = np.asarray(beta, dtype=np.float64)
    C = np.outer(beta, beta)
    np.fill_diagonal(C, 1.0)
    return C


def draw_assets(n_assets, rng):
    """Per asset, in this order: S0 ~ U[80,120], v0 = theta ~ U[0.02,0.09],
    kappa ~ U[1,3], xi ~ U[0.2,0.6], rho ~ U[-0.8,-0.3], beta ~ U[0.45,0.65]."""
    S0, v0, kappa, xi, rho, beta = [], [], [], [], [], []
    for _ in range(n_assets):
        S0.append(rng.uniform(80.0, 120.0))
        v0.append(rng.uniform(0.02, 0.09))
        kappa.append(rng.uniform(1.0, 3.0))
        xi.append(rng.uniform(0.2, 0.6))
        rho.append(rng.uniform(-0.8, -0.3))
        beta.append(rng.uniform(0.45, 0.65))
    v0 = np.array(v0)
    model = {"S0": np.array(S0), "v0": v0.copy(), "kappa": np.array(kappa), "theta": v0.copy(),
             "xi": np.array(xi), "rho": np.array(rho), "r": 0.02}
    return model, one_factor_corr(beta)


def best_of_call(n_assets=5, n_paths=25000, n_steps=252, seed=42, param_seed=42,
                 precision="fp32", mask=MASK_ALL):
    """Correlated Heston assets (random SPD correlation, off-diagonals ~0.3),
    American best-of call K=100, T=1, full Greek set.  n_assets=5 with 25k x 252
    is the 5-asset workload; n_assets=10 with 100k-1M or 200k paths are the
    10-asset ones (the first 5 assets of the 10-asset draw equal the 5-asset
    draw, since assets are drawn in sequence from the same generator)."""
    rng = np.random.default_rng(param_seed)
    model, C = draw_assets(n_assets, rng)
    option = {"cp": "call", "style": "american",
              "underlying": "max_of" if n_assets > 1 else "single", "basis": "auto",
              "K": 100.0, "T": 1.0}
    return {"name": "heston-bestof-call-%dx%dx%d" % (n_assets, n_paths, n_steps), "model": model,
            "corr": C, "option": option, "n_paths": n_paths, "n_steps": n_steps,
            "bumps": default_bumps(mask), "seed": seed, "precision": precision}


# The problem-size classes of the paper's Table 1: (name, assets, daily
# timesteps, paths).  The horizon is one trading day per step, T = steps / 252
# years (6 months for the smallest class, 5 years for the largest).
PAPER_SIZES = (("tiny", 5, 126, 25_000), ("small", 10, 126, 25_000),
               ("medium", 20, 252, 25_000), ("large", 30, 504, 25_000),
               ("huge", 50, 1260, 25_000))


def paper_size(name, seed=42, param_seed=42, n_paths=None):
    """One Table 1 class as a model-only workload (no option, no bumps): the
    best-of parameter draws for that many assets, T = steps / 252."""
    for nm, N, n, P in PAPER_SIZES:
        if nm == name:
            rng = np.random.default_rng(param_seed)
            model, C = draw_assets(N, rng)
            return {"name": "table1-%s-%dx%dx%d" % (nm, N, n, P), "model": model, "corr": C,
                    "n_assets": N, "n_steps": n, "n_paths": P if n_paths is None else n_paths,
                    "T": n / 252.0, "seed": seed}
    raise KeyError(name)


def serving_stream(n_requests, rate_per_s, seed=7, paths=(10_000, 400_000),
                   steps=(52, 126, 252, 504), assets=(1, 20), precision="fp32"):
    """Poisson arrivals of full-Greek-set requests: assets ~ U{1..20}, paths ~
    U[10k, 400k], steps ~ U{52,126,252,504}, parameters as the best-of workload.
    Returns a list of (arrival_time_s, request_dict)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        N = int(rng.integers(assets[0], assets[1] + 1))
        P = int(rng.integers(paths[0], paths[1] + 1))
        n = int(rng.choice(steps))
        model, C = draw_assets(N, rng)
        option = {"cp": "call", "style": "american", "underlying": "max_of", "basis": "auto",
                  "K": 100.0, "T": 1.0}
        req = {"name": "req%d" % i, "model": model, "corr": C, "option": option,
               "n_paths": P, "n_steps": n, "bumps": default_bumps(MASK_ALL),
               "seed": 42 + i, "precision": precision}
        out.append((t, req))
    return out


def gbm_limit_put(S0=100.0, K=100.0, sigma2=0.04, r=0.02, T=1.0, n_paths=20000, n_steps=16,
                  seed=1, style="american"):
    """Single asset with vol-of-vol 0 and v0 = theta: a Black-Scholes world
    (sigma^2 = theta) used by the closed-form pins."""
    model = {"S0": np.array([S0]), "v0": np.array([sigma2]), "kappa": np.array([1.5]),
             "theta": np.array([sigma2]), "xi": np.array([0.0]), "rho": np.array([0.0]),
             "r": r}
    option = {"cp": "put", "style": style, "underlying": "single", "basis": "auto", "K": K,
              "T": T}
    return {"name": "gbm-put", "model": model, "corr": np.eye(1), "option": option,
            "n_paths": n_paths, "n_steps": n_steps, "bumps": default_bumps(MASK_DELTA_GAMMA),
            "seed": seed, "precision": "fp64"}
