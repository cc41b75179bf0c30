/*
 * hs_api.h -- C ABI of the MI355X Heston / Longstaff-Schwartz Greek engine.
 *
 * What it computes (arXiv 2206.03719, "Low-power option Greeks"):
 *   Sec. 2.2 and 2.2.1 -- per-asset Heston stochastic-volatility Monte Carlo
 *   paths advanced in log price and exponentiated, a Longstaff-Schwartz
 *   reduction plus quadratic curve fit for early exercise, and the option's
 *   sensitivities (Greeks) to market moves.
 *   Sec. 4.1 -- the LS path reduction: for each path and timestep, the
 *   maximum value over assets.
 * The paper prints no equations; the discretisation (full-truncation Euler in
 * log price), the random-number layout (Philox4x32-10 with counter
 * (path mod 2^32, step, block, path >> 32) and key = seed), the regression
 * basis and the bump definitions are fixed conventions of this library and
 * are stated next to each entry point below.
 *
 * Conventions for every entry point:
 *   - Plain C; every call returns hs_status (0 = HS_OK, < 0 = error) and never
 *     throws.  On error, hs_last_error() returns a message for this thread and
 *     no output has been written.
 *   - "host" pointers are CPU memory owned by the caller and only read (or,
 *     for outputs, written) during the call.  "device" pointers are HIP
 *     device memory owned by the caller.  The library never allocates device
 *     memory: callers size workspaces with the *_bytes queries.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; calls that return host results synchronize it.
 *   - Arrays of per-asset values have n_assets entries.  Correlation matrices
 *     are n_assets x n_assets, row-major, symmetric, unit diagonal, SPD.
 */
#ifndef HS_API_H
#define HS_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HS_API_VERSION 1
#define HS_MAX_ASSETS 20      /* Greek sets and serving requests               */
#define HS_MAX_PATH_ASSETS 64 /* hs_path_features (the model alone)            */

typedef int32_t hs_status;
#define HS_OK 0
#define HS_EINVAL (-1)     /* an argument is out of its documented range        */
#define HS_ENOTSPD (-2)    /* a correlation matrix (maybe after a bump) not SPD  */
#define HS_ENOMEM (-3)     /* workspace or pool too small                        */
#define HS_EDEVICE (-4)    /* a HIP call failed, or a kernel reported an error   */
#define HS_EBUSY (-5)      /* serving: no free request slot in the queue         */
#define HS_ECANCELLED (-6) /* serving: the request was cancelled                 */
#define HS_ENOTFOUND (-7)  /* serving: unknown ticket                            */

/* option.cp */
#define HS_PUT 0
#define HS_CALL 1
/* option.style: EUROPEAN exercises at maturity only; AMERICAN at every date
 * k*T/n, k = 1..n (not at 0) -- a Bermudan grid on the simulation dates. */
#define HS_EUROPEAN 0
#define HS_AMERICAN 1
/* option.underlying: SINGLE needs n_assets == 1; MAX_OF pays on max_i S_i
 * (the paper's LS path reduction). */
#define HS_SINGLE 0
#define HS_MAX_OF 1
/* option.basis (regression functions of x = (U - cU)/K and w = (A - cA)/tbar,
 * U the underlying, A the mean over assets of max(v, 0), cU and cA their
 * means over the in-the-money paths at that date, tbar the mean long-run
 * variance of the base model):
 *   QUAD     = {1, x, x^2}          (m = 3)
 *   QUAD_VOL = {1, x, x^2, w, x w}  (m = 5)
 *   AUTO     = QUAD for one asset, QUAD_VOL otherwise. */
#define HS_BASIS_AUTO 0
#define HS_BASIS_QUAD 1
#define HS_BASIS_QUAD_VOL 2

/* bumps.mask bits.  Scenario order of a Greek set (fixed): base; spot up for
 * assets 0..N-1; spot down for 0..N-1 [DELTA_GAMMA]; v0 up for 0..N-1
 * [VEGA]; T - T_abs [THETA]; r + r_abs [RHO]; C_ij + corr_abs for i < j in
 * lexicographic order [CORR, N > 1]. */
#define HS_BUMP_DELTA_GAMMA 1u
#define HS_BUMP_VEGA 2u
#define HS_BUMP_THETA 4u
#define HS_BUMP_RHO 8u
#define HS_BUMP_CORR 16u
#define HS_BUMP_ALL 31u

/* opts.precision: HS_FP64 runs the paths in FP64; HS_FP32_PATHS runs the
 * paths in FP32 and stores FP32 features.  In both, payoffs, regression
 * (means, Gram matrix, right-hand side, Cholesky solve), exercise decisions
 * and discounted cash-flow sums are FP64. */
#define HS_FP64 0
#define HS_FP32_PATHS 1

/* opts.scheme: the time step of the Heston paths (Sec. 2.2 and 2.2.1).
 *   EULER_FT: full-truncation Euler in log price, v+ = max(v, 0):
 *     X += (r - v+/2) dt + sqrt(v+ dt) Z^S;
 *     v += kappa (theta - v+) dt + xi sqrt(v+ dt) Z^v.
 *   QE: Andersen's quadratic-exponential step, the benchmark's own scheme:
 *     the next variance matches the CIR conditional mean m and variance s^2
 *     (psi = s^2/m^2 <= 1.5: a (b + Z^v)^2; else 0 with probability
 *     p = (psi-1)/(psi+1), otherwise exponential with mean m/(1-p), drawn
 *     with the uniform Phi(Z^v)); log price
 *     X += r dt + K0 + K1 v + K2 v' + sqrt(K3 v + K4 v') Z^x with
 *     gamma1 = gamma2 = 1/2 and Z^x = sqrt(1-rho^2) Z^S - rho eta, the part
 *     of the spot shock orthogonal to the variance shock (K2 v' carries the
 *     rest).  Needs xi_i > 0 or rho_i = 0 for every asset.
 * In both, Z^S = L eps and Z^v = rho Z^S + sqrt(1-rho^2) eta, with (eps, eta)
 * the Box-Muller pairs of the same Philox counters: both schemes consume
 * identical random numbers, and the spot shocks of assets i and j correlate
 * as C_ij under either. */
#define HS_SCHEME_EULER_FT 0
#define HS_SCHEME_QE 1

/* opts.feature_format: how the per-date path features (U, A) are stored in
 * the workspace between the path kernel and the regression.  NATIVE: in the
 * path precision (8 B per path-step in FP32, 16 B in FP64).  FP16 / BF16:
 * rounded to nearest-even half or bfloat16 (4 B per path-step), a study of
 * reduced-precision storage in the spirit of the paper's numeric-
 * representation experiments (Sec. 4.2, Table 4); FP32 paths with the
 * EULER_FT scheme only.  The regression still reads them into FP64. */
#define HS_FEATURES_NATIVE 0
#define HS_FEATURES_FP16 1
#define HS_FEATURES_BF16 2

/* opts.flags */
#define HS_FLAG_EXPORT_TAU 1u /* write each path's exercise date into greeks.tau */
#define HS_FLAG_TIMING 2u     /* fill greeks.t_*_ms with per-stage device times  */
#define HS_FLAG_GRAPH 4u      /* run each pass as a hipGraph: captured once per
                                 launch shape and workspace, then replayed (needs a
                                 non-null stream; ignored with HS_FLAG_TIMING)      */
#define HS_FLAG_GREEK_SET_KERNEL 8u /* hs_path_features only: compute the features
                                 with the Greek-set path kernel that hs_price_greeks
                                 runs (n_assets <= HS_MAX_ASSETS, waves_per_block
                                 <= 8) instead of the base-model kernel; the two
                                 give the same features bit for bit              */

typedef struct hs_model {
    int32_t n_assets;       /* 1..HS_MAX_ASSETS (hs_path_features: ..64)       */
    const double *S0;       /* host, spot > 0                                  */
    const double *v0;       /* host, initial variance >= 0 (> 0 if VEGA)       */
    const double *kappa;    /* host, mean-reversion speed >= 0                 */
    const double *theta_lr; /* host, long-run variance > 0                     */
    const double *xi;       /* host, vol of vol >= 0                           */
    const double *rho_sv;   /* host, spot/variance correlation, |rho| < 1      */
    double r;               /* risk-free rate (continuous), finite             */
} hs_model;

typedef struct hs_option {
    int32_t cp;         /* HS_PUT | HS_CALL                   */
    int32_t style;      /* HS_EUROPEAN | HS_AMERICAN          */
    int32_t underlying; /* HS_SINGLE | HS_MAX_OF              */
    int32_t basis;      /* HS_BASIS_*                         */
    double K;           /* strike > 0                         */
    double T;           /* maturity in years > 0              */
} hs_option;

typedef struct hs_bumps {
    uint32_t mask;    /* HS_BUMP_* bits; 0 = price only                         */
    double spot_rel;  /* delta/gamma: S0_i (1 +- spot_rel), 0 < spot_rel < 1     */
    double v0_rel;    /* vega: v0_i (1 + v0_rel), > 0                            */
    double T_abs;     /* theta: T - T_abs with the step count fixed, 0 < T_abs < T */
    double r_abs;     /* rho: r + r_abs, != 0                                    */
    double corr_abs;  /* correlation: C_ij + corr_abs (both triangles), != 0     */
} hs_bumps;

typedef struct hs_opts {
    int32_t precision;       /* HS_FP64 | HS_FP32_PATHS                          */
    int32_t waves_per_block; /* path kernel launch shape: 0 = the tuned or
                                planner's choice, else 1..16 waves per block (capped
                                at the variant's most: 16 for FP32 Euler, 8 else, 4
                                for FP64 at 13-16 assets, FP64 QE from 10 and FP64
                                or QE at 17-20).  A block always follows
                                64 paths (one per lane) through every step; its waves
                                split the scenario groups, so this is the library's
                                paths-per-block and work-per-wave knob.  Steps are
                                not tiled: each step needs the previous one's state,
                                so a block runs them in order with the state in
                                registers.  Never changes results.                 */
    uint64_t seed;           /* Philox key                                         */
    uint32_t flags;          /* HS_FLAG_*                                          */
    int32_t sweep_mode;      /* backward sweep: 0 = automatic (cluster when it fits the
                                device), 1 = one workgroup per scenario with the state in
                                registers (n_paths <= 16384), 2 = one workgroup per scenario
                                with the state in the workspace, 3 = cluster of workgroups per
                                scenario (HS_EDEVICE if it cannot be co-resident)          */
    int32_t scheme;          /* HS_SCHEME_EULER_FT (0) | HS_SCHEME_QE (1)          */
    int32_t feature_format;  /* HS_FEATURES_NATIVE (0) | HS_FEATURES_FP16 (1) |
                                HS_FEATURES_BF16 (2)                               */
    int32_t window_dates;    /* American: 0 = the backward sweep runs over all
                                dates at once when the workspace holds them, else
                                in windows of dates with checkpoint-recompute of
                                the paths; > 0 (<= n_steps) = always in windows of
                                this many dates.  Never changes results.           */
    int32_t reserved;        /* must be zero                                       */
} hs_opts;

/* Results of a Greek set.  Caller-allocated host arrays; any may be NULL to
 * skip it.  Greeks not requested by bumps.mask are set to NaN.  Formulas
 * (h = spot_rel, hv = v0_rel):
 *   delta_i = (V(S0_i(1+h)) - V(S0_i(1-h))) / (2 h S0_i)
 *   gamma_i = (V(S0_i(1+h)) - 2 V + V(S0_i(1-h))) / (h S0_i)^2
 *   vega_i  = (V(v0_i(1+hv)) - V) / (hv v0_i)        (w.r.t. the variance v0)
 *   theta   = (V(T - T_abs) - V) / T_abs              (calendar decay)
 *   rho     = (V(r + r_abs) - V) / r_abs
 *   corr_ij = (V(C_ij + corr_abs) - V) / corr_abs,  i < j, lexicographic.
 * V is the mean over paths of the discounted cash flow CF exp(-r tau dt);
 * price_se is its standard error s/sqrt(P) (sample s.d., P-1). */
typedef struct hs_greeks {
    double price, price_se;
    double *delta, *gamma, *vega; /* n_assets each                            */
    double theta, rho;
    double *corr;                 /* n_assets (n_assets - 1) / 2               */
    double *scenario_price;       /* hs_num_scenarios entries, scenario order  */
    double *scenario_se;          /* hs_num_scenarios entries                  */
    int32_t *tau;                 /* HS_FLAG_EXPORT_TAU: scenarios x n_paths,
                                     exercise date index 1..n_steps            */
    int64_t n_scenarios;          /* written                                   */
    int64_t skipped_regressions;  /* sum over scenarios of dates whose fit was
                                     skipped (fewer ITM paths than basis
                                     functions, or a pivot <= 1e-12 of its
                                     diagonal entry)                           */
    double t_paths_ms, t_gram_ms, t_sweep_ms, t_total_ms; /* HS_FLAG_TIMING     */
} hs_greeks;

/* Number of scenarios in the Greek set that bumps->mask describes
 * (1 + 2N + N + 1 + 1 + N(N-1)/2 for HS_BUMP_ALL).  -1 if n_assets is out of
 * range or bumps is NULL.  (A sizing query of this interface: the paper asks
 * for per-asset sensitivities, Sec. 2.2, and names no call of its own.) */
int64_t hs_num_scenarios(int32_t n_assets, const hs_bumps *bumps);

/* Device workspace bytes hs_price_greeks needs to run the whole Greek set in
 * one pass (features of every scenario resident at once).  0 on invalid
 * arguments (see hs_last_error).  (A sizing query of this interface, so that
 * the caller owns all device memory; the paper has no counterpart.) */
size_t hs_workspace_bytes(const hs_model *model, const hs_option *option, int64_t n_paths,
                          int32_t n_steps, const hs_bumps *bumps, const hs_opts *opts);

/* Smallest workspace hs_price_greeks accepts; it then runs the Greek set in
 * several passes over scenario groups and, where one group's features do not
 * fit, in windows of dates that recompute the paths from checkpoints of their
 * state (same results, bit for bit).  With opts.window_dates > 0 both calls
 * size every group in windows of that many dates.  (A sizing query of this
 * interface; the windows answer the capacity problem that the paper meets by
 * batching paths through on-chip memory, Sec. 4.1 and Fig. 3.) */
size_t hs_workspace_min_bytes(const hs_model *model, const hs_option *option, int64_t n_paths,
                              int32_t n_steps, const hs_bumps *bumps, const hs_opts *opts);

/* Price and Greeks of one option under one Heston model (the paper's problem:
 * per-asset Heston configurations, assets x paths x timesteps in; per-asset
 * sensitivities out, Sec. 2.2.1).
 *   model, corr (host), option, bumps, opts: as documented above.
 *   n_paths in 2..2^31, n_steps in 1..4096 (dt = T / n_steps).
 *   d_workspace: device, >= hs_workspace_min_bytes, 256-byte aligned.
 *   out: host struct; its arrays are caller-allocated (see hs_greeks).
 * Validation happens before any device work.  Errors: HS_EINVAL (ranges,
 * NULLs, non-symmetric or non-unit-diagonal corr, theta bump T_abs >= T,
 * vega with v0_i = 0, reserved field non-zero), HS_ENOTSPD (corr or a
 * bumped corr not SPD), HS_ENOMEM (workspace too small), HS_EDEVICE. */
hs_status hs_price_greeks(const hs_model *model, const double *corr, const hs_option *option,
                          int64_t n_paths, int32_t n_steps, const hs_bumps *bumps,
                          const hs_opts *opts, void *d_workspace, size_t workspace_bytes,
                          void *hip_stream, hs_greeks *out);

/* hs_price_greeks without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same Greek set, with the same arguments, errors and
 * results (bit for bit), run in a workspace the library holds itself -- a
 * static device array of HS_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends.  A request whose minimum workspace (hs_workspace_min_bytes)
 * exceeds it is rejected with HS_ENOMEM before any device work; smaller ones
 * run in passes and windows of dates where they do not fit at once.  The
 * call allocates no device memory (HS_FLAG_GRAPH and HS_FLAG_TIMING, which
 * create runtime objects, are rejected with HS_EINVAL).  Every call on a GPU
 * uses that GPU's one array, and each pass rewrites what it reads (tables,
 * status flags, exchange slots): calls that overlap on one GPU race and must
 * not be made. */
#define HS_NOALLOC_SCRATCH_BYTES (64u << 20)
hs_status hs_price_greeks_noalloc(const hs_model *model, const double *corr,
                                  const hs_option *option, int64_t n_paths, int32_t n_steps,
                                  const hs_bumps *bumps, const hs_opts *opts, void *hip_stream,
                                  hs_greeks *out);

/* The paper's measured kernel on its own (Sec. 2.2.1 and 4.1, the problem
 * sizes of its Table 1): Heston paths of the base model and, at each date
 * k = 1..n_steps, the path reduction U = max_i S_i and A = (1/N) sum_i
 * max(v_i, 0), summed in asset order.
 *   model: n_assets in 1..HS_MAX_PATH_ASSETS (1..HS_MAX_ASSETS with
 *          HS_FLAG_GREEK_SET_KERNEL); corr, opts as for hs_price_greeks
 *          (opts.waves_per_block 0 = auto, else 1..16: waves that share a
 *          block of 64 paths, raised to ceil(ceil(n_assets / 2) / 8) if
 *          smaller; never changes the result).  Only HS_FLAG_GREEK_SET_KERNEL
 *          is accepted in opts.flags beyond the common flags, which are ignored.
 *   n_paths in 2..2^31, n_steps in 1..4096, T > 0 (dt = T / n_steps).
 *   d_out (device): [n_steps][n_paths][2] of double (HS_FP64), float
 *          (HS_FP32_PATHS), or half / bfloat16 with opts.feature_format
 *          FP16 / BF16; out_bytes must cover it (else HS_ENOMEM).
 *   d_workspace (device, 256-byte aligned): >= hs_path_features_workspace_bytes,
 *          which holds the model table the kernel reads.
 * Validation as for hs_price_greeks (HS_EINVAL, HS_ENOTSPD) before any device
 * work.  The work is enqueued on hip_stream and the call returns once that
 * stream has drained: the output is complete on return. */
size_t hs_path_features_workspace_bytes(int32_t n_assets);
hs_status hs_path_features(const hs_model *model, const double *corr, int64_t n_paths,
                           int32_t n_steps, double T, const hs_opts *opts, void *d_out,
                           size_t out_bytes, void *d_workspace, size_t workspace_bytes,
                           void *hip_stream);

/* Autotuner of the path kernel's launch shape (waves per block, scenario-group
 * granularity) for requests shaped like this one: times each candidate
 * `repeats` times on hip_stream with the given workspace, in the mode the
 * request will run in (graph replay if opts.flags has HS_FLAG_GRAPH), and
 * stores the fastest in a process-wide table keyed on everything that fixes
 * the launch (assets, path and step classes, scenarios, precision, scheme,
 * feature format, sweep mode and dates per window), which hs_price_greeks
 * and the server consult when opts.waves_per_block == 0.  These parameters
 * never change results (the backward-sweep shape, which does fix the order
 * of FP64 sums, depends only on the request and is not tuned).  *best_ms
 * (host, may be NULL) receives the winning Greek-set time.  Same arguments
 * and errors as hs_price_greeks.  (An interface call of this library: the
 * paper tunes its FPGA design by hand, Sec. 4.) */
hs_status hs_autotune(const hs_model *model, const double *corr, const hs_option *option,
                      int64_t n_paths, int32_t n_steps, const hs_bumps *bumps,
                      const hs_opts *opts, void *d_workspace, size_t workspace_bytes,
                      void *hip_stream, int32_t repeats, double *best_ms);

/* Diagnostics for bit-exactness checks of the device random numbers (the
 * paper streams precomputed random numbers into its kernel, Sec. 4; these
 * expose the ones this library draws on the device, for tests).
 * hs_philox_words: d_out (device uint32) receives, for path p in
 * [0, n_paths), step k in [0, n_steps) and block j in [0, n_blocks), the four
 * Philox4x32-10 words of counter (p mod 2^32, k, j, p >> 32) under key
 * (seed mod 2^32, seed >> 32) at d_out[((p n_steps + k) n_blocks + j) 4 ..].
 * hs_normals: d_eps and d_eta (device, double for HS_FP64 or float for
 * HS_FP32_PATHS) receive the Box-Muller normals of n_assets assets at
 * [(p n_steps + k) n_assets + a].  Both synchronize the stream. */
hs_status hs_philox_words(uint64_t seed, int64_t n_paths, int32_t n_steps, int32_t n_blocks,
                          uint32_t *d_out, void *hip_stream);
hs_status hs_normals(uint64_t seed, int32_t n_assets, int64_t n_paths, int32_t n_steps,
                     int32_t precision, void *d_eps, void *d_eta, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Serving: a continuous-batching request loop (an interface of this library;
 * the paper times single runs).  A server owns a caller-provided device pool
 * (its size is the HBM budget).  An idle slot admits, among the queued
 * requests whose workspace fits the free pool, the one with the least
 * estimated work (path-steps x (scenarios + path tasks)), so small requests
 * do not wait behind large ones; a request is passed by later ones at most
 * 2 x max_slots times, after which the slots wait for it.  Admitted requests
 * run on their own HIP streams: their path and Gram kernels run side by side
 * on the device, and a backward sweep whose workgroups wait on each other
 * runs while no other such sweep does (all its workgroups must be resident).
 * Each request's results are identical, bit for bit, to the same request run
 * alone.  A request larger than the pool runs in several passes in half of
 * it (or its minimum workspace, if larger).
 */
typedef struct hs_server hs_server;

typedef struct hs_request {
    hs_model model;        /* the host arrays are copied at submit time */
    const double *corr;    /* host, copied at submit time               */
    hs_option option;
    int64_t n_paths;
    int32_t n_steps;
    hs_bumps bumps;
    hs_opts opts;
} hs_request;

typedef struct hs_server_stats {
    int64_t submitted, completed, cancelled, failed, running, queued;
    size_t pool_bytes, pool_in_use, pool_peak;
    double path_steps_done;        /* sum over completed requests of S * P * n    */
    int32_t device_max_concurrent; /* most completed requests whose device work
                                      (HIP events on their streams) overlapped   */
    int32_t slots;                 /* max_slots of the server                    */
    double device_overlap_s;       /* seconds with two or more of them on the
                                      device at once                             */
} hs_server_stats;

/* device: HIP device ordinal; d_pool: device, pool_bytes of it (256-byte
 * aligned), owned by the caller until hs_server_destroy returns;
 * max_slots: 1..64 requests in flight; queue capacity is 4096 requests. */
hs_status hs_server_create(int device, void *d_pool, size_t pool_bytes, int32_t max_slots,
                           hs_server **out);
/* Validates and queues a request (HS_EBUSY if the queue is full). */
hs_status hs_submit(hs_server *srv, const hs_request *req, uint64_t *ticket);
/* *done = 1 and results in out once the request has finished (its arrays as
 * in hs_price_greeks, n_assets entries each); *done = 0 otherwise.  A
 * finished request's results can be polled once; then the ticket is retired.
 * Returns the request's own error status if it failed, HS_ECANCELLED if it
 * was cancelled, HS_ENOTFOUND for unknown or retired tickets.
 * Latency (submit to finish, seconds) is written to *latency_s if not NULL. */
hs_status hs_poll(hs_server *srv, uint64_t ticket, hs_greeks *out, int32_t *done,
                  double *latency_s);
/* Cancels a request that has not started (HS_EBUSY if it is already running). */
hs_status hs_cancel(hs_server *srv, uint64_t ticket);
hs_status hs_server_get_stats(hs_server *srv, hs_server_stats *out);
/* Waits for running requests, drops queued ones, frees host resources. */
void hs_server_destroy(hs_server *srv);

/* Message describing this thread's last non-OK status (never NULL). */
const char *hs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HS_API_H */
