// hs_layout.hpp -- plan tables shared by the host planner and the gfx950
// kernels: the per-scenario parameters of a Greek set, the "task" list that
// carries only what differs from the base scenario, and the regression
// records the Gram kernel hands to the backward sweep.
#pragma once
#include <cstddef>
#include <cstdint>

namespace hs {

constexpr int kMaxAssets = 20;
constexpr int kLanes = 64;        // one wave = 64 consecutive paths
constexpr int kMaxWaves = 16;     // most waves per path-kernel block (any variant)
constexpr int kOwnPerWave = 4;    // base assets owned by one wave of a block
// ... in the asset bucket nmax: 5 in the 20-asset bucket, so that four
// waves (one per SIMD) own its base assets
constexpr int paths_own_per_wave(int nmax) { return nmax > 16 ? 5 : kOwnPerWave; }
constexpr int kGramThreads = 256; // Gram kernel block
constexpr int kSweepThreads = 1024;
constexpr int kRegRec = 20;       // doubles per (scenario, date) regression record

// Tasks per wave of the Greek-set path kernel for its asset-count bucket
// nmax (at least nmax: the maturity and rate scenarios have a task per
// asset).  The QE scheme's FP64 variance state and FP64 paths take fewer, so
// that the kernel's registers hold them.
constexpr int paths_tmax_for(bool fp32, bool qe, int nmax)
{
    return !fp32 ? (nmax > 8 ? nmax : 8)
           : qe  ? (nmax > 16 ? nmax : 16)
                 : (nmax <= 8 ? 24 : nmax <= 12 ? 20 : nmax);
}

// Most waves per block of the Greek-set path kernel for a variant: 16 for
// FP32 Euler (at most 128 registers, which its tasks fit), so that all task
// groups of a path chunk can share one block's random numbers and base
// step; 8 otherwise.  FP64 at 13-16 assets needs more than 256 registers per
// lane; at one wave per SIMD
// (4 waves per block) the compiler holds the excess in the accumulation
// registers instead of spilling it to memory (16 assets x 25k paths: 104 ->
// 75 ms of path kernel, 13 assets: 60 -> 41 ms).  At 10 and 12 assets the
// smaller spill costs less than the halved occupancy.  The 20-asset FP64
// and QE variants (20 tasks of FP64 state per wave) and FP64 QE from 10
// assets take the same bound (the 20-asset bucket with five base assets per
// wave), so that no variant spills.
constexpr int paths_max_waves(bool fp32, bool qe, int nmax)
{
    return (fp32 && !qe) ? 16
           : ((!fp32 && nmax == 16) || (!fp32 && qe && nmax >= 10) || nmax == 20) ? 4 : 8;
}


// Storage type of the path features (U, A) in the workspace.
enum FeatType { kFeatF32 = 0, kFeatF64 = 1, kFeatF16 = 2, kFeatBF16 = 3 };
constexpr size_t feat_bytes(int ft) { return ft == kFeatF64 ? 16 : ft == kFeatF32 ? 8 : 4; }

// Quadratic-exponential step constants of one asset of one scenario (host
// FP64): E = exp(-kappa dt), mth = theta (1 - E), c1, c2 with the CIR
// conditional variance s^2 = v c1 + c2, the initial variance v0, the
// log-price coefficients K0 (with r dt), K1..K4, and rho, sqrt(1 - rho^2)
// that split the spot normal into the variance normal and its orthogonal
// part.  All FP64: the variance path and the log-price drift run in FP64 in
// both path precisions (K1 and K2 are near -rho/xi and +rho/xi, and their
// FP32 roundings would not cancel).
template <typename R>
struct QeP {
    double E, mth, c1, c2, v0, K0, K1, K2, K3, K4, rho, rhobar;
};

// One asset of the base scenario.  rhobar = sqrt(1 - rho^2) (host FP64).
template <typename R>
struct AssetP {
    R S0, v0, kappa, theta, xi, rho, rhobar, pad;
    QeP<R> qe;
};

// The base scenario, in the path precision R.
template <typename R>
struct BaseP {
    AssetP<R> a[kMaxAssets];
    R L[kMaxAssets * kMaxAssets];  // chol(C), row-major, upper part zero
    double L64[kMaxAssets * kMaxAssets];  // the same in FP64 (QE: FP64 spot normals)
    R S0_up[kMaxAssets];           // S0_i (1 + h) for the spot-up scenarios
    R S0_dn[kMaxAssets];           // S0_i (1 - h)
    R r, dt, invN, drdt;           // drdt: the rate scenario's (r' - r) dt
};

// A task advances one asset of one bumped scenario whose trajectory differs
// from the base one (v0, T, r or correlation bumps).  Tasks of a scenario
// are contiguous, in asset order, and cover the scenario's own asset range
// [lo, hi); assets outside it are the base scenario's, bit for bit.
//
// The fields of the Euler step come first and in one block, so that the
// kernel reads them with a few wide scalar loads: offsets of the asset's,
// lo's and hi's [asset][lane] rows (x kLanes), the flags first | last << 1,
// the scenario's feature-plane offset, the step constants and the Cholesky
// row.
template <typename R>
struct TaskP {
    int32_t a_el, lo_el, hi_el, flags;
    int64_t fo;       // scen * plane
    R S0, rho, rhobar, dt, r, kappa, theta, xi;
    R L[kMaxAssets];  // the scenario's Cholesky row of `asset` (the base row
                      // where the bump leaves it)
    int32_t asset, own_row, first, last, scen, lo, hi, pad;
    R v0, pad1;
    double L64[kMaxAssets];  // the same in FP64 (QE)
    QeP<R> qe;
};

// One wave's share of a block: its tasks, and whether it writes the base and
// spot-bumped scenarios (which need no state of their own).
struct GroupP {
    int32_t task0, ntask;
    int32_t base_scen;  // feature plane of the base scenario, or -1
    int32_t spot_up0;   // plane of spot-up asset 0 (asset a at +a), or -1
    int32_t spot_dn0;   // plane of spot-down asset 0, or -1
    int32_t rate_scen;  // plane of the rate scenario, or -1
    int32_t pad[2];
};

// Base-scenario path kernel (features of the model alone, no Greek
// scenarios) for up to kMaxPathAssets assets.  A wave owns up to BPW = 1, 2
// or 4 Philox blocks (asset pairs).  Waves per block: up to 16, or up to 8
// where the kernel needs more than 128 registers (the QE scheme, and FP64
// Euler with four blocks per wave), so that it never spills.
constexpr int kMaxPathAssets = 64;
constexpr int kBaseMaxWaves = 16;
constexpr int kBaseMaxBpw = 4;
constexpr int base_max_waves(bool fp32, bool qe, int bpw)
{
    return (qe || (!fp32 && bpw >= 4)) ? 8 : 16;
}

// The model in the path precision R, with the Cholesky factor of the
// correlation in rows of kMaxPathAssets entries (upper part and rows past N
// zero, and two more zero rows, kZeroPair, for slots that own no assets).
constexpr int kZeroPair = kMaxPathAssets / 2;
template <typename R>
struct ModelP {
    AssetP<R> a[kMaxPathAssets];
    R L[(kMaxPathAssets + 2) * kMaxPathAssets];
    double L64[(kMaxPathAssets + 2) * kMaxPathAssets];  // the same in FP64 (QE)
    R r, dt, invN, pad;
};
// Philox blocks per correlation chunk of the base-model kernel (the eps
// buffer in LDS is padded with zeros to a whole number of chunks); fp32: the
// spot normals are FP32 (FP32 Euler paths; under QE they are FP64).
constexpr int base_chunk(bool fp32) { return fp32 ? 4 : 2; }

struct BasePathArgs {
    const void* model;  // ModelP<R>
    void* feat;         // R2 [date][path]
    int64_t P;
    int32_t n, N, W, pad;
    uint32_t key0, key1;
};

// Checkpoint-recompute: a Greek set whose features do not fit its workspace
// runs the backward sweep in windows of ck_every dates, from the last window
// to the first.  The path kernel's first launch runs every step and keeps the
// path state (every base asset and every task, per path) at the dates n - c,
// n - 2c, ... > 0; each later window restarts from its checkpoint and
// recomputes only its own dates' features.  Window w holds dates
// max(1, n - (w + 1) c + 1) .. n - w c; the first launch writes window 0's
// features, and window w >= 1 starts from the state at date n - (w + 1) c,
// checkpoint i = w - 1: ckx [i][slot][P] (log price, R) and ckv [i][slot][P]
// (variance, R or FP64 under QE), slot = asset (base) or N + task index.
struct PathArgs {
    const void* base;      // BaseP<R>
    const void* tasks;     // TaskP<R>[]
    const GroupP* groups;  // [n_blockgroups * W]
    void* feat;            // R2 planes [scen][date][path]
    int64_t P;
    int64_t plane;         // elements per scenario plane (dates stored * P)
    int32_t n, N, W, store_all;
    uint32_t key0, key1;
    int32_t k_begin, k_end;  // steps k_begin..k_end-1 (step k: date k to k + 1)
    int32_t k_feat0;         // step whose date is feature index 0 (store_all)
    int32_t ck_every;        // dates per window (0: no checkpoints)
    int32_t ck_store;        // keep the state at the checkpoint dates
    int32_t ck_slots;        // N + tasks of the pass
    void* ckx;
    void* ckv;
};

// Regression record of one (scenario, date): the inverse of the lower
// Cholesky factor of the Gram matrix, packed row-major (m(m+1)/2 entries), the
// regression-set means, ok flag and set size.
struct RegRec {
    double L[15];
    double cU, cA, ok, cnt, pad;
};
static_assert(sizeof(RegRec) == kRegRec * sizeof(double), "RegRec layout");

struct LsmcArgs {
    const void* feat;      // R2 planes [scen][date - f_date0][path]
    RegRec* reg;           // [scen][date] (date index k-1 for date k)
    const double* disc;    // [scen][n+1] exp(-r j dt), host libm
    const double* idisc;   // [scen][n+1] exp(+r j dt), host libm
    double* out;           // [scen][4]: price, se, skipped, itm-count
    double* cf;            // [scen][P] state in the workspace (cash flows, or
                           // the cluster sweep's discounted cash flows between
                           // windows), else null
    int32_t* tau;          // [scen][P] state / export, or null
    int64_t P;
    int64_t plane;
    int32_t n, m, cp, american;
    double K, inv_K, inv_tbar;
    int32_t export_tau, pad;
    // dates of this launch: regressions k_lo..min(k_hi, n - 1); the first
    // window (win_first, k_hi = n) starts the cash flows from the payoff at
    // date n, the last (win_last, k_lo = 1) prices; features of date d sit
    // at index d - f_date0 of each plane
    int32_t k_lo, k_hi, f_date0, win_first, win_last, pad2;
};

// Cluster sweep: G workgroups of kClusterThreads cooperate on one scenario,
// meeting once per exercise date through per-workgroup partial slots.
constexpr int kClusterThreads = 512;
constexpr int kPartStride = 8;  // doubles per published workgroup partial
constexpr int kMaxClusterGroups = 1024;
constexpr int kPlanComputeUnits = 256;  // MI355X: the cluster sweep plans for this many CUs
// Paths per thread of the cluster sweep: the counts it is compiled for, and
// the most a workgroup holds in registers (two dates of features and the
// discounted cash flow per path, with the compiler's temporaries about 9
// registers per path with 8-byte features, FP32 pairs, and 17 with FP64
// pairs; up to 6 paths per thread (FP64 pairs: 5) two workgroups share a CU,
// above that one workgroup per CU with up to 256 registers, which holds 22
// FP32 pairs (250 registers; 24 spill) and 12 FP64 pairs without spilling).
// More paths per thread mean fewer workgroups per scenario, so more
// scenarios per launch and fewer launches of a large Greek set, each a chain
// of exchanges.
constexpr bool cluster_q_supported(int q, int ft)
{
    return (q >= 1 && q <= 8) || q == 10 || q == 12 ||
           (ft == kFeatF32 && (q == 16 || q == 18 || q == 20 || q == 22));
}
constexpr int cluster_qmax(int ft) { return ft == kFeatF32 ? 22 : 12; }

// Partial slots start as kEmptySlot (a NaN bit pattern that arithmetic never
// produces); a workgroup's published partial is the slot's only write.
constexpr uint64_t kEmptySlot = ~0ull;

// Exchange rows of a scenario: one per exercise date k = 1..n-1 (American
// only) and two for the price sums (rows n and n + 1); row0 is the first
// stored row (0 for American, n for European).
constexpr int cluster_row0(bool american, int n) { return american ? 0 : n; }
constexpr int cluster_rows(bool american, int n) { return n + 2 - cluster_row0(american, n); }

struct ClusterArgs {
    double* partials;     // [scen][rows][G][kPartStride], filled with kEmptySlot
    int32_t* error;       // set to 1 if a wait timed out
    int32_t s0;           // first scenario (plane) of this launch
    int32_t G;            // workgroups per scenario
    int64_t timeout_ticks;  // wall-clock ticks before a wait gives up
};

}  // namespace hs
