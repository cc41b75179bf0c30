// hs_plan.hpp -- host planner of a Greek set: validation, scenario expansion
// (bump-and-revalue with common random numbers), the task/group tables of
// the path kernel, and the workspace layout.  FP64 on the host throughout.
#pragma once
#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hs_api.h"
#include "hs_layout.hpp"

namespace hs {

void set_error(const char* fmt, ...);

// A request copied into host-owned storage.
struct Request {
    int N = 0;
    std::vector<double> S0, v0, kappa, theta, xi, rho;
    double r = 0.0;
    std::vector<double> C;  // N x N
    hs_option opt{};
    int64_t P = 0;
    int32_t n = 0;
    hs_bumps bumps{};
    hs_opts opts{};
};

// max_assets: kMaxAssets for Greek sets, kMaxPathAssets for the base-model
// path features.
hs_status copy_request(const hs_model* model, const double* corr, const hs_option* option,
                       int64_t n_paths, int32_t n_steps, const hs_bumps* bumps,
                       const hs_opts* opts, Request& out, int max_assets = kMaxAssets);
// Ranges and symmetry; max_waves bounds opts.waves_per_block, extra_flags
// are the flag bits the calling entry point accepts beyond the common ones.
hs_status validate(const Request& q, int max_waves = kMaxWaves, uint32_t extra_flags = 0u);

// One scenario of the Greek set (host FP64).
struct Scenario {
    int kind = 0;  // 0 base, 1 spot up, 2 spot down, 3 v0, 4 T, 5 r, 6 corr
    int i = -1, j = -1;
    std::vector<double> S0, v0, L;  // L = chol(C_scenario), N x N
    double r = 0.0, T = 0.0;
    int lo = 0, hi = 0;  // own asset range (assets whose path differs from base)
};

// Scenarios the path kernel derives from the base path without paths of
// their own: the base, the spot bumps (one asset's prices rescaled) and the
// rate bump (r enters the log price only through its drift r dt, so every
// asset's log price moves by (r' - r) t and U by the factor e^{(r' - r) t},
// while A and the variance paths stay the base's).
inline bool from_base_path(int kind) { return kind <= 2 || kind == 5; }

int basis_m(const Request& q);
bool cholesky(int N, const std::vector<double>& C, std::vector<double>& L);
hs_status expand_scenarios(const Request& q, std::vector<Scenario>& out);
int64_t num_scenarios(int N, uint32_t mask);
// The base scenario as the base-model path kernel's table (ModelP in the
// path precision).
std::vector<unsigned char> model_table(const Request& q, const Scenario& base, bool fp32);

// A pass runs a subset of scenarios whose features fit the workspace at once,
// or one unit (base and spots, or one bumped scenario) in windows of `window`
// dates with checkpoint-recompute of the paths (American only).
struct Pass {
    std::vector<int> scen;  // canonical scenario indices, in plane order
    bool has_base_spot = false;
    int window = 0;         // dates per window; 0 = all dates at once
};

// Byte offsets of a pass's regions inside the workspace.
struct Layout {
    size_t base = 0, tasks = 0, groups = 0, disc = 0, reg = 0, out = 0, tau = 0, cf = 0,
           sync = 0, part = 0, ckx = 0, ckv = 0, feat = 0, total = 0;
};

// Checkpoints a pass in windows of c dates keeps: the states at dates
// n - 2c, n - 3c, ... > 0.
inline int checkpoint_count(int n, int c) { return c > 0 ? std::max(0, (n - 1) / c - 1) : 0; }

// Backward-sweep variants.
enum SweepKind { kSweepCluster = 0, kSweepBlockRegs = 1, kSweepBlockState = 2 };

struct Shape {
    bool fp32 = true;
    bool american = true;
    int nmax = 0, tmax = 0;
    int feat = kFeatF32;    // FeatType of the stored features
    int sweep = kSweepCluster;
    int sweep_q = 0;        // single-workgroup sweep: paths per thread (0 = state in workspace)
    int cluster_q = 0;      // cluster sweep: paths per thread
    int cluster_g = 0;      // cluster sweep: workgroups per scenario
};

Shape shape_of(const Request& q);
Layout layout_for(const Request& q, const Shape& sh, int n_scen, int n_tasks, int n_groups,
                  int window = 0);

// Everything one pass uploads and launches.
struct PassPlan {
    std::vector<unsigned char> base;    // BaseP<R>
    std::vector<unsigned char> tasks;   // TaskP<R>[]
    std::vector<GroupP> groups;         // [nbg * W]
    std::vector<double> disc;           // [scen][n+1] exp(-r j dt), then [scen][n+1] exp(+r j dt)
    int W = 1, nbg = 1, nchunks = 1, ntasks = 0;
    int64_t plane = 0;  // feature elements per scenario plane (dates stored x P)
    Layout lay;
};

// target_waves: waves the path kernel aims for; wmax: most waves per block.
PassPlan plan_pass(const Request& q, const Shape& sh, const std::vector<Scenario>& sc,
                   const Pass& pass, int target_waves, int wmax);
// Splits the Greek set into passes that each fit `workspace_bytes` (one pass
// if everything fits); a unit that does not fit alone runs in windows of
// dates (the most dates that fit), and opts.window_dates > 0 runs every unit
// in windows of that many dates.  Empty result = even the smallest windows
// do not fit; *min_bytes then holds the least workspace that works.
std::vector<Pass> make_passes(const Request& q, const Shape& sh, const std::vector<Scenario>& sc,
                              size_t workspace_bytes, size_t* min_bytes);

// Greeks (host FP64) from scenario prices in canonical order.
void greeks_from_prices(const Request& q, const std::vector<double>& price, hs_greeks* out);

}  // namespace hs
