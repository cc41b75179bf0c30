// hs_run.hpp -- one Greek set on one stream (used by the C ABI and the server).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/hs_api.h"
#include "hs_plan.hpp"

namespace hs {

struct RunResult {
    std::vector<double> price, se;
    std::vector<int64_t> skipped;
    std::vector<int32_t> tau;  // [scenario][path] when exported
    double t_paths = 0, t_gram = 0, t_sweep = 0, t_total = 0;
    int n_passes = 0;
};

// Launch shape of the path kernel (0 = default): the autotuner's output.
struct Tune {
    int target_waves = 0;
    int wmax = 0;
};

// The tuned shape for requests like q (default if none was tuned).
Tune tuned_shape(const Request& q);
void store_tuned_shape(const Request& q, const Tune& t);

// Enqueues and completes (synchronizes st) the whole Greek set of a validated
// request in the given workspace; tune == nullptr uses the tuned table.
// shared: other streams of this process run Greek sets on the device at the
// same time (the server); each pass then holds the device to itself only for
// its cluster sweep, not for its path and Gram kernels.
hs_status run_greek_set(const Request& q, void* d_ws, size_t ws_bytes, hipStream_t st,
                        RunResult& res, const Tune* tune, bool shared = false);
void fill_greeks(const Request& q, const RunResult& res, hs_greeks* out);
size_t workspace_bound(const Request& q, bool minimum);
int default_target_waves();

}  // namespace hs
