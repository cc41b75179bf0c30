// hs_api.cpp -- the C ABI: validation, planning, the pass loop that launches
// the path, Gram and sweep kernels on the caller's stream, and the Greeks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/hs_api.h"
#include "hs_kernels.hpp"
#include "hs_plan.hpp"
#include "hs_run.hpp"

namespace hs {

namespace {

bool hip_ok(hipError_t e, const char* what)
{
    if (e == hipSuccess) return true;
    set_error("%s failed: %s", what, hipGetErrorString(e));
    return false;
}

#define HS_HIP(call, what)                   \
    do {                                     \
        if (!hip_ok((call), (what))) return HS_EDEVICE; \
    } while (0)

// Cluster sweeps wait on each other's workgroups, so two of them must never
// compete for residency: one cluster launch sequence at a time per process.
std::mutex g_cluster_mu;

int64_t wall_clock_ticks(double seconds)
{
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;  // 100 MHz
    return static_cast<int64_t>(seconds * 1e3 * khz);
}

double mean_theta(const Request& q)
{
    double t = 0.0;
    for (double x : q.theta) t += x;
    return t / static_cast<double>(q.N);
}

}  // namespace

int default_target_waves() { return 2048; }

hs_status run_greek_set(const Request& q, void* d_ws, size_t ws_bytes, hipStream_t st,
                        RunResult& res, int target_waves)
{
    std::vector<Scenario> sc;
    hs_status rc = expand_scenarios(q, sc);
    if (rc != HS_OK) return rc;
    const Shape sh = shape_of(q);
    size_t mn = 0;
    const std::vector<Pass> passes = make_passes(q, sh, sc, ws_bytes, &mn);
    if (passes.empty()) {
        set_error("workspace of %zu bytes is below the minimum of %zu", ws_bytes, mn);
        return HS_ENOMEM;
    }
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) {
        set_error("workspace must be 256-byte aligned");
        return HS_EINVAL;
    }
    const size_t S = sc.size();
    res.price.assign(S, 0.0);
    res.se.assign(S, 0.0);
    res.skipped.assign(S, 0);
    if (q.opts.flags & HS_FLAG_EXPORT_TAU) res.tau.assign(S * static_cast<size_t>(q.P), 0);
    res.t_paths = res.t_gram = res.t_sweep = res.t_total = 0.0;
    res.n_passes = static_cast<int>(passes.size());

    const bool timing = (q.opts.flags & HS_FLAG_TIMING) != 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (timing)
        for (auto& e : ev) HS_HIP(hipEventCreate(&e), "hipEventCreate");
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard()
        {
            for (int i = 0; i < 4; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } guard{ev};

    unsigned char* ws = static_cast<unsigned char*>(d_ws);
    const int m = basis_m(q);
    const double tbar = mean_theta(q);
    const int tw = target_waves > 0 ? target_waves : default_target_waves();
    for (const Pass& pass : passes) {
        const PassPlan pp = plan_pass(q, sh, sc, pass, tw);
        if (pp.lay.total > ws_bytes) {
            set_error("internal: pass needs %zu bytes of a %zu-byte workspace", pp.lay.total,
                      ws_bytes);
            return HS_ENOMEM;
        }
        for (const GroupP& g : pp.groups)
            if (g.ntask > sh.tmax) {
                set_error("internal: a scenario group has %d tasks, the kernel holds %d", g.ntask,
                          sh.tmax);
                return HS_EINVAL;
            }
        const int Sp = static_cast<int>(pass.scen.size());
        HS_HIP(hipMemcpyAsync(ws + pp.lay.base, pp.base.data(), pp.base.size(),
                              hipMemcpyHostToDevice, st), "upload base");
        HS_HIP(hipMemcpyAsync(ws + pp.lay.tasks, pp.tasks.data(), pp.tasks.size(),
                              hipMemcpyHostToDevice, st), "upload tasks");
        HS_HIP(hipMemcpyAsync(ws + pp.lay.groups, pp.groups.data(),
                              pp.groups.size() * sizeof(GroupP), hipMemcpyHostToDevice, st),
               "upload groups");
        HS_HIP(hipMemcpyAsync(ws + pp.lay.disc, pp.disc.data(), pp.disc.size() * sizeof(double),
                              hipMemcpyHostToDevice, st), "upload discounts");

        PathArgs pa{};
        pa.base = ws + pp.lay.base;
        pa.tasks = ws + pp.lay.tasks;
        pa.groups = reinterpret_cast<const GroupP*>(ws + pp.lay.groups);
        pa.feat = ws + pp.lay.feat;
        pa.P = q.P;
        pa.plane = (sh.american ? static_cast<int64_t>(q.n) : 1) * q.P;
        pa.n = q.n;
        pa.N = q.N;
        pa.W = pp.W;
        pa.store_all = sh.american ? 1 : 0;
        pa.key0 = static_cast<uint32_t>(q.opts.seed);
        pa.key1 = static_cast<uint32_t>(q.opts.seed >> 32);

        LsmcArgs la{};
        la.feat = pa.feat;
        la.reg = reinterpret_cast<RegRec*>(ws + pp.lay.reg);
        la.disc = reinterpret_cast<const double*>(ws + pp.lay.disc);
        la.out = reinterpret_cast<double*>(ws + pp.lay.out);
        la.cf = reinterpret_cast<double*>(ws + pp.lay.cf);
        la.tau = reinterpret_cast<int32_t*>(ws + pp.lay.tau);
        la.P = q.P;
        la.plane = pa.plane;
        la.n = q.n;
        la.m = m;
        la.cp = q.opt.cp;
        la.american = sh.american ? 1 : 0;
        la.K = q.opt.K;
        la.inv_K = 1.0 / q.opt.K;
        la.inv_tbar = 1.0 / tbar;
        la.export_tau = (q.opts.flags & HS_FLAG_EXPORT_TAU) ? 1 : 0;

        if (timing) HS_HIP(hipEventRecord(ev[0], st), "hipEventRecord");
        HS_HIP(launch_paths(sh.fp32, sh.nmax, pa, pp.nchunks, pp.nbg, st), "path kernel launch");
        if (timing) HS_HIP(hipEventRecord(ev[1], st), "hipEventRecord");
        if (sh.american) HS_HIP(launch_gram(sh.fp32, la, Sp, st), "Gram kernel launch");
        if (timing) HS_HIP(hipEventRecord(ev[2], st), "hipEventRecord");
        // backward sweep: a cluster of workgroups per scenario when it fits the
        // device, else one workgroup per scenario with the state in the workspace
        std::unique_lock<std::mutex> cluster_lock(g_cluster_mu, std::defer_lock);
        uint32_t* sync = reinterpret_cast<uint32_t*>(ws + pp.lay.sync);
        int32_t* err_flag = reinterpret_cast<int32_t*>(sync);
        bool cluster = sh.sweep == kSweepCluster;
        int cap = 0;
        if (cluster) {
            cap = cluster_capacity(sh.fp32, sh.cluster_q, cluster_lds_bytes(q.n, sh.cluster_g));
            if (cap < sh.cluster_g) {
                if (q.opts.sweep_mode == 3) {
                    set_error("cluster sweep needs %d co-resident workgroups, the device holds %d",
                              sh.cluster_g, cap);
                    return HS_EDEVICE;
                }
                cluster = false;
            }
        }
        HS_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(sync), 1, 0, st), "clear sweep status");
        if (cluster) {
            HS_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(ws + pp.lay.part),
                                   static_cast<int64_t>(Sp) * (q.n + 2) * sh.cluster_g * kPartStride,
                                   kEmptySlot, st), "clear partial slots");
            ClusterArgs ca{};
            ca.partials = reinterpret_cast<double*>(ws + pp.lay.part);
            ca.error = err_flag;
            ca.G = sh.cluster_g;
            ca.timeout_ticks = wall_clock_ticks(10.0);
            const int per_launch = std::max(1, cap / sh.cluster_g);
            cluster_lock.lock();
            for (int s0 = 0; s0 < Sp; s0 += per_launch) {
                ca.s0 = s0;
                HS_HIP(launch_sweep_cluster(sh.fp32, sh.cluster_q, la, ca,
                                            std::min(per_launch, Sp - s0), st),
                       "cluster sweep launch");
            }
        } else {
            const int qreg = sh.sweep == kSweepBlockRegs ? sh.sweep_q : 0;
            HS_HIP(launch_sweep(sh.fp32, qreg, la, Sp, st), "sweep kernel launch");
        }
        if (timing) HS_HIP(hipEventRecord(ev[3], st), "hipEventRecord");

        std::vector<double> out(static_cast<size_t>(Sp) * 4);
        int32_t err_host = 0;
        HS_HIP(hipMemcpyAsync(out.data(), la.out, out.size() * sizeof(double),
                              hipMemcpyDeviceToHost, st), "download results");
        HS_HIP(hipMemcpyAsync(&err_host, err_flag, sizeof(int32_t), hipMemcpyDeviceToHost, st),
               "download sweep status");
        std::vector<int32_t> tau;
        if (la.export_tau) {
            tau.resize(static_cast<size_t>(Sp) * q.P);
            HS_HIP(hipMemcpyAsync(tau.data(), la.tau, tau.size() * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, st), "download tau");
        }
        HS_HIP(hipStreamSynchronize(st), "stream synchronize");
        if (cluster_lock.owns_lock()) cluster_lock.unlock();
        if (err_host != 0) {
            set_error("cluster sweep: a workgroup barrier timed out (device oversubscribed?)");
            return HS_EDEVICE;
        }
        for (int i = 0; i < Sp; ++i) {
            const int s = pass.scen[i];
            res.price[s] = out[i * 4 + 0];
            res.se[s] = out[i * 4 + 1];
            res.skipped[s] = static_cast<int64_t>(out[i * 4 + 2]);
            if (la.export_tau)
                std::memcpy(res.tau.data() + static_cast<size_t>(s) * q.P,
                            tau.data() + static_cast<size_t>(i) * q.P, q.P * sizeof(int32_t));
        }
        if (timing) {
            float a = 0, b = 0, c = 0;
            HS_HIP(hipEventElapsedTime(&a, ev[0], ev[1]), "hipEventElapsedTime");
            HS_HIP(hipEventElapsedTime(&b, ev[1], ev[2]), "hipEventElapsedTime");
            HS_HIP(hipEventElapsedTime(&c, ev[2], ev[3]), "hipEventElapsedTime");
            res.t_paths += a;
            res.t_gram += b;
            res.t_sweep += c;
            res.t_total += a + b + c;
        }
    }
    return HS_OK;
}

void fill_greeks(const Request& q, const RunResult& res, hs_greeks* out)
{
    const size_t S = res.price.size();
    out->price = res.price[0];
    out->price_se = res.se[0];
    out->n_scenarios = static_cast<int64_t>(S);
    int64_t sk = 0;
    for (int64_t v : res.skipped) sk += v;
    out->skipped_regressions = sk;
    if (out->scenario_price) std::memcpy(out->scenario_price, res.price.data(), S * sizeof(double));
    if (out->scenario_se) std::memcpy(out->scenario_se, res.se.data(), S * sizeof(double));
    if (out->tau && !res.tau.empty())
        std::memcpy(out->tau, res.tau.data(), res.tau.size() * sizeof(int32_t));
    greeks_from_prices(q, res.price, out);
    out->t_paths_ms = res.t_paths;
    out->t_gram_ms = res.t_gram;
    out->t_sweep_ms = res.t_sweep;
    out->t_total_ms = res.t_total;
}

size_t workspace_bound(const Request& q, bool minimum)
{
    const Shape sh = shape_of(q);
    const int N = q.N;
    const int64_t S = num_scenarios(N, q.bumps.mask);
    if (!minimum) return layout_for(q, sh, static_cast<int>(S), static_cast<int>(S * N),
                                    static_cast<int>(S) + 2 * kMaxWaves).total;
    const int head = 1 + ((q.bumps.mask & HS_BUMP_DELTA_GAMMA) ? 2 * N : 0);
    return std::max(layout_for(q, sh, head, N, 1 + 2 * kMaxWaves).total,
                    layout_for(q, sh, 1, N, 1 + 2 * kMaxWaves).total);
}

}  // namespace hs

using namespace hs;

extern "C" {

int64_t hs_num_scenarios(int32_t n_assets, const hs_bumps* bumps)
{
    if (!bumps || n_assets < 1 || n_assets > kMaxAssets) {
        set_error("hs_num_scenarios: n_assets outside 1..%d or null bumps", kMaxAssets);
        return -1;
    }
    return num_scenarios(n_assets, bumps->mask);
}

static size_t ws_query(const hs_model* model, const hs_option* option, int64_t n_paths,
                       int32_t n_steps, const hs_bumps* bumps, const hs_opts* opts, bool minimum)
{
    if (!model || model->n_assets < 1 || model->n_assets > kMaxAssets) {
        set_error("workspace query: bad model");
        return 0;
    }
    // the size does not depend on the correlation values: use the identity
    std::vector<double> I(static_cast<size_t>(model->n_assets) * model->n_assets, 0.0);
    for (int i = 0; i < model->n_assets; ++i) I[i * model->n_assets + i] = 1.0;
    Request q;
    if (copy_request(model, I.data(), option, n_paths, n_steps, bumps, opts, q) != HS_OK) return 0;
    if (validate(q) != HS_OK) return 0;
    return workspace_bound(q, minimum);
}

size_t hs_workspace_bytes(const hs_model* model, const hs_option* option, int64_t n_paths,
                          int32_t n_steps, const hs_bumps* bumps, const hs_opts* opts)
{
    return ws_query(model, option, n_paths, n_steps, bumps, opts, false);
}

size_t hs_workspace_min_bytes(const hs_model* model, const hs_option* option, int64_t n_paths,
                              int32_t n_steps, const hs_bumps* bumps, const hs_opts* opts)
{
    return ws_query(model, option, n_paths, n_steps, bumps, opts, true);
}

hs_status hs_price_greeks(const hs_model* model, const double* corr, const hs_option* option,
                          int64_t n_paths, int32_t n_steps, const hs_bumps* bumps,
                          const hs_opts* opts, void* d_workspace, size_t workspace_bytes,
                          void* hip_stream, hs_greeks* out)
{
    if (!out || !d_workspace) {
        set_error("hs_price_greeks: null out or workspace");
        return HS_EINVAL;
    }
    Request q;
    hs_status rc = copy_request(model, corr, option, n_paths, n_steps, bumps, opts, q);
    if (rc != HS_OK) return rc;
    rc = validate(q);
    if (rc != HS_OK) return rc;
    RunResult res;
    rc = run_greek_set(q, d_workspace, workspace_bytes, static_cast<hipStream_t>(hip_stream), res,
                       0);
    if (rc != HS_OK) return rc;
    fill_greeks(q, res, out);
    return HS_OK;
}

size_t hs_path_features_workspace_bytes(int32_t n_assets)
{
    (void)n_assets;
    return 2 * 256 + sizeof(BaseP<double>) + kMaxWaves * sizeof(GroupP);
}

hs_status hs_path_features(const hs_model* model, const double* corr, int64_t n_paths,
                           int32_t n_steps, double T, const hs_opts* opts, void* d_out,
                           size_t out_bytes, void* d_workspace, size_t workspace_bytes,
                           void* hip_stream)
{
    if (!d_out || !d_workspace) {
        set_error("hs_path_features: null output or workspace");
        return HS_EINVAL;
    }
    hs_option opt{HS_CALL, HS_AMERICAN, HS_MAX_OF, HS_BASIS_AUTO, 1.0, T};
    hs_bumps nob{0u, 0.0, 0.0, 0.0, 0.0, 0.0};
    Request q;
    hs_status rc = copy_request(model, corr, &opt, n_paths, n_steps, &nob, opts, q);
    if (rc != HS_OK) return rc;
    rc = validate(q);
    if (rc != HS_OK) return rc;
    std::vector<Scenario> sc;
    rc = expand_scenarios(q, sc);
    if (rc != HS_OK) return rc;
    const Shape sh = shape_of(q);
    const size_t need = static_cast<size_t>(n_steps) * n_paths * 2 * (sh.fp32 ? 4 : 8);
    if (out_bytes < need) {
        set_error("hs_path_features: output needs %zu bytes, got %zu", need, out_bytes);
        return HS_ENOMEM;
    }
    if (workspace_bytes < hs_path_features_workspace_bytes(q.N)) {
        set_error("hs_path_features: workspace needs %zu bytes",
                  hs_path_features_workspace_bytes(q.N));
        return HS_ENOMEM;
    }
    Pass pass;
    pass.scen = {0};
    pass.has_base_spot = true;
    PassPlan pp = plan_pass(q, sh, sc, pass, default_target_waves());
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    unsigned char* ws = static_cast<unsigned char*>(d_workspace);
    const size_t off_groups = (pp.base.size() + 255) / 256 * 256;
    HS_HIP(hipMemcpyAsync(ws, pp.base.data(), pp.base.size(), hipMemcpyHostToDevice, st),
           "upload base");
    HS_HIP(hipMemcpyAsync(ws + off_groups, pp.groups.data(), pp.groups.size() * sizeof(GroupP),
                          hipMemcpyHostToDevice, st), "upload groups");
    PathArgs pa{};
    pa.base = ws;
    pa.tasks = ws;  // no tasks
    pa.groups = reinterpret_cast<const GroupP*>(ws + off_groups);
    pa.feat = d_out;
    pa.P = q.P;
    pa.plane = static_cast<int64_t>(q.n) * q.P;
    pa.n = q.n;
    pa.N = q.N;
    pa.W = pp.W;
    pa.store_all = 1;
    pa.key0 = static_cast<uint32_t>(q.opts.seed);
    pa.key1 = static_cast<uint32_t>(q.opts.seed >> 32);
    HS_HIP(launch_paths(sh.fp32, sh.nmax, pa, pp.nchunks, pp.nbg, st), "path kernel launch");
    // the host tables must outlive the asynchronous uploads
    HS_HIP(hipStreamSynchronize(st), "stream synchronize");
    return HS_OK;
}

hs_status hs_philox_words(uint64_t seed, int64_t n_paths, int32_t n_steps, int32_t n_blocks,
                          uint32_t* d_out, void* hip_stream)
{
    if (!d_out || n_paths < 1 || n_steps < 1 || n_blocks < 1 ||
        n_paths * n_steps * n_blocks > (int64_t(1) << 31)) {
        set_error("hs_philox_words: bad sizes or null output");
        return HS_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HS_HIP(launch_philox_words(seed, n_paths, n_steps, n_blocks, d_out, st), "Philox launch");
    HS_HIP(hipStreamSynchronize(st), "stream synchronize");
    return HS_OK;
}

hs_status hs_normals(uint64_t seed, int32_t n_assets, int64_t n_paths, int32_t n_steps,
                     int32_t precision, void* d_eps, void* d_eta, void* hip_stream)
{
    if (!d_eps || !d_eta || n_assets < 1 || n_assets > kMaxAssets || n_paths < 1 ||
        n_steps < 1 || (precision != HS_FP64 && precision != HS_FP32_PATHS) ||
        n_paths * n_steps * n_assets > (int64_t(1) << 31)) {
        set_error("hs_normals: bad arguments");
        return HS_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HS_HIP(launch_normals(precision == HS_FP32_PATHS, seed, n_assets, n_paths, n_steps, d_eps,
                          d_eta, st), "normals launch");
    HS_HIP(hipStreamSynchronize(st), "stream synchronize");
    return HS_OK;
}

}  // extern "C"
