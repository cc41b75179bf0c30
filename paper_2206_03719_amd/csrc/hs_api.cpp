// hs_api.cpp -- the C ABI: validation, planning, the pass loop that launches
// the path, Gram and sweep kernels on the caller's stream, and the Greeks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
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

// about three waves per SIMD when paths are few; fewer waves per block (less
// per-wave feature work) once the paths alone fill the device
int default_target_waves() { return 3072; }

// ---------------------------------------------------------------------------
// Tuning table: launch shape of the path kernel per request class.

namespace {

struct TuneKey {
    int N, log2P, n_bucket, S, fp32, scheme, feat, sweep_mode, window, american;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(N, log2P, n_bucket, S, fp32, scheme, feat, sweep_mode, window, american) <
               std::tie(o.N, o.log2P, o.n_bucket, o.S, o.fp32, o.scheme, o.feat, o.sweep_mode,
                        o.window, o.american);
    }
};

std::mutex g_tune_mu;
std::map<TuneKey, Tune> g_tune;

TuneKey tune_key(const Request& q)
{
    int lp = 0;
    while ((int64_t(1) << (lp + 1)) <= q.P) ++lp;
    int nb = 0;
    while ((1 << (nb + 1)) <= q.n) ++nb;
    return {q.N, lp, nb, static_cast<int>(num_scenarios(q.N, q.bumps.mask)),
            q.opts.precision == HS_FP32_PATHS ? 1 : 0, q.opts.scheme, q.opts.feature_format,
            q.opts.sweep_mode, q.opts.window_dates, q.opt.style == HS_AMERICAN ? 1 : 0};
}

// ---------------------------------------------------------------------------
// Graph cache: one instantiated graph per (device, workspace, launch arguments).

std::mutex g_graph_mu;
std::map<std::string, hipGraphExec_t> g_graphs;
constexpr size_t kMaxGraphs = 128;

template <typename T>
void append_bytes(std::string& k, const T& v)
{
    k.append(reinterpret_cast<const char*>(&v), sizeof v);
}

// Everything one pass enqueues after its tables are uploaded.
struct PassLaunch {
    bool fp32 = true, american = true, cluster = false;
    int scheme = HS_SCHEME_EULER_FT;
    int feat = kFeatF32;
    int nmax = 0, nchunks = 0, nbg = 0, Sp = 0, cluster_q = 0, per_launch = 0, sweep_q = 0;
    int window = 0;  // dates per window of a checkpoint-recompute pass, else 0
    int64_t part_count = 0;
    PathArgs pa{};
    LsmcArgs la{};
    ClusterArgs ca{};
    int32_t* err_flag = nullptr;
};

hipError_t enqueue_sweep(const PassLaunch& L, const LsmcArgs& la, hipStream_t st)
{
    hipError_t e;
    if (L.cluster) {
        ClusterArgs ca = L.ca;
        for (int s0 = 0; s0 < L.Sp; s0 += L.per_launch) {
            ca.s0 = s0;
            if ((e = launch_sweep_cluster(L.feat, L.cluster_q, la, ca,
                                          std::min(L.per_launch, L.Sp - s0), st)) != hipSuccess)
                return e;
        }
        return hipSuccess;
    }
    return launch_sweep(L.feat, L.sweep_q, la, L.Sp, st);
}

// Events ev[0..3] (optional) bracket the path kernel, the Gram kernel and the
// sweep; in a windowed pass ev[1] follows the first path launch and the
// windows (recompute, Gram, sweep) count as the sweep.
//
// A one-pass launch sequence in two parts: the front (status and slot fills,
// path kernel, Gram kernel), which may run beside other requests' work, and
// the back (the backward sweep), whose cluster workgroups wait on each other.
hipError_t enqueue_front(const PassLaunch& L, hipStream_t st, hipEvent_t* ev)
{
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
    if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(L.err_flag), 1, 0, st)) != hipSuccess)
        return e;
    if ((e = launch_paths(L.fp32, L.nmax, L.scheme, L.feat, L.pa, L.nchunks, L.nbg, st)) !=
        hipSuccess)
        return e;
    if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
    if (L.american && (e = launch_gram(L.feat, L.la, L.Sp, st)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
    if (L.cluster && (e = launch_fill_u64(reinterpret_cast<uint64_t*>(L.ca.partials),
                                          L.part_count, kEmptySlot, st)) != hipSuccess)
        return e;
    return hipSuccess;
}

hipError_t enqueue_back(const PassLaunch& L, hipStream_t st, hipEvent_t* ev)
{
    hipError_t e;
    if ((e = enqueue_sweep(L, L.la, st)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[3], st)) != hipSuccess) return e;
    return hipSuccess;
}

hipError_t enqueue_pass(const PassLaunch& L, hipStream_t st, hipEvent_t* ev)
{
    hipError_t e;
    if (L.window == 0) {
        if ((e = enqueue_front(L, st, ev)) != hipSuccess) return e;
        return enqueue_back(L, st, ev);
    }
    if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
    if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(L.err_flag), 1, 0, st)) != hipSuccess)
        return e;
    auto fill_slots = [&]() {
        return L.cluster ? launch_fill_u64(reinterpret_cast<uint64_t*>(L.ca.partials),
                                           L.part_count, kEmptySlot, st)
                         : hipSuccess;
    };
    // checkpoint-recompute: every step once, keeping the checkpoints and the
    // last window's features; then window by window from the last date back,
    // recomputing each earlier window's features from its checkpoint
    const int n = L.la.n, c = L.window;
    PathArgs pa = L.pa;
    pa.k_begin = 0;
    pa.k_end = n;
    pa.k_feat0 = n - c;
    pa.ck_store = 1;
    if ((e = launch_paths(L.fp32, L.nmax, L.scheme, L.feat, pa, L.nchunks, L.nbg, st)) !=
        hipSuccess)
        return e;
    if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
    if ((e = fill_slots()) != hipSuccess) return e;
    for (int w = 0;; ++w) {
        const int hi = n - w * c;
        const int lo = std::max(1, hi - c + 1);
        if (w > 0) {
            PathArgs pr = L.pa;
            pr.k_begin = lo - 1;
            pr.k_end = hi;
            pr.k_feat0 = lo - 1;
            pr.ck_store = 0;
            if ((e = launch_paths(L.fp32, L.nmax, L.scheme, L.feat, pr, L.nchunks, L.nbg, st)) !=
                hipSuccess)
                return e;
        }
        LsmcArgs la = L.la;
        la.k_lo = lo;
        la.k_hi = hi;
        la.f_date0 = lo;
        la.win_first = w == 0 ? 1 : 0;
        la.win_last = lo == 1 ? 1 : 0;
        if ((e = launch_gram(L.feat, la, L.Sp, st)) != hipSuccess) return e;
        if ((e = enqueue_sweep(L, la, st)) != hipSuccess) return e;
        if (lo == 1) break;
    }
    if (ev && (e = hipEventRecord(ev[3], st)) != hipSuccess) return e;
    return hipSuccess;
}

hipError_t launch_pass_graph(const PassLaunch& L, void* ws, hipStream_t st)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::string key;
    append_bytes(key, dev);
    append_bytes(key, ws);
    append_bytes(key, L.fp32);
    append_bytes(key, L.american);
    append_bytes(key, L.cluster);
    append_bytes(key, L.nmax);
    append_bytes(key, L.scheme);
    append_bytes(key, L.feat);
    append_bytes(key, L.nchunks);
    append_bytes(key, L.nbg);
    append_bytes(key, L.Sp);
    append_bytes(key, L.cluster_q);
    append_bytes(key, L.per_launch);
    append_bytes(key, L.sweep_q);
    append_bytes(key, L.part_count);
    append_bytes(key, L.window);
    append_bytes(key, L.pa);
    append_bytes(key, L.la);
    append_bytes(key, L.ca);
    append_bytes(key, L.err_flag);
    // held through capture and launch, so no other thread evicts an exec that
    // is about to be launched
    std::lock_guard<std::mutex> lk(g_graph_mu);
    hipGraphExec_t exec = nullptr;
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) exec = it->second;
    if (!exec) {
        if ((e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
        const hipError_t eq = enqueue_pass(L, st, nullptr);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(st, &graph);
        if (eq != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return eq;
        }
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
        if (g_graphs.size() >= kMaxGraphs) {
            // execs already launched on other streams must finish first
            if ((e = hipDeviceSynchronize()) != hipSuccess) {
                (void)hipGraphExecDestroy(exec);
                return e;
            }
            for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
            g_graphs.clear();
        }
        g_graphs.emplace(key, exec);
    }
    return hipGraphLaunch(exec, st);
}

}  // namespace

Tune tuned_shape(const Request& q)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(q));
    return it == g_tune.end() ? Tune{} : it->second;
}

void store_tuned_shape(const Request& q, const Tune& t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(q)] = t;
}

hs_status run_greek_set(const Request& q, void* d_ws, size_t ws_bytes, hipStream_t st,
                        RunResult& res, const Tune* tune, bool shared)
{
    std::vector<Scenario> sc;
    hs_status rc = expand_scenarios(q, sc);
    if (rc != HS_OK) return rc;
    const Shape sh = shape_of(q);
    const std::vector<Pass> passes = make_passes(q, sh, sc, ws_bytes, nullptr);
    if (passes.empty()) {
        size_t mn = 0;
        (void)make_passes(q, sh, sc, 0, &mn);
        set_error("workspace of %zu bytes is below the minimum of %zu", ws_bytes, mn);
        return HS_ENOMEM;
    }
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) {
        set_error("workspace must be 256-byte aligned");
        return HS_EINVAL;
    }
    const Tune tn = tune ? *tune : tuned_shape(q);
    const size_t S = sc.size();
    res.price.assign(S, 0.0);
    res.se.assign(S, 0.0);
    res.skipped.assign(S, 0);
    if (q.opts.flags & HS_FLAG_EXPORT_TAU) res.tau.assign(S * static_cast<size_t>(q.P), 0);
    res.t_paths = res.t_gram = res.t_sweep = res.t_total = 0.0;
    res.n_passes = static_cast<int>(passes.size());

    const bool timing = (q.opts.flags & HS_FLAG_TIMING) != 0;
    const bool graph = !timing && (q.opts.flags & HS_FLAG_GRAPH) && st != nullptr;
    // ev[0..3]: stage times; ev[4]: the end of a pass's front part (shared)
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    if (timing)
        for (int i = 0; i < 4; ++i) HS_HIP(hipEventCreate(&ev[i]), "hipEventCreate");
    if (shared && !graph && !timing)
        HS_HIP(hipEventCreateWithFlags(&ev[4], hipEventDisableTiming), "hipEventCreate");
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard()
        {
            for (int i = 0; i < 5; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } guard{ev};

    unsigned char* ws = static_cast<unsigned char*>(d_ws);
    const int m = basis_m(q);
    const double tbar = mean_theta(q);
    const int tw = tn.target_waves > 0 ? tn.target_waves : default_target_waves();
    for (const Pass& pass : passes) {
        const PassPlan pp = plan_pass(q, sh, sc, pass, tw, tn.wmax);
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
        // the four parameter tables lead the workspace: one upload
        std::vector<unsigned char> up(pp.lay.reg, 0);
        std::memcpy(up.data() + pp.lay.base, pp.base.data(), pp.base.size());
        std::memcpy(up.data() + pp.lay.tasks, pp.tasks.data(), pp.tasks.size());
        std::memcpy(up.data() + pp.lay.groups, pp.groups.data(), pp.groups.size() * sizeof(GroupP));
        std::memcpy(up.data() + pp.lay.disc, pp.disc.data(), pp.disc.size() * sizeof(double));
        HS_HIP(hipMemcpyAsync(ws, up.data(), up.size(), hipMemcpyHostToDevice, st),
               "upload tables");

        PassLaunch L;
        // zero padding too: the graph cache keys on these bytes
        std::memset(static_cast<void*>(&L), 0, sizeof L);
        L.fp32 = sh.fp32;
        L.american = sh.american;
        L.nmax = sh.nmax;
        L.scheme = q.opts.scheme;
        L.feat = sh.feat;
        L.nchunks = pp.nchunks;
        L.nbg = pp.nbg;
        L.Sp = Sp;
        PathArgs& pa = L.pa;
        pa.base = ws + pp.lay.base;
        pa.tasks = ws + pp.lay.tasks;
        pa.groups = reinterpret_cast<const GroupP*>(ws + pp.lay.groups);
        pa.feat = ws + pp.lay.feat;
        pa.P = q.P;
        pa.plane = pp.plane;
        pa.n = q.n;
        pa.N = q.N;
        pa.W = pp.W;
        pa.store_all = sh.american ? 1 : 0;
        pa.key0 = static_cast<uint32_t>(q.opts.seed);
        pa.key1 = static_cast<uint32_t>(q.opts.seed >> 32);
        pa.k_begin = 0;
        pa.k_end = q.n;
        pa.k_feat0 = 0;
        L.window = sh.american ? pass.window : 0;
        pa.ck_every = L.window;
        pa.ck_store = 0;
        pa.ck_slots = q.N + pp.ntasks;
        pa.ckx = ws + pp.lay.ckx;
        pa.ckv = ws + pp.lay.ckv;

        LsmcArgs& la = L.la;
        la.feat = pa.feat;
        la.reg = reinterpret_cast<RegRec*>(ws + pp.lay.reg);
        la.disc = reinterpret_cast<const double*>(ws + pp.lay.disc);
        la.idisc = la.disc + static_cast<size_t>(Sp) * (q.n + 1);
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
        la.k_lo = 1;
        la.k_hi = q.n;
        la.f_date0 = sh.american ? 1 : q.n;
        la.win_first = 1;
        la.win_last = 1;

        // backward sweep: a cluster of workgroups per scenario when it fits the
        // device, else one workgroup per scenario with the state in the workspace
        L.err_flag = reinterpret_cast<int32_t*>(ws + pp.lay.sync);
        L.cluster = sh.sweep == kSweepCluster;
        int cap = 0;
        if (L.cluster) {
            cap = cluster_capacity(sh.feat, sh.cluster_q, L.window > 0,
                                   cluster_lds_bytes(q.n, sh.cluster_g));
            if (cap < sh.cluster_g) {
                if (q.opts.sweep_mode == 3) {
                    set_error("cluster sweep needs %d co-resident workgroups, the device holds %d",
                              sh.cluster_g, cap);
                    return HS_EDEVICE;
                }
                L.cluster = false;
            }
        }
        // windows keep the sweep's state in the workspace between launches
        L.sweep_q = sh.sweep == kSweepBlockRegs && L.window == 0 ? sh.sweep_q : 0;
        if (L.cluster) {
            L.cluster_q = sh.cluster_q;
            L.per_launch = std::max(1, cap / sh.cluster_g);
            L.part_count = static_cast<int64_t>(Sp) * cluster_rows(sh.american, q.n) *
                           sh.cluster_g * kPartStride;
            L.ca.partials = reinterpret_cast<double*>(ws + pp.lay.part);
            L.ca.error = L.err_flag;
            L.ca.G = sh.cluster_g;
            L.ca.timeout_ticks = wall_clock_ticks(10.0);
        }
        std::unique_lock<std::mutex> cluster_lock(g_cluster_mu, std::defer_lock);
        if (graph) {
            if (L.cluster) cluster_lock.lock();
            HS_HIP(launch_pass_graph(L, ws, st), "graph launch");
        } else if (ev[4] && L.cluster && L.window == 0) {
            // shared device (the server): the path and Gram kernels run beside
            // other requests' work; only the cluster sweep, whose workgroups
            // must all be resident at once, waits for the device to itself
            HS_HIP(enqueue_front(L, st, nullptr), "kernel launch");
            HS_HIP(hipEventRecord(ev[4], st), "hipEventRecord");
            HS_HIP(hipEventSynchronize(ev[4]), "hipEventSynchronize");
            cluster_lock.lock();
            HS_HIP(enqueue_back(L, st, nullptr), "kernel launch");
        } else {
            if (L.cluster) cluster_lock.lock();
            HS_HIP(enqueue_pass(L, st, timing ? ev : nullptr), "kernel launch");
        }

        // results [Sp][4] and the status flag right after them: one copy
        std::vector<double> out(static_cast<size_t>(Sp) * 4 + 1);
        HS_HIP(hipMemcpyAsync(out.data(), la.out, static_cast<size_t>(Sp) * 4 * sizeof(double) +
                                                     sizeof(int32_t),
                              hipMemcpyDeviceToHost, st), "download results");
        std::vector<int32_t> tau;
        if (la.export_tau) {
            tau.resize(static_cast<size_t>(Sp) * q.P);
            HS_HIP(hipMemcpyAsync(tau.data(), la.tau, tau.size() * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, st), "download tau");
        }
        HS_HIP(hipStreamSynchronize(st), "stream synchronize");
        if (cluster_lock.owns_lock()) cluster_lock.unlock();
        int32_t err_host = 0;
        std::memcpy(&err_host, out.data() + static_cast<size_t>(Sp) * 4, sizeof(int32_t));
        if (err_host != 0) {
            set_error("cluster sweep: a workgroup wait timed out (device oversubscribed?)");
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
    // one pass over every scenario at once, unless windows are forced
    if (!minimum && q.opts.window_dates == 0)
        return layout_for(q, sh, static_cast<int>(S), static_cast<int>(S * N),
                          static_cast<int>(S) + 2 * kMaxWaves)
            .total;
    // the planner's minimum: the largest unit, in windows of dates where that
    // is smaller (with forced windows every unit runs in them, so this is also
    // the size of one pass); the size does not depend on the correlation values
    std::vector<Scenario> sc;
    if (expand_scenarios(q, sc) != HS_OK) return 0;
    size_t mn = 0;
    (void)make_passes(q, sh, sc, 0, &mn);
    return mn;
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
                       nullptr);
    if (rc != HS_OK) return rc;
    fill_greeks(q, res, out);
    return HS_OK;
}

hs_status hs_autotune(const hs_model* model, const double* corr, const hs_option* option,
                      int64_t n_paths, int32_t n_steps, const hs_bumps* bumps,
                      const hs_opts* opts, void* d_workspace, size_t workspace_bytes,
                      void* hip_stream, int32_t repeats, double* best_ms)
{
    if (!d_workspace || repeats < 1 || repeats > 100) {
        set_error("hs_autotune: null workspace or repeats outside 1..100");
        return HS_EINVAL;
    }
    Request q;
    hs_status rc = copy_request(model, corr, option, n_paths, n_steps, bumps, opts, q);
    if (rc != HS_OK) return rc;
    rc = validate(q);
    if (rc != HS_OK) return rc;
    // candidates run as the request will: graph replay stays on if asked for
    q.opts.flags &= ~(HS_FLAG_TIMING | HS_FLAG_EXPORT_TAU);
    q.opts.waves_per_block = 0;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // target waves (the default first) x the most waves per block (1: as
    // few as the base assets allow)
    const int waves[] = {default_target_waves(), 1024, 8192};
    static const int wmaxes[] = {1, 2, 3, 4, 6, 8, 12, 16};
    const Shape tsh = shape_of(q);
    const int vmax = paths_max_waves(tsh.fp32, q.opts.scheme == HS_SCHEME_QE, tsh.nmax);
    Tune best{};
    double best_t = 1e300;
    for (int tw : waves)
        for (int wm : wmaxes) {
            if (wm > vmax) continue;  // the planner caps it at the variant's most
            const Tune t{tw, wm};
            RunResult res;
            rc = run_greek_set(q, d_workspace, workspace_bytes, st, res, &t);  // warm-up
            if (rc != HS_OK) return rc;
            const auto t0 = std::chrono::steady_clock::now();
            for (int r = 0; r < repeats; ++r) {
                rc = run_greek_set(q, d_workspace, workspace_bytes, st, res, &t);
                if (rc != HS_OK) return rc;
            }
            const double ms = std::chrono::duration<double, std::milli>(
                                  std::chrono::steady_clock::now() - t0).count() / repeats;
            if (ms < best_t) {
                best_t = ms;
                best = t;
            }
        }
    store_tuned_shape(q, best);
    if (best_ms) *best_ms = best_t;
    return HS_OK;
}

size_t hs_path_features_workspace_bytes(int32_t n_assets)
{
    (void)n_assets;
    const size_t greek_set = 2 * 256 + sizeof(BaseP<double>) + kMaxWaves * sizeof(GroupP);
    return std::max(greek_set, sizeof(ModelP<double>));
}


hs_status hs_path_features(const hs_model* model, const double* corr, int64_t n_paths,
                           int32_t n_steps, double T, const hs_opts* opts, void* d_out,
                           size_t out_bytes, void* d_workspace, size_t workspace_bytes,
                           void* hip_stream)
{
    if (!d_out || !d_workspace || !opts) {
        set_error("hs_path_features: null output, workspace or opts");
        return HS_EINVAL;
    }
    const bool greek_set = (opts->flags & HS_FLAG_GREEK_SET_KERNEL) != 0;
    hs_option opt{HS_CALL, HS_AMERICAN, HS_MAX_OF, HS_BASIS_AUTO, 1.0, T};
    hs_bumps nob{0u, 0.0, 0.0, 0.0, 0.0, 0.0};
    Request q;
    hs_status rc = copy_request(model, corr, &opt, n_paths, n_steps, &nob, opts, q,
                                greek_set ? kMaxAssets : kMaxPathAssets);
    if (rc != HS_OK) return rc;
    rc = validate(q, greek_set ? kMaxWaves : kBaseMaxWaves, HS_FLAG_GREEK_SET_KERNEL);
    if (rc != HS_OK) return rc;
    std::vector<Scenario> sc;
    rc = expand_scenarios(q, sc);
    if (rc != HS_OK) return rc;
    const bool fp32 = q.opts.precision == HS_FP32_PATHS;
    const int ft = !fp32 ? kFeatF64
                   : q.opts.feature_format == HS_FEATURES_FP16 ? kFeatF16
                   : q.opts.feature_format == HS_FEATURES_BF16 ? kFeatBF16
                                                               : kFeatF32;
    const size_t need = static_cast<size_t>(n_steps) * n_paths * feat_bytes(ft);
    if (out_bytes < need) {
        set_error("hs_path_features: output needs %zu bytes, got %zu", need, out_bytes);
        return HS_ENOMEM;
    }
    if (workspace_bytes < hs_path_features_workspace_bytes(q.N)) {
        set_error("hs_path_features: workspace needs %zu bytes",
                  hs_path_features_workspace_bytes(q.N));
        return HS_ENOMEM;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    unsigned char* ws = static_cast<unsigned char*>(d_workspace);
    if (!greek_set) {
        // waves: as asked, else (measured on the paper's problem sizes)
        // Euler: one per Philox block up to 12 blocks, beyond that two blocks
        // per wave; QE, whose FP64 variance step gains from several
        // independent assets per wave: at most 4 waves.  Then the nearest
        // count the kernel supports for this asset count, upwards first (at
        // most four blocks per wave; fewer waves where the variant needs more
        // registers).
        const int nblk = (q.N + 1) / 2;
        const int want = q.opts.waves_per_block > 0       ? q.opts.waves_per_block
                         : q.opts.scheme == HS_SCHEME_QE ? std::min(4, nblk)
                         : nblk <= 12                     ? nblk
                                                          : (nblk + 1) / 2;
        int W = -1;
        for (int c = want; c <= kBaseMaxWaves && W < 0; ++c)
            if (paths_base_bpw(fp32, q.opts.scheme, q.N, c) > 0) W = c;
        for (int c = want - 1; c >= 1 && W < 0; --c)
            if (paths_base_bpw(fp32, q.opts.scheme, q.N, c) > 0) W = c;
        if (W < 0) {
            set_error("hs_path_features: no kernel shape for %d assets", q.N);
            return HS_EINVAL;
        }
        const std::vector<unsigned char> tab = model_table(q, sc[0], fp32);
        HS_HIP(hipMemcpyAsync(ws, tab.data(), tab.size(), hipMemcpyHostToDevice, st),
               "upload model");
        BasePathArgs ba{};
        ba.model = ws;
        ba.feat = d_out;
        ba.P = q.P;
        ba.n = q.n;
        ba.N = q.N;
        ba.W = W;
        ba.key0 = static_cast<uint32_t>(q.opts.seed);
        ba.key1 = static_cast<uint32_t>(q.opts.seed >> 32);
        HS_HIP(launch_paths_base(fp32, q.opts.scheme, ft, ba, st), "base path kernel launch");
        // the host table must outlive the asynchronous upload
        HS_HIP(hipStreamSynchronize(st), "stream synchronize");
        return HS_OK;
    }
    const Shape sh = shape_of(q);
    Pass pass;
    pass.scen = {0};
    pass.has_base_spot = true;
    PassPlan pp = plan_pass(q, sh, sc, pass, default_target_waves(), 0);
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
    pa.k_begin = 0;
    pa.k_end = q.n;
    pa.k_feat0 = 0;
    pa.ck_every = 0;  // all dates, no checkpoints
    HS_HIP(launch_paths(sh.fp32, sh.nmax, q.opts.scheme, sh.feat, pa, pp.nchunks, pp.nbg, st),
           "path kernel launch");
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
