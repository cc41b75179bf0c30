// hs_plan.cpp -- validation, scenario expansion, path-kernel task tables,
// workspace layout and Greeks (host, FP64, built with -ffp-contract=off).
#include "hs_plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>

#include "hs_kernels.hpp"

namespace hs {

namespace {
thread_local std::string g_err = "no error";
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
bool finite(double x) { return std::isfinite(x); }
}  // namespace

void set_error(const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

}  // namespace hs

extern "C" const char* hs_last_error(void) { return hs::g_err.c_str(); }

namespace hs {

hs_status copy_request(const hs_model* model, const double* corr, const hs_option* option,
                       int64_t n_paths, int32_t n_steps, const hs_bumps* bumps,
                       const hs_opts* opts, Request& q, int max_assets)
{
    if (!model || !corr || !option || !bumps || !opts) {
        set_error("null argument (model, corr, option, bumps and opts are required)");
        return HS_EINVAL;
    }
    const int N = model->n_assets;
    if (N < 1 || N > max_assets) {
        set_error("n_assets = %d outside 1..%d", N, max_assets);
        return HS_EINVAL;
    }
    const double* arr[6] = {model->S0, model->v0, model->kappa, model->theta_lr, model->xi,
                            model->rho_sv};
    for (const double* a : arr)
        if (!a) {
            set_error("null per-asset model array");
            return HS_EINVAL;
        }
    q.N = N;
    q.S0.assign(model->S0, model->S0 + N);
    q.v0.assign(model->v0, model->v0 + N);
    q.kappa.assign(model->kappa, model->kappa + N);
    q.theta.assign(model->theta_lr, model->theta_lr + N);
    q.xi.assign(model->xi, model->xi + N);
    q.rho.assign(model->rho_sv, model->rho_sv + N);
    q.r = model->r;
    q.C.assign(corr, corr + N * N);
    q.opt = *option;
    q.P = n_paths;
    q.n = n_steps;
    q.bumps = *bumps;
    q.opts = *opts;
    return HS_OK;
}

bool cholesky(int N, const std::vector<double>& C, std::vector<double>& L)
{
    L.assign(static_cast<size_t>(N) * N, 0.0);
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = C[i * N + j];
            for (int k = 0; k < j; ++k) s -= L[i * N + k] * L[j * N + k];
            if (i == j) {
                if (!(s > 0.0)) return false;
                L[i * N + i] = std::sqrt(s);
            } else {
                L[i * N + j] = s / L[j * N + j];
            }
        }
    }
    return true;
}

int64_t num_scenarios(int N, uint32_t mask)
{
    int64_t S = 1;
    if (mask & HS_BUMP_DELTA_GAMMA) S += 2 * static_cast<int64_t>(N);
    if (mask & HS_BUMP_VEGA) S += N;
    if (mask & HS_BUMP_THETA) S += 1;
    if (mask & HS_BUMP_RHO) S += 1;
    if ((mask & HS_BUMP_CORR) && N > 1) S += static_cast<int64_t>(N) * (N - 1) / 2;
    return S;
}

int basis_m(const Request& q)
{
    if (q.opt.basis == HS_BASIS_QUAD) return 3;
    if (q.opt.basis == HS_BASIS_QUAD_VOL) return 5;
    return q.N == 1 ? 3 : 5;
}

hs_status validate(const Request& q, int max_waves, uint32_t extra_flags)
{
    const int N = q.N;
    if (q.P < 2) {
        set_error("n_paths = %lld, need >= 2", static_cast<long long>(q.P));
        return HS_EINVAL;
    }
    if (q.P > (int64_t(1) << 31)) {  // the path kernels run one work-item per path
        set_error("n_paths = %lld above 2^31", static_cast<long long>(q.P));
        return HS_EINVAL;
    }
    if (q.n < 1 || q.n > 4096) {
        set_error("n_steps = %d outside 1..4096", q.n);
        return HS_EINVAL;
    }
    for (int a = 0; a < N; ++a) {
        if (!finite(q.S0[a]) || !(q.S0[a] > 0.0)) {
            set_error("S0[%d] = %g must be finite and > 0", a, q.S0[a]);
            return HS_EINVAL;
        }
        if (!finite(q.v0[a]) || q.v0[a] < 0.0) {
            set_error("v0[%d] = %g must be finite and >= 0", a, q.v0[a]);
            return HS_EINVAL;
        }
        if (!finite(q.kappa[a]) || q.kappa[a] < 0.0) {
            set_error("kappa[%d] = %g must be finite and >= 0", a, q.kappa[a]);
            return HS_EINVAL;
        }
        if (!finite(q.theta[a]) || !(q.theta[a] > 0.0)) {
            set_error("theta_lr[%d] = %g must be finite and > 0", a, q.theta[a]);
            return HS_EINVAL;
        }
        if (!finite(q.xi[a]) || q.xi[a] < 0.0) {
            set_error("xi[%d] = %g must be finite and >= 0", a, q.xi[a]);
            return HS_EINVAL;
        }
        if (!finite(q.rho[a]) || !(std::fabs(q.rho[a]) < 1.0)) {
            set_error("rho_sv[%d] = %g must satisfy |rho| < 1", a, q.rho[a]);
            return HS_EINVAL;
        }
    }
    if (!finite(q.r)) {
        set_error("r must be finite");
        return HS_EINVAL;
    }
    for (int i = 0; i < N; ++i) {
        if (!(std::fabs(q.C[i * N + i] - 1.0) <= 1e-12)) {
            set_error("corr[%d][%d] = %g, need a unit diagonal", i, i, q.C[i * N + i]);
            return HS_EINVAL;
        }
        for (int j = 0; j < N; ++j) {
            const double c = q.C[i * N + j];
            if (!finite(c) || !(std::fabs(c - q.C[j * N + i]) <= 1e-12)) {
                set_error("corr is not symmetric/finite at (%d,%d)", i, j);
                return HS_EINVAL;
            }
        }
    }
    const hs_option& o = q.opt;
    if (o.cp != HS_PUT && o.cp != HS_CALL) {
        set_error("option.cp = %d", o.cp);
        return HS_EINVAL;
    }
    if (o.style != HS_EUROPEAN && o.style != HS_AMERICAN) {
        set_error("option.style = %d", o.style);
        return HS_EINVAL;
    }
    if (o.underlying != HS_SINGLE && o.underlying != HS_MAX_OF) {
        set_error("option.underlying = %d", o.underlying);
        return HS_EINVAL;
    }
    if (o.underlying == HS_SINGLE && N != 1) {
        set_error("HS_SINGLE needs n_assets == 1 (got %d); use HS_MAX_OF", N);
        return HS_EINVAL;
    }
    if (o.basis < HS_BASIS_AUTO || o.basis > HS_BASIS_QUAD_VOL) {
        set_error("option.basis = %d", o.basis);
        return HS_EINVAL;
    }
    if (!finite(o.K) || !(o.K > 0.0) || !finite(o.T) || !(o.T > 0.0)) {
        set_error("option K = %g and T = %g must be finite and > 0", o.K, o.T);
        return HS_EINVAL;
    }
    const hs_bumps& b = q.bumps;
    if (b.mask & ~HS_BUMP_ALL) {
        set_error("bumps.mask = 0x%x has unknown bits", b.mask);
        return HS_EINVAL;
    }
    if ((b.mask & HS_BUMP_DELTA_GAMMA) && !(b.spot_rel > 0.0 && b.spot_rel < 1.0)) {
        set_error("bumps.spot_rel = %g outside (0, 1)", b.spot_rel);
        return HS_EINVAL;
    }
    if (b.mask & HS_BUMP_VEGA) {
        if (!finite(b.v0_rel) || !(b.v0_rel > 0.0)) {
            set_error("bumps.v0_rel = %g must be > 0", b.v0_rel);
            return HS_EINVAL;
        }
        for (int a = 0; a < N; ++a)
            if (!(q.v0[a] > 0.0)) {
                set_error("vega needs v0[%d] > 0 (relative bump)", a);
                return HS_EINVAL;
            }
    }
    if ((b.mask & HS_BUMP_THETA) && !(b.T_abs > 0.0 && b.T_abs < o.T)) {
        set_error("bumps.T_abs = %g outside (0, T)", b.T_abs);
        return HS_EINVAL;
    }
    if ((b.mask & HS_BUMP_RHO) && (!finite(b.r_abs) || b.r_abs == 0.0)) {
        set_error("bumps.r_abs must be finite and non-zero");
        return HS_EINVAL;
    }
    if ((b.mask & HS_BUMP_CORR) && N > 1 && (!finite(b.corr_abs) || b.corr_abs == 0.0)) {
        set_error("bumps.corr_abs must be finite and non-zero");
        return HS_EINVAL;
    }
    const hs_opts& op = q.opts;
    if (op.precision != HS_FP64 && op.precision != HS_FP32_PATHS) {
        set_error("opts.precision = %d", op.precision);
        return HS_EINVAL;
    }
    if (op.waves_per_block < 0 || op.waves_per_block > max_waves) {
        set_error("opts.waves_per_block = %d outside 0..%d", op.waves_per_block, max_waves);
        return HS_EINVAL;
    }
    if (op.flags & ~(HS_FLAG_EXPORT_TAU | HS_FLAG_TIMING | HS_FLAG_GRAPH | extra_flags)) {
        set_error("opts.flags = 0x%x has unknown bits", op.flags);
        return HS_EINVAL;
    }
    if (op.sweep_mode < 0 || op.sweep_mode > 3) {
        set_error("opts.sweep_mode = %d", op.sweep_mode);
        return HS_EINVAL;
    }
    if (op.sweep_mode == 1 && sweep_q_for(q.P) == 0) {
        set_error("opts.sweep_mode = 1 needs n_paths <= %d", 16 * kSweepThreads);
        return HS_EINVAL;
    }
    if (op.reserved != 0) {
        set_error("opts.reserved must be zero");
        return HS_EINVAL;
    }
    if (op.window_dates < 0 || op.window_dates > q.n) {
        set_error("opts.window_dates = %d outside 0..n_steps", op.window_dates);
        return HS_EINVAL;
    }
    if (op.scheme != HS_SCHEME_EULER_FT && op.scheme != HS_SCHEME_QE) {
        set_error("opts.scheme = %d", op.scheme);
        return HS_EINVAL;
    }
    if (op.feature_format < HS_FEATURES_NATIVE || op.feature_format > HS_FEATURES_BF16) {
        set_error("opts.feature_format = %d", op.feature_format);
        return HS_EINVAL;
    }
    if (op.feature_format != HS_FEATURES_NATIVE &&
        (op.precision != HS_FP32_PATHS || op.scheme != HS_SCHEME_EULER_FT)) {
        set_error("16-bit feature storage needs FP32 paths and the Euler scheme");
        return HS_EINVAL;
    }
    if (op.scheme == HS_SCHEME_QE)
        for (int a = 0; a < q.N; ++a)
            if (!(q.xi[a] > 0.0) && q.rho[a] != 0.0) {
                set_error("QE needs xi > 0 or rho = 0 (asset %d: xi = %g, rho = %g)", a, q.xi[a],
                          q.rho[a]);
                return HS_EINVAL;
            }
    return HS_OK;
}

hs_status expand_scenarios(const Request& q, std::vector<Scenario>& out)
{
    const int N = q.N;
    std::vector<double> L0;
    if (!cholesky(N, q.C, L0)) {
        set_error("correlation matrix is not positive definite");
        return HS_ENOTSPD;
    }
    out.clear();
    Scenario base;
    base.kind = 0;
    base.S0 = q.S0;
    base.v0 = q.v0;
    base.L = L0;
    base.r = q.r;
    base.T = q.opt.T;
    out.push_back(base);
    const uint32_t mask = q.bumps.mask;
    if (mask & HS_BUMP_DELTA_GAMMA) {
        for (int d = 0; d < 2; ++d)
            for (int a = 0; a < N; ++a) {
                Scenario s = base;
                s.kind = 1 + d;
                s.i = a;
                s.S0[a] = d == 0 ? q.S0[a] * (1.0 + q.bumps.spot_rel)
                                 : q.S0[a] * (1.0 - q.bumps.spot_rel);
                out.push_back(s);
            }
    }
    if (mask & HS_BUMP_VEGA) {
        for (int a = 0; a < N; ++a) {
            Scenario s = base;
            s.kind = 3;
            s.i = a;
            s.v0[a] = q.v0[a] * (1.0 + q.bumps.v0_rel);
            out.push_back(s);
        }
    }
    if (mask & HS_BUMP_THETA) {
        Scenario s = base;
        s.kind = 4;
        s.T = q.opt.T - q.bumps.T_abs;
        out.push_back(s);
    }
    if (mask & HS_BUMP_RHO) {
        Scenario s = base;
        s.kind = 5;
        s.r = q.r + q.bumps.r_abs;
        out.push_back(s);
    }
    if ((mask & HS_BUMP_CORR) && N > 1) {
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j) {
                Scenario s = base;
                s.kind = 6;
                s.i = i;
                s.j = j;
                std::vector<double> C = q.C;
                C[i * N + j] += q.bumps.corr_abs;
                C[j * N + i] += q.bumps.corr_abs;
                if (!cholesky(N, C, s.L)) {
                    set_error("correlation bumped at (%d,%d) by %g is not positive definite", i, j,
                              q.bumps.corr_abs);
                    return HS_ENOTSPD;
                }
                out.push_back(s);
            }
    }
    // own asset range: assets whose path differs from the base scenario's
    for (Scenario& s : out) {
        if (from_base_path(s.kind)) {
            s.lo = s.hi = 0;
            continue;
        }
        int lo = N, hi = 0;
        for (int a = 0; a < N; ++a) {
            bool own = s.S0[a] != base.S0[a] || s.v0[a] != base.v0[a] || s.r != base.r ||
                       s.T != base.T;
            for (int b = 0; b < N && !own; ++b) own = s.L[a * N + b] != base.L[a * N + b];
            if (own) {
                lo = std::min(lo, a);
                hi = std::max(hi, a + 1);
            }
        }
        if (lo >= hi) {  // a bump that changes nothing: recompute the last asset
            lo = N - 1;
            hi = N;
        }
        s.lo = lo;
        s.hi = hi;
    }
    return HS_OK;
}

Shape shape_of(const Request& q)
{
    Shape sh;
    sh.fp32 = q.opts.precision == HS_FP32_PATHS;
    sh.american = q.opt.style == HS_AMERICAN;
    sh.nmax = paths_nmax_bucket(q.N);
    sh.tmax = paths_tmax(sh.fp32, q.opts.scheme, sh.nmax);
    sh.feat = !sh.fp32 ? kFeatF64
              : q.opts.feature_format == HS_FEATURES_FP16 ? kFeatF16
              : q.opts.feature_format == HS_FEATURES_BF16 ? kFeatBF16
                                                          : kFeatF32;
    // cluster sweep shape from the request alone (never from device load, nor
    // from the workspace): spread the Greek set's scenarios over the compute
    // units, from one path per thread up to the most that one workgroup per
    // CU holds in registers (a set larger than the device runs in several
    // launches, each a chain of exchanges: more paths per thread, fewer
    // launches)
    const int64_t P = q.P;
    const int64_t T = kClusterThreads;
    const int64_t S = num_scenarios(q.N, q.bumps.mask);
    const int64_t qmax = cluster_qmax(sh.feat);
    int64_t gmin = (P + qmax * T - 1) / (qmax * T);
    const int64_t gone = (P + T - 1) / T;
    int64_t G = std::max(gmin, std::min(std::max<int64_t>(1, kPlanComputeUnits / std::max<int64_t>(S, 1)), gone));
    int cq = static_cast<int>((P + G * T - 1) / (G * T));
    while (!cluster_q_supported(cq, sh.feat)) ++cq;  // 9 -> 10, 13 -> 16, ...
    G = (P + cq * T - 1) / (cq * T);
    sh.cluster_q = cq;
    sh.cluster_g = static_cast<int>(G);
    const int mode = q.opts.sweep_mode;
    if (mode == 1) {
        sh.sweep = kSweepBlockRegs;
        sh.sweep_q = sweep_q_for(P);
    } else if (mode == 2 || (mode == 0 && G > kMaxClusterGroups)) {
        sh.sweep = kSweepBlockState;
        sh.sweep_q = 0;
    } else {
        sh.sweep = kSweepCluster;
        sh.sweep_q = 0;
    }
    return sh;
}

Layout layout_for(const Request& q, const Shape& sh, int n_scen, int n_tasks, int n_groups,
                  int window)
{
    const size_t R = sh.fp32 ? 4 : 8;
    const size_t P = static_cast<size_t>(q.P);
    const size_t nd = !sh.american ? 1 : window > 0 ? static_cast<size_t>(window)
                                                    : static_cast<size_t>(q.n);
    const size_t S = static_cast<size_t>(n_scen);
    Layout L;
    size_t off = 0;
    L.base = off;
    off = align_up(off + (sh.fp32 ? sizeof(BaseP<float>) : sizeof(BaseP<double>)));
    L.tasks = off;
    off = align_up(off + static_cast<size_t>(std::max(n_tasks, 1)) *
                             (sh.fp32 ? sizeof(TaskP<float>) : sizeof(TaskP<double>)));
    L.groups = off;
    off = align_up(off + static_cast<size_t>(std::max(n_groups, 1)) * sizeof(GroupP));
    L.disc = off;  // exp(-r j dt), then exp(+r j dt)
    off = align_up(off + 2 * S * (q.n + 1) * sizeof(double));
    L.reg = off;
    off = align_up(off + (sh.american ? S * q.n * sizeof(RegRec) : 0));
    // the results and the status flag side by side: one copy back per pass
    L.out = off;
    off = off + S * 4 * sizeof(double);
    L.sync = off;
    off = align_up(off + (S + 64) * sizeof(uint32_t));
    // exercise dates and cash flows of the workspace-state sweep (also the
    // fallback when a cluster does not fit the device) and the exported dates
    L.tau = off;
    off = align_up(off + S * P * sizeof(int32_t));
    L.cf = off;
    off = align_up(off + S * P * sizeof(double));
    L.part = off;
    if (sh.sweep == kSweepCluster)  // rows: dates 1..n-1, then the two price sums
        off = align_up(off + S * cluster_rows(sh.american, q.n) *
                                 static_cast<size_t>(sh.cluster_g) * kPartStride * sizeof(double));
    // checkpoints of a windowed pass: every base asset and task, log price
    // in R, variance in R (FP64 under QE)
    const size_t ncp = static_cast<size_t>(checkpoint_count(q.n, sh.american ? window : 0));
    const size_t slots = static_cast<size_t>(q.N + n_tasks);
    L.ckx = off;
    off = align_up(off + ncp * slots * P * R);
    L.ckv = off;
    off = align_up(off + ncp * slots * P * (q.opts.scheme == HS_SCHEME_QE ? 8 : R));
    L.feat = off;
    off = align_up(off + S * nd * P * feat_bytes(sh.feat));
    L.total = off;
    return L;
}

namespace {

// Andersen's QE constants for one asset over one step dt (host FP64):
// E = e^{-kappa dt}; m = mth + v E and s^2 = v c1 + c2 are the CIR conditional
// mean and variance; K0 (with r dt) .. K4 the central (gamma = 1/2) log-price
// coefficients, with rho/xi read as 0 when xi = 0 (validation then demands
// rho = 0); rho and sqrt(1 - rho^2) split the asset's spot normal into the
// variance normal and the log price's orthogonal normal.
template <typename R>
QeP<R> qe_params(double v0, double kappa, double theta, double xi, double rho, double r, double dt)
{
    QeP<R> c;
    std::memset(&c, 0, sizeof c);
    const double E = std::exp(-kappa * dt);
    const double f = kappa > 0.0 ? -std::expm1(-kappa * dt) / kappa : dt;  // (1 - E)/kappa
    const double rx = xi > 0.0 ? rho / xi : 0.0;
    c.E = E;
    c.v0 = v0;
    c.mth = theta * (1.0 - E);
    c.c1 = xi * xi * E * f;
    c.c2 = 0.5 * theta * xi * xi * (1.0 - E) * f;
    c.K0 = r * dt - rx * kappa * theta * dt;
    c.K1 = 0.5 * dt * (kappa * rx - 0.5) - rx;
    c.K2 = 0.5 * dt * (kappa * rx - 0.5) + rx;
    c.K3 = 0.5 * dt * (1.0 - rho * rho);
    c.K4 = 0.5 * dt * (1.0 - rho * rho);
    c.rho = rho;
    c.rhobar = std::sqrt(1.0 - rho * rho);
    return c;
}

// The base model in the path precision R for the base-model path kernel.
template <typename R>
std::vector<unsigned char> model_table_t(const Request& q, const Scenario& b0)
{
    ModelP<R> mp;
    std::memset(&mp, 0, sizeof mp);
    const int N = q.N;
    const double dt = q.opt.T / static_cast<double>(q.n);
    for (int a = 0; a < N; ++a) {
        mp.a[a].S0 = static_cast<R>(q.S0[a]);
        mp.a[a].v0 = static_cast<R>(q.v0[a]);
        mp.a[a].kappa = static_cast<R>(q.kappa[a]);
        mp.a[a].theta = static_cast<R>(q.theta[a]);
        mp.a[a].xi = static_cast<R>(q.xi[a]);
        mp.a[a].rho = static_cast<R>(q.rho[a]);
        mp.a[a].rhobar = static_cast<R>(std::sqrt(1.0 - q.rho[a] * q.rho[a]));
        mp.a[a].qe = qe_params<R>(q.v0[a], q.kappa[a], q.theta[a], q.xi[a], q.rho[a], q.r, dt);
        for (int c = 0; c <= a; ++c) {
            mp.L[a * kMaxPathAssets + c] = static_cast<R>(b0.L[a * N + c]);
            mp.L64[a * kMaxPathAssets + c] = b0.L[a * N + c];
        }
    }
    mp.r = static_cast<R>(q.r);
    mp.dt = static_cast<R>(dt);
    mp.invN = static_cast<R>(1.0 / static_cast<double>(N));
    std::vector<unsigned char> out(sizeof mp);
    std::memcpy(out.data(), &mp, sizeof mp);
    return out;
}

template <typename R>
void fill_tables(const Request& q, const Shape& sh, const std::vector<Scenario>& sc,
                 const Pass& pass, const std::vector<std::vector<int>>& group_scen, PassPlan& pp)
{
    const int N = q.N;
    const Scenario& b0 = sc[0];
    BaseP<R> bp;
    std::memset(&bp, 0, sizeof bp);
    for (int a = 0; a < N; ++a) {
        bp.a[a].S0 = static_cast<R>(q.S0[a]);
        bp.a[a].v0 = static_cast<R>(q.v0[a]);
        bp.a[a].kappa = static_cast<R>(q.kappa[a]);
        bp.a[a].theta = static_cast<R>(q.theta[a]);
        bp.a[a].xi = static_cast<R>(q.xi[a]);
        bp.a[a].rho = static_cast<R>(q.rho[a]);
        bp.a[a].rhobar = static_cast<R>(std::sqrt(1.0 - q.rho[a] * q.rho[a]));
        bp.a[a].qe = qe_params<R>(q.v0[a], q.kappa[a], q.theta[a], q.xi[a], q.rho[a], q.r,
                                  q.opt.T / static_cast<double>(q.n));
        for (int c = 0; c < N; ++c) {
            bp.L[a * kMaxAssets + c] = static_cast<R>(b0.L[a * N + c]);
            bp.L64[a * kMaxAssets + c] = b0.L[a * N + c];
        }
        bp.S0_up[a] = static_cast<R>(q.S0[a] * (1.0 + q.bumps.spot_rel));
        bp.S0_dn[a] = static_cast<R>(q.S0[a] * (1.0 - q.bumps.spot_rel));
    }
    bp.r = static_cast<R>(q.r);
    bp.dt = static_cast<R>(q.opt.T / static_cast<double>(q.n));
    // the rate scenario's log-price shift per step, (r' - r) dt
    bp.drdt = R(0);
    for (const Scenario& s : sc)
        if (s.kind == 5) bp.drdt = static_cast<R>((s.r - q.r) * (q.opt.T / static_cast<double>(q.n)));
    bp.invN = static_cast<R>(1.0 / static_cast<double>(N));
    pp.base.resize(sizeof bp);
    std::memcpy(pp.base.data(), &bp, sizeof bp);

    // plane of each canonical scenario in this pass
    std::vector<int> plane(sc.size(), -1);
    for (size_t i = 0; i < pass.scen.size(); ++i) plane[pass.scen[i]] = static_cast<int>(i);

    std::vector<TaskP<R>> tasks;
    pp.groups.assign(static_cast<size_t>(pp.nbg) * pp.W, GroupP{0, 0, -1, -1, -1, -1, {0, 0}});
    for (size_t g = 0; g < group_scen.size(); ++g) {
        GroupP& G = pp.groups[g];
        G.task0 = static_cast<int32_t>(tasks.size());
        if (g == 0 && pass.has_base_spot) {
            G.base_scen = plane[0];
            if (q.bumps.mask & HS_BUMP_DELTA_GAMMA) {
                G.spot_up0 = plane[1];
                G.spot_dn0 = plane[1 + N];
            }
            for (size_t si = 0; si < sc.size(); ++si)
                if (sc[si].kind == 5) G.rate_scen = plane[si];
        }
        for (int si : group_scen[g]) {
            const Scenario& s = sc[si];
            for (int a = s.lo; a < s.hi; ++a) {
                TaskP<R> t;
                std::memset(&t, 0, sizeof t);
                t.asset = a;
                bool own_row = false;
                for (int c = 0; c < N; ++c) own_row |= s.L[a * N + c] != b0.L[a * N + c];
                t.own_row = own_row ? 1 : 0;
                t.first = a == s.lo;
                t.last = a == s.hi - 1;
                t.scen = plane[si];
                t.lo = s.lo;
                t.hi = s.hi;
                t.S0 = static_cast<R>(s.S0[a]);
                t.v0 = static_cast<R>(s.v0[a]);
                t.kappa = static_cast<R>(q.kappa[a]);
                t.theta = static_cast<R>(q.theta[a]);
                t.xi = static_cast<R>(q.xi[a]);
                t.rho = static_cast<R>(q.rho[a]);
                t.rhobar = static_cast<R>(std::sqrt(1.0 - q.rho[a] * q.rho[a]));
                t.r = static_cast<R>(s.r);
                t.dt = static_cast<R>(s.T / static_cast<double>(q.n));
                t.qe = qe_params<R>(s.v0[a], q.kappa[a], q.theta[a], q.xi[a], q.rho[a], s.r,
                                    s.T / static_cast<double>(q.n));
                for (int c = 0; c < N; ++c) {
                    t.L[c] = static_cast<R>(s.L[a * N + c]);
                    t.L64[c] = s.L[a * N + c];
                }
                t.a_el = a * kLanes;
                t.lo_el = s.lo * kLanes;
                t.hi_el = s.hi * kLanes;
                t.flags = (t.first ? 1 : 0) | (t.last ? 2 : 0);
                t.fo = static_cast<int64_t>(t.scen) * pp.plane;
                tasks.push_back(t);
            }
        }
        G.ntask = static_cast<int32_t>(tasks.size()) - G.task0;
    }
    pp.ntasks = static_cast<int>(tasks.size());
    pp.tasks.resize(std::max<size_t>(tasks.size(), 1) * sizeof(TaskP<R>));
    if (!tasks.empty()) std::memcpy(pp.tasks.data(), tasks.data(), tasks.size() * sizeof(TaskP<R>));
    (void)sh;
}

}  // namespace

PassPlan plan_pass(const Request& q, const Shape& sh, const std::vector<Scenario>& sc,
                   const Pass& pass, int target_waves, int wmax)
{
    PassPlan pp;
    const int N = q.N;
    pp.nchunks = static_cast<int>((q.P + kLanes - 1) / kLanes);
    // task scenarios of this pass, heaviest first (stable in canonical order)
    std::vector<int> units;
    int total = 0;
    for (int si : pass.scen)
        if (!from_base_path(sc[si].kind)) {
            units.push_back(si);
            total += sc[si].hi - sc[si].lo;
        }
    std::stable_sort(units.begin(), units.end(), [&](int a, int b) {
        return (sc[a].hi - sc[a].lo) > (sc[b].hi - sc[b].lo);
    });
    const int tmax = sh.tmax;
    const int own = paths_own_per_wave(sh.nmax);
    const int wmin = (N + own - 1) / own;
    int G = std::max(1, (total + tmax - 1) / tmax);
    const int desired = (target_waves + pp.nchunks - 1) / pp.nchunks;
    G = std::max(G, std::min(desired, static_cast<int>(units.size()) + 1));
    if (q.opts.waves_per_block > 0) G = std::max(G, q.opts.waves_per_block);
    // task scenarios into groups, one group per wave: heaviest first, each to
    // the least-loaded group with room (a group past TMAX tasks opens another)
    auto group = [&](int ng) {
        std::vector<std::vector<int>> out(ng);
        std::vector<int> load(ng, 0), cnt(ng, 0);
        if (pass.has_base_spot) load[0] = std::max(1, N / 2);
        for (int si : units) {
            const int w = sc[si].hi - sc[si].lo;
            int best = -1;
            for (int g = 0; g < static_cast<int>(out.size()); ++g)
                if (cnt[g] + w <= tmax && (best < 0 || load[g] < load[best])) best = g;
            if (best < 0) {
                out.emplace_back();
                load.push_back(0);
                cnt.push_back(0);
                best = static_cast<int>(out.size()) - 1;
            }
            out[best].push_back(si);
            load[best] += w;
            cnt[best] += w;
        }
        for (auto& v : out) std::sort(v.begin(), v.end());
        return out;
    };
    std::vector<std::vector<int>> gs = group(G);
    const int vmax = paths_max_waves(sh.fp32, q.opts.scheme == HS_SCHEME_QE, sh.nmax);
    const int wcap = std::max(1, std::min(wmax > 0 ? wmax : vmax, vmax));
    int W = q.opts.waves_per_block > 0 ? q.opts.waves_per_block
                                       : std::min(static_cast<int>(gs.size()), wcap);
    // more task groups than 8 waves hold: 4 waves per block where the base
    // assets fit in 4, else 8 (measured on 8-20 assets at 50k-200k paths: 3
    // or 4 waves per block run 30-42% faster than 8, 4 ahead of 3 at 10
    // assets x 200k; 5 and 6 run slower than 8, and one block of 10 or more
    // waves slower still)
    const int task_groups = (total + tmax - 1) / tmax;
    if (q.opts.waves_per_block == 0 && wmax == 0 && task_groups > std::min(vmax, 8))
        W = wmin <= 4 ? 4 : 8;
    W = std::max(W, wmin);
    W = std::min(W, vmax);
    pp.W = W;
    pp.nbg = static_cast<int>((gs.size() + W - 1) / W);
    // the blocks of a path chunk have nbg W waves: spread the task scenarios
    // over all of them rather than leave some waves without tasks (the same
    // blocks, shorter task chains per wave; results do not depend on the
    // grouping)
    const int slots = pp.nbg * W;
    if (static_cast<int>(gs.size()) < slots && static_cast<int>(units.size()) >= slots) {
        std::vector<std::vector<int>> spread = group(slots);
        if (static_cast<int>(spread.size()) == slots) gs = std::move(spread);
    }
    // dates stored per scenario: all (American), a window of them, or the last
    pp.plane = (sh.american ? static_cast<int64_t>(pass.window > 0 ? pass.window : q.n) : 1) * q.P;
    if (sh.fp32)
        fill_tables<float>(q, sh, sc, pass, gs, pp);
    else
        fill_tables<double>(q, sh, sc, pass, gs, pp);
    // discount factors exp(-r j dt), j = 0..n, per scenario of the pass, then
    // their inverses exp(+r j dt)
    // (scenarios with the same r and T share their rows: computed once)
    const int n = q.n;
    const size_t ns = pass.scen.size();
    const size_t row = static_cast<size_t>(n) + 1;
    pp.disc.resize(2 * ns * row);
    for (size_t i = 0; i < ns; ++i) {
        const Scenario& s = sc[pass.scen[i]];
        size_t same = i;
        for (size_t h = 0; h < i && same == i; ++h) {
            const Scenario& t = sc[pass.scen[h]];
            if (t.r == s.r && t.T == s.T) same = h;
        }
        if (same != i) {
            std::copy_n(pp.disc.begin() + same * row, row, pp.disc.begin() + i * row);
            std::copy_n(pp.disc.begin() + (ns + same) * row, row, pp.disc.begin() + (ns + i) * row);
            continue;
        }
        const double dt = s.T / static_cast<double>(n);
        for (int j = 0; j <= n; ++j) {
            pp.disc[i * row + j] = std::exp(-s.r * static_cast<double>(j) * dt);
            pp.disc[(ns + i) * row + j] = std::exp(s.r * static_cast<double>(j) * dt);
        }
    }
    pp.lay = layout_for(q, sh, static_cast<int>(pass.scen.size()), pp.ntasks,
                        static_cast<int>(pp.groups.size()), pass.window);
    return pp;
}

std::vector<Pass> make_passes(const Request& q, const Shape& sh, const std::vector<Scenario>& sc,
                              size_t workspace_bytes, size_t* min_bytes)
{
    // units: {base + spots} and then each bumped scenario with its own path
    std::vector<std::vector<int>> units;
    std::vector<int> head{0};
    for (size_t i = 1; i < sc.size(); ++i)
        if (from_base_path(sc[i].kind)) head.push_back(static_cast<int>(i));
    units.push_back(head);
    for (size_t i = 1; i < sc.size(); ++i)
        if (!from_base_path(sc[i].kind)) units.push_back({static_cast<int>(i)});
    auto bytes_of = [&](int nscen, int ntask, int nunits, int window) {
        return layout_for(q, sh, nscen, ntask, nunits + 2 * kMaxWaves, window).total;
    };
    auto tasks_of = [&](const std::vector<int>& u) {
        int nt = 0;
        for (int si : u) nt += sc[si].hi - sc[si].lo;
        return nt;
    };
    // windows of dates: American only, and only where they save memory
    const bool can_window = sh.american && q.n >= 2;
    const int forced = can_window ? q.opts.window_dates : 0;
    // the most dates per window with which unit u fits `limit` (0: none)
    auto window_for = [&](const std::vector<int>& u, size_t limit) {
        const int nt = tasks_of(u);
        for (int c = q.n - 1; c >= 1; --c)
            if (bytes_of(static_cast<int>(u.size()), nt, 1, c) <= limit) return c;
        return 0;
    };
    // each unit alone, all dates at once
    size_t unit_max = 0;
    for (auto& u : units)
        unit_max = std::max(unit_max, bytes_of(static_cast<int>(u.size()), tasks_of(u), 1, 0));
    // the least workspace that works (only computed when asked for, or when
    // some unit needs windows of dates)
    size_t mn = unit_max;
    if (min_bytes || forced > 0 || workspace_bytes < unit_max) {
        mn = 0;
        for (auto& u : units) {
            const int nt = tasks_of(u);
            size_t best = forced > 0 ? bytes_of(static_cast<int>(u.size()), nt, 1, forced)
                                     : bytes_of(static_cast<int>(u.size()), nt, 1, 0);
            // the smallest footprint over window lengths: every length up to
            // 64, then lengths about 5% apart (features grow with c,
            // checkpoints shrink with it)
            if (can_window && forced == 0)
                for (int c = 1; c < q.n; c = c < 64 ? c + 1 : c + c / 20)
                    best = std::min(best, bytes_of(static_cast<int>(u.size()), nt, 1, c));
            mn = std::max(mn, best);
        }
    }
    if (min_bytes) *min_bytes = mn;
    std::vector<Pass> passes;
    if (workspace_bytes < mn) return passes;
    Pass cur;
    int cur_tasks = 0, cur_units = 0;
    auto close = [&]() {
        if (!cur.scen.empty()) passes.push_back(cur);
        cur = Pass();
        cur_tasks = 0;
        cur_units = 0;
    };
    for (size_t ui = 0; ui < units.size(); ++ui) {
        const int nt = tasks_of(units[ui]);
        const int us = static_cast<int>(units[ui].size());
        const bool alone_fits = bytes_of(us, nt, 1, 0) <= workspace_bytes;
        if (forced > 0 || !alone_fits) {
            // a unit in windows of dates, in a pass of its own
            close();
            Pass wp;
            wp.scen = units[ui];
            wp.has_base_spot = ui == 0;
            wp.window = forced > 0 ? forced : window_for(units[ui], workspace_bytes);
            if (wp.window <= 0) return {};  // unreachable: mn covers every unit
            passes.push_back(wp);
            continue;
        }
        const size_t need = bytes_of(static_cast<int>(cur.scen.size()) + us, cur_tasks + nt,
                                     cur_units + 1, 0);
        if (!cur.scen.empty() && need > workspace_bytes) close();
        if (ui == 0) cur.has_base_spot = true;
        for (int si : units[ui]) cur.scen.push_back(si);
        cur_tasks += nt;
        cur_units += 1;
    }
    close();
    return passes;
}

void greeks_from_prices(const Request& q, const std::vector<double>& price, hs_greeks* out)
{
    const int N = q.N;
    const uint32_t mask = q.bumps.mask;
    const double nan = std::nan("");
    const double V = price[0];
    size_t s = 1;
    for (int a = 0; a < N; ++a) {
        if (out->delta) out->delta[a] = nan;
        if (out->gamma) out->gamma[a] = nan;
        if (out->vega) out->vega[a] = nan;
    }
    if (out->corr)
        for (int i = 0; i < N * (N - 1) / 2; ++i) out->corr[i] = nan;
    out->theta = nan;
    out->rho = nan;
    if (mask & HS_BUMP_DELTA_GAMMA) {
        for (int a = 0; a < N; ++a) {
            const double up = price[s + a], dn = price[s + N + a];
            const double hs = q.bumps.spot_rel * q.S0[a];
            if (out->delta) out->delta[a] = (up - dn) / (2.0 * hs);
            if (out->gamma) out->gamma[a] = (up - 2.0 * V + dn) / (hs * hs);
        }
        s += 2 * N;
    }
    if (mask & HS_BUMP_VEGA) {
        for (int a = 0; a < N; ++a)
            if (out->vega) out->vega[a] = (price[s + a] - V) / (q.bumps.v0_rel * q.v0[a]);
        s += N;
    }
    if (mask & HS_BUMP_THETA) {
        out->theta = (price[s] - V) / q.bumps.T_abs;
        s += 1;
    }
    if (mask & HS_BUMP_RHO) {
        out->rho = (price[s] - V) / q.bumps.r_abs;
        s += 1;
    }
    if ((mask & HS_BUMP_CORR) && N > 1) {
        int t = 0;
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j, ++t)
                if (out->corr) out->corr[t] = (price[s + t] - V) / q.bumps.corr_abs;
    }
}

std::vector<unsigned char> model_table(const Request& q, const Scenario& base, bool fp32)
{
    return fp32 ? model_table_t<float>(q, base) : model_table_t<double>(q, base);
}

}  // namespace hs
