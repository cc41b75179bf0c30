// hs_lsmc.hip -- gfx950 kernels of the Longstaff-Schwartz stage (Sec. 2.2 and
// 2.2.1: the regression that decides early exercise, here on the GPU in FP64).
//
//   k_gram           per (scenario, date): regression-set means, the Gram
//                    matrix of the centred basis over in-the-money paths, and
//                    its Cholesky factor (all FP64).  Independent of the cash
//                    flows, so all dates run at once.
//   k_sweep          per scenario, one workgroup: the backward sweep
//                    (right-hand side, solve, exercise, cash-flow update) and
//                    the FP64 price and standard error, with the cash-flow
//                    state in registers or in the workspace.
//   k_sweep_cluster  the same sweep with several workgroups per scenario that
//                    meet once per exercise date.
// Reductions use fixed trees (wave butterfly, then waves in index order), so
// every result is a deterministic function of the request.
#include "hs_device.hpp"

namespace hs {
namespace {

// ---------------------------------------------------------------------------
// FP64 block reductions with a fixed tree.  Inside a wave: DPP row shifts by
// 1, 2, 4, 8 (each lane adds its row neighbour; lanes past the row start add
// 0), then the row broadcasts of lanes 15 and 31, leaving the wave's total in
// lane 63.  Across waves: K threads fold the wave totals in wave order.  The
// order of every addition is fixed, so the sum is deterministic.

__device__ __forceinline__ double dpp_f64(double v, int ctrl_tag)
{
    const uint64_t bits = __builtin_bit_cast(uint64_t, v);
    int lo = static_cast<int>(bits), hi = static_cast<int>(bits >> 32);
    switch (ctrl_tag) {
    case 1:
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x111, 0xf, 0xf, true);
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x111, 0xf, 0xf, true);
        break;
    case 2:
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x112, 0xf, 0xf, true);
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x112, 0xf, 0xf, true);
        break;
    case 4:
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x114, 0xf, 0xf, true);
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x114, 0xf, 0xf, true);
        break;
    case 8:
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x118, 0xf, 0xf, true);
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x118, 0xf, 0xf, true);
        break;
    case 15:  // row_bcast15 into rows 1 and 3
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x142, 0xa, 0xf, false);
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x142, 0xa, 0xf, false);
        break;
    default:  // row_bcast31 into rows 2 and 3
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x143, 0xc, 0xf, false);
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x143, 0xc, 0xf, false);
        break;
    }
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint32_t>(lo));
}

// The wave's total, valid in lane 63.
__device__ __forceinline__ double wave_sum_lane63(double v)
{
    v += dpp_f64(v, 1);
    v += dpp_f64(v, 2);
    v += dpp_f64(v, 4);
    v += dpp_f64(v, 8);
    v += dpp_f64(v, 15);
    v += dpp_f64(v, 31);
    return v;
}

template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* scratch /* [nwaves][K] + K */,
                                          int nwaves)
{
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] = wave_sum_lane63(v[i]);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) {
#pragma unroll
        for (int i = 0; i < K; ++i) scratch[wid * K + i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x < K) {
        double s = scratch[threadIdx.x];
        for (int q = 1; q < nwaves; ++q) s += scratch[q * K + threadIdx.x];
        scratch[nwaves * K + threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] = scratch[nwaves * K + i];
    __syncthreads();
}

__device__ __forceinline__ double payoff(int cp, double K, double U)
{
    const double h = cp == 0 ? K - U : U - K;
    return h > 0.0 ? h : 0.0;
}

// phi = {1, x, x^2[, w, x w]}, x = (U - cU)/K, w = (A - cA)/tbar
__device__ __forceinline__ void basis(int m, double U, double Av, double cU, double cA,
                                      double inv_K, double inv_tbar, double (&phi)[5])
{
    const double x = (U - cU) * inv_K;
    const double wv = m == 5 ? (Av - cA) * inv_tbar : 0.0;
    phi[0] = 1.0;
    phi[1] = x;
    phi[2] = x * x;
    phi[3] = wv;
    phi[4] = x * wv;
}

// Packed row-major lower Cholesky of the Gram matrix into the record; a pivot
// at or below 1e-12 of its diagonal entry marks the date as skipped.
__device__ __forceinline__ void gram_finish(int m, const double (&g)[15], double cU, double cA,
                                            double cnt, RegRec* rr)
{
    double L[15];
#pragma unroll
    for (int i = 0; i < 15; ++i) L[i] = 0.0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            if (i < m) {
                double acc = g[i * (i + 1) / 2 + j];
#pragma unroll
                for (int q = 0; q < j; ++q) acc -= L[i * (i + 1) / 2 + q] * L[j * (j + 1) / 2 + q];
                if (i == j) {
                    ok = ok && acc > 1e-12 * g[i * (i + 1) / 2 + i];
                    L[i * (i + 1) / 2 + i] = ok ? sqrt(acc) : 1.0;
                } else {
                    L[i * (i + 1) / 2 + j] = acc / L[j * (j + 1) / 2 + j];
                }
            }
        }
    }
    // store the inverse factor, so a solve is two triangular mat-vecs:
    // beta = L^{-T} (L^{-1} b)
    double Li[15];
#pragma unroll
    for (int i = 0; i < 15; ++i) Li[i] = 0.0;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        if (j < m) {
            Li[j * (j + 1) / 2 + j] = 1.0 / L[j * (j + 1) / 2 + j];
#pragma unroll
            for (int i = j + 1; i < 5; ++i) {
                if (i < m) {
                    double acc = 0.0;
#pragma unroll
                    for (int q = j; q < i; ++q) acc += L[i * (i + 1) / 2 + q] * Li[q * (q + 1) / 2 + j];
                    Li[i * (i + 1) / 2 + j] = -acc / L[i * (i + 1) / 2 + i];
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 15; ++i) rr->L[i] = ok ? Li[i] : 0.0;
    rr->cU = cU;
    rr->cA = cA;
    rr->ok = ok ? 1.0 : 0.0;
    rr->cnt = cnt;
}

// ---------------------------------------------------------------------------
// Gram kernel: block (date k = blockIdx.x + 1, scenario blockIdx.y), one pass
// over the date's features.  Over the in-the-money paths it sums the moments
// S_ab = sum y^a z^b of the fixed-shift variables y = (U - K)/K and
// z = A/tbar - 1 (12 monomials: a <= 4, b <= 2, those the basis products
// need), then shifts them to the regression-set means, d = S_10/S_00 and
// e = S_01/S_00: M_ij = sum (y - d)^i (z - e)^j by the binomial expansion.
// x = y - d and w = z - e are the centred basis variables, so the Gram matrix
// entry of phi_p phi_q is M at the summed exponents.  The shift is small
// against the spread of y and z, so the expansion loses little precision.

// monomial (a, b) -> slot in the moment array
__device__ __host__ constexpr int mono(int a, int b)
{
    return b == 0 ? a : (b == 1 ? 5 + a : 9 + a);  // (0..4,0) (0..3,1) (0..2,2)
}

template <typename R>
__global__ void __launch_bounds__(kGramThreads) k_gram(const LsmcArgs A)
{
    constexpr int U1 = 8;  // loads in flight per thread
    __shared__ double red[(kGramThreads / 64 + 1) * 12];
    const int s = blockIdx.y;
    const int k = blockIdx.x + A.k_lo;
    const R2<R>* __restrict__ F = static_cast<const R2<R>*>(A.feat) + s * A.plane +
                                  static_cast<int64_t>(k - A.f_date0) * A.P;
    const int nw = kGramThreads / 64;
    const int64_t P = A.P;
    const bool two = A.m == 5;  // the basis has w terms

    double S[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) S[i] = 0.0;
    for (int64_t p0 = threadIdx.x; p0 < P; p0 += kGramThreads * U1) {
        // every load issues, with no branch between them (a path past P
        // reads the last path and is masked below), so all U1 are in flight
        R2<R> f[U1];
#pragma unroll
        for (int u = 0; u < U1; ++u) {
            const int64_t p = p0 + u * kGramThreads;
            f[u] = F[p < P ? p : P - 1];
        }
#pragma unroll
        for (int u = 0; u < U1; ++u) {
            const double Uv = static_cast<double>(f[u].u);
            if (p0 + u * kGramThreads < P && payoff(A.cp, A.K, Uv) > 0.0) {
                const double y = (Uv - A.K) * A.inv_K;
                const double y2 = y * y;
                const double y3 = y2 * y;
                S[mono(0, 0)] += 1.0;
                S[mono(1, 0)] += y;
                S[mono(2, 0)] += y2;
                S[mono(3, 0)] += y3;
                S[mono(4, 0)] += y2 * y2;
                if (two) {
                    const double z = static_cast<double>(f[u].a) * A.inv_tbar - 1.0;
                    const double z2 = z * z;
                    S[mono(0, 1)] += z;
                    S[mono(1, 1)] += y * z;
                    S[mono(2, 1)] += y2 * z;
                    S[mono(3, 1)] += y3 * z;
                    S[mono(0, 2)] += z2;
                    S[mono(1, 2)] += y * z2;
                    S[mono(2, 2)] += y2 * z2;
                }
            }
        }
    }
    block_sum<12>(S, red, nw);
    if (threadIdx.x != 0) return;
    RegRec* rr = A.reg + static_cast<int64_t>(s) * A.n + (k - 1);
    const double cnt = S[mono(0, 0)];
    const int m = A.m;
    if (cnt < static_cast<double>(m)) {
        rr->ok = 0.0;
        rr->cnt = cnt;
        return;
    }
    const double d = S[mono(1, 0)] / cnt;
    const double e = two ? S[mono(0, 1)] / cnt : 0.0;
    // powers of -d and -e, binomial coefficients up to 4
    double nd[5], ne[3];
    nd[0] = 1.0;
    ne[0] = 1.0;
#pragma unroll
    for (int i = 1; i < 5; ++i) nd[i] = nd[i - 1] * -d;
    ne[1] = -e;
    ne[2] = e * e;
    constexpr double binom[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0},
                                    {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
    // centred moment M_ij from the fixed-shift sums
    auto M = [&](int i, int j) {
        double acc = 0.0;
        for (int b = 0; b <= j; ++b)
            for (int a = 0; a <= i; ++a)
                acc += binom[i][a] * binom[j][b] * nd[i - a] * ne[j - b] * S[mono(a, b)];
        return acc;
    };
    // basis exponents: phi = {1, x, x^2, w, x w}
    constexpr int ex[5] = {0, 1, 2, 0, 1};
    constexpr int ew[5] = {0, 0, 0, 1, 1};
    double g[15];
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b, ++idx)
            g[idx] = (a < m && b < m) ? M(ex[a] + ex[b], ew[a] + ew[b]) : 0.0;
    gram_finish(m, g, A.K + A.K * d, (1.0 + e) / A.inv_tbar, cnt, rr);
}

// ---------------------------------------------------------------------------
// Backward sweep + price: one block of 1024 threads per scenario.  Thread t
// handles paths t + 1024 i.  With GLB the cash flow and exercise date of each
// path live in the workspace; otherwise in registers (Q paths per thread).

// beta = L^{-T} (L^{-1} b) with Li = L^{-1} packed lower row-major (entries
// past m are 0, so beta past m is 0).
__device__ __forceinline__ void solve_packed(int m, const double (&Li)[15], const double (&b)[5],
                                             double (&beta)[5])
{
    (void)m;
    double y[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q <= i; ++q) acc += Li[i * (i + 1) / 2 + q] * b[q];
        y[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int q = i; q < 5; ++q) acc += Li[q * (q + 1) / 2 + i] * y[q];
        beta[i] = acc;
    }
}

template <typename R, int Q, bool GLB>
__global__ void __launch_bounds__(kSweepThreads) k_sweep(const LsmcArgs A)
{
    extern __shared__ unsigned char hs_smem[];
    double* const sdisc = reinterpret_cast<double*>(hs_smem);         // [n+1]
    double* const red = sdisc + ((A.n + 1 + 1) & ~1);                 // [16 + 1][5]
    constexpr int NW = kSweepThreads / 64;
    const int s = blockIdx.x;
    const int n = A.n;
    const int64_t P = A.P;
    const R2<R>* __restrict__ F = static_cast<const R2<R>*>(A.feat) + s * A.plane;
    for (int j = threadIdx.x; j <= n; j += kSweepThreads) sdisc[j] = A.disc[static_cast<int64_t>(s) * (n + 1) + j];
    __syncthreads();

    // the thread index, opaque at each use: the compiler forms a path's index
    // and address where it needs them instead of keeping Q of them in
    // registers across the date loop
    auto tx = []() {
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
        return t;
    };
    double* const gcf = GLB ? A.cf + static_cast<int64_t>(s) * P : nullptr;
    int32_t* const gtau = GLB ? A.tau + static_cast<int64_t>(s) * P : nullptr;
    const int64_t last = static_cast<int64_t>(n - A.f_date0) * P;  // date n

    // (windows of dates keep the state in the workspace, GLB)
    double cf[GLB ? 1 : Q];
    int tau[GLB ? 1 : Q];
    if (!GLB) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t p = tx() + static_cast<int64_t>(i) * kSweepThreads;
            cf[i] = p < P ? payoff(A.cp, A.K, static_cast<double>(F[last + p].u)) : 0.0;
            tau[i] = n;
        }
    } else if (A.win_first) {
        for (int64_t p = threadIdx.x; p < P; p += kSweepThreads) {
            gcf[p] = payoff(A.cp, A.K, static_cast<double>(F[last + p].u));
            gtau[p] = n;
        }
    }

    double skipped = 0.0;
    const int m = A.m;
    if (A.american) {
        for (int k = min(A.k_hi, n - 1); k >= A.k_lo; --k) {
            const RegRec* rr = A.reg + static_cast<int64_t>(s) * n + (k - 1);
            if (rr->ok == 0.0) {
                skipped += 1.0;
                continue;
            }
            const double cU = rr->cU, cA = rr->cA;
            const R2<R>* __restrict__ Fk = F + static_cast<int64_t>(k - A.f_date0) * P;
            double b[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (!GLB) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const int64_t p = tx() + static_cast<int64_t>(i) * kSweepThreads;
                    if (p < P) {
                        const R2<R> f = Fk[p];
                        const double U = static_cast<double>(f.u);
                        if (payoff(A.cp, A.K, U) > 0.0) {
                            double phi[5];
                            basis(m, U, static_cast<double>(f.a), cU, cA, A.inv_K, A.inv_tbar, phi);
                            const double Y = cf[i] * sdisc[tau[i] - k];
#pragma unroll
                            for (int q = 0; q < 5; ++q)
                                if (q < m) b[q] += phi[q] * Y;
                        }
                    }
                }
            } else {
                for (int64_t p = threadIdx.x; p < P; p += kSweepThreads) {
                    const R2<R> f = Fk[p];
                    const double U = static_cast<double>(f.u);
                    if (payoff(A.cp, A.K, U) > 0.0) {
                        double phi[5];
                        basis(m, U, static_cast<double>(f.a), cU, cA, A.inv_K, A.inv_tbar, phi);
                        const double Y = gcf[p] * sdisc[gtau[p] - k];
#pragma unroll
                        for (int q = 0; q < 5; ++q)
                            if (q < m) b[q] += phi[q] * Y;
                    }
                }
            }
            block_sum<5>(b, red, NW);
            double L[15];
#pragma unroll
            for (int i = 0; i < 15; ++i) L[i] = rr->L[i];
            double beta[5];
            solve_packed(m, L, b, beta);
            if (!GLB) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const int64_t p = tx() + static_cast<int64_t>(i) * kSweepThreads;
                    if (p < P) {
                        const R2<R> f = Fk[p];
                        const double U = static_cast<double>(f.u);
                        const double h = payoff(A.cp, A.K, U);
                        if (h > 0.0) {
                            double phi[5];
                            basis(m, U, static_cast<double>(f.a), cU, cA, A.inv_K, A.inv_tbar, phi);
                            double cont = 0.0;
#pragma unroll
                            for (int q = 0; q < 5; ++q)
                                if (q < m) cont += phi[q] * beta[q];
                            if (h > cont) {
                                cf[i] = h;
                                tau[i] = k;
                            }
                        }
                    }
                }
            } else {
                for (int64_t p = threadIdx.x; p < P; p += kSweepThreads) {
                    const R2<R> f = Fk[p];
                    const double U = static_cast<double>(f.u);
                    const double h = payoff(A.cp, A.K, U);
                    if (h > 0.0) {
                        double phi[5];
                        basis(m, U, static_cast<double>(f.a), cU, cA, A.inv_K, A.inv_tbar, phi);
                        double cont = 0.0;
#pragma unroll
                        for (int q = 0; q < 5; ++q)
                            if (q < m) cont += phi[q] * beta[q];
                        if (h > cont) {
                            gcf[p] = h;
                            gtau[p] = k;
                        }
                    }
                }
            }
        }
    }

    double* const o = A.out + static_cast<int64_t>(s) * 4;
    if (!A.win_last) {  // a window before the last: the state stays in the workspace
        if (threadIdx.x == 0) o[2] = (A.win_first ? 0.0 : o[2]) + skipped;
        return;
    }

    // price: mean of CF exp(-r tau dt), then the sample standard deviation
    double s1[1] = {0.0};
    if (!GLB) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t p = tx() + static_cast<int64_t>(i) * kSweepThreads;
            if (p < P) s1[0] += cf[i] * sdisc[tau[i]];
        }
    } else {
        for (int64_t p = threadIdx.x; p < P; p += kSweepThreads) s1[0] += gcf[p] * sdisc[gtau[p]];
    }
    block_sum<1>(s1, red, NW);
    const double mean = s1[0] / static_cast<double>(P);
    double s2[1] = {0.0};
    if (!GLB) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t p = tx() + static_cast<int64_t>(i) * kSweepThreads;
            if (p < P) {
                const double d = cf[i] * sdisc[tau[i]] - mean;
                s2[0] += d * d;
            }
            if (A.export_tau && p < P) A.tau[static_cast<int64_t>(s) * P + p] = tau[i];
        }
    } else {
        for (int64_t p = threadIdx.x; p < P; p += kSweepThreads) {
            const double d = gcf[p] * sdisc[gtau[p]] - mean;
            s2[0] += d * d;
        }
    }
    block_sum<1>(s2, red, NW);
    if (threadIdx.x == 0) {
        o[0] = mean;
        o[1] = sqrt(s2[0] / static_cast<double>(P - 1) / static_cast<double>(P));
        o[2] = (A.win_first ? 0.0 : o[2]) + skipped;
        o[3] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Cluster sweep: G workgroups per scenario, each holding 512 Q paths' cash
// flow, exercise date and three dates of features in registers.  Once per
// exercise date each wave reduces its right-hand-side partials (a fixed DPP
// tree over its 64 lanes) into LDS; after a barrier, wave q folds component q
// over the waves in order and publishes the workgroup's partial into its slot
// of a per-date row in the workspace.  A slot starts empty (kEmptySlot) and
// receives exactly one 64-bit value, so a reader that sees a non-empty slot
// has the value itself -- no counter, no fence.  Wave q then folds component q
// of the G workgroup partials in one fixed order (lane l takes slots l,
// l + 64, ... in turn, then a DPP tree over the lanes), so all workgroups hold
// the same sum; a second barrier hands it to the other waves, and each thread
// solves for the regression coefficients itself.  A wait longer than
// timeout_ticks of the wall clock sets the error flag and all workgroups
// leave the kernel.

// LDS of the cluster sweep, after the discount table: wave partials [2][NW][8]
// (G == 1), totals [2][8], status flag.
struct ClusterLds {
    double* part;
    double* tot;
    int* flag;
};

// b: this thread's partials.  On return b holds the scenario totals (every
// thread); false if a wait timed out.  par alternates between consecutive
// calls so that no wave overwrites totals another wave has not read yet.
template <int K>
__device__ __forceinline__ bool cluster_exchange(double (&b)[K], int m, double* row, int G, int g,
                                                 int par, const ClusterArgs& C, const ClusterLds& L)
{
    constexpr int NW = kClusterThreads / 64;
    // lane and m made opaque here, so that the compiler recomputes the
    // conditions on them at each exchange instead of keeping their masks in
    // scalar registers across the whole date loop
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    asm volatile("" : "+s"(m));
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int q = 0; q < K; ++q) b[q] = wave_sum_lane63(b[q]);
    if (lane == 63) {
#pragma unroll
        for (int q = 0; q < K; ++q)
            if (q < m) L.part[(par * NW + wid) * kPartStride + q] = b[q];
    }
    __syncthreads();
    if (wid < m) {
        const int q = wid;
        double t = L.part[(par * NW) * kPartStride + q];
        for (int w = 1; w < NW; ++w) t += L.part[(par * NW + w) * kPartStride + q];
        if (G == 1) {
            if (lane == 0) L.tot[par * kPartStride + q] = t;
        } else {
            if (lane == 0)
                __hip_atomic_store(reinterpret_cast<uint64_t*>(row + g * kPartStride + q),
                                   __builtin_bit_cast(uint64_t, t), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            double acc = 0.0;
            bool bad = false;
            for (int j = lane; j < G; j += 64) {
                uint64_t* slot = reinterpret_cast<uint64_t*>(row + j * kPartStride + q);
                uint64_t x = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (x == kEmptySlot) {
                    const long long t0 = wall_clock64();
                    for (;;) {
                        __builtin_amdgcn_s_sleep(1);
                        x = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (x != kEmptySlot) break;
                        if (__hip_atomic_load(C.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                            wall_clock64() - t0 > C.timeout_ticks) {
                            __hip_atomic_store(C.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            bad = true;
                            break;
                        }
                    }
                }
                if (bad) break;
                acc += __builtin_bit_cast(double, x);
            }
            if (bad) *L.flag = 0;
            acc = wave_sum_lane63(acc);
            if (lane == 63) L.tot[par * kPartStride + q] = acc;
        }
    }
    __syncthreads();
    if (*L.flag == 0) return false;
#pragma unroll
    for (int q = 0; q < K; ++q) b[q] = q < m ? L.tot[par * kPartStride + q] : 0.0;
    return true;
}

// Each thread holds the Q paths pbase + i 512 + t (i < Q, pbase = g 512 Q) of
// its workgroup g: their discounted cash flows and two dates of features, in
// registers.  At date k the buffer `cur` holds date k's features and `old`
// date k + 1's: the exercise decision of date k + 1 (its regression solved
// one exchange ago) reads `old`, which then receives date k - 1's loads; the
// right-hand side of date k reads `cur`.  The loads are issued before date
// k's exchange, so they fly during it (the exchange's polls complete after
// them: vector loads of a wave complete in order), and nothing waits for them
// until date k - 1.  The loop is unrolled twice so that the two buffers swap
// roles by renaming.  Up to 6 paths per thread (5 with FP64 features, whose
// two dates take 8 registers per path) two workgroups share a CU (4 waves per
// SIMD, 128 registers); more paths per thread (large Greek sets: fewer
// launches, each a chain of exchanges) take one workgroup per CU and up to
// 256 registers.
template <typename R, int Q, bool WIN>
__global__ void __launch_bounds__(kClusterThreads, Q <= (sizeof(R) == 8 ? 5 : 6) ? 4 : 2)
    k_sweep_cluster(const LsmcArgs A, const ClusterArgs C)
{
    extern __shared__ unsigned char hs_smem[];
    constexpr int NW = kClusterThreads / 64;
    const int n = A.n;
    const int G = C.G;
    ClusterLds Ls;
    Ls.part = reinterpret_cast<double*>(hs_smem);   // [2][NW][8]
    Ls.tot = Ls.part + 2 * NW * kPartStride;        // [2][8]
    Ls.flag = reinterpret_cast<int*>(Ls.tot + 2 * kPartStride);
    const int sl = blockIdx.x / G;
    const int g = blockIdx.x - sl * G;
    const int s = C.s0 + sl;
    const int64_t P = A.P;
    const int m = A.m;
    const int tid = threadIdx.x;
    if (tid == 0) *Ls.flag = 1;
    __syncthreads();

    const int64_t row_len = static_cast<int64_t>(G) * kPartStride;
    const bool amer = A.american != 0;
    double* const part = C.partials +
                         (static_cast<int64_t>(s) * cluster_rows(amer, n) - cluster_row0(amer, n)) *
                             row_len;
    const cptr<RegRec> recs = as_const<RegRec>(A.reg) + static_cast<int64_t>(s) * n;
    const cptr<double> dsc = as_const<double>(A.disc) + static_cast<int64_t>(s) * (n + 1);
    const cptr<double> idsc = as_const<double>(A.idisc) + static_cast<int64_t>(s) * (n + 1);
    // this workgroup's chunk of paths [pbase, pbase + chunk) of scenario s
    const int64_t pbase = static_cast<int64_t>(g) * (kClusterThreads * Q);
    const int chunk = static_cast<int>(min<int64_t>(static_cast<int64_t>(kClusterThreads) * Q,
                                                    P - pbase));
    const int nlive = chunk > tid ? (chunk - tid + kClusterThreads - 1) / kClusterThreads : 0;
    const R2<R>* __restrict__ const F = static_cast<const R2<R>*>(A.feat) + s * A.plane + pbase;
    // a window of dates (WIN), else every date: regressions k_top..k_lo, the
    // features of date d at index d - f0
    const int f0 = WIN ? A.f_date0 : 1;
    const int64_t last = WIN ? static_cast<int64_t>(n - f0) * P  // date n
                             : (A.american ? static_cast<int64_t>(n - 1) * P : 0);
    const int k_lo = WIN ? A.k_lo : 1;
    const int k_top = WIN ? min(A.k_hi, n - 1) : n - 1;
    int par = 0;

    // Q loads of one date into buf, through a buffer resource over this
    // chunk's paths of that date: the whole offset is in the lane's offset,
    // which the buffer unit range-checks, so paths past the chunk read 0
    // (never used) instead of memory past the plane
    // The lane offsets of a date's Q loads are formed afresh at each load from
    // an opaque base (one add each) instead of being kept in Q registers
    // across the sweep.
    const uint32_t voff = static_cast<uint32_t>(tid) * sizeof(R2<R>);
    auto load = [&](int k, R2<R>(&buf)[Q]) {
        const auto rs = buffer_over(F + static_cast<int64_t>(k - f0) * P,
                                    static_cast<uint32_t>(chunk) * sizeof(R2<R>));
        uint32_t vo = voff;
        asm volatile("" : "+v"(vo));
#pragma unroll
        for (int i = 0; i < Q; ++i)
            buf[i] = buffer_load<R2<R>>(rs, vo + i * kClusterThreads * sizeof(R2<R>), 0);
    };

    // State per path: the cash flow discounted to time 0, D = h_tau exp(-r tau
    // dt).  The regression target at date k is D exp(r k dt) =
    // h_tau exp(-r (tau - k) dt), and the price is the mean of D.  The exercise
    // date tau, wanted only for export, goes straight to memory at each
    // exercise (the sweep runs backward, so the last write is the earliest
    // exercise date).
    // (the chunk's base; each store forms its lane's address afresh from an
    // opaque thread index, so that no per-path addresses stay alive)
    int32_t* const tau = A.export_tau ? A.tau + static_cast<int64_t>(s) * P + pbase : nullptr;
    auto put_tau = [&](int i, int v) {
        int t = tid;
        asm volatile("" : "+v"(t));
        tau[t + i * kClusterThreads] = v;
    };
    double D[Q];
    if (!WIN || A.win_first) {
        R2<R> fn[Q];
        const auto rs = buffer_over(F + last, static_cast<uint32_t>(chunk) * sizeof(R2<R>));
#pragma unroll
        for (int i = 0; i < Q; ++i)
            fn[i] = buffer_load<R2<R>>(rs, voff + i * kClusterThreads * sizeof(R2<R>), 0);
        const double dn = dsc[n];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            D[i] = i < nlive ? payoff(A.cp, A.K, static_cast<double>(fn[i].u)) * dn : 0.0;
            if (tau && i < nlive) put_tau(i, n);
        }
    } else {
        const double* const dstate = A.cf + static_cast<int64_t>(s) * P + pbase + tid;
#pragma unroll
        for (int i = 0; i < Q; ++i) D[i] = i < nlive ? dstate[i * kClusterThreads] : 0.0;
    }

    double beta[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    bool have = false;  // beta of the later date k+1 is valid
    double skipped = 0.0;
    // payoff h = max(sg U - sg K, 0) as one FMA (sg = -1 put, +1 call: the
    // same rounding as K - U or U - K); basis x = U/K - cU/K and w = A/tbar -
    // cA/tbar as one FMA each (w = 0 for the quadratic basis)
    const double sg = A.cp == 0 ? -1.0 : 1.0;
    const double sK = sg * A.K;
    const double iw = m == 5 ? A.inv_tbar : 0.0;
    if (A.american) {
        R2<R> fa[Q], fb[Q];
        if (k_top >= k_lo) load(k_top, fa);
        // regression-set flag and means of date k, loaded one date ahead
        double r_ok = k_top >= k_lo ? recs[k_top - 1].ok : 0.0;
        double r_cU = k_top >= k_lo ? recs[k_top - 1].cU : 0.0;
        double r_cA = k_top >= k_lo ? recs[k_top - 1].cA : 0.0;
        double bcU = 0.0, bcA = 0.0;  // regression-set means of date k+1, as cU/K, cA/tbar

        // the exercise decision at date kd with that date's regression (beta,
        // bcU, bcA) and features.  The basis values are recomputed from the
        // features: an empty asm statement hides that they equal the ones the
        // right-hand side formed one exchange earlier, so that the compiler
        // does not keep those (4 more registers per path) across the exchange.
        auto decide = [&](int kd, R2<R>(&f)[Q]) {
            const double d1 = dsc[kd];
            // the live-path count, opaque to the compiler here: it compares
            // i < nl where the decision needs it instead of keeping Q masks
            // (2 Q scalar registers) alive across the whole loop
            int nl = nlive;
            asm volatile("" : "+v"(nl));
            uint32_t exb = 0;  // bit i: path i exercised here
            // four paths at a time, stage by stage, so that their FP64
            // dependency chains interleave
            constexpr int IL = 4;
#pragma unroll
            for (int i0 = 0; i0 < Q; i0 += IL) {
                double U[IL], h[IL], x[IL], w[IL], t[IL], cont[IL];
#pragma unroll
                for (int j = 0; j < IL; ++j)
                    if (i0 + j < Q) asm volatile("" : "+v"(f[i0 + j].u), "+v"(f[i0 + j].a));
#pragma unroll
                for (int j = 0; j < IL; ++j) {
                    if (i0 + j >= Q) continue;
                    U[j] = static_cast<double>(f[i0 + j].u);
                    x[j] = fma(U[j], A.inv_K, -bcU);
                    w[j] = fma(static_cast<double>(f[i0 + j].a), iw, -bcA);
                }
#pragma unroll
                for (int j = 0; j < IL; ++j) {
                    if (i0 + j >= Q) continue;
                    h[j] = fmax(fma(U[j], sg, -sK), 0.0);
                    t[j] = fma(beta[4], w[j], fma(beta[2], x[j], beta[1]));
                }
                // beta_0 + beta_1 x + beta_2 x^2 + beta_3 w + beta_4 x w
#pragma unroll
                for (int j = 0; j < IL; ++j)
                    if (i0 + j < Q) cont[j] = fma(x[j], t[j], fma(beta[3], w[j], beta[0]));
#pragma unroll
                for (int j = 0; j < IL; ++j) {
                    const int i = i0 + j;
                    if (i >= Q) continue;
                    // non-short-circuit: no branch around the continuation value
                    const bool ex = (i < nl) & (h[j] > 0.0) & (h[j] > cont[j]);
                    D[i] = ex ? h[j] * d1 : D[i];
                    exb |= ex ? (1u << i) : 0u;
                }
            }
            // exercise dates, only when exported: a store under a branch in
            // the loop above would cut it into one block per path, and the
            // compiler could no longer interleave the paths' FP64 chains
            if (tau) {
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    if (exb & (1u << i)) put_tau(i, kd);
            }
        };

        // one date k (cur: date k, old: date k + 1); false if a wait timed out
        auto step = [&](int k, R2<R>(&cur)[Q], R2<R>(&old)[Q]) -> bool {
            const bool ok = r_ok != 0.0;
            const double cU = r_cU * A.inv_K, cA = r_cA * iw;
            if (k > k_lo) {
                r_ok = recs[k - 2].ok;
                r_cU = recs[k - 2].cU;
                r_cA = recs[k - 2].cA;
            }
            // exercise at date k+1 with its regression, then the next date's
            // loads into its buffer, then this date's right-hand side with the
            // updated cash flows
            if (have) decide(k + 1, old);
            // unconditional (the last date reloads itself, unused): a load
            // under a branch would leave the compiler unsure how many loads
            // are in flight, and it would wait for all of them before the
            // right-hand side
            load(max(k - 1, k_lo), old);
            // -0.0 + y == y for every y, so the first path's terms need no add
            double b[5] = {-0.0, -0.0, -0.0, -0.0, -0.0};
            if (ok) {
                const double ik = idsc[k];
                // four paths at a time, stage by stage (the sums still add
                // the paths in order)
                constexpr int IL = 4;
#pragma unroll
                for (int i0 = 0; i0 < Q; i0 += IL) {
                    double x[IL], w[IL], Y[IL], xY[IL];
#pragma unroll
                    for (int j = 0; j < IL; ++j) {
                        const int i = i0 + j;
                        if (i >= Q) continue;
                        const double U = static_cast<double>(cur[i].u);
                        x[j] = fma(U, A.inv_K, -cU);
                        w[j] = fma(static_cast<double>(cur[i].a), iw, -cA);
                        // paths out of the money add exact zeros, and so do
                        // paths past P (their D stays 0: decide never
                        // exercises them)
                        Y[j] = fma(U, sg, -sK) > 0.0 ? D[i] * ik : 0.0;
                        xY[j] = x[j] * Y[j];
                    }
#pragma unroll
                    for (int j = 0; j < IL; ++j) {
                        if (i0 + j >= Q) continue;
                        b[0] += Y[j];
                        b[1] += xY[j];
                        b[2] = fma(x[j], xY[j], b[2]);
                        b[3] = fma(w[j], Y[j], b[3]);
                        b[4] = fma(w[j], xY[j], b[4]);
                    }
                }
                // the inverse factor's loads fly during the exchange
                double Lk[15];
#pragma unroll
                for (int i = 0; i < 15; ++i) Lk[i] = recs[k - 1].L[i];
                if (!cluster_exchange<5>(b, m, part + static_cast<int64_t>(k) * row_len, G, g, par,
                                         C, Ls))
                    return false;
                par ^= 1;
                solve_packed(m, Lk, b, beta);
                bcU = cU;
                bcA = cA;
                have = true;
            } else {
                skipped += 1.0;
                have = false;
            }
            return true;
        };

        for (int k = k_top; k >= k_lo;) {
            if (!step(k, fa, fb)) return;
            if (--k < k_lo) break;
            if (!step(k, fb, fa)) return;
            --k;
        }
        if (have) {  // exercise at date k_lo (1 in the last window): its buffer was cur last
            if ((k_top - k_lo) % 2 == 0)
                decide(k_lo, fa);
            else
                decide(k_lo, fb);
        }
    }

    if (WIN && !A.win_last) {  // a window before the last: D waits in the workspace
        double* const dstate = A.cf + static_cast<int64_t>(s) * P + pbase + tid;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            if (i < nlive) dstate[i * kClusterThreads] = D[i];
        if (g == 0 && tid == 0) {
            double* o = A.out + static_cast<int64_t>(s) * 4;
            o[2] = (A.win_first ? 0.0 : o[2]) + skipped;
        }
        return;
    }

    // price and standard error over the whole scenario
    double s1[1] = {0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (i < nlive) s1[0] += D[i];
    if (!cluster_exchange<1>(s1, 1, part + static_cast<int64_t>(n) * row_len, G, g, par, C, Ls))
        return;
    par ^= 1;
    const double mean = s1[0] / static_cast<double>(P);
    double s2[1] = {0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (i < nlive) {
            const double d = D[i] - mean;
            s2[0] += d * d;
        }
    }
    if (!cluster_exchange<1>(s2, 1, part + static_cast<int64_t>(n + 1) * row_len, G, g, par, C,
                             Ls))
        return;
    if (g == 0 && tid == 0) {
        double* o = A.out + static_cast<int64_t>(s) * 4;
        o[0] = mean;
        o[1] = sqrt(s2[0] / static_cast<double>(P - 1) / static_cast<double>(P));
        o[2] = WIN && !A.win_first ? o[2] + skipped : skipped;
        o[3] = 0.0;
    }
}

__global__ void k_fill_u64(uint64_t* p, int64_t count, uint64_t value)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += stride)
        p[i] = value;
}

template <typename R, int Q, bool GLB>
hipError_t launch_sweep_t(const LsmcArgs& a, int S, hipStream_t st)
{
    const size_t lds = sizeof(double) * (((a.n + 2) & ~1) + (kSweepThreads / 64 + 1) * 5);
    hipLaunchKernelGGL((k_sweep<R, Q, GLB>), dim3(S), dim3(kSweepThreads), lds, st, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_sweep_r(int q, const LsmcArgs& a, int S, hipStream_t st)
{
    switch (q) {
    case 0: return launch_sweep_t<R, 1, true>(a, S, st);
    case 1: return launch_sweep_t<R, 1, false>(a, S, st);
    case 2: return launch_sweep_t<R, 2, false>(a, S, st);
    case 4: return launch_sweep_t<R, 4, false>(a, S, st);
    case 8: return launch_sweep_t<R, 8, false>(a, S, st);
    case 16: return launch_sweep_t<R, 16, false>(a, S, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int Q, bool WIN>
hipError_t launch_cluster_t(const LsmcArgs& a, const ClusterArgs& c, int S_launch, size_t lds,
                            hipStream_t st)
{
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&k_sweep_cluster<R, Q, WIN>),
            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_sweep_cluster<R, Q, WIN>), dim3(S_launch * c.G), dim3(kClusterThreads),
                       lds, st, a, c);
    return hipGetLastError();
}

template <typename R, int Q, bool WIN>
int cluster_capacity_t(size_t lds)
{
    const void* f = reinterpret_cast<const void*>(&k_sweep_cluster<R, Q, WIN>);
    if (lds > 65536 && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds)) != hipSuccess)
        return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kClusterThreads, lds) !=
        hipSuccess)
        return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

// The feature storage code of a feature type.
template <typename FT>
constexpr int feat_code()
{
    return std::is_same_v<FT, float>      ? kFeatF32
           : std::is_same_v<FT, double>   ? kFeatF64
           : std::is_same_v<FT, _Float16> ? kFeatF16
                                          : kFeatBF16;
}

// Calls f with the paths-per-thread count q as a compile-time constant, for
// the counts cluster_q_supported admits with features FT (others return bad
// and are never instantiated).
template <typename FT, typename Ret, typename Fn>
Ret with_q(int q, Ret bad, Fn&& f)
{
    switch (q) {
#define HS_Q(Q)                                                        \
    case Q:                                                            \
        if constexpr (cluster_q_supported(Q, feat_code<FT>()))         \
            return f(std::integral_constant<int, Q>{});                \
        else                                                           \
            return bad;
        HS_Q(1) HS_Q(2) HS_Q(3) HS_Q(4) HS_Q(5) HS_Q(6) HS_Q(7) HS_Q(8) HS_Q(10) HS_Q(12)
        HS_Q(16) HS_Q(18) HS_Q(20) HS_Q(22)
#undef HS_Q
    default: return bad;
    }
}

}  // namespace

size_t cluster_lds_bytes(int n, int G)
{
    (void)n;
    (void)G;
    return sizeof(double) * (2 * (kClusterThreads / 64) * kPartStride + 2 * kPartStride) + 16;
}

int cluster_capacity(int ft, int q, bool win, size_t lds)
{
    if (!cluster_q_supported(q, ft)) return 0;
    return with_feat(ft, 0, [&](auto tag) -> int {
        using FT = std::remove_pointer_t<decltype(tag)>;
        return with_q<FT>(q, 0, [&](auto qc) -> int {
            constexpr int Q = decltype(qc)::value;
            return win ? cluster_capacity_t<FT, Q, true>(lds) : cluster_capacity_t<FT, Q, false>(lds);
        });
    });
}

hipError_t launch_sweep_cluster(int ft, int q, const LsmcArgs& a, const ClusterArgs& c,
                                int S_launch, hipStream_t st)
{
    const size_t lds = cluster_lds_bytes(a.n, c.G);
    const bool win = a.k_lo != 1 || a.k_hi != a.n || !a.win_first || !a.win_last;
    if (win && (!a.american || !a.cf || a.k_lo < 1 || a.k_hi > a.n || a.f_date0 > a.k_lo))
        return hipErrorInvalidValue;
    if (!cluster_q_supported(q, ft)) return hipErrorInvalidValue;
    return with_feat(ft, hipErrorInvalidValue, [&](auto tag) -> hipError_t {
        using FT = std::remove_pointer_t<decltype(tag)>;
        return with_q<FT>(q, hipErrorInvalidValue, [&](auto qc) -> hipError_t {
            constexpr int Q = decltype(qc)::value;
            return win ? launch_cluster_t<FT, Q, true>(a, c, S_launch, lds, st)
                       : launch_cluster_t<FT, Q, false>(a, c, S_launch, lds, st);
        });
    });
}

hipError_t launch_fill_u64(uint64_t* p, int64_t count, uint64_t value, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill_u64, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, p, count,
                       value);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gram_r(const LsmcArgs& a, int S, hipStream_t st)
{
    const int top = std::min(a.k_hi, a.n - 1);
    hipLaunchKernelGGL((k_gram<R>), dim3(top - a.k_lo + 1, S), dim3(kGramThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gram(int ft, const LsmcArgs& a, int S, hipStream_t st)
{
    if (std::min(a.k_hi, a.n - 1) < a.k_lo) return hipSuccess;
    if (a.k_lo < 1 || a.k_hi > a.n || a.f_date0 < 1 || a.f_date0 > a.k_lo)
        return hipErrorInvalidValue;
    return with_feat(ft, hipErrorInvalidValue, [&](auto tag) {
        return launch_gram_r<std::remove_pointer_t<decltype(tag)>>(a, S, st);
    });
}

int sweep_q_for(int64_t P)
{
    static const int qs[] = {1, 2, 4, 8, 16};
    for (int q : qs)
        if (P <= static_cast<int64_t>(q) * kSweepThreads) return q;
    return 0;  // state in the workspace
}

hipError_t launch_sweep(int ft, int q, const LsmcArgs& a, int S, hipStream_t st)
{
    return with_feat(ft, hipErrorInvalidValue, [&](auto tag) {
        return launch_sweep_r<std::remove_pointer_t<decltype(tag)>>(q, a, S, st);
    });
}

}  // namespace hs
