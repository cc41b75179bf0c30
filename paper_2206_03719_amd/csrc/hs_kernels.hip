// hs_kernels.hip -- gfx950 kernels of the Heston / Longstaff-Schwartz Greek
// engine (arXiv 2206.03719, Sec. 2.2.1 and 4.1: Heston paths in log price,
// exponentiation, the max-over-assets path reduction, and the LS regression
// that decides early exercise).
//
//   k_paths     one pass over all steps of a block of 64 paths for a whole
//               Greek set: Philox4x32-10 normals shared by every scenario
//               (common random numbers), Cholesky correlation, full-truncation
//               Euler in log price, the per-date reduction (U = max_i S_i,
//               A = mean_i max(v_i, 0)), coalesced feature stores.  The waves
//               of a block split the random numbers and the base scenario's
//               assets, meet in LDS, then each advances only the assets that
//               its bumped scenarios change.
//   k_gram      per (scenario, date): regression-set means, the Gram matrix of
//               the centred basis over in-the-money paths, and its Cholesky
//               factor (all FP64).  Independent of the cash flows, so all
//               dates run at once.
//   k_sweep     per scenario: the backward sweep (right-hand side, solve,
//               exercise, cash-flow update) and the FP64 price and standard
//               error, with the cash-flow state in registers or in the
//               workspace.
// Reductions use fixed trees (wave butterfly, then waves in index order), so
// every result is a deterministic function of the request.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "hs_kernels.hpp"
#include "hs_layout.hpp"

namespace hs {
namespace {

// ---------------------------------------------------------------------------
// Random numbers.

struct Words {
    uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): per round, the 64-bit
// products of counter words 0 and 2 with two odd constants; their high halves
// are mixed with the other counter words and the key, their low halves move
// into place; the key advances by two Weyl constants between rounds.
__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        if (i) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
    }
    return {c0, c1, c2, c3};
}

// The odd multiples of 2^-24 in (0,1): exact in FP32 and FP64 alike.
__device__ __forceinline__ float unit_f32(uint32_t w)
{
    return static_cast<float>(2u * (w >> 9) + 1u) * 0x1p-24f;
}
__device__ __forceinline__ double unit_f64(uint32_t w)
{
    return static_cast<double>(2u * (w >> 9) + 1u) * 0x1p-24;
}

// Box-Muller: R = sqrt(-2 ln u1), (eps, eta) = R (cos 2 pi u2, sin 2 pi u2);
// sincospi takes 2 u2 exactly, so no rounding of the angle.
__device__ __forceinline__ void box_muller(uint32_t w1, uint32_t w2, float& e, float& h)
{
    const float R = sqrtf(-2.0f * logf(unit_f32(w1)));
    float s, c;
    sincospif(2.0f * unit_f32(w2), &s, &c);
    e = R * c;
    h = R * s;
}
__device__ __forceinline__ void box_muller(uint32_t w1, uint32_t w2, double& e, double& h)
{
    const double R = sqrt(-2.0 * log(unit_f64(w1)));
    double s, c;
    sincospi(2.0 * unit_f64(w2), &s, &c);
    e = R * c;
    h = R * s;
}

__device__ __forceinline__ float exp_r(float x) { return expf(x); }
__device__ __forceinline__ double exp_r(double x) { return exp(x); }
__device__ __forceinline__ float sqrt_r(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }

template <typename R>
struct alignas(2 * sizeof(R)) R2 {
    R u, a;
};

// Uniform (wave-wide) select of arr[i] as a chain of selects with constant
// indices (instantiated per index, so the array stays in registers).
template <int J, typename R, int NM>
__device__ __forceinline__ R pick_from(const R (&arr)[NM], int i, R acc)
{
    if constexpr (J >= NM) {
        return acc;
    } else {
        return pick_from<J + 1>(arr, i, i == J ? arr[J] : acc);
    }
}
template <typename R, int NM>
__device__ __forceinline__ R pick(const R (&arr)[NM], int i)
{
    return pick_from<1>(arr, i, arr[0]);
}

// ---------------------------------------------------------------------------
// Path kernel.
//
// Block = W waves x 64 lanes; lane l of every wave follows path
// 64 * blockIdx.x + l.  blockIdx.y selects a "block group": W groups (one per
// wave) of tasks.  LDS holds, double-buffered by step parity, the step's
// normals (eps, eta), the base scenario's correlated normals Z^S, exp(X) and
// max(v, 0), each [asset][lane].
template <typename R, int NMAX, int TMAX>
__global__ void __launch_bounds__(kLanes * kMaxWaves) k_paths(const PathArgs A)
{
    extern __shared__ unsigned char hs_smem[];
    constexpr int SLAB = NMAX * kLanes;  // one [asset][lane] array
    R* const lds = reinterpret_cast<R*>(hs_smem);

    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int W = A.W;
    const int N = A.N;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kLanes + lane;
    const bool live = p < A.P;

    const BaseP<R>* __restrict__ bp = static_cast<const BaseP<R>*>(A.base);
    const int gidx = static_cast<int>(blockIdx.y) * W + w;
    const GroupP grp = A.groups[gidx];
    const TaskP<R>* __restrict__ tk = static_cast<const TaskP<R>*>(A.tasks) + grp.task0;
    const int ntask = grp.ntask;

    const R dt = bp->dt;
    const R r = bp->r;
    const R invN = bp->invN;
    const R half = R(0.5);
    const uint32_t plo = static_cast<uint32_t>(p);
    const uint32_t phi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    R2<R>* __restrict__ feat = static_cast<R2<R>*>(A.feat);
    const int64_t P = A.P;
    const int nblk = (N + 1) / 2;

    // base assets owned by this wave: a = w + i W
    R Xo[kOwnPerWave], Vo[kOwnPerWave];
#pragma unroll
    for (int i = 0; i < kOwnPerWave; ++i) {
        const int a = w + i * W;
        Xo[i] = R(0);
        Vo[i] = (a < N) ? bp->a[a].v0 : R(0);
    }
    R tX[TMAX], tV[TMAX];
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
        tX[t] = R(0);
        tV[t] = (t < ntask) ? tk[t].v0 : R(0);
    }

    for (int k = 0; k < A.n; ++k) {
        R* const buf = lds + (k & 1) * 5 * SLAB;
        R* const s_eps = buf;
        R* const s_eta = buf + SLAB;
        R* const s_zs = buf + 2 * SLAB;
        R* const s_e = buf + 3 * SLAB;
        R* const s_vp = buf + 4 * SLAB;

        // 1) Philox blocks j = w, w + W, ...: pair 2j <- (w0, w1), 2j+1 <- (w2, w3)
        for (int j = w; j < nblk; j += W) {
            const Words q = philox10(plo, static_cast<uint32_t>(k), static_cast<uint32_t>(j), phi,
                                     A.key0, A.key1);
            R e, h;
            box_muller(q.x, q.y, e, h);
            s_eps[(2 * j) * kLanes + lane] = e;
            s_eta[(2 * j) * kLanes + lane] = h;
            if (2 * j + 1 < N) {
                box_muller(q.z, q.w, e, h);
                s_eps[(2 * j + 1) * kLanes + lane] = e;
                s_eta[(2 * j + 1) * kLanes + lane] = h;
            }
        }
        __syncthreads();

        // 2) the base scenario's owned assets: Z^S = L eps, full-truncation Euler
#pragma unroll
        for (int i = 0; i < kOwnPerWave; ++i) {
            const int a = w + i * W;
            if (a < N) {
                R z = R(0);
                for (int b = 0; b <= a; ++b) z += bp->L[a * kMaxAssets + b] * s_eps[b * kLanes + lane];
                const AssetP<R> q = bp->a[a];
                const R zv = q.rho * z + q.rhobar * s_eta[a * kLanes + lane];
                const R vp = Vo[i] > R(0) ? Vo[i] : R(0);
                const R sq = sqrt_r(vp * dt);
                Xo[i] = Xo[i] + (r - half * vp) * dt + sq * z;
                Vo[i] = Vo[i] + q.kappa * (q.theta - vp) * dt + q.xi * sq * zv;
                s_zs[a * kLanes + lane] = z;
                s_e[a * kLanes + lane] = exp_r(Xo[i]);
                s_vp[a * kLanes + lane] = Vo[i] > R(0) ? Vo[i] : R(0);
            }
        }
        __syncthreads();

        // 3) features
        const bool store = A.store_all || k == A.n - 1;
        const int64_t off = (A.store_all ? static_cast<int64_t>(k) * P : 0) + p;
        R eps[NMAX], E[NMAX], Sb[NMAX], vpb[NMAX], pm[NMAX], sm[NMAX], ps[NMAX];
#pragma unroll
        for (int a = 0; a < NMAX; ++a) {
            if (a < N) {
                eps[a] = s_eps[a * kLanes + lane];
                E[a] = s_e[a * kLanes + lane];
                Sb[a] = bp->a[a].S0 * E[a];
                vpb[a] = s_vp[a * kLanes + lane];
            } else {
                eps[a] = R(0);
                E[a] = R(0);
                Sb[a] = R(0);
                vpb[a] = R(0);
            }
        }
        // prefix max / prefix sum / suffix max of the base scenario (entries
        // past N are 0, and every S > 0, so the padding never wins a max)
        R bsum = R(0);
        pm[0] = Sb[0];
#pragma unroll
        for (int a = 1; a < NMAX; ++a) pm[a] = Sb[a] > pm[a - 1] ? Sb[a] : pm[a - 1];
#pragma unroll
        for (int a = 0; a < NMAX; ++a) {
            if (a < N) bsum = bsum + vpb[a];
            ps[a] = bsum;
        }
        sm[NMAX - 1] = Sb[NMAX - 1];
#pragma unroll
        for (int a = NMAX - 2; a >= 0; --a) sm[a] = Sb[a] > sm[a + 1] ? Sb[a] : sm[a + 1];
        const R bA = bsum * invN;

        if (store && live) {
            if (grp.base_scen >= 0) {
                R2<R> f;
                f.u = sm[0];
                f.a = bA;
                feat[grp.base_scen * A.plane + off] = f;
            }
            if (grp.spot_up0 >= 0) {
#pragma unroll
                for (int a = 0; a < NMAX; ++a) {
                    if (a < N) {
                        const R lo = a > 0 ? pm[a > 0 ? a - 1 : 0] : R(0);
                        const R hi = a + 1 < NMAX ? sm[a + 1 < NMAX ? a + 1 : a] : R(0);
                        const R ex = lo > hi ? lo : hi;
                        const R su = bp->S0_up[a] * E[a];
                        const R sd = bp->S0_dn[a] * E[a];
                        R2<R> f;
                        f.a = bA;
                        f.u = su > ex ? su : ex;
                        feat[(grp.spot_up0 + a) * A.plane + off] = f;
                        f.u = sd > ex ? sd : ex;
                        feat[(grp.spot_dn0 + a) * A.plane + off] = f;
                    }
                }
            }
        }

        // 4) this wave's tasks (assets of bumped scenarios that leave the base path)
        R runM = R(0), runS = R(0);
#pragma unroll
        for (int t = 0; t < TMAX; ++t) {
            if (t < ntask) {
                const TaskP<R>& T = tk[t];
                const int a = T.asset;
                R z;
                if (T.own_row) {
                    z = R(0);
#pragma unroll
                    for (int b = 0; b < NMAX; ++b) z += T.L[b] * eps[b];
                } else {
                    z = s_zs[a * kLanes + lane];
                }
                const R zv = T.rho * z + T.rhobar * s_eta[a * kLanes + lane];
                const R vp = tV[t] > R(0) ? tV[t] : R(0);
                const R sq = sqrt_r(vp * T.dt);
                tX[t] = tX[t] + (T.r - half * vp) * T.dt + sq * z;
                tV[t] = tV[t] + T.kappa * (T.theta - vp) * T.dt + T.xi * sq * zv;
                const R S = T.S0 * exp_r(tX[t]);
                const R vpt = tV[t] > R(0) ? tV[t] : R(0);
                if (T.first) {
                    runM = T.lo > 0 ? pick(pm, T.lo - 1) : R(0);
                    runS = T.lo > 0 ? pick(ps, T.lo - 1) : R(0);
                }
                runM = S > runM ? S : runM;
                runS = runS + vpt;
                if (T.last) {
                    if (T.hi < N) {
                        const R tail = pick(sm, T.hi);
                        runM = tail > runM ? tail : runM;
                        runS = runS + (bsum - pick(ps, T.hi - 1));
                    }
                    if (store && live) {
                        R2<R> f;
                        f.u = runM;
                        f.a = runS * invN;
                        feat[T.scen * A.plane + off] = f;
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 block reductions with a fixed tree: xor butterfly inside each wave
// (every lane ends with the same bits), then the waves' sums in index order.

template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* scratch /* [nwaves][K] */,
                                          int nwaves)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int i = 0; i < K; ++i) v[i] += __shfl_xor(v[i], off, 64);
    }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < K; ++i) scratch[wid * K + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < K; ++i) {
        double s = scratch[i];
        for (int q = 1; q < nwaves; ++q) s += scratch[q * K + i];
        v[i] = s;
    }
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

// ---------------------------------------------------------------------------
// Gram kernel: block (date k = blockIdx.x + 1, scenario blockIdx.y).

template <typename R>
__global__ void __launch_bounds__(kGramThreads) k_gram(const LsmcArgs A)
{
    __shared__ double red[(kGramThreads / 64) * 15];
    const int s = blockIdx.y;
    const int k = blockIdx.x + 1;
    const R2<R>* __restrict__ F =
        static_cast<const R2<R>*>(A.feat) + s * A.plane + static_cast<int64_t>(k - 1) * A.P;
    const int nw = kGramThreads / 64;

    double c3[3] = {0.0, 0.0, 0.0};
    for (int64_t p = threadIdx.x; p < A.P; p += kGramThreads) {
        const R2<R> f = F[p];
        const double U = static_cast<double>(f.u);
        if (payoff(A.cp, A.K, U) > 0.0) {
            c3[0] += 1.0;
            c3[1] += U;
            c3[2] += static_cast<double>(f.a);
        }
    }
    block_sum<3>(c3, red, nw);
    RegRec* rr = A.reg + static_cast<int64_t>(s) * A.n + (k - 1);
    const double cnt = c3[0];
    if (cnt < static_cast<double>(A.m)) {
        if (threadIdx.x == 0) {
            rr->ok = 0.0;
            rr->cnt = cnt;
        }
        return;
    }
    const double cU = c3[1] / cnt;
    const double cA = c3[2] / cnt;
    const int m = A.m;
    double g[15];
#pragma unroll
    for (int i = 0; i < 15; ++i) g[i] = 0.0;
    for (int64_t p = threadIdx.x; p < A.P; p += kGramThreads) {
        const R2<R> f = F[p];
        const double U = static_cast<double>(f.u);
        if (payoff(A.cp, A.K, U) > 0.0) {
            double phi[5];
            basis(m, U, static_cast<double>(f.a), cU, cA, A.inv_K, A.inv_tbar, phi);
            int idx = 0;
#pragma unroll
            for (int i = 0; i < 5; ++i)
#pragma unroll
                for (int j = 0; j <= i; ++j, ++idx)
                    if (i < m) g[idx] += phi[i] * phi[j];
        }
    }
    block_sum<15>(g, red, nw);
    if (threadIdx.x == 0) {
        // packed row-major lower Cholesky; a pivot at or below 1e-12 of its
        // diagonal entry marks the date as skipped
        double L[15];
        bool ok = true;
        for (int i = 0; i < m && ok; ++i) {
            for (int j = 0; j <= i; ++j) {
                double acc = g[i * (i + 1) / 2 + j];
                for (int q = 0; q < j; ++q) acc -= L[i * (i + 1) / 2 + q] * L[j * (j + 1) / 2 + q];
                if (i == j) {
                    if (!(acc > 1e-12 * g[i * (i + 1) / 2 + i])) {
                        ok = false;
                        break;
                    }
                    L[i * (i + 1) / 2 + i] = sqrt(acc);
                } else {
                    L[i * (i + 1) / 2 + j] = acc / L[j * (j + 1) / 2 + j];
                }
            }
        }
        for (int i = 0; i < 15; ++i) rr->L[i] = ok ? L[i] : 0.0;
        rr->cU = cU;
        rr->cA = cA;
        rr->ok = ok ? 1.0 : 0.0;
        rr->cnt = cnt;
    }
}

// ---------------------------------------------------------------------------
// Backward sweep + price: one block of 1024 threads per scenario.  Thread t
// handles paths t + 1024 i.  With GLB the cash flow and exercise date of each
// path live in the workspace; otherwise in registers (Q paths per thread).

// L L^T beta = b with L packed lower row-major (m = 3 or 5); the entries of
// beta past m are 0.
__device__ __forceinline__ void solve_packed(int m, const double (&L)[15], const double (&b)[5],
                                             double (&beta)[5])
{
    double y[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double acc = b[i];
#pragma unroll
        for (int q = 0; q < i; ++q) acc -= L[i * (i + 1) / 2 + q] * y[q];
        y[i] = i < m ? acc / L[i * (i + 1) / 2 + i] : 0.0;
    }
#pragma unroll
    for (int i = 4; i >= 0; --i) {
        double acc = y[i];
#pragma unroll
        for (int q = i + 1; q < 5; ++q) acc -= L[q * (q + 1) / 2 + i] * beta[q];
        beta[i] = i < m ? acc / L[i * (i + 1) / 2 + i] : 0.0;
    }
}

template <typename R, int Q, bool GLB>
__global__ void __launch_bounds__(kSweepThreads) k_sweep(const LsmcArgs A)
{
    extern __shared__ unsigned char hs_smem[];
    double* const sdisc = reinterpret_cast<double*>(hs_smem);         // [n+1]
    double* const red = sdisc + ((A.n + 1 + 1) & ~1);                 // [16][5]
    constexpr int NW = kSweepThreads / 64;
    const int s = blockIdx.x;
    const int n = A.n;
    const int64_t P = A.P;
    const R2<R>* __restrict__ F = static_cast<const R2<R>*>(A.feat) + s * A.plane;
    for (int j = threadIdx.x; j <= n; j += kSweepThreads) sdisc[j] = A.disc[static_cast<int64_t>(s) * (n + 1) + j];
    __syncthreads();

    double* const gcf = GLB ? A.cf + static_cast<int64_t>(s) * P : nullptr;
    int32_t* const gtau = GLB ? A.tau + static_cast<int64_t>(s) * P : nullptr;
    const int64_t last = A.american ? static_cast<int64_t>(n - 1) * P : 0;

    double cf[GLB ? 1 : Q];
    int tau[GLB ? 1 : Q];
    if (!GLB) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t p = threadIdx.x + static_cast<int64_t>(i) * kSweepThreads;
            cf[i] = p < P ? payoff(A.cp, A.K, static_cast<double>(F[last + p].u)) : 0.0;
            tau[i] = n;
        }
    } else {
        for (int64_t p = threadIdx.x; p < P; p += kSweepThreads) {
            gcf[p] = payoff(A.cp, A.K, static_cast<double>(F[last + p].u));
            gtau[p] = n;
        }
    }

    double skipped = 0.0;
    const int m = A.m;
    if (A.american) {
        for (int k = n - 1; k >= 1; --k) {
            const RegRec* rr = A.reg + static_cast<int64_t>(s) * n + (k - 1);
            if (rr->ok == 0.0) {
                skipped += 1.0;
                continue;
            }
            const double cU = rr->cU, cA = rr->cA;
            const R2<R>* __restrict__ Fk = F + static_cast<int64_t>(k - 1) * P;
            double b[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (!GLB) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const int64_t p = threadIdx.x + static_cast<int64_t>(i) * kSweepThreads;
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
                    const int64_t p = threadIdx.x + static_cast<int64_t>(i) * kSweepThreads;
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

    // price: mean of CF exp(-r tau dt), then the sample standard deviation
    double s1[1] = {0.0};
    if (!GLB) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t p = threadIdx.x + static_cast<int64_t>(i) * kSweepThreads;
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
            const int64_t p = threadIdx.x + static_cast<int64_t>(i) * kSweepThreads;
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
        double* o = A.out + static_cast<int64_t>(s) * 4;
        o[0] = mean;
        o[1] = sqrt(s2[0] / static_cast<double>(P - 1) / static_cast<double>(P));
        o[2] = skipped;
        o[3] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Diagnostics.

__global__ void k_philox_words(uint32_t k0, uint32_t k1, int64_t P, int n, int nb, uint32_t* out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t total = P * n * nb;
    if (i >= total) return;
    const int j = static_cast<int>(i % nb);
    const int k = static_cast<int>((i / nb) % n);
    const int64_t p = i / (static_cast<int64_t>(nb) * n);
    const Words q = philox10(static_cast<uint32_t>(p), static_cast<uint32_t>(k),
                             static_cast<uint32_t>(j),
                             static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32), k0, k1);
    out[i * 4 + 0] = q.x;
    out[i * 4 + 1] = q.y;
    out[i * 4 + 2] = q.z;
    out[i * 4 + 3] = q.w;
}

template <typename R>
__global__ void k_normals(uint32_t k0, uint32_t k1, int N, int64_t P, int n, R* eps, R* eta)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int nb = (N + 1) / 2;
    const int64_t total = P * n * nb;
    if (i >= total) return;
    const int j = static_cast<int>(i % nb);
    const int k = static_cast<int>((i / nb) % n);
    const int64_t p = i / (static_cast<int64_t>(nb) * n);
    const Words q = philox10(static_cast<uint32_t>(p), static_cast<uint32_t>(k),
                             static_cast<uint32_t>(j),
                             static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32), k0, k1);
    const int64_t row = (p * n + k) * N;
    R e, h;
    box_muller(q.x, q.y, e, h);
    eps[row + 2 * j] = e;
    eta[row + 2 * j] = h;
    if (2 * j + 1 < N) {
        box_muller(q.z, q.w, e, h);
        eps[row + 2 * j + 1] = e;
        eta[row + 2 * j + 1] = h;
    }
}

template <typename R, int NMAX, int TMAX>
hipError_t launch_paths_t(const PathArgs& a, int nchunks, int nbg, hipStream_t st)
{
    const size_t lds = 2u * 5u * NMAX * kLanes * sizeof(R);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_paths<R, NMAX, TMAX>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    dim3 grid(nchunks, nbg), block(kLanes, a.W);
    hipLaunchKernelGGL((k_paths<R, NMAX, TMAX>), grid, block, lds, st, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_paths_r(int nmax, const PathArgs& a, int nchunks, int nbg, hipStream_t st)
{
    constexpr bool F = sizeof(R) == 4;
    switch (nmax) {
    case 1: return launch_paths_t<R, 1, F ? 32 : 16>(a, nchunks, nbg, st);
    case 2: return launch_paths_t<R, 2, F ? 32 : 16>(a, nchunks, nbg, st);
    case 3: return launch_paths_t<R, 3, F ? 32 : 16>(a, nchunks, nbg, st);
    case 4: return launch_paths_t<R, 4, F ? 32 : 16>(a, nchunks, nbg, st);
    case 5: return launch_paths_t<R, 5, F ? 32 : 16>(a, nchunks, nbg, st);
    case 6: return launch_paths_t<R, 6, F ? 32 : 16>(a, nchunks, nbg, st);
    case 8: return launch_paths_t<R, 8, F ? 32 : 16>(a, nchunks, nbg, st);
    case 10: return launch_paths_t<R, 10, F ? 24 : 16>(a, nchunks, nbg, st);
    case 12: return launch_paths_t<R, 12, F ? 24 : 16>(a, nchunks, nbg, st);
    case 16: return launch_paths_t<R, 16, F ? 20 : 16>(a, nchunks, nbg, st);
    case 20: return launch_paths_t<R, 20, 20>(a, nchunks, nbg, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int Q, bool GLB>
hipError_t launch_sweep_t(const LsmcArgs& a, int S, hipStream_t st)
{
    const size_t lds = sizeof(double) * (((a.n + 2) & ~1) + (kSweepThreads / 64) * 5);
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

}  // namespace

int paths_tmax(bool fp32, int nmax)
{
    if (fp32) return nmax <= 8 ? 32 : nmax <= 12 ? 24 : 20;
    return nmax <= 16 ? 16 : 20;
}

int paths_nmax_bucket(int N)
{
    static const int b[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20};
    for (int v : b)
        if (N <= v) return v;
    return -1;
}

size_t paths_lds_bytes(bool fp32, int nmax)
{
    return 2u * 5u * static_cast<size_t>(nmax) * kLanes * (fp32 ? 4u : 8u);
}

hipError_t launch_paths(bool fp32, int nmax, const PathArgs& a, int nchunks, int nbg,
                        hipStream_t st)
{
    return fp32 ? launch_paths_r<float>(nmax, a, nchunks, nbg, st)
                : launch_paths_r<double>(nmax, a, nchunks, nbg, st);
}

hipError_t launch_gram(bool fp32, const LsmcArgs& a, int S, hipStream_t st)
{
    if (a.n < 2) return hipSuccess;
    dim3 grid(a.n - 1, S), block(kGramThreads);
    if (fp32)
        hipLaunchKernelGGL((k_gram<float>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_gram<double>), grid, block, 0, st, a);
    return hipGetLastError();
}

int sweep_q_for(int64_t P)
{
    static const int qs[] = {1, 2, 4, 8, 16};
    for (int q : qs)
        if (P <= static_cast<int64_t>(q) * kSweepThreads) return q;
    return 0;  // state in the workspace
}

hipError_t launch_sweep(bool fp32, int q, const LsmcArgs& a, int S, hipStream_t st)
{
    return fp32 ? launch_sweep_r<float>(q, a, S, st) : launch_sweep_r<double>(q, a, S, st);
}

hipError_t launch_philox_words(uint64_t seed, int64_t P, int n, int nb, uint32_t* out,
                               hipStream_t st)
{
    const int64_t total = P * n * nb;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_philox_words, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                       static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), P, n, nb,
                       out);
    return hipGetLastError();
}

hipError_t launch_normals(bool fp32, uint64_t seed, int N, int64_t P, int n, void* eps, void* eta,
                          hipStream_t st)
{
    const int64_t total = P * n * ((N + 1) / 2);
    const int64_t blocks = (total + 255) / 256;
    const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
    if (fp32)
        hipLaunchKernelGGL((k_normals<float>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                           st, k0, k1, N, P, n, static_cast<float*>(eps), static_cast<float*>(eta));
    else
        hipLaunchKernelGGL((k_normals<double>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                           st, k0, k1, N, P, n, static_cast<double*>(eps),
                           static_cast<double*>(eta));
    return hipGetLastError();
}

}  // namespace hs
