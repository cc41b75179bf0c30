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

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "../../include/hs_api.h"
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

// Box-Muller: R = sqrt(-2 ln u1), (eps, eta) = R (cos 2 pi u2, sin 2 pi u2).
// FP32 uses the hardware transcendentals: v_log_f32 is log2 (so -2 ln u =
// -2 ln 2 log2 u), and v_sin_f32 / v_cos_f32 take their argument in turns, so
// u2 goes in exactly with no 2 pi rounding.  Each is good to a few ulp, far
// inside the FP32 path's error budget, at a fraction of the library calls'
// instruction count.  FP64 keeps the correctly rounded library functions
// (sincospi takes 2 u2 exactly).
__device__ __forceinline__ void box_muller(uint32_t w1, uint32_t w2, float& e, float& h)
{
    const float R = __builtin_amdgcn_sqrtf(-1.38629436112f * __builtin_amdgcn_logf(unit_f32(w1)));
    const float u2 = unit_f32(w2);
    e = R * __builtin_amdgcn_cosf(u2);
    h = R * __builtin_amdgcn_sinf(u2);
}
__device__ __forceinline__ void box_muller(uint32_t w1, uint32_t w2, double& e, double& h)
{
    const double R = sqrt(-2.0 * log(unit_f64(w1)));
    double s, c;
    sincospi(2.0 * unit_f64(w2), &s, &c);
    e = R * c;
    h = R * s;
}

// FP32: e^x = 2^(x log2 e) on v_exp_f32, and v_sqrt_f32 (arguments here are
// >= 0 and far from overflow); FP64: the library functions.
// Box-Muller with eta in FP64 and eps in R (the QE variance path's normal).
__device__ __forceinline__ void box_muller_mixed(uint32_t w1, uint32_t w2, float& e, double& h)
{
    const double R = sqrt(-2.0 * log(unit_f64(w1)));
    double sn, cs;
    sincospi(2.0 * unit_f64(w2), &sn, &cs);
    e = static_cast<float>(R * cs);
    h = R * sn;
}
__device__ __forceinline__ void box_muller_mixed(uint32_t w1, uint32_t w2, double& e, double& h)
{
    box_muller(w1, w2, e, h);
}

__device__ __forceinline__ float exp_r(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504089f); }
__device__ __forceinline__ double exp_r(double x) { return exp(x); }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }

// FP32: hardware log2 and reciprocal; FP64: the library / IEEE division.
__device__ __forceinline__ float log_r(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945f; }
__device__ __forceinline__ double log_r(double x) { return log(x); }
__device__ __forceinline__ float div_r(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double div_r(double a, double b) { return a / b; }
// standard normal distribution function
__device__ __forceinline__ float ncdf_r(float z) { return 0.5f * erfcf(-z * 0.707106781186548f); }
__device__ __forceinline__ double ncdf_r(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

template <typename R>
struct alignas(2 * sizeof(R)) R2 {
    R u, a;
};

// Read-only parameter tables are read through the constant address space:
// their loads are uniform across a wave and become scalar (SMEM) loads even
// though the kernels store to other global buffers.
template <typename T>
using cptr = const T __attribute__((address_space(4)))*;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const void* p)
{
    return reinterpret_cast<cptr<T>>(reinterpret_cast<uintptr_t>(p));
}

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
// Andersen's quadratic-exponential step of one asset from (X, v) with the
// correlated normal zx and the independent normal zv (constants c: QeP).  The
// variance path -- its normal, its state and the whole step, including the
// branch test psi <= 1.5 -- runs in FP64 in both path precisions: the two
// branches map the same normal to different variances, so an FP32 variance
// state that strays by rounding across psi = 1.5 would send the path off the
// FP64 one for good.  The log price's drift K0 + K1 v + K2 v' is FP64 too
// (K1 and K2 are near -rho/xi and rho/xi, so the sum cancels); its diffusion
// term and the log price itself run in R.
template <typename R, typename CP>
__device__ __forceinline__ void qe_step(CP c, R zx, double zv, R& X, double& v)
{
    const double m = c->mth + v * c->E;
    const double s2 = v * c->c1 + c->c2;
    double vn;
    if (!(s2 > 0.0)) {
        vn = m;
    } else {
        const double psi = s2 / (m * m);
        if (psi <= 1.5) {
            const double t = 2.0 / psi;
            const double b2 = t - 1.0 + sqrt(t) * sqrt(t - 1.0);
            const double a = m / (1.0 + b2);
            const double b = sqrt(b2);
            vn = a * (b + zv) * (b + zv);
        } else {
            const double pm = (psi - 1.0) / (psi + 1.0);
            const double beta = (1.0 - pm) / m;
            const double u = ncdf_r(zv);
            vn = u <= pm ? 0.0 : log((1.0 - pm) / (1.0 - u)) / beta;
        }
    }
    if constexpr (sizeof(R) == 8) {
        X = X + c->K0 + c->K1 * v + c->K2 * vn + sqrt(c->K3 * v + c->K4 * vn) * zx;
    } else {
        // drift in FP64 (K1 v + K2 v' nearly cancels), diffusion in R
        const double drift = c->K0 + c->K1 * v + c->K2 * vn;
        X = X + static_cast<R>(drift) +
            sqrt_r(static_cast<R>(c->K3 * v + c->K4 * vn)) * zx;
    }
    v = vn;
}

// ---------------------------------------------------------------------------
// Path kernel.
//
// Block = W waves x 64 lanes; lane l of every wave follows path
// 64 * blockIdx.x + l.  blockIdx.y selects a "block group": W groups (one per
// wave) of tasks.  LDS holds, double-buffered by step parity, the step's
// normals (eps, eta), the base scenario's correlated normals Z^S, exp(X) and
// max(v, 0), each [asset][lane]; under QE the variance normal eta and the
// variance state are FP64 (VT) in both path precisions.
template <typename R, int NMAX, int TMAX, int SCHEME, typename FT, bool CK>
__global__ void __launch_bounds__(kLanes * paths_max_waves(sizeof(R) == 4, NMAX))
    k_paths(const PathArgs A)
{
    using VT = std::conditional_t<SCHEME == HS_SCHEME_QE, double, R>;
    extern __shared__ unsigned char hs_smem[];
    constexpr int SLAB = NMAX * kLanes;  // one [asset][lane] array
    R* const lds = reinterpret_cast<R*>(hs_smem);
    VT* const lds_eta = reinterpret_cast<VT*>(hs_smem + 2 * 5 * SLAB * sizeof(R));

    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int W = A.W;
    const int N = A.N;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kLanes + lane;
    const bool live = p < A.P;

    const cptr<BaseP<R>> bp = as_const<BaseP<R>>(A.base);
    const int gidx = static_cast<int>(blockIdx.y) * W + w;
    const cptr<GroupP> gp = as_const<GroupP>(A.groups) + gidx;
    const int g_task0 = gp->task0, ntask = gp->ntask, g_base = gp->base_scen,
              g_up0 = gp->spot_up0, g_dn0 = gp->spot_dn0;
    const cptr<TaskP<R>> tk = as_const<TaskP<R>>(A.tasks) + g_task0;

    const R dt = bp->dt;
    const R r = bp->r;
    const R invN = bp->invN;
    const R half = R(0.5);
    const uint32_t plo = static_cast<uint32_t>(p);
    const uint32_t phi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    R2<FT>* __restrict__ feat = static_cast<R2<FT>*>(A.feat);
    const int64_t P = A.P;
    const int nblk = (N + 1) / 2;

    // base assets owned by this wave: a = w + i W
    R Xo[kOwnPerWave];
    VT Vo[kOwnPerWave];
#pragma unroll
    for (int i = 0; i < kOwnPerWave; ++i) {
        const int a = w + i * W;
        Xo[i] = R(0);
        Vo[i] = (a < N) ? static_cast<VT>(SCHEME == HS_SCHEME_QE ? bp->a[a].qe.v0 : bp->a[a].v0)
                        : VT(0);
    }
    R tX[TMAX];
    VT tV[TMAX];
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
        tX[t] = R(0);
        tV[t] = (t < ntask) ? static_cast<VT>(SCHEME == HS_SCHEME_QE ? tk[t].qe.v0 : tk[t].v0)
                            : VT(0);
    }

    // checkpoint-recompute: the state at date n - (i + 2) c, checkpoint i,
    // lives at [(i slots + slot) P + p]; the base assets are kept by block
    // group 0 and read by every group, a task by the wave that owns it (one
    // lane pointer per array and wave-uniform slot offsets; compiled in only
    // for windowed passes, CK)
    if constexpr (CK) if (A.k_begin > 0 && live) {
        const int64_t row0 =
            static_cast<int64_t>((A.n - A.k_begin) / A.ck_every - 2) * A.ck_slots;
        const R* const bx = static_cast<const R*>(A.ckx) + row0 * P + p;
        const VT* const bv = static_cast<const VT*>(A.ckv) + row0 * P + p;
#pragma unroll
        for (int i = 0; i < kOwnPerWave; ++i) {
            const int a = w + i * W;
            if (a < N) {
                Xo[i] = bx[static_cast<int64_t>(a) * P];
                Vo[i] = bv[static_cast<int64_t>(a) * P];
            }
        }
        const int64_t t0 = static_cast<int64_t>(N + g_task0) * P;
#pragma unroll
        for (int t = 0; t < TMAX; ++t) {
            if (t < ntask) {
                tX[t] = bx[t0 + static_cast<int64_t>(t) * P];
                tV[t] = bv[t0 + static_cast<int64_t>(t) * P];
            }
        }
    }

    for (int k = CK ? A.k_begin : 0; k < (CK ? A.k_end : A.n); ++k) {
        R* const buf = lds + (k & 1) * 5 * SLAB;
        R* const s_eps = buf;
        VT* const s_eta = SCHEME == HS_SCHEME_QE ? lds_eta + (k & 1) * SLAB
                                                 : reinterpret_cast<VT*>(buf + SLAB);
        R* const s_zs = buf + 2 * SLAB;
        R* const s_e = buf + 3 * SLAB;
        R* const s_vp = buf + 4 * SLAB;

        // 1) Philox blocks j = w, w + W, ...: pair 2j <- (w0, w1), 2j+1 <- (w2, w3)
        for (int j = w; j < nblk; j += W) {
            const Words q = philox10(plo, static_cast<uint32_t>(k), static_cast<uint32_t>(j), phi,
                                     A.key0, A.key1);
            R e;
            VT h;
            if constexpr (SCHEME == HS_SCHEME_QE)
                box_muller_mixed(q.x, q.y, e, h);
            else
                box_muller(q.x, q.y, e, h);
            s_eps[(2 * j) * kLanes + lane] = e;
            s_eta[(2 * j) * kLanes + lane] = h;
            if (2 * j + 1 < N) {
                if constexpr (SCHEME == HS_SCHEME_QE)
                    box_muller_mixed(q.z, q.w, e, h);
                else
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
                const cptr<AssetP<R>> q = bp->a + a;
                if constexpr (SCHEME == HS_SCHEME_QE) {
                    qe_step(&q->qe, z, s_eta[a * kLanes + lane], Xo[i], Vo[i]);
                } else {
                    const R zv = q->rho * z + q->rhobar * s_eta[a * kLanes + lane];
                    const R vp = Vo[i] > R(0) ? Vo[i] : R(0);
                    const R sq = sqrt_r(vp * dt);
                    Xo[i] = Xo[i] + (r - half * vp) * dt + sq * z;
                    Vo[i] = Vo[i] + q->kappa * (q->theta - vp) * dt + q->xi * sq * zv;
                }
                s_zs[a * kLanes + lane] = z;
                s_e[a * kLanes + lane] = exp_r(Xo[i]);
                s_vp[a * kLanes + lane] = static_cast<R>(Vo[i] > VT(0) ? Vo[i] : VT(0));
            }
        }
        __syncthreads();

        // 3) features
        // (checkpoint runs store the dates from k_feat0 + 1 on, at index 0)
        const bool store = CK ? (A.store_all ? k >= A.k_feat0 : k == A.n - 1)
                              : (A.store_all || k == A.n - 1);
        const int64_t off =
            (A.store_all ? static_cast<int64_t>(CK ? k - A.k_feat0 : k) * P : 0) + p;
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
            if (g_base >= 0) {
                R2<FT> f;
                f.u = static_cast<FT>(sm[0]);
                f.a = static_cast<FT>(bA);
                feat[g_base * A.plane + off] = f;
            }
            if (g_up0 >= 0) {
#pragma unroll
                for (int a = 0; a < NMAX; ++a) {
                    if (a < N) {
                        const R lo = a > 0 ? pm[a > 0 ? a - 1 : 0] : R(0);
                        const R hi = a + 1 < NMAX ? sm[a + 1 < NMAX ? a + 1 : a] : R(0);
                        const R ex = lo > hi ? lo : hi;
                        const R su = bp->S0_up[a] * E[a];
                        const R sd = bp->S0_dn[a] * E[a];
                        R2<FT> f;
                        f.a = static_cast<FT>(bA);
                        f.u = static_cast<FT>(su > ex ? su : ex);
                        feat[(g_up0 + a) * A.plane + off] = f;
                        f.u = static_cast<FT>(sd > ex ? sd : ex);
                        feat[(g_dn0 + a) * A.plane + off] = f;
                    }
                }
            }
        }

        // 4) this wave's tasks (assets of bumped scenarios that leave the base path)
        R runM = R(0), runS = R(0);
#pragma unroll
        for (int t = 0; t < TMAX; ++t) {
            if (t < ntask) {
                const cptr<TaskP<R>> T = tk + t;
                const int a = T->asset;
                R z;
                if (T->own_row) {
                    z = R(0);
#pragma unroll
                    for (int b = 0; b < NMAX; ++b) z += T->L[b] * eps[b];
                } else {
                    z = s_zs[a * kLanes + lane];
                }
                if constexpr (SCHEME == HS_SCHEME_QE) {
                    qe_step(&T->qe, z, s_eta[a * kLanes + lane], tX[t], tV[t]);
                } else {
                    const R zv = T->rho * z + T->rhobar * s_eta[a * kLanes + lane];
                    const R vp = tV[t] > R(0) ? tV[t] : R(0);
                    const R sq = sqrt_r(vp * T->dt);
                    tX[t] = tX[t] + (T->r - half * vp) * T->dt + sq * z;
                    tV[t] = tV[t] + T->kappa * (T->theta - vp) * T->dt + T->xi * sq * zv;
                }
                const R S = T->S0 * exp_r(tX[t]);
                const R vpt = static_cast<R>(tV[t] > VT(0) ? tV[t] : VT(0));
                if (T->first) {
                    runM = T->lo > 0 ? pick(pm, T->lo - 1) : R(0);
                    runS = T->lo > 0 ? pick(ps, T->lo - 1) : R(0);
                }
                runM = S > runM ? S : runM;
                runS = runS + vpt;
                if (T->last) {
                    if (T->hi < N) {
                        const R tail = pick(sm, T->hi);
                        runM = tail > runM ? tail : runM;
                        runS = runS + (bsum - pick(ps, T->hi - 1));
                    }
                    if (store && live) {
                        R2<FT> f;
                        f.u = static_cast<FT>(runM);
                        f.a = static_cast<FT>(runS * invN);
                        feat[T->scen * A.plane + off] = f;
                    }
                }
            }
        }

        // 5) the state at a checkpoint date (where a window other than the
        //    last two dates' windows starts over)
        if constexpr (CK) if (A.ck_store && (A.n - k - 1) % A.ck_every == 0 &&
                              (A.n - k - 1) / A.ck_every >= 2 && live) {
            const int64_t row0 =
                static_cast<int64_t>((A.n - k - 1) / A.ck_every - 2) * A.ck_slots;
            R* const bx = static_cast<R*>(A.ckx) + row0 * P + p;
            VT* const bv = static_cast<VT*>(A.ckv) + row0 * P + p;
            if (blockIdx.y == 0) {
#pragma unroll
                for (int i = 0; i < kOwnPerWave; ++i) {
                    const int a = w + i * W;
                    if (a < N) {
                        bx[static_cast<int64_t>(a) * P] = Xo[i];
                        bv[static_cast<int64_t>(a) * P] = Vo[i];
                    }
                }
            }
            const int64_t t0 = static_cast<int64_t>(N + g_task0) * P;
#pragma unroll
            for (int t = 0; t < TMAX; ++t) {
                if (t < ntask) {
                    bx[t0 + static_cast<int64_t>(t) * P] = tX[t];
                    bv[t0 + static_cast<int64_t>(t) * P] = tV[t];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Base-scenario path kernel: Heston paths of one model and the per-date path
// reduction (the paper's measured stage, Sec. 2.2.1 and 4.1), for up to
// kMaxPathAssets assets.
//
// Block = W waves x 64 lanes; lane l of every wave follows path
// 64 * blockIdx.x + l.  Wave w owns the Philox blocks own_block(w, i, W)
// (i < BPW) and with them the asset pairs (2j, 2j + 1): it draws their
// normals, keeps eta in registers and publishes eps to LDS.  After the step's
// one barrier, every wave forms Z^S = L eps for its own assets from the
// published eps (in the order b = 0, 1, ..., as the Greek-set kernel does),
// advances them, and leaves the largest S over its assets and each asset's
// max(v, 0) in LDS.  After the next barrier wave 0, whose rows of L are the
// shortest, folds them into the date's feature: U = max over waves, A = (1/N)
// x the sum of max(v_i, 0) in asset order, so that the feature is the same
// for every W and bit for bit the Greek-set kernel's base feature.  LDS is
// double buffered by step parity: eps [2][blocks, padded to CH][64] pairs, max(v, 0)
// [2][2 blocks][64], wave maxima [2][W][64].
// Philox block i of wave w among W: blocks are dealt in a snake (w, then
// 2W - 1 - w, then 2W + w, ...), so that the triangular correlation work
// (block j needs j + 1 rows of eps) evens out over the waves, and each
// wave's blocks increase with i.
__device__ __forceinline__ int own_block(int w, int i, int W)
{
    return (i & 1) ? (i + 1) * W - 1 - w : i * W + w;
}

template <typename R, int BPW, int SCHEME, typename FT>
__global__ void __launch_bounds__(kLanes * base_max_waves(sizeof(R) == 4, SCHEME == HS_SCHEME_QE, BPW))
    k_paths_base(const BasePathArgs A)
{
    using VT = std::conditional_t<SCHEME == HS_SCHEME_QE, double, R>;
    extern __shared__ unsigned char hs_smem[];
    const int N = A.N;
    const int W = A.W;
    const int nblk = (N + 1) / 2;
    constexpr int CH = base_chunk(sizeof(R) == 4);
    const int nblk_pad = (nblk + CH - 1) / CH * CH;
    R2<R>* const s_eps = reinterpret_cast<R2<R>*>(hs_smem);
    R* const s_vp = reinterpret_cast<R*>(s_eps + 2 * nblk_pad * kLanes);
    R* const s_max = s_vp + 2 * (2 * nblk) * kLanes;

    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kLanes + lane;
    const bool live = p < A.P;
    const int64_t P = A.P;
    const cptr<ModelP<R>> mp = as_const<ModelP<R>>(A.model);
    const R dt = mp->dt;
    const R r = mp->r;
    const R invN = mp->invN;
    const R half = R(0.5);
    const uint32_t plo = static_cast<uint32_t>(p);
    const uint32_t phi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    R2<FT>* __restrict__ feat = static_cast<R2<FT>*>(A.feat);

    // own slot s: block w + (s / 2) W, asset 2 (w + (s / 2) W) + (s & 1)
    R X[2 * BPW];
    VT V[2 * BPW];
    VT eta[2 * BPW];
#pragma unroll
    for (int s = 0; s < 2 * BPW; ++s) {
        const int a = 2 * own_block(w, s / 2, W) + (s & 1);
        const int ac = a < N ? a : 0;  // the table is read in bounds either way
        const VT v0 = static_cast<VT>(SCHEME == HS_SCHEME_QE ? mp->a[ac].qe.v0 : mp->a[ac].v0);
        X[s] = R(0);
        V[s] = a < N ? v0 : VT(0);
        eta[s] = VT(0);
    }

    // eps pairs past the last block stay 0 (their L columns are 0 too)
    for (int j = nblk + w; j < nblk_pad; j += W) {
        s_eps[j * kLanes + lane] = R2<R>{R(0), R(0)};
        s_eps[(nblk_pad + j) * kLanes + lane] = R2<R>{R(0), R(0)};
    }

    // the feature of the date after step kk, from the buffers of parity kk & 1
    auto fold = [&](int kk) {
        const R* const vb = s_vp + (kk & 1) * (2 * nblk) * kLanes;
        const R* const mb = s_max + (kk & 1) * W * kLanes;
        R M = mb[lane];
        for (int v = 1; v < W; ++v) {
            const R x = mb[v * kLanes + lane];
            M = x > M ? x : M;
        }
        R sum = R(0);
        for (int a = 0; a < N; ++a) sum = sum + vb[a * kLanes + lane];
        if (live) {
            R2<FT> f;
            f.u = static_cast<FT>(M);
            f.a = static_cast<FT>(sum * invN);
            feat[static_cast<int64_t>(kk) * P + p] = f;
        }
    };

    for (int k = 0; k < A.n; ++k) {
        R2<R>* const eb = s_eps + (k & 1) * nblk_pad * kLanes;
        R* const vb = s_vp + (k & 1) * (2 * nblk) * kLanes;
        R* const mb = s_max + (k & 1) * W * kLanes;

        // 1) own Philox blocks: pair 2j <- (w0, w1), 2j+1 <- (w2, w3); the
        //    pair past an odd N is published as 0 (its L column is 0)
#pragma unroll
        for (int i = 0; i < BPW; ++i) {
            const int j = own_block(w, i, W);
            if (j < nblk) {
                const Words q = philox10(plo, static_cast<uint32_t>(k), static_cast<uint32_t>(j),
                                         phi, A.key0, A.key1);
                R2<R> e;
                if constexpr (SCHEME == HS_SCHEME_QE)
                    box_muller_mixed(q.x, q.y, e.u, eta[2 * i]);
                else
                    box_muller(q.x, q.y, e.u, eta[2 * i]);
                if (2 * j + 1 < N) {
                    if constexpr (SCHEME == HS_SCHEME_QE)
                        box_muller_mixed(q.z, q.w, e.a, eta[2 * i + 1]);
                    else
                        box_muller(q.z, q.w, e.a, eta[2 * i + 1]);
                } else {
                    e.a = R(0);
                    eta[2 * i + 1] = VT(0);
                }
                eb[j * kLanes + lane] = e;
            }
        }
        __syncthreads();

        // 2) the previous date's feature
        if (w == 0 && k > 0) fold(k - 1);

        // 3) own assets: Z^S over the published blocks 0..j of each owned
        //    block j, CH blocks at a time with one wait for the chunk's LDS
        //    and scalar loads; the upper part of L is 0, so the columns a
        //    chunk adds past a row's diagonal add 0, and slots that own no
        //    block read the zero rows
        R z[2 * BPW];
#pragma unroll
        for (int s = 0; s < 2 * BPW; ++s) z[s] = R(0);
        int jb = 0;
#pragma unroll
        for (int i = 0; i < BPW; ++i) {
            const int ji = own_block(w, i, W);
            const int jend = ji < nblk ? ji : -1;
            for (; jb <= jend; jb += CH) {
                R2<R> e[CH];
#pragma unroll
                for (int c = 0; c < CH; ++c) e[c] = eb[(jb + c) * kLanes + lane];
#pragma unroll
                for (int t = i; t < BPW; ++t) {
                    const int jt = own_block(w, t, W);
                    const int row = 2 * (jt < nblk ? jt : kZeroPair);
                    const cptr<R> l0 = mp->L + row * kMaxPathAssets + 2 * jb;
                    const cptr<R> l1 = l0 + kMaxPathAssets;
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        z[2 * t] += l0[2 * c] * e[c].u;
                        z[2 * t] += l0[2 * c + 1] * e[c].a;
                        z[2 * t + 1] += l1[2 * c] * e[c].u;
                        z[2 * t + 1] += l1[2 * c + 1] * e[c].a;
                    }
                }
            }
        }
        R m = R(0);  // every S > 0
#pragma unroll
        for (int s = 0; s < 2 * BPW; ++s) {
            const int a = 2 * own_block(w, s / 2, W) + (s & 1);
            if (a < N) {
                const cptr<AssetP<R>> q = mp->a + a;
                if constexpr (SCHEME == HS_SCHEME_QE) {
                    qe_step(&q->qe, z[s], eta[s], X[s], V[s]);
                } else {
                    const R zv = q->rho * z[s] + q->rhobar * eta[s];
                    const R vp = V[s] > R(0) ? V[s] : R(0);
                    const R sq = sqrt_r(vp * dt);
                    X[s] = X[s] + (r - half * vp) * dt + sq * z[s];
                    V[s] = V[s] + q->kappa * (q->theta - vp) * dt + q->xi * sq * zv;
                }
                const R S = q->S0 * exp_r(X[s]);
                m = S > m ? S : m;
                vb[a * kLanes + lane] = static_cast<R>(V[s] > VT(0) ? V[s] : VT(0));
            }
        }
        mb[w * kLanes + lane] = m;
    }
    __syncthreads();
    if (w == 0 && A.n > 0) fold(A.n - 1);
}

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

    double* const gcf = GLB ? A.cf + static_cast<int64_t>(s) * P : nullptr;
    int32_t* const gtau = GLB ? A.tau + static_cast<int64_t>(s) * P : nullptr;
    const int64_t last = static_cast<int64_t>(n - A.f_date0) * P;  // date n

    // (windows of dates keep the state in the workspace, GLB)
    double cf[GLB ? 1 : Q];
    int tau[GLB ? 1 : Q];
    if (!GLB) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t p = threadIdx.x + static_cast<int64_t>(i) * kSweepThreads;
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
    const int lane = threadIdx.x & 63;
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

// KEEP: each path keeps the payoff and centred basis variables of the date it
// last entered the regression, so that date's exercise decision needs no
// recomputation (more registers: one workgroup per CU).  Otherwise the
// decision recomputes them from that date's features, within 128 registers so
// that two workgroups share a CU (4 waves per SIMD), for Greek sets larger
// than one workgroup per CU can hold.  Both give the same numbers.
template <typename R, int Q, bool KEEP, bool WIN>
__global__ void __launch_bounds__(kClusterThreads,
                                  (!KEEP && !WIN && Q <= cluster_qmax_shared(sizeof(R) <= 4)) ? 4
                                                                                             : 2)
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
    const R2<R>* __restrict__ F = static_cast<const R2<R>*>(A.feat) + s * A.plane;
    if (threadIdx.x == 0) *Ls.flag = 1;
    __syncthreads();

    const int64_t row_len = static_cast<int64_t>(G) * kPartStride;
    const bool amer = A.american != 0;
    double* const part = C.partials +
                         (static_cast<int64_t>(s) * cluster_rows(amer, n) - cluster_row0(amer, n)) *
                             row_len;
    const cptr<RegRec> recs = as_const<RegRec>(A.reg) + static_cast<int64_t>(s) * n;
    const cptr<double> dsc = as_const<double>(A.disc) + static_cast<int64_t>(s) * (n + 1);
    const cptr<double> idsc = as_const<double>(A.idisc) + static_cast<int64_t>(s) * (n + 1);
    const int64_t pbase = static_cast<int64_t>(g) * (kClusterThreads * Q) + threadIdx.x;
    // a window of dates (WIN), else every date: regressions k_top..k_lo, the
    // features of date d at index d - f0
    const int f0 = WIN ? A.f_date0 : 1;
    const int64_t last = WIN ? static_cast<int64_t>(n - f0) * P  // date n
                             : (A.american ? static_cast<int64_t>(n - 1) * P : 0);
    const int k_lo = WIN ? A.k_lo : 1;
    const int k_top = WIN ? min(A.k_hi, n - 1) : n - 1;
    int par = 0;

    // State per path: the cash flow discounted to time 0, D = h_tau exp(-r tau
    // dt).  The regression target at date k is D exp(r k dt) =
    // h_tau exp(-r (tau - k) dt), and the price is the mean of D.  The exercise
    // date tau, wanted only for export, goes straight to memory at each
    // exercise (the sweep runs backward, so the last write is the earliest
    // exercise date).
    // Path pbase + i kClusterThreads exists iff i < nlive (the last workgroup
    // of a scenario may be ragged).
    const int64_t room = P - pbase;
    const int nlive = room <= 0 ? 0 : (room + kClusterThreads - 1) / kClusterThreads;
    int32_t* const tau = A.export_tau ? A.tau + static_cast<int64_t>(s) * P + pbase : nullptr;
    // (a window after the first takes D from the workspace, where the
    // previous window left it)
    double D[Q];
    if (!WIN || A.win_first) {
        const double dn = dsc[n];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t p = pbase + i * kClusterThreads;
            D[i] = i < nlive ? payoff(A.cp, A.K, static_cast<double>(F[last + p].u)) * dn : 0.0;
            if (tau && i < nlive) tau[i * kClusterThreads] = n;
        }
    } else {
        const double* const dstate = A.cf + static_cast<int64_t>(s) * P + pbase;
#pragma unroll
        for (int i = 0; i < Q; ++i) D[i] = i < nlive ? dstate[i * kClusterThreads] : 0.0;
    }

    double beta[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    bool have = false;  // beta of the later date k+1 is valid
    double skipped = 0.0;
    if (A.american) {
        // Three feature buffers take turns: at date k, cur holds date k (this
        // regression), nxt date k-1 (loaded one date ago) and old date k+1
        // (without KEEP, its decision's features); after the exchange old
        // receives date k-2.  The loop is unrolled three times so the roles
        // rotate by renaming and a load's destination is not read until two
        // dates later: the loads fly across the next date's work.
        R bu[3][Q], ba[3][Q];
        // payoff and centred basis variables of each path at the date last
        // regressed, kept for that date's exercise decision (h = 0: out of
        // the money, no decision)
        double hh[Q], xx[Q], ww[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t p = pbase + i * kClusterThreads;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                bu[j][i] = R(0);
                ba[j][i] = R(0);
            }
            hh[i] = 0.0;
            xx[i] = 0.0;
            ww[i] = 0.0;
            if (i < nlive && k_top >= k_lo) {
                const R2<R> f = F[static_cast<int64_t>(k_top - f0) * P + p];
                bu[0][i] = f.u;
                ba[0][i] = f.a;
            }
            if (i < nlive && k_top - 1 >= k_lo) {
                const R2<R> f = F[static_cast<int64_t>(k_top - 1 - f0) * P + p];
                bu[1][i] = f.u;
                ba[1][i] = f.a;
            }
        }
        // regression-set flag and means of date k, loaded one date ahead
        double r_ok = k_top >= k_lo ? recs[k_top - 1].ok : 0.0;
        double r_cU = k_top >= k_lo ? recs[k_top - 1].cU : 0.0;
        double r_cA = k_top >= k_lo ? recs[k_top - 1].cA : 0.0;
        double bcU = 0.0, bcA = 0.0;  // regression-set means of date k+1

        // the exercise decision at date kd with the regression of that date
        // (beta, bcU, bcA), from the kept values or from that date's features
        auto decide = [&](int kd, const R (&du)[Q], const R (&da)[Q]) {
            const double d1 = dsc[kd];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                double h, x, w;
                if constexpr (KEEP) {
                    h = hh[i];
                    x = xx[i];
                    w = ww[i];
                } else {
                    const double U = static_cast<double>(du[i]);
                    h = i < nlive ? payoff(A.cp, A.K, U) : 0.0;
                    double phi[5];
                    basis(m, U, static_cast<double>(da[i]), bcU, bcA, A.inv_K, A.inv_tbar, phi);
                    x = phi[1];
                    w = phi[3];
                }
                if (h > 0.0) {
                    const double cont = beta[0] + beta[1] * x + beta[2] * (x * x) + beta[3] * w +
                                        beta[4] * (x * w);
                    if (h > cont) {
                        D[i] = h * d1;
                        if (tau) tau[i * kClusterThreads] = kd;
                    }
                }
            }
        };

        // one date k with buffers cur = C, old = O; false if a wait timed out
        auto step = [&](int k, auto Ci, auto Oi) -> bool {
            constexpr int CB = decltype(Ci)::value, OB = decltype(Oi)::value;
            const bool ok = r_ok != 0.0;
            const double cU = r_cU, cA = r_cA;
            if (k > k_lo) {
                r_ok = recs[k - 2].ok;
                r_cU = recs[k - 2].cU;
                r_cA = recs[k - 2].cA;
            }
            const double ik = idsc[k];
            // exercise at date k+1 with its regression, then this date's
            // right-hand side with the updated cash flows
            if (have) decide(k + 1, bu[OB], ba[OB]);
            double b[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if constexpr (KEEP) hh[i] = 0.0;
                if (ok) {
                    const double U = static_cast<double>(bu[CB][i]);
                    const double h = payoff(A.cp, A.K, U);
                    if (i < nlive && h > 0.0) {
                        double phi[5];
                        basis(m, U, static_cast<double>(ba[CB][i]), cU, cA, A.inv_K, A.inv_tbar,
                              phi);
                        const double Y = D[i] * ik;
#pragma unroll
                        for (int q = 0; q < 5; ++q)
                            if (q < m) b[q] += phi[q] * Y;
                        if constexpr (KEEP) {
                            hh[i] = h;
                            xx[i] = phi[1];
                            ww[i] = phi[3];
                        }
                    }
                }
            }
            if (ok) {
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
            // date k-2 into old, issued after the exchange, whose slot polls
            // would otherwise wait for these loads (vector loads complete in
            // order)
            // (all Q loads issue without branches: a path past P reads the
            // last path, whose value no decision or sum uses)
            if (k - 2 >= k_lo) {
                const R2<R>* __restrict__ Fn = F + static_cast<int64_t>(k - 2 - f0) * P;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const int64_t p = pbase + i * kClusterThreads;
                    const R2<R> f = Fn[p < P ? p : P - 1];
                    bu[OB][i] = f.u;
                    ba[OB][i] = f.a;
                }
            }
            return true;
        };

        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        for (int k = k_top; k >= k_lo;) {
            if (!step(k, I0{}, I2{})) return;
            if (--k < k_lo) break;
            if (!step(k, I1{}, I0{})) return;
            if (--k < k_lo) break;
            if (!step(k, I2{}, I1{})) return;
            --k;
        }
        if (have) {  // exercise at date k_lo (1 in the last window): its buffer was cur last
            switch ((k_top - k_lo) % 3) {
            case 0: decide(k_lo, bu[0], ba[0]); break;
            case 1: decide(k_lo, bu[1], ba[1]); break;
            default: decide(k_lo, bu[2], ba[2]); break;
            }
        }
    }

    if (WIN && !A.win_last) {  // a window before the last: D waits in the workspace
        double* const dstate = A.cf + static_cast<int64_t>(s) * P + pbase;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            if (i < nlive) dstate[i * kClusterThreads] = D[i];
        if (g == 0 && threadIdx.x == 0) {
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
    if (g == 0 && threadIdx.x == 0) {
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

template <typename R, int NMAX, int TMAX, int SCHEME, typename FT, bool CK>
hipError_t launch_paths_ck(const PathArgs& a, int nchunks, int nbg, hipStream_t st)
{
    const size_t lds = 2u * 5u * NMAX * kLanes * sizeof(R) +
                       (SCHEME == HS_SCHEME_QE ? 2u * NMAX * kLanes * sizeof(double) : 0u);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_paths<R, NMAX, TMAX, SCHEME, FT, CK>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    dim3 grid(nchunks, nbg), block(kLanes, a.W);
    hipLaunchKernelGGL((k_paths<R, NMAX, TMAX, SCHEME, FT, CK>), grid, block, lds, st, a);
    return hipGetLastError();
}

template <typename R, int NMAX, int TMAX, int SCHEME, typename FT>
hipError_t launch_paths_t(const PathArgs& a, int nchunks, int nbg, hipStream_t st)
{
    return a.ck_every > 0 ? launch_paths_ck<R, NMAX, TMAX, SCHEME, FT, true>(a, nchunks, nbg, st)
                          : launch_paths_ck<R, NMAX, TMAX, SCHEME, FT, false>(a, nchunks, nbg, st);
}

template <typename R, int SCHEME, typename FT>
hipError_t launch_paths_r(int nmax, const PathArgs& a, int nchunks, int nbg, hipStream_t st)
{
    constexpr bool F = sizeof(R) == 4, Q = SCHEME == HS_SCHEME_QE;
    switch (nmax) {
    case 1: return launch_paths_t<R, 1, paths_tmax_for(F, Q, 1), SCHEME, FT>(a, nchunks, nbg, st);
    case 2: return launch_paths_t<R, 2, paths_tmax_for(F, Q, 2), SCHEME, FT>(a, nchunks, nbg, st);
    case 3: return launch_paths_t<R, 3, paths_tmax_for(F, Q, 3), SCHEME, FT>(a, nchunks, nbg, st);
    case 4: return launch_paths_t<R, 4, paths_tmax_for(F, Q, 4), SCHEME, FT>(a, nchunks, nbg, st);
    case 5: return launch_paths_t<R, 5, paths_tmax_for(F, Q, 5), SCHEME, FT>(a, nchunks, nbg, st);
    case 6: return launch_paths_t<R, 6, paths_tmax_for(F, Q, 6), SCHEME, FT>(a, nchunks, nbg, st);
    case 8: return launch_paths_t<R, 8, paths_tmax_for(F, Q, 8), SCHEME, FT>(a, nchunks, nbg, st);
    case 10: return launch_paths_t<R, 10, paths_tmax_for(F, Q, 10), SCHEME, FT>(a, nchunks, nbg, st);
    case 12: return launch_paths_t<R, 12, paths_tmax_for(F, Q, 12), SCHEME, FT>(a, nchunks, nbg, st);
    case 16: return launch_paths_t<R, 16, paths_tmax_for(F, Q, 16), SCHEME, FT>(a, nchunks, nbg, st);
    case 20: return launch_paths_t<R, 20, paths_tmax_for(F, Q, 20), SCHEME, FT>(a, nchunks, nbg, st);
    default: return hipErrorInvalidValue;
    }
}

// Calls f with a null pointer of the feature storage type of code ft.
template <typename Ret, typename Fn>
Ret with_feat(int ft, Ret bad, Fn&& f)
{
    switch (ft) {
    case kFeatF32: return f(static_cast<float*>(nullptr));
    case kFeatF64: return f(static_cast<double*>(nullptr));
    case kFeatF16: return f(static_cast<_Float16*>(nullptr));
    case kFeatBF16: return f(static_cast<__bf16*>(nullptr));
    default: return bad;
    }
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

template <typename R, int Q, bool KEEP, bool WIN>
hipError_t launch_cluster_t(const LsmcArgs& a, const ClusterArgs& c, int S_launch, size_t lds,
                            hipStream_t st)
{
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&k_sweep_cluster<R, Q, KEEP, WIN>),
            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_sweep_cluster<R, Q, KEEP, WIN>), dim3(S_launch * c.G),
                       dim3(kClusterThreads), lds, st, a, c);
    return hipGetLastError();
}

template <typename R, int Q, bool KEEP, bool WIN>
int cluster_capacity_t(size_t lds)
{
    const void* f = reinterpret_cast<const void*>(&k_sweep_cluster<R, Q, KEEP, WIN>);
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

}  // namespace

size_t cluster_lds_bytes(int n, int G)
{
    (void)n;
    (void)G;
    return sizeof(double) * (2 * (kClusterThreads / 64) * kPartStride + 2 * kPartStride) + 16;
}

int cluster_capacity(int ft, int q, bool keep, bool win, size_t lds)
{
    if (keep && win) return 0;  // windows run the variant without kept basis values
    return with_feat(ft, 0, [&](auto tag) -> int {
        using FT = std::remove_pointer_t<decltype(tag)>;
        switch (q) {
#define HS_CAP(Q)                                                                          \
    case Q:                                                                                \
        return keep  ? cluster_capacity_t<FT, Q, true, false>(lds)                         \
               : win ? cluster_capacity_t<FT, Q, false, true>(lds)                         \
                     : cluster_capacity_t<FT, Q, false, false>(lds);
            HS_CAP(1) HS_CAP(2) HS_CAP(3) HS_CAP(4) HS_CAP(5) HS_CAP(6) HS_CAP(7) HS_CAP(8)
#undef HS_CAP
        default: return 0;
        }
    });
}

hipError_t launch_sweep_cluster(int ft, int q, bool keep, const LsmcArgs& a,
                                const ClusterArgs& c, int S_launch, hipStream_t st)
{
    const size_t lds = cluster_lds_bytes(a.n, c.G);
    const bool win = a.k_lo != 1 || a.k_hi != a.n || !a.win_first || !a.win_last;
    if (win && (keep || !a.american || !a.cf || a.k_lo < 1 || a.k_hi > a.n || a.f_date0 > a.k_lo))
        return hipErrorInvalidValue;
    return with_feat(ft, hipErrorInvalidValue, [&](auto tag) -> hipError_t {
        using FT = std::remove_pointer_t<decltype(tag)>;
        switch (q) {
#define HS_LAUNCH(Q)                                                                    \
    case Q:                                                                             \
        return keep  ? launch_cluster_t<FT, Q, true, false>(a, c, S_launch, lds, st)    \
               : win ? launch_cluster_t<FT, Q, false, true>(a, c, S_launch, lds, st)    \
                     : launch_cluster_t<FT, Q, false, false>(a, c, S_launch, lds, st);
            HS_LAUNCH(1) HS_LAUNCH(2) HS_LAUNCH(3) HS_LAUNCH(4) HS_LAUNCH(5) HS_LAUNCH(6)
            HS_LAUNCH(7) HS_LAUNCH(8)
#undef HS_LAUNCH
        default: return hipErrorInvalidValue;
        }
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

int paths_tmax(bool fp32, int scheme, int nmax)
{
    return paths_tmax_for(fp32, scheme == HS_SCHEME_QE, nmax);
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

hipError_t launch_paths(bool fp32, int nmax, int scheme, int ft, const PathArgs& a, int nchunks,
                        int nbg, hipStream_t st)
{
    // the step range, and a restart only from a kept checkpoint
    if (a.k_begin < 0 || a.k_end > a.n || a.k_begin > a.k_end || a.k_feat0 < 0 ||
        a.ck_every < 0)
        return hipErrorInvalidValue;
    if (a.ck_every == 0 && (a.k_begin != 0 || a.ck_store))
        return hipErrorInvalidValue;
    if (a.ck_every > 0 && a.k_begin > 0 &&
        ((a.n - a.k_begin) % a.ck_every != 0 || (a.n - a.k_begin) / a.ck_every < 2))
        return hipErrorInvalidValue;
    // the block must fit the variant's launch bound
    if (a.W < 1 || a.W > paths_max_waves(fp32, nmax)) return hipErrorInvalidValue;
    if (!fp32) {
        if (ft != kFeatF64) return hipErrorInvalidValue;
        return scheme == HS_SCHEME_QE
                   ? launch_paths_r<double, HS_SCHEME_QE, double>(nmax, a, nchunks, nbg, st)
                   : launch_paths_r<double, HS_SCHEME_EULER_FT, double>(nmax, a, nchunks, nbg, st);
    }
    if (scheme == HS_SCHEME_QE)
        return ft == kFeatF32 ? launch_paths_r<float, HS_SCHEME_QE, float>(nmax, a, nchunks, nbg, st)
                              : hipErrorInvalidValue;
    switch (ft) {
    case kFeatF32:
        return launch_paths_r<float, HS_SCHEME_EULER_FT, float>(nmax, a, nchunks, nbg, st);
    case kFeatF16:
        return launch_paths_r<float, HS_SCHEME_EULER_FT, _Float16>(nmax, a, nchunks, nbg, st);
    case kFeatBF16:
        return launch_paths_r<float, HS_SCHEME_EULER_FT, __bf16>(nmax, a, nchunks, nbg, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int BPW, int SCHEME, typename FT>
hipError_t launch_paths_base_t(const BasePathArgs& a, hipStream_t st)
{
    const size_t lds = paths_base_lds_bytes(sizeof(R) == 4, a.N, a.W);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&k_paths_base<R, BPW, SCHEME, FT>),
            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    const int64_t nb = (a.P + kLanes - 1) / kLanes;
    dim3 grid(static_cast<unsigned>(nb)), block(kLanes, a.W);
    hipLaunchKernelGGL((k_paths_base<R, BPW, SCHEME, FT>), grid, block, lds, st, a);
    return hipGetLastError();
}

template <typename R, int SCHEME, typename FT>
hipError_t launch_paths_base_r(int bpw, const BasePathArgs& a, hipStream_t st)
{
    switch (bpw) {
    case 1: return launch_paths_base_t<R, 1, SCHEME, FT>(a, st);
    case 2: return launch_paths_base_t<R, 2, SCHEME, FT>(a, st);
    case 4: return launch_paths_base_t<R, 4, SCHEME, FT>(a, st);
    default: return hipErrorInvalidValue;
    }
}

int paths_base_bpw(bool fp32, int scheme, int N, int W)
{
    const int nblk = (N + 1) / 2;
    if (N < 1 || N > kMaxPathAssets || W < 1 || W > kBaseMaxWaves) return -1;
    const int need = (nblk + W - 1) / W;
    for (int b = 1; b <= kBaseMaxBpw; b *= 2)
        if (need <= b) return W <= base_max_waves(fp32, scheme == HS_SCHEME_QE, b) ? b : -1;
    return -1;
}

size_t paths_base_lds_bytes(bool fp32, int N, int W)
{
    const size_t R = fp32 ? 4u : 8u;
    const size_t nblk = static_cast<size_t>((N + 1) / 2);
    const size_t ch = static_cast<size_t>(base_chunk(fp32));
    const size_t nblk_pad = (nblk + ch - 1) / ch * ch;
    return 2u * nblk_pad * kLanes * 2u * R + 2u * (2u * nblk) * kLanes * R +
           2u * static_cast<size_t>(W) * kLanes * R;
}

hipError_t launch_paths_base(bool fp32, int scheme, int ft, const BasePathArgs& a, hipStream_t st)
{
    const int bpw = paths_base_bpw(fp32, scheme, a.N, a.W);
    if (bpw < 0 || a.P < 1 || a.n < 1) return hipErrorInvalidValue;
    if (!fp32) {
        if (ft != kFeatF64) return hipErrorInvalidValue;
        return scheme == HS_SCHEME_QE
                   ? launch_paths_base_r<double, HS_SCHEME_QE, double>(bpw, a, st)
                   : launch_paths_base_r<double, HS_SCHEME_EULER_FT, double>(bpw, a, st);
    }
    if (scheme == HS_SCHEME_QE)
        return ft == kFeatF32 ? launch_paths_base_r<float, HS_SCHEME_QE, float>(bpw, a, st)
                              : hipErrorInvalidValue;
    switch (ft) {
    case kFeatF32: return launch_paths_base_r<float, HS_SCHEME_EULER_FT, float>(bpw, a, st);
    case kFeatF16: return launch_paths_base_r<float, HS_SCHEME_EULER_FT, _Float16>(bpw, a, st);
    case kFeatBF16: return launch_paths_base_r<float, HS_SCHEME_EULER_FT, __bf16>(bpw, a, st);
    default: return hipErrorInvalidValue;
    }
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
