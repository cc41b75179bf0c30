// hs_paths.hpp -- the Greek-set path kernel k_paths and its launch templates.
// Each path-kernel source (one per path precision, scheme and feature storage
// group) includes this header and instantiates its own variants, so the
// variants compile in parallel.
//
// k_paths: one pass over all steps of a block of 64 paths for a whole Greek
// set: Philox4x32-10 normals shared by every scenario (common random
// numbers), Cholesky correlation, the time step in log price (full-truncation
// Euler or Andersen's QE), the per-date path reduction of Sec. 4.1 (U =
// max_i S_i, A = mean_i max(v_i, 0)), coalesced feature stores.  The waves of
// a block split the random numbers and the base scenario's assets, meet in
// LDS, then each advances only the assets that its bumped scenarios change.
#pragma once
#include "hs_device.hpp"

namespace hs {
namespace {

// ---------------------------------------------------------------------------
// Path kernel.
//
// Block = W waves x 64 lanes; lane l of every wave follows path
// 64 * blockIdx.x + l.  blockIdx.y selects a "block group": W groups (one per
// wave) of tasks.  LDS holds, each [asset][lane]: the step's normals (eps,
// eta), double-buffered by step parity (a fast wave draws step k + 1 while a
// slow one still reads step k's eta); the base scenario's correlated normals
// Z^S, exp(X) and max(v, 0), and the prefix tables of the base features
// (single buffers: a step's writes come after its first barrier, which every
// wave reaches only once it has finished the previous step).  Under QE the
// normals eps, eta, Z^S and the variance state are FP64 (ZT, VT) in both
// path precisions, so the variance path is the FP64 one.
template <typename R, int NMAX, int TMAX, int SCHEME, typename FT, bool CK>
__global__ void __launch_bounds__(kLanes * paths_max_waves(sizeof(R) == 4, SCHEME == HS_SCHEME_QE, NMAX))
    k_paths(const PathArgs A)
{
    using VT = std::conditional_t<SCHEME == HS_SCHEME_QE, double, R>;
    using ZT = VT;  // the spot normals eps and Z^S = L eps
    extern __shared__ unsigned char hs_smem[];
    constexpr int SLAB = NMAX * kLanes;          // one [asset][lane] array
    constexpr int XSLAB = (NMAX + 1) * kLanes;   // one prefix table
    constexpr size_t SZ = SLAB * sizeof(ZT), SR = SLAB * sizeof(R), SX = XSLAB * sizeof(R);
    constexpr size_t PAR = 2 * SZ;               // eps and eta of one parity
    ZT* const s_zs = reinterpret_cast<ZT*>(hs_smem + 2 * PAR);
    R* const s_e = reinterpret_cast<R*>(hs_smem + 2 * PAR + SZ);
    R* const s_vp = reinterpret_cast<R*>(hs_smem + 2 * PAR + SZ + SR);
    // prefix tables of the base scenario, entry j of [0, N]: the largest
    // price and the sum of max(v, 0) over assets < j (pmx, psx), the largest
    // price over assets >= j (smx; 0 at j = N)
    R* const s_pmx = reinterpret_cast<R*>(hs_smem + 2 * PAR + SZ + 2 * SR);
    R* const s_psx = reinterpret_cast<R*>(hs_smem + 2 * PAR + SZ + 2 * SR + SX);
    R* const s_smx = reinterpret_cast<R*>(hs_smem + 2 * PAR + SZ + 2 * SR + 2 * SX);

    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int W = A.W;
    const int N0 = A.N;
    const int N = N0;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kLanes + lane;
    const bool live = p < A.P;

    const cptr<BaseP<R>> bp = as_const<BaseP<R>>(A.base);
    cptr<ZT> bL;
    if constexpr (std::is_same_v<ZT, R>)
        bL = bp->L;
    else
        bL = bp->L64;
    const int gidx = static_cast<int>(blockIdx.y) * W + w;
    const cptr<GroupP> gp = as_const<GroupP>(A.groups) + gidx;
    const int g_task0 = gp->task0, ntask = gp->ntask, g_base = gp->base_scen,
              g_up0 = gp->spot_up0, g_dn0 = gp->spot_dn0, g_rate = gp->rate_scen;
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
    constexpr int OWN = paths_own_per_wave(NMAX);
    R Xo[OWN];
    VT Vo[OWN];
#pragma unroll
    for (int i = 0; i < OWN; ++i) {
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
        for (int i = 0; i < OWN; ++i) {
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
        // the asset count (shadowing the kernel's), opaque here: the compiler
        // compares a < N where needed instead of keeping per-asset masks in
        // (spilled) scalar registers across the step loop
        int N = N0;
        asm volatile("" : "+s"(N));
        unsigned char* const pb = hs_smem + (k & 1) * PAR;
        ZT* const s_eps = reinterpret_cast<ZT*>(pb);
        VT* const s_eta = reinterpret_cast<VT*>(pb + SZ);

        // 1) Philox blocks j = w, w + W, ...: pair 2j <- (w0, w1), 2j+1 <- (w2, w3)
        for (int j = w; j < nblk; j += W) {
            const Words q = philox10(plo, static_cast<uint32_t>(k), static_cast<uint32_t>(j), phi,
                                     A.key0, A.key1);
            ZT e;
            VT h;
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

        // 2) the base scenario's owned assets: Z^S = L eps, then the time step
#pragma unroll
        for (int i = 0; i < OWN; ++i) {
            const int a = w + i * W;
            if (a < N) {
                ZT z = ZT(0);
                for (int b = 0; b <= a; ++b) z += bL[a * kMaxAssets + b] * s_eps[b * kLanes + lane];
                const cptr<AssetP<R>> q = bp->a + a;
                if constexpr (SCHEME == HS_SCHEME_QE) {
                    qe_step(&q->qe, z, s_eta[a * kLanes + lane], Xo[i], Vo[i]);
                } else {
                    const R zv = q->rho * z + q->rhobar * s_eta[a * kLanes + lane];
                    const R vp = pos_r(Vo[i]);
                    const R sq = sqrt_r(vp * dt);
                    Xo[i] = Xo[i] + (r - half * vp) * dt + sq * z;
                    Vo[i] = Vo[i] + q->kappa * (q->theta - vp) * dt + q->xi * sq * zv;
                }
                s_zs[a * kLanes + lane] = z;
                s_e[a * kLanes + lane] = exp_r(Xo[i]);
                s_vp[a * kLanes + lane] = static_cast<R>(pos_r(Vo[i]));
            }
        }
        __syncthreads();

        // 3) features
        // (checkpoint runs store the dates from k_feat0 + 1 on, at index 0)
        const bool store = CK ? (A.store_all ? k >= A.k_feat0 : k == A.n - 1)
                              : (A.store_all || k == A.n - 1);
        const int64_t off =
            (A.store_all ? static_cast<int64_t>(CK ? k - A.k_feat0 : k) * P : 0) + p;
        // the base scenario's prices Sb and prefix tables, streamed into LDS:
        // every wave writes the same tables (identical values from identical
        // inputs) and then reads entries back -- relaxed atomic accesses, so
        // the overlapping writes are no data race, and a wave's own write
        // precedes its reads
        ZT eps[NMAX];
        R Sb[NMAX];
        R bsum = R(0), run = R(0);
        lds_put(s_pmx + lane, R(0));
        lds_put(s_psx + lane, R(0));
#pragma unroll
        for (int a = 0; a < NMAX; ++a) {
            if (a < N) {
                eps[a] = s_eps[a * kLanes + lane];
                Sb[a] = bp->a[a].S0 * s_e[a * kLanes + lane];
                run = a == 0 ? Sb[0] : (Sb[a] > run ? Sb[a] : run);
                bsum = bsum + s_vp[a * kLanes + lane];
                lds_put(s_pmx + (a + 1) * kLanes + lane, run);
                lds_put(s_psx + (a + 1) * kLanes + lane, bsum);
            } else {
                eps[a] = ZT(0);
                Sb[a] = R(0);
            }
        }
        // suffix maxima (every S > 0; 0 past the last asset)
        R suf = R(0);
        lds_put(s_smx + N * kLanes + lane, R(0));
#pragma unroll
        for (int a = NMAX - 1; a >= 0; --a) {
            if (a < N) {
                suf = Sb[a] > suf ? Sb[a] : suf;
                lds_put(s_smx + a * kLanes + lane, suf);
            }
        }
        const R bA = bsum * invN;

        if (store && live) {
            if (g_base >= 0) {
                R2<FT> f;
                f.u = static_cast<FT>(suf);
                f.a = static_cast<FT>(bA);
                feat[g_base * A.plane + off] = f;
            }
            if (g_rate >= 0) {
                // the rate bump shifts every log price by (r' - r) t at date
                // t = (k + 1) dt: U scales by e^{(r' - r) t}, A is the base's.
                // U + U (e^x - 1): the small change keeps its full relative
                // precision (the rate Greek is that change over the bump)
                R2<FT> f;
                f.u = static_cast<FT>(
                    fma(suf, expm1_r(bp->drdt * static_cast<R>(k + 1)), suf));
                f.a = static_cast<FT>(bA);
                feat[g_rate * A.plane + off] = f;
            }
            if (g_up0 >= 0) {
                // a spot bump rescales one asset of the base path; the other
                // assets' largest price comes from the prefix tables
#pragma unroll
                for (int a = 0; a < NMAX; ++a) {
                    if (a < N) {
                        const R lo = lds_get(s_pmx + a * kLanes + lane);
                        const R hi = lds_get(s_smx + (a + 1) * kLanes + lane);
                        const R ex = lo > hi ? lo : hi;
                        const R E = s_e[a * kLanes + lane];
                        const R su = bp->S0_up[a] * E;
                        const R sd = bp->S0_dn[a] * E;
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

        // 4) this wave's tasks (assets of bumped scenarios that leave the base
        //    path); a scenario's own assets [lo, hi) are consecutive tasks,
        //    joined to the base's assets outside them through the prefix tables
        R runM = R(0), runS = R(0);
        // the task count, opaque here: the compiler compares t < nt at each
        // task instead of keeping TMAX masks in (spilled) scalar registers
        int nt = ntask;
        asm volatile("" : "+s"(nt));
#pragma unroll
        for (int t = 0; t < TMAX; ++t) {
            if (t < nt) {
                const cptr<TaskP<R>> T = tk + t;
                // the Euler step's constants lead the record: a few wide
                // scalar loads
                const int a_el = T->a_el, lo_el = T->lo_el, hi_el = T->hi_el, flags = T->flags;
                ZT z = ZT(0);
                if constexpr (SCHEME == HS_SCHEME_QE) {
                    if (T->own_row) {
#pragma unroll
                        for (int b = 0; b < NMAX; ++b) z += T->L64[b] * eps[b];
                    } else {
                        z = s_zs[a_el + lane];
                    }
                    qe_step(&T->qe, z, s_eta[a_el + lane], tX[t], tV[t]);
                } else {
                    // the scenario's Cholesky row (the base row where the bump
                    // leaves it): the same FMA chain as the base step's, so
                    // equal rows give equal Z^S
#pragma unroll
                    for (int b = 0; b < NMAX; ++b) z += T->L[b] * eps[b];
                    const R zv = T->rho * z + T->rhobar * s_eta[a_el + lane];
                    const R vp = pos_r(tV[t]);
                    const R sq = sqrt_r(vp * T->dt);
                    tX[t] = tX[t] + (T->r - half * vp) * T->dt + sq * z;
                    tV[t] = tV[t] + T->kappa * (T->theta - vp) * T->dt + T->xi * sq * zv;
                }
                const R S = T->S0 * exp_r(tX[t]);
                const R vpt = static_cast<R>(pos_r(tV[t]));
                if (flags & 1) {  // a scenario's first task: the base assets below lo
                    runM = lds_get(s_pmx + lo_el + lane);
                    runS = lds_get(s_psx + lo_el + lane);
                }
                runM = S > runM ? S : runM;
                runS = runS + vpt;
                if (flags & 2) {
                    const R tail = lds_get(s_smx + hi_el + lane);
                    runM = tail > runM ? tail : runM;
                    runS = runS + (lds_get(s_psx + N * kLanes + lane) -
                                   lds_get(s_psx + hi_el + lane));
                    if (store && live) {
                        R2<FT> f;
                        f.u = static_cast<FT>(runM);
                        f.a = static_cast<FT>(runS * invN);
                        feat[T->fo + off] = f;
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
                for (int i = 0; i < OWN; ++i) {
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

template <typename R, int NMAX, int TMAX, int SCHEME, typename FT, bool CK>
hipError_t launch_paths_ck(const PathArgs& a, int nchunks, int nbg, hipStream_t st)
{
    const size_t lds = paths_lds_bytes(sizeof(R) == 4, SCHEME, NMAX);
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

}  // namespace
}  // namespace hs
