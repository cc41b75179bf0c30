// hs_paths_base.hip -- the base-model path kernel k_paths_base: Heston paths of
// one model and the per-date path reduction (the paper's measured stage, Sec.
// 2.2.1 and 4.1) for up to 64 assets, behind hs_path_features.
#include "hs_device.hpp"

namespace hs {
namespace {

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
    using ZT = VT;  // spot normals eps and Z^S (FP64 under QE: the variance path is the FP64 one)
    extern __shared__ unsigned char hs_smem[];
    const int N = A.N;
    const int W = A.W;
    const int nblk = (N + 1) / 2;
    constexpr int CH = base_chunk(sizeof(ZT) == 4);
    const int nblk_pad = (nblk + CH - 1) / CH * CH;
    R2<ZT>* const s_eps = reinterpret_cast<R2<ZT>*>(hs_smem);
    R* const s_vp = reinterpret_cast<R*>(s_eps + 2 * nblk_pad * kLanes);
    R* const s_max = s_vp + 2 * (2 * nblk) * kLanes;

    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kLanes + lane;
    const bool live = p < A.P;
    const int64_t P = A.P;
    const cptr<ModelP<R>> mp = as_const<ModelP<R>>(A.model);
    cptr<ZT> mL;
    if constexpr (std::is_same_v<ZT, R>)
        mL = mp->L;
    else
        mL = mp->L64;
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
        s_eps[j * kLanes + lane] = R2<ZT>{ZT(0), ZT(0)};
        s_eps[(nblk_pad + j) * kLanes + lane] = R2<ZT>{ZT(0), ZT(0)};
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
        R2<ZT>* const eb = s_eps + (k & 1) * nblk_pad * kLanes;
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
                R2<ZT> e;
                box_muller(q.x, q.y, e.u, eta[2 * i]);
                if (2 * j + 1 < N) {
                    box_muller(q.z, q.w, e.a, eta[2 * i + 1]);
                } else {
                    e.a = ZT(0);
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
        ZT z[2 * BPW];
#pragma unroll
        for (int s = 0; s < 2 * BPW; ++s) z[s] = ZT(0);
        int jb = 0;
#pragma unroll
        for (int i = 0; i < BPW; ++i) {
            const int ji = own_block(w, i, W);
            const int jend = ji < nblk ? ji : -1;
            for (; jb <= jend; jb += CH) {
                R2<ZT> e[CH];
#pragma unroll
                for (int c = 0; c < CH; ++c) e[c] = eb[(jb + c) * kLanes + lane];
#pragma unroll
                for (int t = i; t < BPW; ++t) {
                    const int jt = own_block(w, t, W);
                    const int row = 2 * (jt < nblk ? jt : kZeroPair);
                    const cptr<ZT> l0 = mL + row * kMaxPathAssets + 2 * jb;
                    const cptr<ZT> l1 = l0 + kMaxPathAssets;
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

}  // namespace

template <typename R, int BPW, int SCHEME, typename FT>
hipError_t launch_paths_base_t(const BasePathArgs& a, hipStream_t st)
{
    const size_t lds = paths_base_lds_bytes(sizeof(R) == 4, SCHEME, a.N, a.W);
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

size_t paths_base_lds_bytes(bool fp32, int scheme, int N, int W)
{
    // eps pairs (FP64 under QE), max(v, 0) and the wave maxima, two parities
    const size_t R = fp32 ? 4u : 8u, Z = scheme == HS_SCHEME_QE ? 8u : R;
    const size_t nblk = static_cast<size_t>((N + 1) / 2);
    const size_t ch = static_cast<size_t>(base_chunk(Z == 4u));
    const size_t nblk_pad = (nblk + ch - 1) / ch * ch;
    return 2u * nblk_pad * kLanes * 2u * Z + 2u * (2u * nblk) * kLanes * R +
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

}  // namespace hs
