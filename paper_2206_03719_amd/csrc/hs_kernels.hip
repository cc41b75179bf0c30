// hs_kernels.hip -- host-side dispatch of the Greek-set path kernel variants
// (compiled in hs_paths_*.hip), its shape helpers, and the diagnostic kernels
// that expose the random numbers (Philox words and Box-Muller normals).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "../../include/hs_api.h"
#include "hs_kernels.hpp"
#include "hs_layout.hpp"
#include "hs_device.hpp"

namespace hs {
namespace {

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

}  // namespace

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

size_t paths_lds_bytes(bool fp32, int scheme, int nmax)
{
    // two parities of eps and eta, one of Z^S (FP64 under QE), exp(X) and
    // max(v, 0), and three prefix tables of nmax + 1 entries
    const size_t r = fp32 ? 4u : 8u, z = scheme == HS_SCHEME_QE ? 8u : r;
    const size_t slab = static_cast<size_t>(nmax) * kLanes;
    return slab * (5u * z + 2u * r) + 3u * static_cast<size_t>(nmax + 1) * kLanes * r;
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
    if (a.W < 1 || a.W > paths_max_waves(fp32, scheme == HS_SCHEME_QE, nmax)) return hipErrorInvalidValue;
    if (!fp32)
        return scheme == HS_SCHEME_QE ? launch_paths_f64q(nmax, ft, a, nchunks, nbg, st)
                                      : launch_paths_f64e(nmax, ft, a, nchunks, nbg, st);
    if (scheme == HS_SCHEME_QE) return launch_paths_f32q(nmax, ft, a, nchunks, nbg, st);
    return ft == kFeatF32 ? launch_paths_f32e(nmax, ft, a, nchunks, nbg, st)
                          : launch_paths_f32h(nmax, ft, a, nchunks, nbg, st);
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
