// hs_kernels.hpp -- host-side launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "hs_layout.hpp"

namespace hs {

// Path kernel: the asset-count bucket (1,2,3,4,5,6,8,10,12,16,20) that holds N,
// tasks per wave for a bucket, and the dynamic LDS it needs.
int paths_nmax_bucket(int N);
int paths_tmax(bool fp32, int scheme, int nmax);
size_t paths_lds_bytes(bool fp32, int scheme, int nmax);
hipError_t launch_paths(bool fp32, int nmax, int scheme, int feat, const PathArgs& a, int nchunks,
                        int nblockgroups, hipStream_t st);
// The variants behind launch_paths, one source each: FP32 Euler with FP32
// features (f32e) or 16-bit features (f32h), FP32 QE (f32q), FP64 Euler
// (f64e) and FP64 QE (f64q).
hipError_t launch_paths_f32e(int nmax, int ft, const PathArgs& a, int nchunks, int nbg, hipStream_t st);
hipError_t launch_paths_f32h(int nmax, int ft, const PathArgs& a, int nchunks, int nbg, hipStream_t st);
hipError_t launch_paths_f32q(int nmax, int ft, const PathArgs& a, int nchunks, int nbg, hipStream_t st);
hipError_t launch_paths_f64e(int nmax, int ft, const PathArgs& a, int nchunks, int nbg, hipStream_t st);
hipError_t launch_paths_f64q(int nmax, int ft, const PathArgs& a, int nchunks, int nbg, hipStream_t st);

// Base-scenario path kernel (features of the model alone): Philox blocks per
// wave for N assets and W waves (1, 2 or 4; -1 if this W does not fit), its
// dynamic LDS, and the launch over ceil(P / 64) blocks of W waves.
int paths_base_bpw(bool fp32, int scheme, int N, int W);
size_t paths_base_lds_bytes(bool fp32, int scheme, int N, int W);
hipError_t launch_paths_base(bool fp32, int scheme, int feat, const BasePathArgs& a,
                             hipStream_t st);

// The kernels after the path kernel are compiled per feature storage type
// (FeatType: FP32, FP64, FP16, BF16), the path kernel per path precision,
// scheme and storage type.

// Gram matrices and their Cholesky factors for dates 1..n-1 of S scenarios.
hipError_t launch_gram(int feat, const LsmcArgs& a, int S, hipStream_t st);

// Backward sweep + price of S scenarios.  q = paths per thread with the state
// in registers (1,2,4,8,16), or 0 for the state in the workspace.
int sweep_q_for(int64_t P);
hipError_t launch_sweep(int feat, int q, const LsmcArgs& a, int S, hipStream_t st);

// Cluster sweep: Q paths per thread (cluster_q_supported), G workgroups per
// scenario, S_launch scenarios (planes c.s0 ..) per launch; capacity =
// workgroups that fit on the device at once.  A launch over a window of
// dates (LsmcArgs k_lo, k_hi, win_first, win_last not the whole sweep) runs a
// variant of its own.
size_t cluster_lds_bytes(int n, int G);
int cluster_capacity(int feat, int q, bool win, size_t lds);
hipError_t launch_sweep_cluster(int feat, int q, const LsmcArgs& a, const ClusterArgs& c,
                                int S_launch, hipStream_t st);
hipError_t launch_fill_u64(uint64_t* p, int64_t count, uint64_t value, hipStream_t st);

hipError_t launch_philox_words(uint64_t seed, int64_t P, int n, int nb, uint32_t* out,
                               hipStream_t st);
hipError_t launch_normals(bool fp32, uint64_t seed, int N, int64_t P, int n, void* eps,
                          void* eta, hipStream_t st);

}  // namespace hs
