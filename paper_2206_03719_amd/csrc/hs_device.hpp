// hs_device.hpp -- device helpers shared by the gfx950 kernels of the Heston /
// Longstaff-Schwartz Greek engine: the Philox4x32-10 generator, the exact
// uniform map, Box-Muller, the path-precision transcendentals, the constant
// address space, and Andersen's quadratic-exponential step.  Each kernel
// source includes this header; its functions have internal linkage.
#pragma once
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

__device__ __forceinline__ float exp_r(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504089f); }
__device__ __forceinline__ double exp_r(double x) { return exp(x); }
// max(x, 0) for a finite x: one v_med3 in FP32 (a compare-select there
// became a quieting max plus a max)
__device__ __forceinline__ float pos_r(float x)
{
    return __builtin_amdgcn_fmed3f(x, 0.0f, __builtin_huge_valf());
}
__device__ __forceinline__ double pos_r(double x) { return x > 0.0 ? x : 0.0; }
// e^x - 1 to full relative precision for small x (library functions)
__device__ __forceinline__ float expm1_r(float x) { return expm1f(x); }
__device__ __forceinline__ double expm1_r(double x) { return expm1(x); }
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

// Raw buffer access to `bytes` bytes from p: a load whose lane offset (voff)
// is at or past the end reads 0 (the buffer unit's range check covers the
// lane offset, so callers put the whole offset there and pass soff = 0), and
// a ragged last chunk of paths needs no clamped addresses.  Descriptor word
// 3, 0x00020000, is the raw (unformatted) buffer of the GFX9 family's
// resource layout.  p and bytes must be wave-uniform: they are read from the
// first active lane, so the descriptor lives in scalar registers (a
// descriptor the compiler takes for divergent costs a loop per load).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_over(const void* p, uint32_t bytes)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a >> 32));
    void* const q = reinterpret_cast<void*>((static_cast<uint64_t>(hi) << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(q, 0,
                                             static_cast<int>(__builtin_amdgcn_readfirstlane(bytes)),
                                             0x00020000);
}
template <typename T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16, "buffer_load size");
    if constexpr (sizeof(T) == 16)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    else if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
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

// Relaxed workgroup-scope atomic LDS accesses (plain ds_write / ds_read).
template <typename T>
__device__ __forceinline__ void lds_put(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ T lds_get(T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---------------------------------------------------------------------------
// Andersen's quadratic-exponential step of one asset from (X, v) (constants
// c: QeP) with the asset's correlated spot normal zs = (L eps)_i and its own
// normal eta.  The K2 v' term carries rho times the variance shock, so the
// log price takes the orthogonal part of the spot shock:
//   z_v = rho zs + sqrt(1 - rho^2) eta,  z_x = sqrt(1 - rho^2) zs - rho eta,
// independent unit normals with rho z_v + sqrt(1 - rho^2) z_x = zs, so the
// spot shocks of different assets keep the correlation C (as under the Euler
// scheme).  The variance path -- zs and eta, z_v, the state and the whole
// step, including the branch test psi <= 1.5 -- runs in FP64 in both path
// precisions: the two branches map the same normal to different variances,
// so an FP32 variance state that strays by rounding across psi = 1.5 would
// send the path off the FP64 one for good.  The log price's drift K0 + K1 v +
// K2 v' is FP64 too (K1 and K2 are near -rho/xi and rho/xi, so the sum
// cancels); its diffusion term and the log price itself run in R.
template <typename R, typename CP>
__device__ __forceinline__ void qe_step(CP c, double zs, double eta, R& X, double& v)
{
    const double zv = c->rho * zs + c->rhobar * eta;
    const R zx = static_cast<R>(c->rhobar * zs - c->rho * eta);
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

}  // namespace
}  // namespace hs
