// Device building blocks of the path kernels: the counter-based generator,
// the uniform and normal maps, and wavefront reductions.  gfx950 (CDNA4),
// wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heston {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round
// multiplies counter words 0 and 2 by fixed 32-bit constants (full 64-bit
// products), mixes the high halves with words 1, 3 and the key, and the key
// then advances by the two Weyl constants.  From the third round on every
// word is per-lane, and each three-way XOR is one v_bitop3_b32 (truth table
// 0x96); the first two rounds are left to the compiler, which keeps their
// wave-uniform parts on the scalar unit.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)M0 * c.x;
        const uint64_t p1 = (uint64_t)M1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        if (i >= 2)
            c = U4{(uint32_t)__builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96), lo1,
                   (uint32_t)__builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96), lo0};
        else
            c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// Uniform in (0,1) from the top 23 bits of a word: (m + 1/2) 2^-23, exact in
// binary32 and binary64.  Single precision builds 1 + m 2^-23 by placing m
// under the exponent of 1.0 and subtracts 1 - 2^-24; the difference is
// representable, so it is exact (no integer-to-float conversion).
__device__ __forceinline__ float uniform_f32(uint32_t w)
{
    return __uint_as_float(0x3F800000u | (w >> 9)) - 0x1.fffffep-1f;
}
__device__ __forceinline__ double uniform_f64(uint32_t w)
{
    return (double)(w >> 9) * 0x1p-23 + 0x1p-24;
}

// Box-Muller pair from two uniforms: (sqrt(-2 ln ua) cos 2 pi ub, sqrt(-2 ln ua) sin 2 pi ub).
// Single precision uses the hardware transcendental units: v_log_f32 (log2),
// v_sqrt_f32, and v_cos_f32 / v_sin_f32, whose argument is in revolutions.
__device__ __forceinline__ void box_muller(float ua, float ub, float &za, float &zb)
{
    constexpr float M2LN2 = -1.38629436111989061883f; // -2 ln 2
    const float rad = __builtin_amdgcn_sqrtf(M2LN2 * __builtin_amdgcn_logf(ua));
    za = rad * __builtin_amdgcn_cosf(ub);
    zb = rad * __builtin_amdgcn_sinf(ub);
}
// The same pair divided by SQRT_2LN2 = sqrt(2 ln 2): sqrt(-log2 ua) (cos 2 pi ub,
// sin 2 pi ub), for callers that fold the factor into the constants the
// normals multiply.
constexpr double SQRT_2LN2 = 1.17741002251547469101;
__device__ __forceinline__ void box_muller_log2(float ua, float ub, float &za, float &zb)
{
    const float rad = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(ua));
    za = rad * __builtin_amdgcn_cosf(ub);
    zb = rad * __builtin_amdgcn_sinf(ub);
}
__device__ __forceinline__ void box_muller(double ua, double ub, double &za, double &zb)
{
    const double rad = sqrt(-2.0 * log(ua));
    double s, c;
    sincospi(2.0 * ub, &s, &c);
    za = rad * c;
    zb = rad * s;
}

// Inverse standard normal CDF on the lower half, u in [2^-31, 1/2].
// Single precision: Wichura's algorithm AS 241 (Applied Statistics 37, 1988),
// its single-precision form PPND7 (relative accuracy about 1e-7), evaluated
// branch-free: the central rational in r = 0.180625 - q^2, q = u - 1/2, for
// u >= 0.075 and the first tail rational in t = sqrt(-ln u) - 1.6 below: both
// polynomials computed, numerator and denominator selected, one reciprocal.
// All coefficients are positive and r, t >= 0 on their ranges, so neither
// polynomial cancels in binary32.  The second tail
// (sqrt(-ln u) > 5, u < 1.4e-11) lies outside the stated domain.
// Double precision: the device math library's normcdfinv.
__device__ __forceinline__ float inv_normal_lower(float u)
{
    const float q = u - 0.5f, r = 0.180625f - q * q;
    const float num_c = ((59.109374720f * r + 159.29113202f) * r + 50.434271938f) * r + 3.3871327179f;
    const float den_c = ((67.187563600f * r + 78.757757664f) * r + 17.895169469f) * r + 1.0f;
    // -ln u = -ln2 log2 u
    const float t =
        __builtin_amdgcn_sqrtf(-0.69314718055994530942f * __builtin_amdgcn_logf(u)) - 1.6f;
    const float num_t = ((0.17023821103f * t + 1.3067284816f) * t + 2.7568153900f) * t + 1.4234372777f;
    const float den_t = (0.12021132975f * t + 0.73700164250f) * t + 1.0f;
    // one reciprocal, of the selected denominator
    const bool tail = u < 0.075f;
    return (tail ? -num_t : q * num_c) * __builtin_amdgcn_rcpf(tail ? den_t : den_c);
}
__device__ __forceinline__ double inv_normal_lower(double u) { return normcdfinv(u); }

// Real-typed helpers.
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fast_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double fast_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float fast_exp(float x)
{
    return __builtin_amdgcn_exp2f(x * 1.44269504088896340736f);
}
__device__ __forceinline__ double fast_exp(double x) { return exp(x); }

template <class R> __device__ __forceinline__ R to_real(double v) { return (R)v; }

// ---------------------------------------------------------------------------
// Wavefront sum of a double, butterfly over the 64 lanes (fixed order, so the
// result is bitwise reproducible).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

} // namespace heston
