// Device building blocks of the path kernels: the counter-based generator,
// the uniform and normal maps, and wavefront reductions.  gfx950 (CDNA4),
// wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "inv_normal_coef.hpp"

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

// Inverse standard normal CDF on the lower half.
// Single precision, from 30-bit coordinates: xs in [0, 2^29) stands for
// u = (xs + 1/2) 2^-30.  In the erfinv variable of Giles (2011), w =
// -ln(4u(1-u)), Phi^{-1}(u) = -(1 - 2u) Q(w) with Q smooth: a degree-10
// polynomial in w - 4 for w <= 8 and a degree-7 polynomial in sqrt(w) - 3.6
// beyond (u < 8.4e-5, down to 2^-31), both fitted to relative error 2.1e-7
// in binary32 (coefficients and their fit: inv_normal_coef.hpp).  One
// logarithm per normal.  2u = (2 xs + 1) 2^-30 is exact in binary32 after
// rounding the integer, and 4u(1-u) = 2u (2 - 2u) keeps full relative
// precision as u -> 0.
template <int K>
__device__ __forceinline__ float horner(const float (&c)[K], float t)
{
    float q = c[0];
#pragma unroll
    for (int k = 1; k < K; ++k)
        q = q * t + c[k];
    return q;
}

// Two normals at once (the two coordinates of a bridge node): one branch
// into the tail piece for both, which a wave takes only when one of its lanes
// needs it for either.
__device__ __forceinline__ void inv_normal_lower_bits2(uint32_t xa, uint32_t xb, float &za,
                                                       float &zb)
{
    constexpr float LN2F = 0.69314718055994530942f;
    const float a0 = (float)(2u * xa + 1u) * 0x1p-30f, a1 = (float)(2u * xb + 1u) * 0x1p-30f; // 2u
    const float l0 = __builtin_amdgcn_logf(a0 * (2.0f - a0)); // log2(4u(1-u)) <= 0
    const float l1 = __builtin_amdgcn_logf(a1 * (2.0f - a1));
    float q0 = horner(INV_NORMAL_CENTRAL, l0 * -LN2F - INV_NORMAL_CENTER);
    float q1 = horner(INV_NORMAL_CENTRAL, l1 * -LN2F - INV_NORMAL_CENTER);
    constexpr float SPLIT = -INV_NORMAL_W_SPLIT / LN2F;
    const bool t0 = l0 < SPLIT, t1 = l1 < SPLIT;
    if (t0 || t1) {
        const float p0 = horner(INV_NORMAL_TAIL,
                                __builtin_amdgcn_sqrtf(l0 * -LN2F) - INV_NORMAL_TAIL_CENTER);
        const float p1 = horner(INV_NORMAL_TAIL,
                                __builtin_amdgcn_sqrtf(l1 * -LN2F) - INV_NORMAL_TAIL_CENTER);
        q0 = t0 ? p0 : q0;
        q1 = t1 ? p1 : q1;
    }
    za = (a0 - 1.0f) * q0; // -(1 - 2u) Q
    zb = (a1 - 1.0f) * q1;
}
// Double precision, from u in (0, 1/2]: the device math library's normcdfinv.
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
