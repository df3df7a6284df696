// Double-precision complex arithmetic for device code (the semi-analytic
// geometric price and the exact sampler's characteristic function): plain
// struct, principal branches throughout.
#pragma once

#include <hip/hip_runtime.h>

namespace heston {

struct Cx {
    double re, im;
};
__device__ __forceinline__ Cx operator+(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cx operator-(Cx a, Cx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ Cx operator*(Cx a, Cx b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ Cx operator*(Cx a, double s) { return {a.re * s, a.im * s}; }
// Smith's division (no overflow of |b|^2 for large operands), two real
// divisions.
__device__ __forceinline__ Cx operator/(Cx a, Cx b)
{
    if (fabs(b.re) >= fabs(b.im)) {
        const double t = b.im / b.re, inv = 1.0 / (b.re + b.im * t);
        return {(a.re + a.im * t) * inv, (a.im - a.re * t) * inv};
    }
    const double t = b.re / b.im, inv = 1.0 / (b.re * t + b.im);
    return {(a.re * t + a.im) * inv, (a.im * t - a.re) * inv};
}
__device__ __forceinline__ Cx cexp(Cx z)
{
    double s, c;
    sincos(z.im, &s, &c);
    const double e = exp(z.re);
    return {e * c, e * s};
}
// Principal branch.
__device__ __forceinline__ Cx clog(Cx z) { return {log(hypot(z.re, z.im)), atan2(z.im, z.re)}; }
// Principal square root (non-negative real part).
__device__ __forceinline__ Cx csqrt(Cx z)
{
    const double m = hypot(z.re, z.im);
    if (m == 0.0)
        return {0.0, 0.0};
    const double t = sqrt(0.5 * (m + fabs(z.re)));
    if (z.re >= 0.0)
        return {t, z.im / (2.0 * t)};
    return {fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}
__device__ __forceinline__ Cx operator*(double s, Cx a) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ Cx operator-(Cx a) { return {-a.re, -a.im}; }
__device__ __forceinline__ double cabs(Cx z) { return hypot(z.re, z.im); }

} // namespace heston
