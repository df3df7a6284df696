// The Milstein step shared by the pricing kernel and the adjoint's forward
// recomputation (paper: algorithm "Milstein approximation under Heston model").
#pragma once

#include "device_math.hpp"
#include "internal.hpp"

namespace heston {

template <class R> struct Coef {
    R dt, sqrt_dt, r_dt, half_dt, kdt, ktdt, qdt;
};

template <class R> __device__ __forceinline__ Coef<R> coef(const StepCoef &s)
{
    return Coef<R>{(R)s.dt, (R)s.sqrt_dt, (R)s.r_dt, (R)s.half_dt, (R)s.kappa_dt,
                   (R)s.kappa_theta_dt, (R)s.quarter_sigma2_dt};
}

// One step of (x = ln S/S0, V) on grid c: the log-price step carries no
// Milstein term; the variance step carries mil = sigma^2 dt (Z2^2 - 1) / 4.
// sz2 = sigma Z2.  FT: full truncation (V+ in drift and diffusion, V carried);
// otherwise absorption (V clamped at 0 after the step).
template <class R, bool FT>
__device__ __forceinline__ void mil_step(R &x, R &v, const Coef<R> &c, R z1, R sz2, R mil)
{
    const R vp = v > R(0) ? v : R(0);
    const R s = fast_sqrt(vp * c.dt);
    x += (c.r_dt - c.half_dt * vp) + s * z1;
    const R vb = FT ? v : vp;
    v = vb + (c.ktdt - c.kdt * vp) + sz2 * s + mil;
    if (!FT)
        v = v > R(0) ? v : R(0);
}

// Step j+1 is a fixing date (every step when the mask is absent).
__device__ __forceinline__ bool is_fixing(const uint32_t *fix_bits, uint32_t jf)
{
    return fix_bits == nullptr || ((fix_bits[jf >> 5] >> (jf & 31u)) & 1u);
}

// Normals of steps (j, j+1) from one Philox block: counter (j >> 1, lo32 p, hi32 p, 0).
template <class R>
__device__ __forceinline__ void philox_normals(uint32_t j, uint32_t plo, uint32_t phi, uint32_t k0,
                                               uint32_t k1, R &za0, R &zb0, R &za1, R &zb1)
{
    const U4 w = philox4x32_10(U4{j >> 1, plo, phi, 0u}, k0, k1);
    if constexpr (sizeof(R) == 4) {
        box_muller(uniform_f32(w.x), uniform_f32(w.y), za0, zb0);
        box_muller(uniform_f32(w.z), uniform_f32(w.w), za1, zb1);
    } else {
        box_muller(uniform_f64(w.x), uniform_f64(w.y), za0, zb0);
        box_muller(uniform_f64(w.z), uniform_f64(w.w), za1, zb1);
    }
}

} // namespace heston
