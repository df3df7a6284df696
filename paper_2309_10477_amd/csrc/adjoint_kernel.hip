// Reverse-mode (adjoint) sensitivities of each path's discounted payoff to
// theta = (S0, v0, r, kappa, theta, sigma, rho), over checkpointed step states.
//
// The forward pricing launch stores (x, V) every SEG steps and the final
// (x_N, A).  Per path this kernel walks the segments from last to first:
// it recomputes the segment's SEG steps from the checkpoint with the same
// Philox normals (kept with the step's V+, sqrt(V+ dt) and fixing term in
// registers), then runs the reverse recurrence of the Milstein step
// (paper: algorithm "Milstein approximation under Heston model") with the
// conventions d max(y,0)/dy = 1{y > 0} and d sqrt(V+ dt)/dV = 0 where V+ = 0.
// The payoff seeds follow the pathwise estimators of the paper's section
// "Pathwise method for greeks estimation" (chain rule through S_T or the
// discrete average); dS0 and dr reproduce the pathwise Delta and Rho.
#include "device_math.hpp"
#include "internal.hpp"
#include "path_step.hpp"

namespace heston {
namespace {

template <class R, bool ASIAN, bool FT, int SEG>
__global__ __launch_bounds__(BLOCK) void adjoint_kernel(const PriceLaunch L, double seed_grad,
                                                        double *__restrict__ per_path)
{
    __shared__ double red[BLOCK / 64][N_ACC];
    const uint64_t np = L.n_paths;
    const uint64_t row = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool active = row < np;
    const uint64_t rr = active ? row : 0;
    const uint64_t p = L.first_path + rr;
    const uint32_t N = L.n_steps;
    const R *ck = reinterpret_cast<const R *>(L.ckpt);
    const uint64_t nck = ckpt_count(N, SEG);

    const Coef<R> c = coef<R>(L.base);
    const R rho = (R)L.rho, rho_bar = (R)L.rho_bar, sigma = (R)L.sigma, theta = (R)L.theta;
    const R rho_ratio = (R)(L.rho_bar > 0 ? L.rho / L.rho_bar : 0.0); // -d rho_bar / d rho
    const R half_sigma_dt = (R)(0.5 * L.sigma * L.base.dt);            // d(qdt)/d sigma
    const R two_qdt = (R)(2.0 * L.base.quarter_sigma2_dt);
    const uint32_t k0 = (uint32_t)L.seed, k1 = (uint32_t)(L.seed >> 32);
    const uint32_t plo = (uint32_t)p, phi = (uint32_t)(p >> 32);

    // payoff and its seeds (FP64, as in the pricing kernel's epilogue)
    const double S0 = L.S0, D = exp(-L.r * L.T), inv_nfix = 1.0 / (double)L.n_fix;
    const R xN = ck[(2 * nck) * np + rr];
    const R AN = ck[(2 * nck + 1) * np + rr];
    const double rel = ASIAN ? (double)AN * inv_nfix : exp((double)xN);
    const double X = S0 * rel;
    const bool call = L.opt_type == 0 || L.opt_type == 2;
    const double sgn = call ? 1.0 : -1.0;
    const double in = sgn * (X - L.K);
    const bool itm = in > 0.0;
    const double y = itm ? D * in : 0.0;
    const double g_S0 = itm ? sgn * D * rel : 0.0;
    const R c_fix = (R)(itm ? sgn * D * S0 * inv_nfix : 0.0); // dy / d e^{x_i} at a fixing

    R xbar = (!ASIAN && itm) ? (R)(sgn * D * X) : R(0); // dy/dx_N for a European
    R vbar = 0, sum_xbar = 0, kbar = 0, thbar = 0, sbar = 0, rhobar = 0;

    for (int64_t seg = (int64_t)nck - 1; seg >= 0; --seg) {
        const uint32_t s0 = (uint32_t)seg * SEG;
        const uint32_t len = N - s0 < (uint32_t)SEG ? N - s0 : (uint32_t)SEG;
        R x = ck[(2 * (uint64_t)seg) * np + rr];
        R v = ck[(2 * (uint64_t)seg + 1) * np + rr];
        R a_vp[SEG], a_s[SEG], a_za[SEG], a_zb[SEG], a_f[SEG];
        bool a_clip[SEG];
        // forward recomputation of the segment
#pragma unroll
        for (int k = 0; k < SEG; k += 2) {
            if ((uint32_t)k < len) {
                R za[2], zb[2];
                philox_normals<R>(s0 + k, plo, phi, k0, k1, za[0], zb[0], za[1], zb[1]);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int kk = k + h;
                    if ((uint32_t)kk < len) {
                        const R z2 = rho * za[h] + rho_bar * zb[h];
                        const R vp = v > R(0) ? v : R(0);
                        a_vp[kk] = vp;
                        a_s[kk] = fast_sqrt(vp * c.dt);
                        a_za[kk] = za[h];
                        a_zb[kk] = zb[h];
                        const R vb = FT ? v : vp;
                        const R vpre =
                            vb + (c.ktdt - c.kdt * vp) + (sigma * z2) * a_s[kk] + c.qdt * (z2 * z2 - R(1));
                        mil_step<R, FT>(x, v, c, za[h], sigma * z2, c.qdt * (z2 * z2 - R(1)));
                        a_clip[kk] = !FT && !(vpre > R(0));
                        a_f[kk] = (ASIAN && is_fixing(L.fix_bits, s0 + kk + 1)) ? c_fix * fast_exp(x)
                                                                               : R(0);
                    }
                }
            }
        }
        // reverse sweep
#pragma unroll
        for (int k = SEG - 1; k >= 0; --k) {
            if ((uint32_t)k < len) {
                xbar += a_f[k]; // now the adjoint of x_{j+1}
                if (!FT && a_clip[k])
                    vbar = R(0); // V_{j+1} = max(pre, 0) with pre <= 0
                sum_xbar += xbar;
                const R vp = a_vp[k], s = a_s[k], za = a_za[k], zb = a_zb[k];
                const R z2 = rho * za + rho_bar * zb;
                const R dz2 = za - rho_ratio * zb;
                const bool pos = vp > R(0);
                const R dsdv = pos ? c.half_dt / s : R(0);
                const R g = xbar * (za * dsdv - c.half_dt) + vbar * (sigma * z2 * dsdv - c.kdt);
                kbar += vbar * (theta - vp);
                thbar += vbar;
                sbar += vbar * (s * z2 + half_sigma_dt * (z2 * z2 - R(1)));
                rhobar += vbar * (sigma * s + two_qdt * z2) * dz2;
                vbar = FT ? vbar + (pos ? g : R(0)) : (pos ? vbar + g : R(0));
            }
        }
    }

    double out[8];
    out[ADJ_PRICE] = y;
    out[ADJ_S0] = g_S0;
    out[ADJ_V0] = (double)vbar;
    out[ADJ_R] = (double)sum_xbar * L.base.dt - L.T * y;
    out[ADJ_KAPPA] = (double)kbar * L.base.dt;
    out[ADJ_THETA] = (double)thbar * L.base.kappa_dt;
    out[ADJ_SIGMA] = (double)sbar;
    out[ADJ_RHO] = (double)rhobar;
#pragma unroll
    for (int e = 1; e < 8; ++e)
        out[e] *= seed_grad;
    if (per_path != nullptr && active)
#pragma unroll
        for (int e = 0; e < 8; ++e)
            per_path[row * 8 + e] = out[e];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const double ye = active ? out[e] : 0.0;
        const double s1 = wave_sum(ye);
        const double s2 = wave_sum(ye * ye);
        if (lane == 0) {
            red[wave][2 * e] = s1;
            red[wave][2 * e + 1] = s2;
        }
    }
    __syncthreads();
    if (threadIdx.x < N_ACC) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w)
            t += red[w][threadIdx.x];
        L.partials[(uint64_t)blockIdx.x * N_ACC + threadIdx.x] = t;
    }
}

template <class R, bool ASIAN, bool FT>
hipError_t launch_seg(const PriceLaunch &L, double g, double *pp, hipStream_t s)
{
    const dim3 grid((uint32_t)((L.n_paths + BLOCK - 1) / BLOCK));
    if (L.ckpt_every == 8)
        hipLaunchKernelGGL((adjoint_kernel<R, ASIAN, FT, 8>), grid, dim3(BLOCK), 0, s, L, g, pp);
    else
        hipLaunchKernelGGL((adjoint_kernel<R, ASIAN, FT, 16>), grid, dim3(BLOCK), 0, s, L, g, pp);
    return hipGetLastError();
}

template <class R>
hipError_t launch_r(const PriceLaunch &L, double g, double *pp, hipStream_t s)
{
    const bool asian = L.opt_type >= 2;
    if (asian)
        return L.scheme == 0 ? launch_seg<R, true, true>(L, g, pp, s)
                             : launch_seg<R, true, false>(L, g, pp, s);
    return L.scheme == 0 ? launch_seg<R, false, true>(L, g, pp, s)
                         : launch_seg<R, false, false>(L, g, pp, s);
}

} // namespace

hipError_t launch_adjoint(const PriceLaunch &L, double seed_grad, double *per_path,
                          hipStream_t stream)
{
    return L.precision == 0 ? launch_r<double>(L, seed_grad, per_path, stream)
                            : launch_r<float>(L, seed_grad, per_path, stream);
}

} // namespace heston
