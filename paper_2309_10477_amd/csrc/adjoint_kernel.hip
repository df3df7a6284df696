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

// The forward pass of the adjoint: one path per lane, checkpoints of (x, V)
// every `every` steps and the final (x_N, A), then the payoff and pathwise
// estimators into FP64 block partials (price, Delta, Rho in the N_ACC layout).
template <class R, bool ASIAN, bool FT>
__global__ __launch_bounds__(BLOCK) void adjoint_forward_kernel(const PriceLaunch L)
{
    __shared__ double red[BLOCK / 64][N_ACC];
    const uint64_t np = L.n_paths;
    const uint64_t row = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool active = row < np;
    const uint64_t rr = active ? row : 0;
    const PathConsts k = path_consts(L);
    R x, v, A, B;
    R *ck = reinterpret_cast<R *>(L.ckpt);
    forward_path<R, ASIAN, FT>(k, L.first_path + rr, x, v, A, B, active ? ck : nullptr, np, rr,
                               L.ckpt_every);
    double out[3];
    path_estimators<ASIAN>(k, (double)x, (double)A, (double)B, out[0], out[1], out[2]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < N_EST; ++e) {
        const double ye = (active && e < 3) ? out[e < 3 ? e : 0] : 0.0;
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

template <class R, bool ASIAN, bool FT, int SEG>
__global__ __launch_bounds__(BLOCK) void adjoint_kernel(const PriceLaunch L, double seed_grad,
                                                        double *__restrict__ per_path)
{
    __shared__ double red[BLOCK / 64][N_ACC];
    const uint64_t np = L.n_paths;
    const uint64_t row = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool active = row < np;
    const uint64_t rr = active ? row : 0;
    const PathConsts k = path_consts(L);
    double out[8];
    adjoint_path<R, ASIAN, FT, SEG>(k, L.first_path + rr, reinterpret_cast<const R *>(L.ckpt), np,
                                    rr, out);
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

template <class R>
hipError_t launch_fwd_r(const PriceLaunch &L, hipStream_t s)
{
    const dim3 grid((uint32_t)((L.n_paths + BLOCK - 1) / BLOCK));
    const bool asian = L.opt_type >= 2;
    if (asian) {
        if (L.scheme == 0)
            hipLaunchKernelGGL((adjoint_forward_kernel<R, true, true>), grid, dim3(BLOCK), 0, s, L);
        else
            hipLaunchKernelGGL((adjoint_forward_kernel<R, true, false>), grid, dim3(BLOCK), 0, s, L);
    } else {
        if (L.scheme == 0)
            hipLaunchKernelGGL((adjoint_forward_kernel<R, false, true>), grid, dim3(BLOCK), 0, s, L);
        else
            hipLaunchKernelGGL((adjoint_forward_kernel<R, false, false>), grid, dim3(BLOCK), 0, s, L);
    }
    return hipGetLastError();
}

} // namespace

hipError_t launch_adjoint_forward(const PriceLaunch &L, hipStream_t stream)
{
    return L.precision == 0 ? launch_fwd_r<double>(L, stream) : launch_fwd_r<float>(L, stream);
}

hipError_t launch_adjoint(const PriceLaunch &L, double seed_grad, double *per_path,
                          hipStream_t stream)
{
    return L.precision == 0 ? launch_r<double>(L, seed_grad, per_path, stream)
                            : launch_r<float>(L, seed_grad, per_path, stream);
}

} // namespace heston
