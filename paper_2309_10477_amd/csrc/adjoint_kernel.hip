// Reverse-mode (adjoint) sensitivities of each path's discounted payoff to
// theta = (S0, v0, r, kappa, theta, sigma, rho), over checkpointed step states.
//
// The forward pricing launch stores (x, V) every SEG steps and the final
// (x_N, A).  Per path this kernel walks the segments from last to first:
// it recomputes the segment's SEG steps from the checkpoint with the same
// Philox normals (kept with the step's V+, sqrt(V+ dt) and fixing term in
// registers), then runs the reverse recurrence of the Milstein step
// (paper: algorithm "Milstein approximation under Heston model") with the
// conventions d max(y,0)/dy = 1{y > 0} and d sqrt(V+ dt)/dV = 0 where V+ = 0,
// or, under Andersen's QE scheme (the paper's Future Work), the reverse
// recurrence of the QE step with its branch decisions held fixed.
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
template <class R, bool ASIAN, int SC>
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
    if constexpr (SC == 2)
        forward_path_qe<R, ASIAN>(k, L.first_path + rr, x, v, A, B, active ? ck : nullptr, np, rr,
                                  L.ckpt_every);
    else
        forward_path<R, ASIAN, SC == 0>(k, L.first_path + rr, x, v, A, B, active ? ck : nullptr,
                                        np, rr, L.ckpt_every);
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

template <class R, bool ASIAN, int SC, int SEG>
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
    if constexpr (SC == 2)
        adjoint_path_qe<R, ASIAN, SEG>(k, L.first_path + rr, reinterpret_cast<const R *>(L.ckpt),
                                       np, rr, out);
    else
        adjoint_path<R, ASIAN, SC == 0, SEG>(k, L.first_path + rr,
                                             reinterpret_cast<const R *>(L.ckpt), np, rr, out);
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

template <class R, bool ASIAN, int SC>
hipError_t launch_seg(const PriceLaunch &L, double g, double *pp, hipStream_t s)
{
    const dim3 grid((uint32_t)((L.n_paths + BLOCK - 1) / BLOCK));
    if (L.ckpt_every == 8)
        hipLaunchKernelGGL((adjoint_kernel<R, ASIAN, SC, 8>), grid, dim3(BLOCK), 0, s, L, g, pp);
    else
        hipLaunchKernelGGL((adjoint_kernel<R, ASIAN, SC, 16>), grid, dim3(BLOCK), 0, s, L, g, pp);
    return hipGetLastError();
}

// L.scheme: 0 Milstein with full truncation, 1 with absorption, 2 QE.
template <class R, bool ASIAN>
hipError_t launch_sc(const PriceLaunch &L, double g, double *pp, hipStream_t s)
{
    return L.scheme == 0   ? launch_seg<R, ASIAN, 0>(L, g, pp, s)
           : L.scheme == 1 ? launch_seg<R, ASIAN, 1>(L, g, pp, s)
                           : launch_seg<R, ASIAN, 2>(L, g, pp, s);
}

template <class R>
hipError_t launch_r(const PriceLaunch &L, double g, double *pp, hipStream_t s)
{
    return L.opt_type >= 2 ? launch_sc<R, true>(L, g, pp, s) : launch_sc<R, false>(L, g, pp, s);
}

template <class R, bool ASIAN, int SC> void launch_fwd_t(const PriceLaunch &L, hipStream_t s)
{
    const dim3 grid((uint32_t)((L.n_paths + BLOCK - 1) / BLOCK));
    hipLaunchKernelGGL((adjoint_forward_kernel<R, ASIAN, SC>), grid, dim3(BLOCK), 0, s, L);
}

template <class R, bool ASIAN> void launch_fwd_sc(const PriceLaunch &L, hipStream_t s)
{
    if (L.scheme == 0)
        launch_fwd_t<R, ASIAN, 0>(L, s);
    else if (L.scheme == 1)
        launch_fwd_t<R, ASIAN, 1>(L, s);
    else
        launch_fwd_t<R, ASIAN, 2>(L, s);
}

template <class R>
hipError_t launch_fwd_r(const PriceLaunch &L, hipStream_t s)
{
    if (L.opt_type >= 2)
        launch_fwd_sc<R, true>(L, s);
    else
        launch_fwd_sc<R, false>(L, s);
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
