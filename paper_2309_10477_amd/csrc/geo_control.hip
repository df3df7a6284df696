// Semi-analytic price of the geometric-average Asian option under Heston, on
// the device: the expectation of the control in the arithmetic-Asian
// control-variate estimator.
//
// ln G = (1/n) sum_i ln S(t_i) is a linear functional of the affine state
// (ln S, V), so E[exp(u ln G)] = exp(u ln S0 + A + B v0).  Going backwards
// from the last fixing date, the coefficient a of ln S is u/n times the number
// of dates still ahead, and over each gap between dates (A, B) follow the
// Riccati equations of the Heston model with that a, whose solution is closed
// form: with c2 = sigma^2/2, c1 = rho sigma a - kappa, c0 = (a^2 - a)/2 and the
// roots r_- (attracting) and r_+ of c2 x^2 + c1 x + c0,
//   B(tau) = (r_- - r_+ g e^{-d tau}) / (1 - g e^{-d tau}),  g = (B0 - r_-)/(B0 - r_+),
//   A(tau) = A0 + r a tau + kappa theta (r_- tau - ln((1 - g e^{-d tau})/(1 - g)) / c2).
// The call price is e^{-rT} ((E[G] - K)/2 + (1/pi) int_0^inf Re[e^{-iv ln K}
// (M(1+iv) - K M(iv)) / (iv)] dv) (Gil-Pelaez), integrated by 16-point
// Gauss-Legendre on panels of width GEO_PANEL_WIDTH up to a power of two v_max
// where the integrand's modulus bound is below 1e-15 (E[G] + K).
//
// Each thread evaluates one transform (a sequential pass over the fixing
// dates), so a launch is bound by that chain's latency, not by throughput.
// The first pass integrates over [0, g.v_max] (a range the host sizes from
// the variance of ln G) in one node launch that also evaluates the bound at
// its end; only if that bound is not small does the caller run the search: a bound kernel (one wave) at v =
// 2^k, then nodes up to the first 2^k whose bound is small (a fixed grid whose
// blocks beyond it only write a zero partial).  A finish kernel sums the block
// partials in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cplx.hpp"
#include "device_math.hpp"
#include "internal.hpp"

namespace heston {
namespace {

constexpr int GEO_MAX_LOG2_RANGE = 14; // v_max <= 2^14
// Panel width: the integrand varies on the scale of 1 / sd(ln G) and is
// analytic in a strip about the real axis, so 16 nodes per 4 units resolve
// it to rounding (checked against adaptive quadrature: 1e-13 relative up to
// width 8 on the tested parameter sets).
constexpr uint32_t GEO_PANEL_WIDTH = 4;
static_assert(GEO_MAX_LOG2_RANGE < GEO_BOUND_POINTS, "bound table too short");
static_assert(2 * GEO_BOUND_POINTS < 64, "one wave evaluates every bound and E[G]");
constexpr uint32_t GEO_NODE_THREADS = 32u << GEO_MAX_LOG2_RANGE; // 16 nodes x 2 transforms
constexpr uint32_t GEO_NODE_BLOCKS = GEO_NODE_THREADS / BLOCK;
constexpr double GEO_TOL = 1e-15;

__device__ __forceinline__ double fix_time(const GeoControl &g, uint32_t i)
{
    return (g.steps ? (double)g.steps[i] : (double)(i + 1)) * g.dt;
}

// (A, B) carried over a gap tau with the coefficient a of ln S.
__device__ __forceinline__ void riccati(const GeoControl &g, Cx a, double tau, Cx &A, Cx &B)
{
    const double c2 = 0.5 * g.sigma * g.sigma;
    const Cx c1 = a * (g.rho * g.sigma) - Cx{g.kappa, 0.0};
    const Cx c0 = (a * a - a) * 0.5;
    Cx d = csqrt(c1 * c1 - c0 * (4.0 * c2));
    if (d.re < 0.0)
        d = Cx{-d.re, -d.im};
    const double h = 0.5 / c2;
    const Cx rm = (Cx{-c1.re, -c1.im} - d) * h;
    const Cx rp = (Cx{-c1.re, -c1.im} + d) * h;
    const Cx q = (B - rm) / (B - rp);
    const Cx e = cexp(d * (-tau));
    const Cx qe = q * e;
    const Cx one{1.0, 0.0};
    const Cx Bn = (rm - rp * qe) / (one - qe);
    const Cx intB = rm * tau - clog((one - qe) / (one - q)) * (1.0 / c2);
    A = A + a * (g.r * tau) + intB * (g.kappa * g.theta);
    B = Bn;
}

// Exponent of E[exp(u ln G)]: u ln S0 + A + B v0.
__device__ Cx log_transform(const GeoControl &g, Cx u)
{
    const Cx w = u * (1.0 / (double)g.n_fix);
    Cx a = w, A{0.0, 0.0}, B{0.0, 0.0};
    for (uint32_t k = g.n_fix; k-- > 0;) {
        const double tk = fix_time(g, k), tp = k ? fix_time(g, k - 1) : 0.0;
        riccati(g, a, tk - tp, A, B);
        if (k)
            a = a + w;
    }
    return a * g.lnS0 + A + B * g.v0;
}

// Part `which` of the Gil-Pelaez integrand at v: which 0 gives
// Im(e^{-iv ln K} M(1+iv)) / v, which 1 gives -K Im(e^{-iv ln K} M(iv)) / v.
__device__ double integrand_part(const GeoControl &g, double v, int which)
{
    const Cx u{which ? 0.0 : 1.0, v};
    const Cx m = cexp(log_transform(g, u) - Cx{0.0, v * g.lnK});
    return (which ? -g.K : 1.0) * m.im / v;
}

// Modulus bound of one part: |M(u)| (times K for part 1) / v.
__device__ double bound_part(const GeoControl &g, double v, int which)
{
    const Cx u{which ? 0.0 : 1.0, v};
    return (which ? g.K : 1.0) * exp(log_transform(g, u).re) / v;
}

__global__ __launch_bounds__(64) void geo_bound_kernel(const GeoControl g, double *bound,
                                                       double *out)
{
    const int t = threadIdx.x;
    if (t < 2 * GEO_BOUND_POINTS)
        bound[t] = bound_part(g, ldexp(1.0, t >> 1), t & 1);
    else if (t == 2 * GEO_BOUND_POINTS)
        out[2] = exp(log_transform(g, Cx{1.0, 0.0}).re); // E[G]
}

// Range of the integral: the first 2^k (k <= GEO_MAX_LOG2_RANGE) whose bound
// is below tolerance, or 0 if none is.
__device__ uint32_t range_from(const double *bound, double EG, double K)
{
    const double tol = GEO_TOL * (EG + K);
    for (int k = 0; k <= GEO_MAX_LOG2_RANGE; ++k)
        if (bound[2 * k] + bound[2 * k + 1] <= tol)
            return 1u << k;
    return 0u;
}

// Gauss-Legendre nodes of the integral over [0, range], two transforms per
// node.  With a `fixed` range the three threads after the nodes evaluate the
// modulus bound at v = fixed (out[4], out[5]) and E[G] (out[2]); otherwise the
// range comes from the bound table of geo_bound_kernel.
__global__ __launch_bounds__(BLOCK) void geo_node_kernel(const GeoControl g, uint32_t fixed,
                                                         const double *bound, double *out,
                                                         double *partials)
{
    __shared__ double red[BLOCK / 64];
    const uint32_t range = fixed ? fixed : range_from(bound, out[2], g.K);
    const uint32_t width = range < GEO_PANEL_WIDTH ? range : GEO_PANEL_WIDTH;
    const uint32_t panels = width ? range / width : 0u;
    const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
    const uint32_t n_node_threads = 32u * panels;
    double val = 0.0;
    if (t < n_node_threads) {
        const uint32_t node = t >> 1, panel = node >> 4, j = node & 15;
        const double x = j < 8 ? -g.gl_x[7 - j] : g.gl_x[j - 8];
        const double w = j < 8 ? g.gl_w[7 - j] : g.gl_w[j - 8];
        const double v = ((double)panel + 0.5 + 0.5 * x) * (double)width;
        val = 0.5 * (double)width * w * integrand_part(g, v, (int)(t & 1));
    } else if (fixed && t < n_node_threads + 2) {
        out[4 + (t - n_node_threads)] = bound_part(g, (double)fixed, (int)(t - n_node_threads));
    } else if (fixed && t == n_node_threads + 2) {
        out[2] = exp(log_transform(g, Cx{1.0, 0.0}).re); // E[G]
    }
    const double s = wave_sum(val);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w)
            b += red[w];
        partials[blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(BLOCK) void geo_finish_kernel(const GeoControl g, uint32_t fixed,
                                                           uint32_t n_blocks, const double *bound,
                                                           const double *partials, double *out)
{
    __shared__ double red[BLOCK];
    double s = 0.0;
    for (uint32_t b = threadIdx.x; b < n_blocks; b += BLOCK)
        s += partials[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (threadIdx.x < (unsigned)h)
            red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double EG = out[2], I = red[0];
        const double D = exp(-g.r * g.T);
        const bool ok = fixed ? out[4] + out[5] <= GEO_TOL * (EG + g.K)
                              : range_from(bound, EG, g.K) != 0u;
        const double call = D * (0.5 * (EG - g.K) + I / M_PI);
        const double nan = __builtin_nan("");
        out[0] = ok ? call : nan;
        out[1] = ok ? call - D * (EG - g.K) : nan;
        out[3] = I;
    }
}

} // namespace

uint32_t geo_node_blocks() { return GEO_NODE_BLOCKS; }

hipError_t launch_geo_price_fixed(const GeoControl &g, double *partials, double *buf,
                                  hipStream_t stream)
{
    static_assert((32u * GEO_MAX_FIXED_RANGE + 3u + BLOCK - 1) / BLOCK <= GEO_NODE_BLOCKS,
                  "fixed range within the partials buffer");
    if (g.v_max < GEO_PANEL_WIDTH || g.v_max > GEO_MAX_FIXED_RANGE || g.v_max % GEO_PANEL_WIDTH)
        return hipErrorInvalidValue;
    const uint32_t blocks = (32u * (g.v_max / GEO_PANEL_WIDTH) + 3u + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(geo_node_kernel, dim3(blocks), dim3(BLOCK), 0, stream, g, g.v_max,
                       (const double *)buf, buf + GEO_OUT, partials);
    hipLaunchKernelGGL(geo_finish_kernel, dim3(1), dim3(BLOCK), 0, stream, g, g.v_max, blocks,
                       (const double *)buf, (const double *)partials, buf + GEO_OUT);
    return hipGetLastError();
}

hipError_t launch_geo_price_search(const GeoControl &g, double *partials, double *buf,
                                   hipStream_t stream)
{
    hipLaunchKernelGGL(geo_bound_kernel, dim3(1), dim3(64), 0, stream, g, buf, buf + GEO_OUT);
    hipLaunchKernelGGL(geo_node_kernel, dim3(GEO_NODE_BLOCKS), dim3(BLOCK), 0, stream, g, 0u,
                       (const double *)buf, buf + GEO_OUT, partials);
    hipLaunchKernelGGL(geo_finish_kernel, dim3(1), dim3(BLOCK), 0, stream, g, 0u,
                       GEO_NODE_BLOCKS, (const double *)buf, (const double *)partials,
                       buf + GEO_OUT);
    return hipGetLastError();
}

} // namespace heston
