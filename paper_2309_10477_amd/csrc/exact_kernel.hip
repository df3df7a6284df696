// Exact simulation of the Heston model (paper: algorithm "Broadie and Kaya
// exact simulation algorithm", section "Heston Model Exact simulation", and
// the sections on its two bottlenecks), FP64, one path per lane at a time.
//
// Step of length D from (x = ln S/S0, V_u):
//  1. V_t = c X, X non-central chi-square with d = 4 kappa theta / sigma^2
//     degrees of freedom and non-centrality lambda = V_u e^{-kappa D} / c,
//     c = sigma^2 (1 - e^{-kappa D}) / (4 kappa): for d > 1,
//     X = 2 Gamma((d-1)/2) + (Zv + sqrt(lambda))^2; for d <= 1,
//     X = 2 Gamma(d/2 + N), N ~ Poisson(lambda / 2) by inversion.  Gamma draws
//     by Marsaglia and Tsang (ACM TOMS 26(3), 2000; full acceptance test,
//     shapes below one raised by one and multiplied by U^(1/shape)).
//  2. I = int_u^t V given (V_u, V_t): inversion of its CDF, F(x) = h x / pi +
//     (2/pi) sum_j sin(h j x)/j Re Phi(h j), at a uniform U, where Phi is the
//     conditional characteristic function of the paper (exponents negative,
//     the Bessel-function ratio I_nu(z(a)) / I_nu(z(0)), nu = d/2 - 1, taken
//     on the branch continuous along the grid, ln z summed from its factors).  The grid spacing h = pi / u_eps
//     with u_eps = mean + 12 sd (from the slope and curvature of log Phi at
//     0), the grid length the first power of two >= 64 at which |Phi|/J falls
//     below pi 1e-10 / 2, truncated after the last point above it.  Inversion:
//     bisection on [0, u_eps] with Newton steps, to |F - U| < 1e-13.
//  3. x += r D - I/2 + rho (V_t - V_u - kappa theta D + kappa I) / sigma
//          + sqrt(1 - rho^2) sqrt(I) Zs.
// I_nu(z) = (z/2)^nu S(z) / Gamma(nu + 1) with S(z) = sum_k (z^2/4)^k
// Gamma(nu+1) / (k! Gamma(k+nu+1)), summed directly: the Gamma(nu + 1) cancels
// in the ratio, and (z/2)^nu takes the continuous argument of z.  The sum loses
// about e^{|z| - Re z} times the rounding unit; a path whose grid needs
// |z| - Re z > 20 or |z| > 600, more than EXACT_MAX_GRID points, a Poisson
// mean above EXACT_MAX_POISSON_MEAN or EXACT_MAX_GAMMA_ATTEMPTS rejections is
// counted as failed (payoff 0) and the call reports it.
//
// Random inputs: block k of step j of path p is Philox4x32-10 at counter
// (j, lo32 p, hi32 p, 5 + 256 k).  Block 0: Box-Muller of words 0, 1 gives
// (Zv, Zs), word 2 the uniform U of the inversion, word 3 the Poisson
// uniform; blocks k >= 1 are the gamma sampler's attempts (the first normal
// of words 0, 1 and the acceptance uniform of word 2; word 3 of block 1 is
// the uniform that lowers a shape below one).
//
// The Re Phi of the current draw live in `scratch`, one column per lane
// ([point][lane], coalesced); each lane walks paths lane, lane + n_lanes, ...
// and keeps FP64 sums of its estimators, reduced per block at the end.
#include <hip/hip_runtime.h>

#include "cplx.hpp"
#include "device_math.hpp"
#include "internal.hpp"
#include "path_step.hpp"

namespace heston {
namespace {

constexpr double PI = 3.14159265358979323846;
constexpr double GRID_EPS = 1e-10;

// Philox blocks of one (path, step).
struct Draw {
    uint32_t plo, phi, step, k0, k1;
    __device__ U4 block(uint32_t k) const
    {
        return philox4x32_10(U4{step, plo, phi, EXACT_COUNTER_TAG + (k << 8)}, k0, k1);
    }
};

// Gamma(alpha, 1); NaN after too many rejections.
__device__ double gamma_draw(double alpha, const Draw &dr)
{
    const double a = alpha < 1.0 ? alpha + 1.0 : alpha;
    const double d = a - 1.0 / 3.0, c = 1.0 / sqrt(9.0 * d);
    double g = __builtin_nan(""), boost = 1.0;
    for (int k = 1; k <= EXACT_MAX_GAMMA_ATTEMPTS; ++k) {
        const U4 w = dr.block((uint32_t)k);
        if (k == 1)
            boost = uniform_f64(w.w);
        double x, unused;
        box_muller(uniform_f64(w.x), uniform_f64(w.y), x, unused);
        double v = 1.0 + c * x;
        if (v <= 0.0)
            continue;
        v = v * v * v;
        if (log(uniform_f64(w.z)) < 0.5 * x * x + d - d * v + d * log(v)) {
            g = d * v;
            break;
        }
    }
    if (alpha < 1.0)
        g *= pow(boost, 1.0 / alpha);
    return g;
}

// Smallest k with u <= P(N <= k), N ~ Poisson(mu); NaN above the mean limit.
__device__ double poisson_inverse(double mu, double u)
{
    if (mu > EXACT_MAX_POISSON_MEAN)
        return __builtin_nan("");
    double pk = exp(-mu), F = pk;
    const int cap = (int)(mu + 40.0 * sqrt(mu) + 100.0);
    int k = 0;
    while (u > F && k < cap) {
        ++k;
        pk *= mu / k;
        F += pk;
    }
    return (double)k;
}

// S(z) = sum_k (z^2/4)^k / (k! (nu+1)_k); `bad` set if the sum does not
// settle or would lose too much to cancellation.
__device__ Cx bessel_sum(Cx z, double nu, bool &bad)
{
    const double az = cabs(z);
    if (az > 600.0 || az - z.re > 20.0)
        bad = true;
    const Cx q = z * z * 0.25;
    Cx t{1.0, 0.0}, s{1.0, 0.0};
    for (int k = 1; k < 2000; ++k) {
        // 1 / (k (k + nu)): hardware reciprocal and one Newton step
        const double den = (double)k * ((double)k + nu);
        double rc = __builtin_amdgcn_rcp(den);
        rc = rc * fma(-den, rc, 2.0);
        t = t * q * rc;
        s = s + t;
        // |t| < 1e-17 |s|, compared squared
        if ((double)k > 0.5 * az &&
            t.re * t.re + t.im * t.im < 1e-34 * (s.re * s.re + s.im * s.im))
            return s;
    }
    bad = true;
    return s;
}

// Per-draw constants of Phi: the Bessel terms at a = 0 and the endpoint sums.
struct PhiCtx {
    double vu, vt, r, sum_v;   // r = sqrt(vu vt)
    double log_zk;             // ln z(0) (r > 0)
    double log_s_zk;           // ln S(z(0))
};

// log Phi(a) = lp + ln S(z(a)) (lp returned, S(z(a)) in *s; S = 1 when r = 0).
// ln z(a) is summed from its factors (ln r + ln 4g - g D/2 -
// ln(sigma^2 (1 - e^{-gD}))): it cannot underflow, and its imaginary part is
// an argument of z continuous along a >= 0, the branch of (z/2)^nu.
__device__ Cx log_phi_part(const ExactLaunch &L, const PhiCtx &pc, double a, Cx *s, bool &bad)
{
    const Cx g = csqrt(Cx{L.kappa2, -L.two_sigma2 * a});
    const Cx eg = cexp(g * (-L.D));
    const Cx one{1.0, 0.0};
    const Cx ome = one - eg;
    const Cx lg = clog(g), lome = clog(ome);
    const Cx t1 = lg - g * (0.5 * L.D) + Cx{L.t1_const, 0.0} - lome;
    const Cx t2 = (Cx{L.coth_k, 0.0} - g * (one + eg) / ome) * (pc.sum_v * L.inv_sigma2);
    // ln z(a) / r
    const Cx lz0 = lg - g * (0.5 * L.D) - lome + Cx{L.log4_over_sigma2, 0.0};
    if (pc.r == 0.0) { // I_nu(z) ~ (z/2)^nu / Gamma(nu+1) as z -> 0
        *s = Cx{1.0, 0.0};
        return t1 + t2 + (lz0 - Cx{L.log_zk_scale, 0.0}) * L.nu;
    }
    const Cx lz{lz0.re + log(pc.r), lz0.im};
    *s = bessel_sum(cexp(lz), L.nu, bad);
    return t1 + t2 + Cx{L.nu * (lz.re - pc.log_zk) - pc.log_s_zk, L.nu * lz.im};
}

// log Phi(a), for the moments at small a.
__device__ Cx log_phi(const ExactLaunch &L, const PhiCtx &pc, double a, bool &bad)
{
    Cx s;
    const Cx lp = log_phi_part(L, pc, a, &s, bad);
    return lp + clog(s);
}

// Phi(a) on the grid: the Bessel sum multiplies instead of entering a logarithm.
__device__ Cx phi(const ExactLaunch &L, const PhiCtx &pc, double a, bool &bad)
{
    Cx s;
    const Cx lp = log_phi_part(L, pc, a, &s, bad);
    return cexp(lp) * s;
}

// Conditional mean and standard deviation of I from log Phi at a = h, 2h.
__device__ void moments(const ExactLaunch &L, const PhiCtx &pc, double &mu, double &sd, bool &bad)
{
    const double guess = fmax(0.5 * (pc.vu + pc.vt) * L.D, 1e-10);
    const double h = 1e-3 / guess;
    const Cx l0 = log_phi(L, pc, h, bad);
    const Cx l1 = log_phi(L, pc, 2.0 * h, bad);
    mu = (8.0 * l0.im - l1.im) / (6.0 * h);
    const double var = -(16.0 * l0.re - l1.re) / (6.0 * h * h);
    sd = sqrt(fmax(var, (1e-3 * mu) * (1e-3 * mu)));
}

// F(x) - u and the density at x from the stored grid (rotation recurrence,
// re-anchored every 64 points).
__device__ void cdf_pdf(const double *col, uint32_t stride, uint32_t K, double h, double x,
                        double &F, double &f)
{
    const double th = h * x;
    double s1, c1;
    sincos(th, &s1, &c1);
    double sf = 0.0, sp = 0.0, sj = 0.0, cj = 1.0;
    for (uint32_t j = 1; j <= K; ++j) {
        if ((j & 63u) == 0u) {
            sincos(th * (double)j, &sj, &cj);
        } else {
            const double sn = sj * c1 + cj * s1;
            cj = cj * c1 - sj * s1;
            sj = sn;
        }
        const double rp = col[(size_t)(j - 1) * stride];
        sf += sj / (double)j * rp;
        sp += cj * rp;
    }
    F = h * x / PI + (2.0 / PI) * sf;
    f = h / PI + (2.0 * h / PI) * sp;
}

// One draw of I given (vu, vt) at the uniform u; `col` is the lane's scratch
// column (stride n_lanes).
__device__ double sample_integral(const ExactLaunch &L, double vu, double vt, double u,
                                  double *col, bool &bad)
{
    PhiCtx pc;
    pc.vu = vu;
    pc.vt = vt;
    pc.sum_v = vu + vt;
    pc.r = sqrt(vu * vt);
    pc.log_zk = 0.0;
    pc.log_s_zk = 0.0;
    if (pc.r != 0.0) {
        pc.log_zk = log(pc.r) + L.log_zk_scale;
        pc.log_s_zk = log(bessel_sum(Cx{exp(pc.log_zk), 0.0}, L.nu, bad).re);
    }
    double mu, sd;
    moments(L, pc, mu, sd, bad);
    const double ueps = mu + 12.0 * sd;
    const double h = PI / ueps;
    const double thr = PI * GRID_EPS / 2.0;
    // grid: doubled from 64 points until |Phi| / J at its last point is below
    // the threshold; kept up to the last point whose |Phi| / j reaches it
    uint32_t J = 64, j = 0, K = 0;
    for (;;) {
        double last = 0.0;
        for (; j < J; ++j) {
            const Cx ph = phi(L, pc, h * (double)(j + 1), bad);
            col[(size_t)j * L.n_lanes] = ph.re;
            last = cabs(ph);
            if (last / (double)(j + 1) >= thr)
                K = j + 1;
        }
        if (last / (double)J < thr)
            break;
        if (J >= EXACT_MAX_GRID || bad) { // the next points would not fit
            bad = true;
            break;
        }
        J *= 2;
    }
    if (K == 0)
        K = 1;
    if (bad || !(ueps > 0.0))
        return __builtin_nan("");
    double lo = 0.0, hi = ueps;
    double x = fmin(fmax(mu, 1e-12), ueps);
    for (int it = 0; it < 200; ++it) {
        double F, f;
        cdf_pdf(col, L.n_lanes, K, h, x, F, f);
        const double e = F - u;
        if (fabs(e) < 1e-13)
            return x;
        if (e > 0.0)
            hi = x;
        else
            lo = x;
        if (hi - lo < 1e-14 * fmax(1.0, hi))
            return x;
        const double xn = f > 0.0 ? x - e / f : 0.5 * (lo + hi);
        x = (lo < xn && xn < hi) ? xn : 0.5 * (lo + hi);
    }
    return x;
}

__global__ __launch_bounds__(BLOCK) void exact_kernel(const ExactLaunch L)
{
    __shared__ double red[BLOCK / 64][EXACT_REC];
    const uint32_t lane = blockIdx.x * BLOCK + threadIdx.x;
    // sums of price, pathwise Delta and Rho (value, square) and the failures
    double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const bool asian = L.opt_type >= 2, geo = L.opt_type >= 4;
    const bool call = L.opt_type == 0 || L.opt_type == 2 || L.opt_type == 4;
    const double sgn = call ? 1.0 : -1.0;
    const double disc = exp(-L.r * L.T), lnS0 = log(L.S0), nfix = (double)L.n_fix;
    const double D = L.D;
    if (lane < L.n_lanes) {
        double *col = L.scratch + lane;
        for (uint64_t i = lane; i < L.n_paths; i += L.n_lanes) {
            const uint64_t p = L.first_path + i;
            Draw dr{(uint32_t)p, (uint32_t)(p >> 32), 0u, (uint32_t)L.seed,
                    (uint32_t)(L.seed >> 32)};
            double x = 0.0, V = L.v0, A = 0.0, B = 0.0, Itot = 0.0;
            bool bad = false;
            for (uint32_t j = 0; j < L.n_steps && !bad; ++j) {
                dr.step = j;
                const U4 w = dr.block(0);
                double zv, zs;
                box_muller(uniform_f64(w.x), uniform_f64(w.y), zv, zs);
                const double lam = V * L.ekD / L.c;
                double X;
                if (L.d > 1.0) {
                    const double sq = zv + sqrt(lam);
                    X = 2.0 * gamma_draw(0.5 * (L.d - 1.0), dr) + sq * sq;
                } else {
                    const double n = poisson_inverse(0.5 * lam, uniform_f64(w.w));
                    X = n == n ? 2.0 * gamma_draw(0.5 * L.d + n, dr) : __builtin_nan("");
                }
                const double vt = L.c * X;
                if (!(vt >= 0.0)) {
                    bad = true;
                    break;
                }
                const double I = sample_integral(L, V, vt, uniform_f64(w.z), col, bad);
                if (bad)
                    break;
                Itot += I;
                const double isq = (vt - V - L.kappa * L.theta * D + L.kappa * I) / L.sigma;
                x += L.r * D - 0.5 * I + L.rho * isq + L.rho_bar * sqrt(fmax(I, 0.0)) * zs;
                V = vt;
                if (asian && is_fixing(L.fix_bits, j + 1)) {
                    const double t = (double)(j + 1) * D;
                    if (geo) {
                        A += lnS0 + x;
                        B += t;
                    } else {
                        const double S = L.S0 * exp(x);
                        A += S;
                        B += t * S;
                    }
                }
            }
            const double ST = L.S0 * exp(x);
            const double Xv = geo ? exp(A / nfix) : asian ? A / nfix : ST;
            if (geo)
                B = Xv * B;
            const bool itm = sgn * (Xv - L.K) > 0.0;
            double est[3];
            est[0] = itm ? disc * sgn * (Xv - L.K) : 0.0;
            est[1] = itm ? sgn * disc * Xv / L.S0 : 0.0;
            est[2] = !itm ? 0.0
                     : asian ? disc * (sgn * B / nfix - L.T * sgn * (Xv - L.K))
                             : sgn * disc * L.K * L.T;
            if (bad) {
                acc[6] += 1.0;
            } else {
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    acc[2 * e] += est[e];
                    acc[2 * e + 1] += est[e] * est[e];
                }
            }
            if (L.dump != nullptr) {
                double *rec = L.dump + i * DUMP_WIDTH;
                const double nan = __builtin_nan("");
                rec[0] = bad ? nan : ST;
                rec[1] = bad ? nan : V;
                rec[2] = bad ? nan : Xv;
                rec[3] = bad ? nan : est[0];
                rec[4] = bad ? nan : est[1];
                rec[5] = bad ? nan : est[2];
#pragma unroll
                for (int k = 6; k < 14; ++k)
                    rec[k] = nan;
                rec[14] = bad ? nan : x;
                rec[15] = bad ? nan : Itot;
            }
        }
    }
    const int wl = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < EXACT_REC; ++k) {
        const double v = k < 6 ? acc[k] : k == N_ACC ? acc[6] : 0.0;
        const double s = wave_sum(v);
        if (wl == 0)
            red[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < EXACT_REC) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w)
            s += red[w][threadIdx.x];
        L.partials[(uint64_t)blockIdx.x * EXACT_REC + threadIdx.x] = s;
    }
}

} // namespace

hipError_t launch_exact(const ExactLaunch &L, hipStream_t stream)
{
    if (L.n_lanes == 0 || L.n_lanes % BLOCK != 0 || L.n_lanes > EXACT_MAX_LANES)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(exact_kernel, dim3(L.n_lanes / BLOCK), dim3(BLOCK), 0, stream, L);
    return hipGetLastError();
}

} // namespace heston
