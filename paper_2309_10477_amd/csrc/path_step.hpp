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
// otherwise absorption (V clamped at 0 after the step).  sdt is the time step
// under the square root: dt, or dt NS^2 with scaled normals (NormalScale).
// Returns the variance before the absorption clamp.
template <class R, bool FT>
__device__ __forceinline__ R mil_step(R &x, R &v, const Coef<R> &c, R z1, R sz2, R mil, R sdt)
{
    const R vp = v > R(0) ? v : R(0);
    const R s = fast_sqrt(vp * sdt);
    x += (c.r_dt - c.half_dt * vp) + s * z1;
    const R vb = FT ? v : vp;
    const R pre = vb + (c.ktdt - c.kdt * vp) + sz2 * s + mil;
    v = FT ? pre : (pre > R(0) ? pre : R(0));
    return pre;
}

// Step j+1 is a fixing date (every step when the mask is absent).
__device__ __forceinline__ bool is_fixing(const uint32_t *fix_bits, uint32_t jf)
{
    return fix_bits == nullptr || ((fix_bits[jf >> 5] >> (jf & 31u)) & 1u);
}

// Normals of steps (j, j+1) from one Philox block: counter (j >> 1, lo32 p, hi32 p, 0).
// LOG2_SCALED (single precision only): the normals come divided by
// sqrt(2 ln 2) (box_muller_log2).
template <class R, bool LOG2_SCALED = false>
__device__ __forceinline__ void philox_normals(uint32_t j, uint32_t plo, uint32_t phi, uint32_t k0,
                                               uint32_t k1, R &za0, R &zb0, R &za1, R &zb1)
{
    const U4 w = philox4x32_10(U4{j >> 1, plo, phi, 0u}, k0, k1);
    if constexpr (sizeof(R) == 4 && LOG2_SCALED) {
        box_muller_log2(uniform_f32(w.x), uniform_f32(w.y), za0, zb0);
        box_muller_log2(uniform_f32(w.z), uniform_f32(w.w), za1, zb1);
    } else if constexpr (sizeof(R) == 4) {
        box_muller(uniform_f32(w.x), uniform_f32(w.y), za0, zb0);
        box_muller(uniform_f32(w.z), uniform_f32(w.w), za1, zb1);
    } else {
        box_muller(uniform_f64(w.x), uniform_f64(w.y), za0, zb0);
        box_muller(uniform_f64(w.z), uniform_f64(w.w), za1, zb1);
    }
}

// Constants that multiply the normals.  Single precision takes its Philox
// normals divided by NS = sqrt(2 ln 2) (box_muller_log2) and folds NS into
// them: rho and rho_bar turn the scaled pair into Z2; the square root is taken
// of V+ dt NS^2, which puts NS onto the log-price's Z1; sigma / NS then leaves
// the variance diffusion sigma Z2 sqrt(V+ dt) unchanged.  Double precision
// keeps the plain normals (NS = 1).
template <class R> struct NormalScale {
    R rho, rho_bar, sigma, sdt, ns;
};
template <class R> __device__ __forceinline__ NormalScale<R> normal_scale(const PathConsts &k)
{
    const double ns = sizeof(R) == 4 ? SQRT_2LN2 : 1.0;
    return NormalScale<R>{(R)(k.rho * ns), (R)(k.rho_bar * ns), (R)(k.sigma / ns),
                          (R)(k.c.dt * ns * ns), (R)ns};
}

__host__ __device__ inline PathConsts path_consts(const PriceLaunch &L)
{
    PathConsts k;
    k.c = L.base;
    k.S0 = L.S0;
    k.K = L.K;
    k.r = L.r;
    k.T = L.T;
    k.v0 = L.v0;
    k.rho = L.rho;
    k.rho_bar = L.rho_bar;
    k.sigma = L.sigma;
    k.theta = L.theta;
    k.seed = L.seed;
    k.fix_bits = L.fix_bits;
    k.n_steps = L.n_steps;
    k.n_fix = L.n_fix;
    k.type = L.opt_type;
    k.wide = L.wide_paths ? 1u : 0u;
    return k;
}

// One path's forward pass (single scenario): x_N, V_N, the fixing sums
// A = sum e^x and B = sum t e^x; when ck is set, stores (x, V) before steps
// 0, every, 2 every, ... and the final (x_N, A) in the checkpoint layout
// with `stride` paths per row.
template <class R, bool ASIAN, bool FT>
__device__ __forceinline__ void forward_path(const PathConsts &k, uint64_t p, R &x, R &v, R &A,
                                             R &B, R *ck, uint64_t stride, uint64_t row,
                                             uint32_t every)
{
    const Coef<R> c = coef<R>(k.c);
    const NormalScale<R> ns = normal_scale<R>(k);
    const uint32_t k0 = (uint32_t)k.seed, k1 = (uint32_t)(k.seed >> 32);
    const uint32_t plo = (uint32_t)p, phi = k.wide ? (uint32_t)(p >> 32) : 0u;
    const uint32_t N = k.n_steps;
    x = R(0);
    v = (R)k.v0;
    A = R(0);
    B = R(0);
    auto step = [&](uint32_t j, R za, R zb) {
        const R z2 = ns.rho * za + ns.rho_bar * zb;
        mil_step<R, FT>(x, v, c, za, ns.sigma * z2, c.qdt * (z2 * z2 - R(1)), ns.sdt);
        if constexpr (ASIAN) {
            if (is_fixing(k.fix_bits, j + 1)) {
                const R e = fast_exp(x);
                A += e;
                B += (R)(j + 1) * c.dt * e;
            }
        }
    };
    for (uint32_t j = 0; j < N; j += 2) {
        if (ck != nullptr && j % every == 0) {
            const uint64_t cc = j / every;
            ck[(2 * cc) * stride + row] = x;
            ck[(2 * cc + 1) * stride + row] = v;
        }
        R za0, zb0, za1, zb1;
        philox_normals<R, sizeof(R) == 4>(j, plo, phi, k0, k1, za0, zb0, za1, zb1);
        step(j, za0, zb0);
        if (j + 1 < N)
            step(j + 1, za1, zb1);
    }
    if (ck != nullptr) {
        const uint64_t cc = ckpt_count(N, every);
        ck[(2 * cc) * stride + row] = x;
        ck[(2 * cc + 1) * stride + row] = A;
    }
}

// Discounted payoff and the paper's pathwise Delta / Rho of one path, in FP64.
template <bool ASIAN>
__device__ __forceinline__ void path_estimators(const PathConsts &k, double x, double A, double B,
                                                double &pay, double &pw_delta, double &pw_rho)
{
    const double D = exp(-k.r * k.T);
    const double inv_nfix = 1.0 / (double)k.n_fix;
    const double rel = ASIAN ? A * inv_nfix : exp(x);
    const double X = k.S0 * rel;
    const bool call = k.type == 0 || k.type == 2;
    const double sgn = call ? 1.0 : -1.0;
    const double in = sgn * (X - k.K);
    const bool itm = in > 0.0;
    pay = itm ? D * in : 0.0;
    pw_delta = itm ? sgn * D * rel : 0.0;
    if (ASIAN)
        pw_rho = itm ? D * (sgn * k.S0 * B * inv_nfix - k.T * in) : 0.0;
    else
        pw_rho = itm ? sgn * D * k.K * k.T : 0.0;
}

// Reverse sweep of one path over its checkpoints (see adjoint_kernel.hip):
// out = (payoff, d/dS0, d/dv0, d/dr, d/dkappa, d/dtheta, d/dsigma, d/drho).
template <class R, bool ASIAN, bool FT, int SEG>
__device__ __forceinline__ void adjoint_path(const PathConsts &k, uint64_t p, const R *ck,
                                             uint64_t stride, uint64_t row, double out[8])
{
    const uint32_t N = k.n_steps;
    const uint64_t nck = ckpt_count(N, SEG);
    const Coef<R> c = coef<R>(k.c);
    const NormalScale<R> ns = normal_scale<R>(k);
    const R sigma = (R)k.sigma, theta = (R)k.theta;
    const R half_dt_ns = (R)(0.5 * k.c.dt * (double)ns.ns); // ds/dV+ = half_dt_ns rs / NS
    const R rho_ratio = (R)(k.rho_bar > 0 ? k.rho / k.rho_bar : 0.0); // -d rho_bar / d rho
    const R half_sigma_dt = (R)(0.5 * k.sigma * k.c.dt);              // d(qdt)/d sigma
    const R two_qdt = (R)(2.0 * k.c.quarter_sigma2_dt);
    const uint32_t k0 = (uint32_t)k.seed, k1 = (uint32_t)(k.seed >> 32);
    const uint32_t plo = (uint32_t)p, phi = k.wide ? (uint32_t)(p >> 32) : 0u;

    // payoff and its seeds (FP64, as in the pricing epilogue)
    const double S0 = k.S0, D = exp(-k.r * k.T), inv_nfix = 1.0 / (double)k.n_fix;
    const R xN = ck[(2 * nck) * stride + row];
    const R AN = ck[(2 * nck + 1) * stride + row];
    const double rel = ASIAN ? (double)AN * inv_nfix : exp((double)xN);
    const double X = S0 * rel;
    const bool call = k.type == 0 || k.type == 2;
    const double sgn = call ? 1.0 : -1.0;
    const double in = sgn * (X - k.K);
    const bool itm = in > 0.0;
    const double y = itm ? D * in : 0.0;
    const double g_S0 = itm ? sgn * D * rel : 0.0;
    const R c_fix = (R)(itm ? sgn * D * S0 * inv_nfix : 0.0); // dy / d e^{x_i} at a fixing

    R xbar = (!ASIAN && itm) ? (R)(sgn * D * X) : R(0); // dy/dx_N for a European
    R vbar = 0, sum_xbar = 0, kbar = 0, thbar = 0, sbar = 0, rhobar = 0;

    for (int64_t seg = (int64_t)nck - 1; seg >= 0; --seg) {
        const uint32_t s0 = (uint32_t)seg * SEG;
        const uint32_t len = N - s0 < (uint32_t)SEG ? N - s0 : (uint32_t)SEG;
        R x = ck[(2 * (uint64_t)seg) * stride + row];
        R v = ck[(2 * (uint64_t)seg + 1) * stride + row];
        R a_vp[SEG], a_za[SEG], a_zb[SEG], a_f[SEG];
        bool a_clip[SEG];
        // forward recomputation of the segment
#pragma unroll
        for (int q = 0; q < SEG; q += 2) {
            if ((uint32_t)q < len) {
                R za[2], zb[2];
                philox_normals<R, sizeof(R) == 4>(s0 + q, plo, phi, k0, k1, za[0], zb[0], za[1],
                                                  zb[1]);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int qq = q + h;
                    if ((uint32_t)qq < len) {
                        const R z2 = ns.rho * za[h] + ns.rho_bar * zb[h];
                        const R vp = v > R(0) ? v : R(0);
                        a_vp[qq] = vp;
                        a_za[qq] = za[h];
                        a_zb[qq] = zb[h];
                        // the clip flag comes from the very value the step clamped
                        const R vpre = mil_step<R, FT>(x, v, c, za[h], ns.sigma * z2,
                                                       c.qdt * (z2 * z2 - R(1)), ns.sdt);
                        a_clip[qq] = !FT && !(vpre > R(0));
                        a_f[qq] = (ASIAN && is_fixing(k.fix_bits, s0 + qq + 1)) ? c_fix * fast_exp(x)
                                                                               : R(0);
                    }
                }
            }
        }
        // reverse sweep
#pragma unroll
        for (int q = SEG - 1; q >= 0; --q) {
            if ((uint32_t)q < len) {
                xbar += a_f[q]; // now the adjoint of x_{j+1}
                if (!FT && a_clip[q])
                    vbar = R(0); // V_{j+1} = max(pre, 0) with pre <= 0
                sum_xbar += xbar;
                // za, zb are the scaled normals (true ones times 1 / NS)
                const R vp = a_vp[q], za = a_za[q], zb = a_zb[q];
                const R z2 = ns.rho * za + ns.rho_bar * zb;
                const R dz2 = za - rho_ratio * zb; // dZ2/drho / NS
                const bool pos = vp > R(0);
                // s = sqrt(V+ dt) and NS ds/dV+ = NS dt / (2 s) from one reciprocal
                // square root
                const R s2 = vp * c.dt;
                const R rs = pos ? fast_rsqrt(s2) : R(0);
                const R s = s2 * rs;
                const R dsdv = half_dt_ns * rs;
                const R g = xbar * (za * dsdv - c.half_dt) + vbar * (ns.sigma * z2 * dsdv - c.kdt);
                kbar += vbar * (theta - vp);
                thbar += vbar;
                sbar += vbar * (s * z2 + half_sigma_dt * (z2 * z2 - R(1)));
                rhobar += vbar * (sigma * s + two_qdt * z2) * dz2;
                vbar = FT ? vbar + (pos ? g : R(0)) : (pos ? vbar + g : R(0));
            }
        }
    }
    out[0] = y;
    out[1] = g_S0;
    out[2] = (double)vbar;
    out[3] = (double)sum_xbar * k.c.dt - k.T * y;
    out[4] = (double)kbar * k.c.dt;
    out[5] = (double)thbar * k.c.kappa_dt;
    out[6] = (double)sbar;
    out[7] = (double)rhobar * (double)ns.ns;
}


// ---------------------------------------------------------------------------
// Andersen's QE scheme in the adjoint skeleton (the paper's Future Work; L.
// Andersen, "Simple and efficient simulation of the Heston stochastic
// volatility model", 2008): the same Philox inputs, checkpoints and reductions
// as the Milstein adjoint, with the variance step and the log-price step of
// QE.  State (x = ln S/S0, V) unscaled; inputs of step j from one Philox block
// with counter (j, lo32 p, hi32 p, QE_COUNTER_TAG): words 0, 1 give the
// Box-Muller pair (Zs for the log-price, Zv for the quadratic branch), word 2
// the uniform Uv of the exponential branch.
//   m = E V + theta (1 - E), s2 = cs1 V + cs0, psi = s2 / m^2, E = e^{-kappa dt},
//   cs1 = sigma^2 E (1 - E) / kappa, cs0 = theta sigma^2 (1 - E)^2 / (2 kappa);
//   psi <= 3/2: V' = a (b + Zv)^2, b^2 = 2/psi - 1 + sqrt(2/psi (2/psi - 1)),
//               a = m / (1 + b^2);
//   else:       p = (psi - 1) / (psi + 1), V' = 0 if Uv <= p, else
//               V' = m / (1 - p) ln((1 - p) / (1 - Uv));
//   x' = x + r dt + K0 + K1 V + K2 V' + sqrt(Kq (V + V')) Zs  (central weights 1/2:
//   K0 = -rho kappa theta dt / sigma, K1,2 = dt (kappa rho / sigma - 1/2) / 2 -/+ rho / sigma,
//   Kq = dt (1 - rho^2) / 2).
constexpr double QE_PSI_C = 1.5;

template <class R> struct QECoef {
    R E, mth, cs1, cs0, K0, K1, K2, Kq, r_dt, dt;
    // partial derivatives, in the order (kappa, theta, sigma, rho) where used
    R dE_k, dmth_k, dmth_t, dcs1_k, dcs1_s, dcs0_k, dcs0_t, dcs0_s;
    R dK0[4], dK1[4], dK2[4], dKq_r;
};

template <class R> __device__ __forceinline__ QECoef<R> qe_coef(const PathConsts &k)
{
    const double dt = k.c.dt, kap = k.c.kappa_dt / dt, th = k.theta, sig = k.sigma, rho = k.rho;
    const double E = exp(-kap * dt), dE = -dt * E, s2s = sig * sig;
    const double A1 = E * (1.0 - E) / kap, A0 = (1.0 - E) * (1.0 - E) / (2.0 * kap);
    const double dA1 = dE * (1.0 - 2.0 * E) / kap - A1 / kap;
    const double dA0 = -(1.0 - E) * dE / kap - A0 / kap;
    const double c = kap * rho / sig - 0.5;
    const double dc[4] = {rho / sig, 0.0, -kap * rho / (sig * sig), kap / sig};
    QECoef<R> q;
    q.E = (R)E;
    q.mth = (R)(th * (1.0 - E));
    q.cs1 = (R)(s2s * A1);
    q.cs0 = (R)(th * s2s * A0);
    q.K0 = (R)(-rho * kap * th * dt / sig);
    q.K1 = (R)(0.5 * dt * c - rho / sig);
    q.K2 = (R)(0.5 * dt * c + rho / sig);
    q.Kq = (R)(0.5 * dt * (1.0 - rho * rho));
    q.r_dt = (R)k.c.r_dt;
    q.dt = (R)dt;
    q.dE_k = (R)dE;
    q.dmth_k = (R)(-th * dE);
    q.dmth_t = (R)(1.0 - E);
    q.dcs1_k = (R)(s2s * dA1);
    q.dcs1_s = (R)(2.0 * sig * A1);
    q.dcs0_k = (R)(th * s2s * dA0);
    q.dcs0_t = (R)(s2s * A0);
    q.dcs0_s = (R)(2.0 * sig * th * A0);
    const double dK0[4] = {-rho * th * dt / sig, -rho * kap * dt / sig, rho * kap * th * dt / s2s,
                           -kap * th * dt / sig};
    const double dR[4] = {0.0, 0.0, rho / s2s, -1.0 / sig}; // d(-rho / sigma)
    for (int i = 0; i < 4; ++i) {
        q.dK0[i] = (R)dK0[i];
        q.dK1[i] = (R)(0.5 * dt * dc[i] + dR[i]);
        q.dK2[i] = (R)(0.5 * dt * dc[i] - dR[i]);
    }
    q.dKq_r = (R)(-dt * rho);
    return q;
}

// The QE inputs of step j: (Zs, Zv, Uv).
template <class R>
__device__ __forceinline__ void qe_draws(uint32_t j, uint32_t plo, uint32_t phi, uint32_t k0,
                                         uint32_t k1, R &zs, R &zv, R &uv)
{
    const U4 w = philox4x32_10(U4{j, plo, phi, QE_COUNTER_TAG}, k0, k1);
    if constexpr (sizeof(R) == 4) {
        box_muller(uniform_f32(w.x), uniform_f32(w.y), zs, zv);
        uv = uniform_f32(w.z);
    } else {
        box_muller(uniform_f64(w.x), uniform_f64(w.y), zs, zv);
        uv = uniform_f64(w.z);
    }
}

__device__ __forceinline__ float qe_log(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994530942f; }
__device__ __forceinline__ double qe_log(double x) { return log(x); }

// b + Zv as a plain rounded sum, never contracted with the Box-Muller product
// that made Zv: the reverse sweep recomputes the step from the stored (rounded)
// Zv, and where b + Zv cancels, V' = a (b + Zv)^2 taken from an FMA with the
// unrounded product would differ from that recomputation by far more than a
// rounding of V' (its relative change is 2 ulp(Zv) / |b + Zv|).
template <class R> __device__ __forceinline__ R qe_shift(R b, R zv)
{
#pragma clang fp contract(off)
    return b + zv;
}

// The variance step: V' and (in *quad) the branch it took.
template <class R>
__device__ __forceinline__ R qe_variance_step(const QECoef<R> &q, R v, R zv, R uv, bool &quad)
{
    const R m = q.E * v + q.mth, s2 = q.cs1 * v + q.cs0;
    const R psi = s2 / (m * m);
    quad = psi <= (R)QE_PSI_C;
    if (quad) {
        const R inv = R(2) / psi;
        const R b2 = inv - R(1) + fast_sqrt(inv * (inv - R(1)));
        const R bz = qe_shift(fast_sqrt(b2), zv);
        return m / (R(1) + b2) * bz * bz;
    }
    const R p = (psi - R(1)) / (psi + R(1));
    return uv <= p ? R(0) : m / (R(1) - p) * qe_log((R(1) - p) / (R(1) - uv));
}

// One QE step of (x, V); returns the step's branch-dependent random input
// (Zv in the quadratic branch, Uv in the exponential one), which with V and
// Zs is all the reverse sweep needs.
template <class R>
__device__ __forceinline__ R qe_step(R &x, R &v, const QECoef<R> &q, R zs, R zv, R uv)
{
    bool quad;
    const R vn = qe_variance_step(q, v, zv, uv, quad);
    x += q.r_dt + q.K0 + q.K1 * v + q.K2 * vn + fast_sqrt(q.Kq * (v + vn)) * zs;
    v = vn;
    return quad ? zv : uv;
}

// Forward pass under QE, as forward_path (same checkpoint layout).
template <class R, bool ASIAN>
__device__ __forceinline__ void forward_path_qe(const PathConsts &k, uint64_t p, R &x, R &v, R &A,
                                                R &B, R *ck, uint64_t stride, uint64_t row,
                                                uint32_t every)
{
    const QECoef<R> q = qe_coef<R>(k);
    const uint32_t k0 = (uint32_t)k.seed, k1 = (uint32_t)(k.seed >> 32);
    const uint32_t plo = (uint32_t)p, phi = k.wide ? (uint32_t)(p >> 32) : 0u;
    const uint32_t N = k.n_steps;
    x = R(0);
    v = (R)k.v0;
    A = R(0);
    B = R(0);
    for (uint32_t j = 0; j < N; ++j) {
        if (ck != nullptr && j % every == 0) {
            const uint64_t cc = j / every;
            ck[(2 * cc) * stride + row] = x;
            ck[(2 * cc + 1) * stride + row] = v;
        }
        R zs, zv, uv;
        qe_draws<R>(j, plo, phi, k0, k1, zs, zv, uv);
        qe_step(x, v, q, zs, zv, uv);
        if constexpr (ASIAN) {
            if (is_fixing(k.fix_bits, j + 1)) {
                const R e = fast_exp(x);
                A += e;
                B += (R)(j + 1) * q.dt * e;
            }
        }
    }
    if (ck != nullptr) {
        const uint64_t cc = ckpt_count(N, every);
        ck[(2 * cc) * stride + row] = x;
        ck[(2 * cc + 1) * stride + row] = A;
    }
}

// Reverse sweep under QE (see adjoint_path): per segment the steps are
// recomputed from the checkpoint, keeping V, Zs, the branch input and the
// fixing term; the reverse step recomputes m, s2, psi, the branch and V' from
// V and differentiates them with the branch held fixed.
template <class R, bool ASIAN, int SEG>
__device__ __forceinline__ void adjoint_path_qe(const PathConsts &k, uint64_t p, const R *ck,
                                                uint64_t stride, uint64_t row, double out[8])
{
    const uint32_t N = k.n_steps;
    const uint64_t nck = ckpt_count(N, SEG);
    const QECoef<R> q = qe_coef<R>(k);
    const uint32_t k0 = (uint32_t)k.seed, k1 = (uint32_t)(k.seed >> 32);
    const uint32_t plo = (uint32_t)p, phi = k.wide ? (uint32_t)(p >> 32) : 0u;

    const double S0 = k.S0, D = exp(-k.r * k.T), inv_nfix = 1.0 / (double)k.n_fix;
    const R xN = ck[(2 * nck) * stride + row];
    const R AN = ck[(2 * nck + 1) * stride + row];
    const double rel = ASIAN ? (double)AN * inv_nfix : exp((double)xN);
    const double X = S0 * rel;
    const bool call = k.type == 0 || k.type == 2;
    const double sgn = call ? 1.0 : -1.0;
    const double in = sgn * (X - k.K);
    const bool itm = in > 0.0;
    const double y = itm ? D * in : 0.0;
    const double g_S0 = itm ? sgn * D * rel : 0.0;
    const R c_fix = (R)(itm ? sgn * D * S0 * inv_nfix : 0.0);

    R xbar = (!ASIAN && itm) ? (R)(sgn * D * X) : R(0);
    R vbar = 0, sum_xbar = 0, kbar = 0, thbar = 0, sbar = 0, rhobar = 0;

    for (int64_t seg = (int64_t)nck - 1; seg >= 0; --seg) {
        const uint32_t s0 = (uint32_t)seg * SEG;
        const uint32_t len = N - s0 < (uint32_t)SEG ? N - s0 : (uint32_t)SEG;
        R x = ck[(2 * (uint64_t)seg) * stride + row];
        R v = ck[(2 * (uint64_t)seg + 1) * stride + row];
        R a_v[SEG], a_zs[SEG], a_u[SEG], a_f[SEG];
#pragma unroll
        for (int qq = 0; qq < SEG; ++qq) {
            if ((uint32_t)qq < len) {
                R zs, zv, uv;
                qe_draws<R>(s0 + qq, plo, phi, k0, k1, zs, zv, uv);
                a_v[qq] = v;
                a_zs[qq] = zs;
                a_u[qq] = qe_step(x, v, q, zs, zv, uv);
                a_f[qq] = (ASIAN && is_fixing(k.fix_bits, s0 + qq + 1)) ? c_fix * fast_exp(x) : R(0);
            }
        }
#pragma unroll
        for (int qq = SEG - 1; qq >= 0; --qq) {
            if ((uint32_t)qq < len) {
                xbar += a_f[qq]; // the adjoint of x_{j+1}
                sum_xbar += xbar;
                const R vj = a_v[qq], zs = a_zs[qq], u = a_u[qq];
                // recompute the step
                const R m = q.E * vj + q.mth, s2 = q.cs1 * vj + q.cs0;
                const R psi = s2 / (m * m);
                R vn, dvn_dm, dvn_ds2;
                if (psi <= (R)QE_PSI_C) {
                    const R inv = R(2) / psi;
                    const R r = fast_sqrt(inv * (inv - R(1)));
                    const R b2 = inv - R(1) + r;
                    const R b = fast_sqrt(b2);
                    const R g = qe_shift(b, u); // u = Zv
                    const R a = m / (R(1) + b2);
                    vn = a * g * g;
                    // dV'/db2 at fixed m, then through inv = 2 m^2 / s2
                    const R dvn_db2 = a * g / b - vn / (R(1) + b2);
                    const R db2_dinv = R(1) + (R(2) * inv - R(1)) / (R(2) * r);
                    const R t = dvn_db2 * db2_dinv;
                    dvn_dm = g * g / (R(1) + b2) + t * (R(2) * inv / m);
                    dvn_ds2 = -t * inv / s2;
                } else {
                    const R p = (psi - R(1)) / (psi + R(1));
                    if (u <= p) { // u = Uv: the point mass at zero
                        vn = R(0);
                        dvn_dm = R(0);
                        dvn_ds2 = R(0);
                    } else {
                        const R L = qe_log((R(1) - p) / (R(1) - u));
                        const R om = R(1) / (R(1) - p);
                        vn = m * om * L;
                        // dV'/dp = m (L - 1) / (1-p)^2, dp/dpsi = 2 / (psi+1)^2
                        const R dvn_dpsi = m * (L - R(1)) * om * om * (R(2) / ((psi + R(1)) * (psi + R(1))));
                        dvn_dm = om * L - dvn_dpsi * (R(2) * psi / m);
                        dvn_ds2 = dvn_dpsi / (m * m);
                    }
                }
                // log-price step: x' = x + r dt + K0 + K1 V + K2 V' + sqrt(Kq (V + V')) Zs
                const R qv = q.Kq * (vj + vn);
                const R sq = fast_sqrt(qv);
                const R dsq = qv > R(0) ? R(0.5) / sq : R(0); // d sqrt / d(qv)
                const R vnbar = vbar + xbar * (q.K2 + q.Kq * dsq * zs);
                const R vbar_x = xbar * (q.K1 + q.Kq * dsq * zs);
                const R sdq = xbar * zs * dsq * (vj + vn); // adjoint of Kq
                kbar += xbar * (q.dK0[0] + q.dK1[0] * vj + q.dK2[0] * vn);
                thbar += xbar * (q.dK0[1] + q.dK1[1] * vj + q.dK2[1] * vn);
                sbar += xbar * (q.dK0[2] + q.dK1[2] * vj + q.dK2[2] * vn);
                rhobar += xbar * (q.dK0[3] + q.dK1[3] * vj + q.dK2[3] * vn) + sdq * q.dKq_r;
                // variance step
                const R mbar = vnbar * dvn_dm, s2bar = vnbar * dvn_ds2;
                kbar += mbar * (q.dE_k * vj + q.dmth_k) + s2bar * (q.dcs1_k * vj + q.dcs0_k);
                thbar += mbar * q.dmth_t + s2bar * q.dcs0_t;
                sbar += s2bar * (q.dcs1_s * vj + q.dcs0_s);
                vbar = vbar_x + mbar * q.E + s2bar * q.cs1;
            }
        }
    }
    out[0] = y;
    out[1] = g_S0;
    out[2] = (double)vbar;
    out[3] = (double)sum_xbar * k.c.dt - k.T * y;
    out[4] = (double)kbar;
    out[5] = (double)thbar;
    out[6] = (double)sbar;
    out[7] = (double)rhobar;
}

} // namespace heston
