// Pricing kernel: Milstein paths of the Heston model, payoffs, pathwise and
// bump-and-revalue Greek samples, and their FP64 cross-path sums.
//
// Paper mapping:
//  - normals and their correlation: Background, algorithm "Generation of two
//    correlated Normal random variables" (Z1 = Za, Z2 = rho Za + rho_bar Zb);
//  - the step: algorithm "Milstein approximation under Heston model" -- the
//    log-price step has no Milstein term, the variance step carries
//    1/4 sigma^2 dt (Z2^2 - 1); truncation by absorption (the paper's
//    V <- max(V, 0)) or full truncation;
//  - payoffs and discounting: Background (European/Asian payoffs, risk-neutral
//    pricing) and algorithm "Monte Carlo option pricing estimation";
//  - pathwise Delta/Rho: section "Pathwise method for greeks estimation".
//
// One path per lane, all path state in VGPRs; x = ln(S/S0) is carried instead
// of S (the log-price form of the step, which the paper derives before
// exponentiating).  Nothing per step touches HBM: Philox normals are generated
// in registers; Sobol normals come from direction numbers read through the
// scalar cache and a Brownian-bridge stack in LDS.  Each block writes one FP64
// partial record; a second kernel sums the partials in a fixed order.
#include <type_traits>

#include "device_math.hpp"
#include "internal.hpp"
#include "path_step.hpp"

namespace heston {
namespace {

struct Payoff {
    int type;
    double K, inv_nfix;
    __device__ __forceinline__ bool call() const { return type == 0 || type == 2 || type == 4; }
    __device__ __forceinline__ double operator()(double D, double X) const
    {
        const double in = call() ? X - K : K - X;
        return in > 0.0 ? D * in : 0.0;
    }
};

// Sobol coordinate d of point with Gray code g, digitally shifted; 30-bit.
__device__ __forceinline__ uint32_t sobol_coord(const uint32_t *__restrict__ dirs, uint32_t d,
                                                uint32_t g, int nbits, uint32_t shift)
{
    uint32_t x = shift;
    const uint32_t *v = dirs + 32u * d;
    for (int b = 0; b < nbits; ++b)
        x ^= ((g >> b) & 1u) ? v[b] : 0u;
    return x;
}

// Standard normal of the 30-bit coordinate x, u = (x + 1/2) 2^-30.  The upper
// half is mapped through its exact complement, z = -Phi^{-1}(1 - u), so that
// single precision keeps full relative precision in both tails.
template <class R>
__device__ __forceinline__ void sobol_normals(uint32_t x0, uint32_t x1, R &z0, R &z1)
{
    if constexpr (sizeof(R) == 4) {
        // bit 29 marks the upper half: m is all ones there, and the mirror
        // 0x3FFFFFFF - x of a 30-bit x is x with its 30 bits complemented
        // (one bitop3: (m & 0x3FFFFFFF) ^ x); the sign is restored by flipping
        // the float's sign bit (no selects)
        const uint32_t m0 = (uint32_t)__builtin_amdgcn_sbfe((int)x0, 29, 1);
        const uint32_t m1 = (uint32_t)__builtin_amdgcn_sbfe((int)x1, 29, 1);
        float a, b;
        inv_normal_lower_bits2(__builtin_amdgcn_bitop3_b32(m0, 0x3FFFFFFFu, x0, 0x6A),
                               __builtin_amdgcn_bitop3_b32(m1, 0x3FFFFFFFu, x1, 0x6A), a, b);
        z0 = __uint_as_float(__float_as_uint(a) ^ (m0 & 0x80000000u));
        z1 = __uint_as_float(__float_as_uint(b) ^ (m1 & 0x80000000u));
    } else {
        auto one = [](uint32_t x) {
            const bool upper = x >= (1u << 29);
            const uint32_t xs = upper ? 0x3FFFFFFFu - x : x;
            const R z = inv_normal_lower(((R)xs + R(0.5)) * R(0x1p-30));
            return upper ? -z : z;
        };
        z0 = one(x0);
        z1 = one(x1);
    }
}

// The low six Gray-code bits of a lane's point select direction numbers
// v[0..5]; `m` holds all-ones or zero masks for them.
__device__ __forceinline__ uint32_t sobol_low(const uint32_t *__restrict__ v, const uint32_t m[6])
{
    uint32_t x = m[0] & v[0];
#pragma unroll
    for (int b = 1; b < 6; ++b)
        x = __builtin_amdgcn_bitop3_b32(m[b], v[b], x, 0x6A); // (m & v) ^ x
    return x;
}

// The fused kernel carries each scenario's state scaled: y = ln(S/S0) / ln 2,
// so the fixing exponential is a single exp2, and w = V dt, so the diffusion
// coefficient is sqrt(w+); the constants of each time grid absorb the scales.
// Per step and scenario this is the same Milstein step (paper: algorithm
// "Milstein approximation under Heston model") multiplied through by 1/ln 2
// and by dt respectively.
constexpr double LOG2E = 1.4426950408889634074;
constexpr double LN2 = 0.69314718055994530942;

template <class R> struct Grid {
    R kdt;   // kappa dt
    R ktdt2; // kappa theta dt^2
    R qdt2;  // sigma^2 dt^2 / 4
    R sdt;   // sigma dt
    R dt;
    R kdt_h; // kappa dt / 2
};

template <class R> __device__ __forceinline__ Grid<R> grid(const StepCoef &c, double sigma)
{
    return Grid<R>{(R)c.kappa_dt, (R)(c.kappa_theta_dt * c.dt), (R)(c.quarter_sigma2_dt * c.dt),
                   (R)(sigma * c.dt), (R)c.dt, (R)(0.5 * c.kappa_dt)};
}

// max(w, 0) as one v_med3 (no NaN canonicalisation of the loop-carried w).
__device__ __forceinline__ float clamp0(float w) { return __builtin_amdgcn_fmed3f(w, 0.0f, 3.0e38f); }
__device__ __forceinline__ double clamp0(double w) { return w > 0.0 ? w : 0.0; }
__device__ __forceinline__ float exp2r(float y) { return __builtin_amdgcn_exp2f(y); }
__device__ __forceinline__ double exp2r(double y) { return exp2(y); }

// One scaled step on grid g; z1l = Z1 / ln 2, a_g = kappa theta dt^2 +
// sigma^2 dt^2 (Z2^2 - 1) / 4, s_g = sigma dt Z2.  y leaves out the
// deterministic drift r t / ln 2, which is added back where S is needed: at
// the end of the path, and at a fixing date through the weight e^{r t_j}.
// Under full truncation the clamp is taken as w + |w| = 2 max(w, 0), one
// plain add (exact), and the factor 2 is carried by the constants: the caller
// passes z1l and s_g divided by sqrt 2 (FT_SCALE).
template <class R, bool FT> constexpr R FT_SCALE = FT ? (R)0.70710678118654752440 : R(1);

template <class R, bool FT>
__device__ __forceinline__ void scaled_step(R &y, R &w, const Grid<R> &g, R z1l, R a_g, R s_g)
{
    if constexpr (FT) {
        constexpr R QUARTER_LOG2E = (R)(0.25 * LOG2E);
        const R vp2 = w + fabs(w);
        const R s = fast_sqrt(vp2); // sqrt 2 x sqrt(V+ dt)
        y = y - QUARTER_LOG2E * vp2;
        y = y + s * z1l;
        w = w + (a_g - g.kdt_h * vp2);
        w = w + s * s_g;
        return;
    }
    constexpr R HALF_LOG2E = (R)(0.5 * LOG2E);
    const R vp = clamp0(w);
    const R s = fast_sqrt(vp);
    y = y - HALF_LOG2E * vp;
    y = y + s * z1l;
    const R wb = FT ? w : vp;
    w = wb + (a_g - g.kdt * vp);
    w = w + s * s_g;
    if (!FT)
        w = clamp0(w);
}

// Partial truncation (reflect = false) and reflection (reflect = true) of the
// variance, in the f1/f2/f3 form of Lord, Koekkoek and van Dijk (2010):
// w' = f1(w) + (a_g - kappa dt f2(w)) + sqrt(f3(w)) s_g, with the log-price
// step taking f3; partial truncation f1 = f2 = identity, f3 = max(., 0);
// reflection f1 = f2 = f3 = |.|.  The choice is wave-uniform (a launch
// parameter), so both variants share one kernel.
template <class R>
__device__ __forceinline__ void scaled_step_fix(R &y, R &w, const Grid<R> &g, R z1l, R a_g, R s_g,
                                                bool reflect)
{
    constexpr R HALF_LOG2E = (R)(0.5 * LOG2E);
    const R aw = fabs(w);
    const R f12 = reflect ? aw : w;
    const R f3 = reflect ? aw : clamp0(w);
    const R s = fast_sqrt(f3);
    y = y - HALF_LOG2E * f3;
    y = y + s * z1l;
    w = f12 + (a_g - g.kdt * f12);
    w = w + s * s_g;
}

// Andersen's quadratic-exponential (QE) scheme on one time grid, in the same
// scaled state (y = ln(S/S0)/ln 2 without the drift r t, w = V dt).  With
// E = e^{-kappa dt}, the square-root process's conditional mean and variance
// of w' = V(t+dt) dt given w are m = E w + theta dt (1-E) and
// s2 = cs1 w + cs0, cs1 = sigma^2 dt E (1-E) / kappa,
// cs0 = theta sigma^2 dt^2 (1-E)^2 / (2 kappa); the log-price step is
// (K0 + K1 V + K2 V' + sqrt(K3 V + K4 V') Zs) / ln 2 with Andersen's central
// weights gamma1 = gamma2 = 1/2, here k0 = K0/ln 2, k1 = K1/(dt ln 2),
// k2 = K2/(dt ln 2), k3 = K3/dt, k4 = K4/dt (the 1/ln 2 of the diffusion term
// rides on Zs).
template <class R> struct QEGrid {
    R E, mth, cs1, cs0, k0, k1, k2, k3, k4;
};

template <class R> __device__ __forceinline__ QEGrid<R> qe_grid(const StepCoef &c, const PriceLaunch &L)
{
    const double dt = c.dt, E = exp(-L.kappa * dt), s2s = L.sigma * L.sigma;
    const double kr = L.kappa * L.rho / L.sigma - 0.5;
    QEGrid<R> g;
    g.E = (R)E;
    g.mth = (R)(L.theta * dt * (1.0 - E));
    g.cs1 = (R)(s2s * dt * E * (1.0 - E) / L.kappa);
    g.cs0 = (R)(L.theta * s2s * dt * dt * (1.0 - E) * (1.0 - E) / (2.0 * L.kappa));
    g.k0 = (R)(-L.rho * L.kappa * L.theta * dt / L.sigma * LOG2E);
    g.k1 = (R)((0.5 * dt * kr - L.rho / L.sigma) / dt * LOG2E);
    g.k2 = (R)((0.5 * dt * kr + L.rho / L.sigma) / dt * LOG2E);
    g.k3 = (R)(0.5 * (1.0 - L.rho * L.rho));
    g.k4 = g.k3;
    return g;
}

__device__ __forceinline__ float fast_log(float x) { return __builtin_amdgcn_logf(x) * (float)LN2; }
__device__ __forceinline__ double fast_log(double x) { return log(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

// One QE step of one scenario, in two parts; z1l = Zs / ln 2, zv the normal
// of the quadratic branch, uv the uniform of the exponential branch.
// psi = s2 / m^2 <= 3/2 takes the scaled squared normal a (b + zv)^2, else V'
// is 0 with probability p = (psi-1)/(psi+1) and exponential above it.
// qe_pre gives m, s2 and the branch (psi <= 3/2 tested as s2 <= 3/2 m^2, no
// division); qe_post evaluates a branch only when some lane of the wave takes
// it (quad, expo: wave-uniform votes over all scenarios), psi itself only in
// the exponential branch.
// Away from zero variance every lane takes the quadratic branch, so whole
// waves skip the exponential one and its logarithm; each lane still selects
// by its own psi, so the result is that of evaluating both.
template <class R> struct QEPre {
    R m, s2;
    bool quad; // psi = s2 / m^2 <= 3/2
};

template <class R> __device__ __forceinline__ QEPre<R> qe_pre(R w, const QEGrid<R> &g)
{
    const R m = w * g.E + g.mth;
    const R s2 = w * g.cs1 + g.cs0;
    return QEPre<R>{m, s2, s2 <= R(1.5) * (m * m)};
}

template <class R>
__device__ __forceinline__ void qe_post(R &y, R &w, const QEGrid<R> &g, const QEPre<R> &q, R z1l,
                                        R zv, R uv, bool quad, bool expo)
{
    const R m = q.m, s2 = q.s2;
    R wq = R(0), we = R(0);
    if (quad) {
        const R inv = R(2) * m * m * fast_rcp(s2);
        const R b2 = inv - R(1) + fast_sqrt(inv * (inv - R(1)));
        const R b = fast_sqrt(b2);
        const R a = m * fast_rcp(R(1) + b2);
        const R bz = b + zv;
        wq = a * bz * bz;
    }
    if (expo) {
        // p = (psi - 1) / (psi + 1), 1 - p = 2 / (psi + 1), 1 / beta = m (psi + 1) / 2;
        // uv <= p is tested as uv (psi + 1) <= psi - 1 and ln((1 - p) / (1 - uv))
        // as -ln((psi + 1)(1 - uv) / 2)
        const R rm = fast_rcp(m);
        const R psi = s2 * rm * rm;
        const R pp1 = psi + R(1);
        we = uv * pp1 <= psi - R(1) ? R(0)
                                    : -(R(0.5) * m * pp1) * fast_log(R(0.5) * pp1 * (R(1) - uv));
    }
    const R wn = q.quad ? wq : we;
    y = y + g.k0 + g.k1 * w + g.k2 * wn + fast_sqrt(g.k3 * w + g.k4 * wn) * z1l;
    w = wn;
}

// Wave-uniform: does some lane of the wave have c set?  (Every lane of the
// wave runs the step loop, so the vote covers all 64.)
__device__ __forceinline__ bool any_lane(bool c)
{
    return __builtin_amdgcn_ballot_w64(c) != 0u;
}

// Single-precision QE asks for six waves per SIMD: left to itself the compiler
// spends 140-147 VGPRs on it (three waves); bounded, it fits in 76 without
// spilling and runs 4% faster.  The other variants keep the default.
// SPLIT (small FP64 launches with fused bumps, Milstein, Philox, European or
// arithmetic Asian): each lane runs one scenario of one path -- lane l of a
// wave takes path l / 5 of the wave's SPLIT_PATHS_PER_WAVE and scenario l % 5
// (base, v0+, v0-, T+, T-; lanes 60-63 idle) -- with that scenario's grid,
// initial variance and fixing weight, and the base lane gathers the other four
// final states before the payoffs.  Every scenario takes the same operations
// as in the fused layout, so the per-path values are the same.  With the
// path's draws shared by its five lanes a wave's step is about a fifth of the
// fused layout's for a fifth of its paths: shorter waves, slightly more
// instructions per path, which pays while the launch has few waves per SIMD.
template <class R, int RNG, int AV, bool BUMPS, int SCH, bool SPLIT = false>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(SCH == 2 && sizeof(R) == 4 ? 6 : 1))) void price_kernel(
    const PriceLaunch L)
{
    static_assert(!SPLIT || (sizeof(R) == 8 && RNG == 0 && BUMPS && (AV == 0 || AV == 1) &&
                             (SCH == 0 || SCH == 1)),
                  "scenario-split layout: FP64, Philox, fused bumps, Milstein, no geometric average");
    // AV: 0 European, 1 arithmetic average, 2 geometric average over the
    // fixings, 3 arithmetic average with the geometric one as its control.
    // SCH: 0 Milstein with full truncation, 1 Milstein with absorption, 2 QE,
    // 3 Milstein with partial truncation or reflection (L.reflect)
    constexpr bool ASIAN = AV != 0, GEO = AV == 2, CV = AV == 3;
    constexpr int NE = CV ? N_EST_CV : N_EST, NA = 2 * NE;
    constexpr bool FT = SCH == 0;
    extern __shared__ unsigned char smem_raw[];
    __shared__ double red[BLOCK / 64][NA];

    const uint32_t rep = L.rep0 + blockIdx.y;
    const uint64_t M = L.paths_per_rep;
    const uint64_t rep_lo = (uint64_t)rep * M;
    const uint64_t lo = L.first_path > rep_lo ? L.first_path : rep_lo;
    const uint64_t end = L.first_path + L.n_paths;
    const uint64_t hi = end < rep_lo + M ? end : rep_lo + M;
    const uint32_t scen = SPLIT ? (threadIdx.x & 63) % 5 : 0; // scenario of the lane (SPLIT)
    const uint64_t p = SPLIT ? lo + (uint64_t)blockIdx.x * (BLOCK / 64 * SPLIT_PATHS_PER_WAVE) +
                                   (threadIdx.x >> 6) * SPLIT_PATHS_PER_WAVE + (threadIdx.x & 63) / 5
                             : lo + (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    bool active = p < hi && (!SPLIT || (threadIdx.x & 63) < 5 * SPLIT_PATHS_PER_WAVE);

    const uint32_t N = L.n_steps;
    const Grid<R> gb = grid<R>(L.base, L.sigma);
    const R rho = (R)L.rho, rho_bar = (R)L.rho_bar, log2e = (R)LOG2E;

    R y = 0, w = (R)(L.v0 * L.base.dt), A = 0, B = 0, C = 0, D3 = 0;
    // bump scenarios that need their own paths: v0 +/- and T +/-
    Grid<R> gu{}, gd{};
    R yv0 = 0, yv1 = 0, wv0 = (R)((L.v0 + L.hv) * L.base.dt), wv1 = (R)((L.v0 - L.hv) * L.base.dt);
    R yt0 = 0, yt1 = 0, wt0 = (R)(L.v0 * L.tup.dt), wt1 = (R)(L.v0 * L.tdn.dt);
    R Av0 = 0, Av1 = 0, At0 = 0, At1 = 0;
    R Gs = 0; // control: sum of y over the fixings (base scenario)
    if constexpr (BUMPS) {
        gu = grid<R>(L.tup, L.sigma);
        gd = grid<R>(L.tdn, L.sigma);
    }
    // SPLIT: the lane's scenario grid and initial w (as the fused layout's states start)
    Grid<R> gs = gb;
    if constexpr (SPLIT) {
        gs = scen == 3 ? gu : scen == 4 ? gd : gb;
        w = scen == 1 ? wv0 : scen == 2 ? wv1 : scen == 3 ? wt0 : scen == 4 ? wt1 : w;
    }
    QEGrid<R> qb{}, qu{}, qd{};
    if constexpr (SCH == 2) {
        qb = qe_grid<R>(L.base, L);
        if constexpr (BUMPS) {
            qu = qe_grid<R>(L.tup, L);
            qd = qe_grid<R>(L.tdn, L);
        }
    }

    // Fixing sums after step j (the fixing at t = (j+1) dt): weights e^{rt},
    // t e^{rt}, t^2 e^{rt}, t^3 e^{rt} (base grid), e^{rt} on the T +/- grids.
    auto fixing = [&](uint32_t j) {
        if constexpr (GEO) {
            // geometric average: the same registers sum each scenario's y
            if (is_fixing(L.fix_bits, j + 1)) {
                A += y;
                if constexpr (BUMPS) {
                    Av0 += yv0;
                    Av1 += yv1;
                    At0 += yt0;
                    At1 += yt1;
                }
            }
        } else if constexpr (ASIAN && SPLIT) {
            // the lane's own scenario: weight e^{rt} of its grid; B, C, D3 (base
            // grid) matter on the base lane only
            if (is_fixing(L.fix_bits, j + 1)) {
                const R *tw = reinterpret_cast<const R *>(L.step_weights) + STEP_WEIGHTS * j;
                const R e = exp2r(y);
                A += tw[scen == 3 ? 4 : scen == 4 ? 5 : 0] * e;
                B += tw[1] * e;
                C += tw[2] * e;
                D3 += tw[3] * e;
            }
        } else if constexpr (ASIAN) {
            if (is_fixing(L.fix_bits, j + 1)) {
                const R *tw = reinterpret_cast<const R *>(L.step_weights) + STEP_WEIGHTS * j;
                const R e = exp2r(y);
                A += tw[0] * e;
                B += tw[1] * e;
                if constexpr (CV)
                    Gs += y;
                if constexpr (BUMPS) {
                    C += tw[2] * e;
                    if constexpr (sizeof(R) == 8)
                        D3 += tw[3] * e;
                    Av0 += tw[0] * exp2r(yv0);
                    Av1 += tw[0] * exp2r(yv1);
                    At0 += tw[4] * exp2r(yt0);
                    At1 += tw[5] * exp2r(yt1);
                }
            }
        }
    };

    // Multipliers of the normals: Z1 / ln 2 (times FT_SCALE) and the
    // correlation; the single-precision Philox walk folds the factor
    // sqrt(2 ln 2) of its Box-Muller radius into them.
    R z1c = log2e * FT_SCALE<R, FT>, rhoc = rho, rhobc = rho_bar;

    // One Milstein step given the independent normals (za, zb) of step j.
    auto step = [&](uint32_t j, R za, R zb) {
        constexpr R FS = FT_SCALE<R, FT>;
        const R z1l = za * z1c;
        const R z2 = rhoc * za + rhobc * zb;
        const R z2m1 = z2 * z2 - R(1);
        if constexpr (SPLIT) {
            scaled_step<R, FT>(y, w, gs, z1l, gs.ktdt2 + gs.qdt2 * z2m1, (gs.sdt * FS) * z2);
            fixing(j);
            return;
        }
        const R ab = gb.ktdt2 + gb.qdt2 * z2m1, sb = (gb.sdt * FS) * z2;
        if constexpr (SCH == 3) {
            const bool rf = L.reflect;
            scaled_step_fix<R>(y, w, gb, z1l, ab, sb, rf);
            if constexpr (BUMPS) {
                scaled_step_fix<R>(yv0, wv0, gb, z1l, ab, sb, rf);
                scaled_step_fix<R>(yv1, wv1, gb, z1l, ab, sb, rf);
                scaled_step_fix<R>(yt0, wt0, gu, z1l, gu.ktdt2 + gu.qdt2 * z2m1, gu.sdt * z2, rf);
                scaled_step_fix<R>(yt1, wt1, gd, z1l, gd.ktdt2 + gd.qdt2 * z2m1, gd.sdt * z2, rf);
            }
        } else {
            scaled_step<R, FT>(y, w, gb, z1l, ab, sb);
            if constexpr (BUMPS) {
                scaled_step<R, FT>(yv0, wv0, gb, z1l, ab, sb);
                scaled_step<R, FT>(yv1, wv1, gb, z1l, ab, sb);
                scaled_step<R, FT>(yt0, wt0, gu, z1l, gu.ktdt2 + gu.qdt2 * z2m1, (gu.sdt * FS) * z2);
                scaled_step<R, FT>(yt1, wt1, gd, z1l, gd.ktdt2 + gd.qdt2 * z2m1, (gd.sdt * FS) * z2);
            }
        }
        fixing(j);
    };

    if constexpr (SCH == 2) {
        // QE: one Philox block per step, counter (j, lo32 p, hi32 p, 4); words 0, 1
        // give the Box-Muller pair (Zs, Zv), word 2 the uniform Uv.
        const uint32_t k0 = (uint32_t)L.seed, k1 = (uint32_t)(L.seed >> 32);
        const uint32_t plo = (uint32_t)p, phi = L.wide_paths ? (uint32_t)(p >> 32) : 0u;
        for (uint32_t j = 0; j < N; ++j) {
            const U4 q = philox4x32_10(U4{j, plo, phi, QE_COUNTER_TAG}, k0, k1);
            R zs, zv;
            R uv;
            if constexpr (sizeof(R) == 4) {
                box_muller(uniform_f32(q.x), uniform_f32(q.y), zs, zv);
                uv = uniform_f32(q.z);
            } else {
                box_muller(uniform_f64(q.x), uniform_f64(q.y), zs, zv);
                uv = uniform_f64(q.z);
            }
            const R z1l = zs * log2e;
            const QEPre<R> q0 = qe_pre<R>(w, qb);
            QEPre<R> q1{}, q2{}, q3{}, q4{};
            bool lo = q0.quad, hi = !lo;
            if constexpr (BUMPS) {
                q1 = qe_pre<R>(wv0, qb);
                q2 = qe_pre<R>(wv1, qb);
                q3 = qe_pre<R>(wt0, qu);
                q4 = qe_pre<R>(wt1, qd);
                for (const bool qd_ : {q1.quad, q2.quad, q3.quad, q4.quad}) {
                    lo = lo || qd_;
                    hi = hi || !qd_;
                }
            }
            const bool quad = any_lane(lo), expo = any_lane(hi);
            qe_post<R>(y, w, qb, q0, z1l, zv, uv, quad, expo);
            if constexpr (BUMPS) {
                qe_post<R>(yv0, wv0, qb, q1, z1l, zv, uv, quad, expo);
                qe_post<R>(yv1, wv1, qb, q2, z1l, zv, uv, quad, expo);
                qe_post<R>(yt0, wt0, qu, q3, z1l, zv, uv, quad, expo);
                qe_post<R>(yt1, wt1, qd, q4, z1l, zv, uv, quad, expo);
            }
            fixing(j);
        }
    } else if constexpr (RNG == 0) {
        // Philox: counter (j >> 1, lo32 p, hi32 p, 0); words (0,1) even step, (2,3) odd step.
        const uint32_t k0 = (uint32_t)L.seed, k1 = (uint32_t)(L.seed >> 32);
        // Paths below 2^32 have a zero high counter word: the first round's
        // second product is then zero and the compiler keeps it scalar.
        const uint32_t plo = (uint32_t)p, phi = L.wide_paths ? (uint32_t)(p >> 32) : 0u;
        constexpr bool SCALED = sizeof(R) == 4;
        if constexpr (SCALED) {
            constexpr double NS = SQRT_2LN2;
            z1c = (R)(LOG2E * (double)FT_SCALE<R, FT> * NS);
            rhoc = (R)(L.rho * NS);
            rhobc = (R)(L.rho_bar * NS);
        }
        if constexpr (SPLIT) {
            // The five lanes of a path share its normals.  Over a group of
            // ten steps the lane of scenario s draws the Philox block of steps
            // j0 + 2s and j0 + 2s + 1, and each lane reads every step's pair
            // from the lane that drew it, so a lane computes a fifth of the
            // path's draws.  The next group is drawn while the current one is
            // stepped.  (Lanes 60-63 read within their group or lane 63.)
            constexpr uint32_t G = 10;
            const int src0 = (int)(threadIdx.x & 63u) - (int)scen;
            R a0, b0, a1, b1, za[G], zb[G];
            philox_normals<R, false>(2 * scen, plo, phi, k0, k1, a0, b0, a1, b1);
            auto gather = [&]() {
#pragma unroll
                for (uint32_t k = 0; k < G; ++k) {
                    const int src = min(src0 + (int)(k >> 1), 63);
                    za[k] = __shfl((k & 1) ? a1 : a0, src, 64);
                    zb[k] = __shfl((k & 1) ? b1 : b0, src, 64);
                }
            };
            uint32_t j0 = 0;
            for (; j0 + G <= N; j0 += G) {
                gather();
                philox_normals<R, false>(j0 + G + 2 * scen, plo, phi, k0, k1, a0, b0, a1, b1);
#pragma unroll
                for (uint32_t k = 0; k < G; ++k)
                    step(j0 + k, za[k], zb[k]);
            }
            if (j0 < N) {
                gather();
#pragma unroll
                for (uint32_t k = 0; k < G; ++k)
                    if (j0 + k < N)
                        step(j0 + k, za[k], zb[k]);
            }
        } else {
            uint32_t j = 0;
            for (; j + 1 < N; j += 2) {
                R za0, zb0, za1, zb1;
                philox_normals<R, SCALED>(j, plo, phi, k0, k1, za0, zb0, za1, zb1);
                step(j, za0, zb0);
                step(j + 1, za1, zb1);
            }
            if (j < N) {
                R za0, zb0, za1, zb1;
                philox_normals<R, SCALED>(j, plo, phi, k0, k1, za0, zb0, za1, zb1);
                step(j, za0, zb0);
            }
        }
    } else {
        // Sobol point i of replicate `rep`, Brownian bridge walked in time order
        // with the right end-points of the enclosing intervals on an LDS stack.
        R *stk = reinterpret_cast<R *>(smem_raw); // [depth][2][BLOCK]
        const uint32_t tid = threadIdx.x;
        auto slot = [&](int level, int motion) -> R & {
            return stk[(level * 2 + motion) * BLOCK + tid];
        };
        const uint64_t i = active ? p - rep_lo : 0;
        const uint32_t g = (uint32_t)(i ^ (i >> 1));
        int nbits = 0;
        while (nbits < 30 && (M - 1) >> nbits)
            ++nbits;
        const uint32_t *shift = L.sobol_shift + (uint64_t)rep * 2u * N;
        uint32_t m[6];
#pragma unroll
        for (int b = 0; b < 6; ++b)
            m[b] = 0u - ((g >> b) & 1u);
        // Two walks.  Fast (the launch's waves cover 64-point-aligned blocks and
        // the host built position-ordered tables): the node consumed at position
        // pos (0 = root, o + 1 = bridge op o) reads the wave's row of the
        // per-block table and the replicate's shift at addresses that depend only
        // on pos, so an op's loads do not wait on the op record, and each lane
        // reads the XOR of its low six Gray-code bits' direction numbers from the
        // low-bit table (the wave's 64 lanes read one 512-byte row, which the
        // next position's load fetches one op ahead).  Otherwise dimensions are
        // addressed through the op's node index and each lane combines the
        // direction numbers of its own Gray code.
        auto walk = [&](auto fast_tag) {
            constexpr bool FAST = decltype(fast_tag)::value;
            const uint32_t *hi_row =
                FAST ? L.sobol_hi + (uint64_t)(__builtin_amdgcn_readfirstlane((uint32_t)i) >> 6) * 2u * N
                     : nullptr;
            // When every wave covers 64 consecutive points starting at a multiple
            // of 64, Gray-code bits 6 and up are the same in all its lanes: their
            // XOR of direction numbers is wave-uniform (scalar), and each lane only
            // combines six direction numbers under its fixed masks.
            const bool aligned = (M % 64 == 0) && ((lo - rep_lo) % 64 == 0);
            const uint32_t g_hi = __builtin_amdgcn_readfirstlane(g) & ~63u;
            auto coord = [&](uint32_t d) -> uint32_t {
                const uint32_t *v = L.sobol_dirs + 32u * d;
                if (aligned) {
                    uint32_t u = shift[d];
                    for (uint32_t bits = g_hi; bits; bits &= bits - 1)
                        u ^= v[__builtin_ctz(bits)];
                    return u ^ sobol_low(v, m);
                }
                return sobol_coord(L.sobol_dirs, d, g, nbits, shift[d]);
            };
            // the lane's entry of the low-bit table at a walk position (row N is
            // the zero pad that the last position's look-ahead reads)
            const uint32_t g_lo = g & 63u;
            auto low_at = [&](uint32_t pos) -> uint2 {
                return reinterpret_cast<const uint2 *>(L.sobol_low + 128u * pos)[g_lo];
            };
            uint2 low_next = FAST ? low_at(0u) : uint2{0u, 0u};
            // normals of the node at walk position pos (node index k); positions
            // are consumed in order 0, 1, ..., N - 1
            auto node_normals = [&](uint32_t pos, int k, R &wa, R &wb) {
                if constexpr (FAST) {
                    const uint2 lw = low_next;
                    low_next = low_at(pos + 1u);
                    const uint32_t c = 2u * pos;
                    sobol_normals<R>(shift[c] ^ hi_row[c] ^ lw.x, shift[c + 1] ^ hi_row[c + 1] ^ lw.y,
                                     wa, wb);
                } else {
                    const uint32_t d = 2u * (uint32_t)k;
                    sobol_normals<R>(coord(d), coord(d + 1), wa, wb);
                }
            };
            R ca = 0, cbm = 0; // B_j of the two motions
            {
                R wa, wb;
                node_normals(0u, 0, wa, wb);
                const R sc = (R)L.bridge_root_scale;
                slot(0, 0) = sc * wa;
                slot(0, 1) = sc * wb;
            }
            int sp = 1;
            for (uint32_t j = 0; j < N; ++j) {
                const int op_end = L.bridge_start[j + 1];
                for (int o = L.bridge_start[j]; o < op_end; ++o) {
                    const BridgeOp op = L.bridge_ops[o];
                    R wa, wb;
                    node_normals((uint32_t)o + 1u, op.node, wa, wb);
                    R a, b, c;
                    if constexpr (sizeof(R) == 4) {
                        a = op.a; b = op.b; c = op.c;
                    } else {
                        a = op.ad; b = op.bd; c = op.cd;
                    }
                    const R ta = slot(sp - 1, 0), tb = slot(sp - 1, 1);
                    slot(sp, 0) = a * ca + b * ta + c * wa;
                    slot(sp, 1) = a * cbm + b * tb + c * wb;
                    ++sp;
                }
                --sp;
                const R na = slot(sp, 0), nb = slot(sp, 1);
                const R za = na - ca, zb = nb - cbm;
                ca = na;
                cbm = nb;
                step(j, za, zb);
            }
        };
        if (L.sobol_low != nullptr)
            walk(std::true_type{});
        else
            walk(std::false_type{});
    }

    if constexpr (SPLIT) {
        // the base lane takes the bumped scenarios' final states from its four
        // neighbours; only it contributes to the sums
        const int l = (int)(threadIdx.x & 63);
        yv0 = __shfl(y, l + 1, 64);
        yv1 = __shfl(y, l + 2, 64);
        yt0 = __shfl(y, l + 3, 64);
        yt1 = __shfl(y, l + 4, 64);
        if constexpr (ASIAN) {
            Av0 = __shfl(A, l + 1, 64);
            Av1 = __shfl(A, l + 2, 64);
            At0 = __shfl(A, l + 3, 64);
            At1 = __shfl(A, l + 4, 64);
        }
        active = active && scen == 0;
    }

    // ---- payoffs and Greek samples, in FP64 ----
    double est[NE];
    const Payoff pay{L.opt_type, L.K, 1.0 / (double)L.n_fix};
    const double S0 = L.S0, D = exp(-L.r * L.T);
    const double x = (double)y * LN2 + L.r * L.T;
    const double eT = exp(x);
    const double ST = S0 * eT;
    // geometric averages: the fixing times of each grid sum to dt times the
    // sum of the fixing step indices; G / S0 = exp(mean of (y ln 2 + r t_i))
    const double tsum = L.base.dt * L.fix_step_sum;
    auto geo_rel = [&](double ysum, double ts) {
        return exp(((double)ysum * LN2 + L.r * ts) * pay.inv_nfix);
    };
    // Sbar / S0 (or G / S0, or S_T / S0), and the dSbar/dr term of the pathwise Rho
    const double rel = GEO ? geo_rel((double)A, tsum) : ASIAN ? (double)A * pay.inv_nfix : eT;
    const double dBr = GEO ? rel * tsum : (double)B;
    const double X = S0 * rel;
    const double sgn = pay.call() ? 1.0 : -1.0;
    const bool itm = sgn * (X - L.K) > 0.0;
    est[EST_PRICE] = pay(D, X);
    est[EST_PW_DELTA] = itm ? sgn * D * rel : 0.0;
    if (ASIAN)
        est[EST_PW_RHO] = itm ? D * (sgn * S0 * dBr * pay.inv_nfix - L.T * sgn * (X - L.K)) : 0.0;
    else
        est[EST_PW_RHO] = itm ? sgn * D * L.K * L.T : 0.0;

    double sc[8] = {0, 0, 0, 0, 0, 0, 0, 0}; // S0+, S0-, v0+, v0-, r+, r-, T+, T-
    if constexpr (BUMPS) {
        const double hS = L.hS, hr = L.hr;
        sc[0] = pay(D, (S0 + hS) * rel);
        sc[1] = pay(D, (S0 - hS) * rel);
        const double Xv0 = S0 * (GEO     ? geo_rel((double)Av0, tsum)
                                 : ASIAN ? (double)Av0 * pay.inv_nfix
                                         : exp((double)yv0 * LN2 + L.r * L.T));
        const double Xv1 = S0 * (GEO     ? geo_rel((double)Av1, tsum)
                                 : ASIAN ? (double)Av1 * pay.inv_nfix
                                         : exp((double)yv1 * LN2 + L.r * L.T));
        sc[2] = pay(D, Xv0);
        sc[3] = pay(D, Xv1);
        const double Dup = exp(-(L.r + hr) * L.T), Ddn = exp(-(L.r - hr) * L.T);
        double Xu, Xd;
        if (GEO) {
            // r enters ln G as r times the mean fixing time: exact
            const double tb = tsum * pay.inv_nfix;
            Xu = X * exp(hr * tb);
            Xd = X * exp(-hr * tb);
        } else if (ASIAN) {
            // e^{+-h t_i} summed over the fixings by its Taylor series in h.
            const double a = (double)A, b = (double)B, c = (double)C, d3 = (double)D3;
            const double even = a + 0.5 * hr * hr * c, odd = hr * b + hr * hr * hr / 6.0 * d3;
            Xu = S0 * (even + odd) * pay.inv_nfix;
            Xd = S0 * (even - odd) * pay.inv_nfix;
        } else {
            Xu = ST * exp(hr * L.T);
            Xd = ST * exp(-hr * L.T);
        }
        sc[4] = pay(Dup, Xu);
        sc[5] = pay(Ddn, Xd);
        const double Tu = L.T + L.hT, Td = L.T - L.hT;
        const double Xt0 = S0 * (GEO     ? geo_rel((double)At0, L.tup.dt * L.fix_step_sum)
                                 : ASIAN ? (double)At0 * pay.inv_nfix
                                         : exp((double)yt0 * LN2 + L.r * Tu));
        const double Xt1 = S0 * (GEO     ? geo_rel((double)At1, L.tdn.dt * L.fix_step_sum)
                                 : ASIAN ? (double)At1 * pay.inv_nfix
                                         : exp((double)yt1 * LN2 + L.r * Td));
        sc[6] = pay(exp(-L.r * Tu), Xt0);
        sc[7] = pay(exp(-L.r * Td), Xt1);
        est[EST_DELTA] = (sc[0] - sc[1]) / (2.0 * hS);
        est[EST_GAMMA] = (sc[0] - 2.0 * est[EST_PRICE] + sc[1]) / (hS * hS);
        est[EST_VEGA] = (sc[2] - sc[3]) / (2.0 * L.hv);
        est[EST_RHO] = (sc[4] - sc[5]) / (2.0 * hr);
        est[EST_THETA] = -(sc[6] - sc[7]) / (2.0 * L.hT);
    } else {
#pragma unroll
        for (int e = EST_DELTA; e < N_EST; ++e)
            est[e] = 0.0;
    }

    double gpay = 0.0; // control payoff
    if constexpr (CV) {
        gpay = pay(D, S0 * geo_rel((double)Gs, tsum));
        est[EST_CV_GEO] = gpay;
        est[EST_CV_DIFF] = est[EST_PRICE] - gpay;
    }

    if (L.pay_out != nullptr && active)
        L.pay_out[p - L.first_path] = est[EST_PRICE];

    if (L.dump != nullptr && active) {
        double *rec = L.dump + (p - L.first_path) * DUMP_WIDTH;
        rec[0] = ST;
        rec[1] = (double)w / L.base.dt;
        rec[2] = X;
        rec[3] = est[EST_PRICE];
        rec[4] = est[EST_PW_DELTA];
        rec[5] = est[EST_PW_RHO];
        const double nan = __builtin_nan("");
#pragma unroll
        for (int k = 0; k < 8; ++k)
            rec[6 + k] = BUMPS ? sc[k] : nan;
        rec[14] = x;
        rec[15] = gpay;
    }

    // ---- FP64 sums: wavefront butterfly, then the block's waves in order ----
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const double ye = active ? est[e] : 0.0;
        const double s1 = wave_sum(ye);
        const double s2 = wave_sum(ye * ye);
        if (lane == 0) {
            red[wave][2 * e] = s1;
            red[wave][2 * e + 1] = s2;
        }
    }
    __syncthreads();
    if (threadIdx.x < NA) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w)
            s += red[w][threadIdx.x];
        L.partials[((uint64_t)blockIdx.y * L.blocks_per_rep + blockIdx.x) * NA + threadIdx.x] = s;
    }
}

// Sums runs of partial records (W doubles each) in a fixed order.  Block
// (x, y) adds records [x chunk, min((x + 1) chunk, rep_rows)) of replicate y
// (records y rep_rows + ...) into out[(y gridDim.x + x) W + ...].  Thread t
// owns column t % W of row group t / W: it adds rows g, g + G, g + 2G, ...
// (G = RB / W groups), so consecutive threads read consecutive doubles, into
// U running sums (row g + (U i + u) G into sum u); the U sums, then the G
// group sums of each column, are added in order.  One workgroup reads at a
// few tens of GB/s, so long replicates are first cut into chunks of
// REDUCE_CHUNK records, one block each, and the chunk sums reduced again.
constexpr int RB = 1024; // threads of a reduction block
template <int W>
__global__ __launch_bounds__(RB) void reduce_partials(const double *__restrict__ in,
                                                      uint32_t rep_rows, uint32_t chunk,
                                                      double *__restrict__ out)
{
    constexpr int G = RB / W, U = 8;
    __shared__ double red[G][W];
    const uint32_t first = blockIdx.x * chunk;
    const uint32_t rows = rep_rows - first < chunk ? rep_rows - first : chunk;
    const double *base = in + ((uint64_t)blockIdx.y * rep_rows + first) * W;
    const int t = threadIdx.x, col = t % W, grp = t / W;
    if (grp < G) {
        double acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            acc[u] = 0.0;
        for (uint32_t b = grp; b < rows; b += U * G) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t row = b + (uint32_t)(u * G);
                if (row < rows)
                    acc[u] += base[(uint64_t)row * W + col];
            }
        }
        double sum = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            sum += acc[u];
        red[grp][col] = sum;
    }
    __syncthreads();
    if (t < W) {
        double s = 0.0;
        for (int g = 0; g < G; ++g)
            s += red[g][t];
        out[((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * W + t] = s;
    }
}

template <int W>
hipError_t launch_reduce_w(const PriceLaunch &L, double *rep_sums, hipStream_t stream)
{
    const uint32_t chunks = (L.blocks_per_rep + REDUCE_CHUNK - 1) / REDUCE_CHUNK;
    if (chunks <= 1) {
        hipLaunchKernelGGL(reduce_partials<W>, dim3(1, L.n_reps), dim3(RB), 0, stream, L.partials,
                           L.blocks_per_rep, L.blocks_per_rep, rep_sums);
        return hipGetLastError();
    }
    if (L.reduce_tmp == nullptr)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(reduce_partials<W>, dim3(chunks, L.n_reps), dim3(RB), 0, stream,
                       L.partials, L.blocks_per_rep, REDUCE_CHUNK, L.reduce_tmp);
    hipLaunchKernelGGL(reduce_partials<W>, dim3(1, L.n_reps), dim3(RB), 0, stream,
                       (const double *)L.reduce_tmp, chunks, chunks, rep_sums);
    return hipGetLastError();
}

// Plain bump-and-revalue: per-path central differences of stored payoff rows.
__global__ __launch_bounds__(BLOCK) void bump_combine_kernel(const double *__restrict__ pay,
                                                             uint64_t n, uint32_t n_bump,
                                                             const BumpScales sc,
                                                             double *__restrict__ partials)
{
    __shared__ double red[BLOCK / 64][BUMP_W];
    double acc[BUMP_W];
#pragma unroll
    for (int k = 0; k < BUMP_W; ++k)
        acc[k] = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) {
        const double b = pay[i];
        acc[0] += b;
        acc[1] += b * b;
#pragma unroll
        for (int k = 0; k < MAX_BUMPS; ++k) {
            if (k < (int)n_bump) {
                const double u = pay[(1 + 2 * (uint64_t)k) * n + i];
                const double d = pay[(2 + 2 * (uint64_t)k) * n + i];
                const double g1 = (u - d) * sc.first[k];
                const double g2 = (u - 2.0 * b + d) * sc.second[k];
                acc[2 + 4 * k] += g1;
                acc[3 + 4 * k] += g1 * g1;
                acc[4 + 4 * k] += g2;
                acc[5 + 4 * k] += g2 * g2;
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < BUMP_W; ++k) {
        const double t = wave_sum(acc[k]);
        if (lane == 0)
            red[wave][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < BUMP_W) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w)
            t += red[w][threadIdx.x];
        partials[(uint64_t)blockIdx.x * BUMP_W + threadIdx.x] = t;
    }
}

// Fixed-order sum of `rows` records of width w (w <= BLOCK): the block's
// floor(BLOCK / w) groups of w threads take rows g, g + groups, ... (thread k
// of a group owns column k); the group sums are then added in group order.
__global__ __launch_bounds__(BLOCK) void reduce_rows_kernel(const double *__restrict__ partials,
                                                            uint32_t rows, uint32_t w,
                                                            double *__restrict__ out)
{
    __shared__ double red[BLOCK];
    const uint32_t groups = BLOCK / w;
    const uint32_t grp = threadIdx.x / w, col = threadIdx.x % w;
    double t = 0.0;
    if (grp < groups)
        for (uint32_t r = grp; r < rows; r += groups)
            t += partials[(uint64_t)r * w + col];
    red[threadIdx.x] = t;
    __syncthreads();
    if (threadIdx.x < w) {
        double s = 0.0;
        for (uint32_t g = 0; g < groups; ++g)
            s += red[g * w + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

template <class R>
__global__ void step_weights_kernel(uint32_t n, double r, double dt, double dt_up, double dt_dn,
                                    R *out)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n)
        return;
    const double t = (double)(j + 1) * dt, g = exp(r * t);
    R *o = out + (uint64_t)STEP_WEIGHTS * j;
    o[0] = (R)g;
    o[1] = (R)(t * g);
    o[2] = (R)(t * t * g);
    o[3] = (R)(t * t * t * g);
    o[4] = (R)exp(r * (double)(j + 1) * dt_up);
    o[5] = (R)exp(r * (double)(j + 1) * dt_dn);
    o[6] = (R)0;
    o[7] = (R)0;
}

// Column c of the position-ordered tables holds dimension 2 node(c / 2) + c % 2,
// where node(pos) is the bridge node consumed at walk position pos; without a
// permutation column c is dimension c.
__device__ __forceinline__ uint32_t table_dim(const int32_t *perm, uint32_t c)
{
    return perm ? 2u * (uint32_t)perm[c >> 1] + (c & 1u) : c;
}

// Per 64-point block b of a replicate and column c: the XOR of the direction
// numbers v[d][k] of dimension d = table_dim(c) over the set bits k >= 6 of
// the Gray code of 64 b, which every point of the block shares (Gray code
// g(i) = i ^ (i >> 1)).
__global__ void sobol_hi_kernel(const uint32_t *dirs, const int32_t *perm, uint32_t dims,
                                uint32_t n_blk, uint32_t *out)
{
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (uint64_t)dims * n_blk)
        return;
    const uint32_t b = (uint32_t)(idx / dims), c = (uint32_t)(idx - (uint64_t)b * dims);
    const uint32_t i = b << 6;
    const uint32_t *v = dirs + 32u * table_dim(perm, c);
    uint32_t x = 0;
    for (uint32_t bits = (i ^ (i >> 1)) & ~63u; bits; bits &= bits - 1)
        x ^= v[__builtin_ctz(bits)];
    out[idx] = x;
}

// out[pos][l][h] = XOR of the direction numbers k < 6 of dimension h of the
// node at walk position pos over the set bits k of l (l = a point's low six
// Gray-code bits); row N is zero.
__global__ void sobol_low_kernel(const uint32_t *dir12, uint32_t N, uint32_t *out)
{
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (N + 1u) * 128u)
        return;
    const uint32_t pos = idx >> 7, l = (idx >> 1) & 63u, h = idx & 1u;
    uint32_t x = 0;
    if (pos < N)
        for (uint32_t b = 0; b < 6; ++b)
            if ((l >> b) & 1u)
                x ^= dir12[pos * 12u + h * 6u + b];
    out[idx] = x;
}

// Digital shifts of the Sobol replicates: shift[r][c] = top 30 bits of word 0
// of Philox4x32-10(counter (d, r, 0, 1), key = seed), d = table_dim(c).
__global__ void sobol_shift_kernel(uint64_t seed, const int32_t *perm, uint32_t dims, uint32_t reps,
                                   uint32_t *out)
{
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= dims * reps)
        return;
    const uint32_t r = idx / dims, c = idx - r * dims;
    const uint32_t d = table_dim(perm, c);
    const U4 w = philox4x32_10(U4{d, r, 0u, 1u}, (uint32_t)seed, (uint32_t)(seed >> 32));
    out[idx] = w.x >> 2;
}

template <class R, int RNG, int AV, bool BUMPS, int SCH>
hipError_t launch_t(const PriceLaunch &L, hipStream_t s)
{
    const dim3 grid(L.blocks_per_rep, L.n_reps);
    const size_t smem = RNG == 1 ? (size_t)L.bridge_depth * 2 * BLOCK * sizeof(R) : 0;
    if constexpr (sizeof(R) == 8 && RNG == 0 && BUMPS && (AV == 0 || AV == 1) &&
                  (SCH == 0 || SCH == 1)) {
        if (L.split) {
            hipLaunchKernelGGL((price_kernel<R, RNG, AV, BUMPS, SCH, true>), grid, dim3(BLOCK), 0,
                               s, L);
            return hipGetLastError();
        }
    }
    if (L.split)
        return hipErrorInvalidValue; // the host offers the split layout only where it exists
    hipLaunchKernelGGL((price_kernel<R, RNG, AV, BUMPS, SCH>), grid, dim3(BLOCK), smem, s, L);
    return hipGetLastError();
}

template <class R, int RNG, int AV, bool BUMPS>
hipError_t launch_ft(const PriceLaunch &L, hipStream_t s)
{
    if (L.scheme == 0)
        return launch_t<R, RNG, AV, BUMPS, 0>(L, s);
    if (L.scheme == 1)
        return launch_t<R, RNG, AV, BUMPS, 1>(L, s);
    if (L.scheme == 3)
        return launch_t<R, RNG, AV, BUMPS, 3>(L, s);
    if constexpr (RNG == 0)
        return launch_t<R, RNG, AV, BUMPS, 2>(L, s);
    return hipErrorInvalidValue; // QE draws Philox inputs only (checked by the host)
}

template <class R, int RNG, int AV>
hipError_t launch_b(const PriceLaunch &L, hipStream_t s)
{
    return L.bumps ? launch_ft<R, RNG, AV, true>(L, s) : launch_ft<R, RNG, AV, false>(L, s);
}

template <class R, int RNG> hipError_t launch_a(const PriceLaunch &L, hipStream_t s)
{
    if (L.opt_type == 2 || L.opt_type == 3)
        return L.cv ? launch_b<R, RNG, 3>(L, s) : launch_b<R, RNG, 1>(L, s);
    if (L.opt_type == 4 || L.opt_type == 5)
        return launch_b<R, RNG, 2>(L, s);
    return launch_b<R, RNG, 0>(L, s);
}

template <class R> hipError_t launch_r(const PriceLaunch &L, hipStream_t s)
{
    return L.rng == 0 ? launch_a<R, 0>(L, s) : launch_a<R, 1>(L, s);
}

} // namespace

hipError_t launch_step_weights(const PriceLaunch &L, void *out, hipStream_t stream)
{
    const uint32_t n = L.n_steps;
    const double du = L.bumps ? L.tup.dt : L.base.dt, dd = L.bumps ? L.tdn.dt : L.base.dt;
    if (L.precision == 0)
        hipLaunchKernelGGL(step_weights_kernel<double>, dim3((n + 255) / 256), dim3(256), 0, stream,
                           n, L.r, L.base.dt, du, dd, (double *)out);
    else
        hipLaunchKernelGGL(step_weights_kernel<float>, dim3((n + 255) / 256), dim3(256), 0, stream,
                           n, L.r, L.base.dt, du, dd, (float *)out);
    return hipGetLastError();
}

hipError_t launch_sobol_hi(const uint32_t *dirs, const int32_t *perm, uint32_t dims, uint32_t n_blk,
                           uint32_t *out, hipStream_t stream)
{
    const uint64_t n = (uint64_t)dims * n_blk;
    hipLaunchKernelGGL(sobol_hi_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       dirs, perm, dims, n_blk, out);
    return hipGetLastError();
}

hipError_t launch_sobol_low(const uint32_t *dir12, uint32_t N, uint32_t *out, hipStream_t stream)
{
    const uint32_t n = (N + 1u) * 128u;
    hipLaunchKernelGGL(sobol_low_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, dir12, N, out);
    return hipGetLastError();
}

hipError_t launch_sobol_shifts(uint64_t seed, const int32_t *perm, uint32_t dims, uint32_t reps,
                               uint32_t *out, hipStream_t stream)
{
    const uint32_t n = dims * reps;
    hipLaunchKernelGGL(sobol_shift_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, seed, perm,
                       dims, reps, out);
    return hipGetLastError();
}

hipError_t launch_paths(const PriceLaunch &L, hipStream_t stream)
{
    return L.precision == 0 ? launch_r<double>(L, stream) : launch_r<float>(L, stream);
}

hipError_t launch_bump_combine(const double *pay, uint64_t n_paths, uint32_t n_bump,
                               const BumpScales &sc, double *partials, uint32_t blocks,
                               hipStream_t stream)
{
    hipLaunchKernelGGL(bump_combine_kernel, dim3(blocks), dim3(BLOCK), 0, stream, pay, n_paths,
                       n_bump, sc, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_rows(const double *partials, uint32_t rows, uint32_t w, double *out,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(BLOCK), 0, stream, partials, rows, w,
                       out);
    return hipGetLastError();
}

hipError_t launch_reduce(const PriceLaunch &L, double *rep_sums, hipStream_t stream)
{
    return L.cv ? launch_reduce_w<N_ACC_CV>(L, rep_sums, stream)
                : launch_reduce_w<N_ACC>(L, rep_sums, stream);
}

} // namespace heston
