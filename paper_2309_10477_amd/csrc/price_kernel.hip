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
#include "device_math.hpp"
#include "internal.hpp"
#include "path_step.hpp"

namespace heston {
namespace {

struct Payoff {
    int type;
    double K, inv_nfix;
    __device__ __forceinline__ bool call() const { return type == 0 || type == 2; }
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
template <class R> __device__ __forceinline__ R sobol_normal(uint32_t x)
{
    const bool upper = x >= (1u << 29);
    const uint32_t xs = upper ? 0x3FFFFFFFu - x : x;
    const R z = inv_normal(((R)xs + R(0.5)) * R(0x1p-30));
    return upper ? -z : z;
}

template <class R, int RNG, bool ASIAN, bool BUMPS, bool FT>
__global__ __launch_bounds__(BLOCK) void price_kernel(const PriceLaunch L)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ double red[BLOCK / 64][N_ACC];

    const uint32_t rep = L.rep0 + blockIdx.y;
    const uint64_t M = L.paths_per_rep;
    const uint64_t rep_lo = (uint64_t)rep * M;
    const uint64_t lo = L.first_path > rep_lo ? L.first_path : rep_lo;
    const uint64_t end = L.first_path + L.n_paths;
    const uint64_t hi = end < rep_lo + M ? end : rep_lo + M;
    const uint64_t p = lo + (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool active = p < hi;

    const uint32_t N = L.n_steps;
    const Coef<R> cb = coef<R>(L.base);
    const R rho = (R)L.rho, rho_bar = (R)L.rho_bar, sigma = (R)L.sigma;

    R x = 0, v = (R)L.v0, A = 0, B = 0, C = 0, D3 = 0;
    // bump scenarios that need their own paths: v0 +/- and T +/-
    Coef<R> cu{}, cd{};
    R xv0 = 0, xv1 = 0, vv0 = (R)(L.v0 + L.hv), vv1 = (R)(L.v0 - L.hv), Av0 = 0, Av1 = 0;
    R xt0 = 0, xt1 = 0, vt0 = (R)L.v0, vt1 = (R)L.v0, At0 = 0, At1 = 0;
    if constexpr (BUMPS) {
        cu = coef<R>(L.tup);
        cd = coef<R>(L.tdn);
    }

    // One step given the independent normals (za, zb) of step j.
    auto step = [&](uint32_t j, R za, R zb) {
        const R z1 = za;
        const R z2 = rho * za + rho_bar * zb;
        const R sz2 = sigma * z2;
        const R z2m1 = z2 * z2 - R(1);
        mil_step<R, FT>(x, v, cb, z1, sz2, cb.qdt * z2m1);
        if constexpr (BUMPS) {
            const R mb = cb.qdt * z2m1;
            mil_step<R, FT>(xv0, vv0, cb, z1, sz2, mb);
            mil_step<R, FT>(xv1, vv1, cb, z1, sz2, mb);
            mil_step<R, FT>(xt0, vt0, cu, z1, sz2, cu.qdt * z2m1);
            mil_step<R, FT>(xt1, vt1, cd, z1, sz2, cd.qdt * z2m1);
        }
        if constexpr (ASIAN) {
            const uint32_t jf = j + 1;
            const bool fix = is_fixing(L.fix_bits, jf);
            if (fix) {
                const R e = fast_exp(x);
                const R t = (R)jf * cb.dt;
                A += e;
                const R te = t * e;
                B += te;
                if constexpr (BUMPS) {
                    const R tte = t * te;
                    C += tte;
                    if constexpr (sizeof(R) == 8)
                        D3 += t * tte;
                    Av0 += fast_exp(xv0);
                    Av1 += fast_exp(xv1);
                    At0 += fast_exp(xt0);
                    At1 += fast_exp(xt1);
                }
            }
        }
    };

    if constexpr (RNG == 0) {
        // Philox: counter (j >> 1, lo32 p, hi32 p, 0); words (0,1) even step, (2,3) odd step.
        const uint32_t k0 = (uint32_t)L.seed, k1 = (uint32_t)(L.seed >> 32);
        const uint32_t plo = (uint32_t)p, phi = (uint32_t)(p >> 32);
        R *ck = reinterpret_cast<R *>(L.ckpt);
        const uint64_t np = L.n_paths, row = p - L.first_path;
        uint32_t j = 0;
        for (; j + 1 < N; j += 2) {
            if (ck != nullptr && j % L.ckpt_every == 0 && active) {
                const uint64_t c = j / L.ckpt_every;
                ck[(2 * c) * np + row] = x;
                ck[(2 * c + 1) * np + row] = v;
            }
            const U4 w = philox4x32_10(U4{j >> 1, plo, phi, 0u}, k0, k1);
            R za, zb;
            if constexpr (sizeof(R) == 4)
                box_muller(uniform_f32(w.x), uniform_f32(w.y), za, zb);
            else
                box_muller(uniform_f64(w.x), uniform_f64(w.y), za, zb);
            step(j, za, zb);
            if constexpr (sizeof(R) == 4)
                box_muller(uniform_f32(w.z), uniform_f32(w.w), za, zb);
            else
                box_muller(uniform_f64(w.z), uniform_f64(w.w), za, zb);
            step(j + 1, za, zb);
        }
        if (j < N) {
            if (ck != nullptr && j % L.ckpt_every == 0 && active) {
                const uint64_t c = j / L.ckpt_every;
                ck[(2 * c) * np + row] = x;
                ck[(2 * c + 1) * np + row] = v;
            }
            const U4 w = philox4x32_10(U4{j >> 1, plo, phi, 0u}, k0, k1);
            R za, zb;
            if constexpr (sizeof(R) == 4)
                box_muller(uniform_f32(w.x), uniform_f32(w.y), za, zb);
            else
                box_muller(uniform_f64(w.x), uniform_f64(w.y), za, zb);
            step(j, za, zb);
        }
        if (ck != nullptr && active) {
            const uint64_t c = ckpt_count(N, L.ckpt_every);
            ck[(2 * c) * np + row] = x;
            ck[(2 * c + 1) * np + row] = A;
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
        auto node_normals = [&](int k, R &wa, R &wb) {
            const uint32_t d = 2u * (uint32_t)k;
            wa = sobol_normal<R>(sobol_coord(L.sobol_dirs, d, g, nbits, shift[d]));
            wb = sobol_normal<R>(sobol_coord(L.sobol_dirs, d + 1, g, nbits, shift[d + 1]));
        };
        R ca = 0, cbm = 0; // B_j of the two motions
        {
            R wa, wb;
            node_normals(0, wa, wb);
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
                node_normals(op.node, wa, wb);
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
    }

    // ---- payoffs and Greek samples, in FP64 ----
    double y[N_EST];
    const Payoff pay{L.opt_type, L.K, 1.0 / (double)L.n_fix};
    const double S0 = L.S0, D = exp(-L.r * L.T);
    const double eT = exp((double)x);
    const double ST = S0 * eT;
    const double rel = ASIAN ? (double)A * pay.inv_nfix : eT; // Sbar / S0 (or S_T / S0)
    const double X = S0 * rel;
    const double sgn = pay.call() ? 1.0 : -1.0;
    const bool itm = sgn * (X - L.K) > 0.0;
    y[EST_PRICE] = pay(D, X);
    y[EST_PW_DELTA] = itm ? sgn * D * rel : 0.0;
    if (ASIAN)
        y[EST_PW_RHO] = itm ? D * (sgn * S0 * (double)B * pay.inv_nfix - L.T * sgn * (X - L.K)) : 0.0;
    else
        y[EST_PW_RHO] = itm ? sgn * D * L.K * L.T : 0.0;

    double sc[8] = {0, 0, 0, 0, 0, 0, 0, 0}; // S0+, S0-, v0+, v0-, r+, r-, T+, T-
    if constexpr (BUMPS) {
        const double hS = L.hS, hr = L.hr;
        sc[0] = pay(D, (S0 + hS) * rel);
        sc[1] = pay(D, (S0 - hS) * rel);
        const double Xv0 = S0 * (ASIAN ? (double)Av0 * pay.inv_nfix : exp((double)xv0));
        const double Xv1 = S0 * (ASIAN ? (double)Av1 * pay.inv_nfix : exp((double)xv1));
        sc[2] = pay(D, Xv0);
        sc[3] = pay(D, Xv1);
        const double Dup = exp(-(L.r + hr) * L.T), Ddn = exp(-(L.r - hr) * L.T);
        double Xu, Xd;
        if (ASIAN) {
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
        const double Xt0 = S0 * (ASIAN ? (double)At0 * pay.inv_nfix : exp((double)xt0));
        const double Xt1 = S0 * (ASIAN ? (double)At1 * pay.inv_nfix : exp((double)xt1));
        sc[6] = pay(exp(-L.r * Tu), Xt0);
        sc[7] = pay(exp(-L.r * Td), Xt1);
        y[EST_DELTA] = (sc[0] - sc[1]) / (2.0 * hS);
        y[EST_GAMMA] = (sc[0] - 2.0 * y[EST_PRICE] + sc[1]) / (hS * hS);
        y[EST_VEGA] = (sc[2] - sc[3]) / (2.0 * L.hv);
        y[EST_RHO] = (sc[4] - sc[5]) / (2.0 * hr);
        y[EST_THETA] = -(sc[6] - sc[7]) / (2.0 * L.hT);
    } else {
#pragma unroll
        for (int e = EST_DELTA; e < N_EST; ++e)
            y[e] = 0.0;
    }

    if (L.pay_out != nullptr && active)
        L.pay_out[p - L.first_path] = y[EST_PRICE];

    if (L.dump != nullptr && active) {
        double *rec = L.dump + (p - L.first_path) * DUMP_WIDTH;
        rec[0] = ST;
        rec[1] = (double)v;
        rec[2] = X;
        rec[3] = y[EST_PRICE];
        rec[4] = y[EST_PW_DELTA];
        rec[5] = y[EST_PW_RHO];
        const double nan = __builtin_nan("");
#pragma unroll
        for (int k = 0; k < 8; ++k)
            rec[6 + k] = BUMPS ? sc[k] : nan;
        rec[14] = (double)x;
        rec[15] = 0.0;
    }

    // ---- FP64 sums: wavefront butterfly, then the block's waves in order ----
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < N_EST; ++e) {
        const double ye = active ? y[e] : 0.0;
        const double s1 = wave_sum(ye);
        const double s2 = wave_sum(ye * ye);
        if (lane == 0) {
            red[wave][2 * e] = s1;
            red[wave][2 * e + 1] = s2;
        }
    }
    __syncthreads();
    if (threadIdx.x < N_ACC) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w)
            s += red[w][threadIdx.x];
        L.partials[((uint64_t)blockIdx.y * L.blocks_per_rep + blockIdx.x) * N_ACC + threadIdx.x] = s;
    }
}

// Sums the partial records of each replicate in a fixed order.
__global__ __launch_bounds__(BLOCK) void reduce_partials(const double *__restrict__ partials,
                                                         uint32_t blocks_per_rep,
                                                         double *__restrict__ rep_sums)
{
    __shared__ double red[BLOCK][N_ACC + 1];
    const double *base = partials + (uint64_t)blockIdx.x * blocks_per_rep * N_ACC;
    double acc[N_ACC];
#pragma unroll
    for (int k = 0; k < N_ACC; ++k)
        acc[k] = 0.0;
    for (uint32_t b = threadIdx.x; b < blocks_per_rep; b += BLOCK)
#pragma unroll
        for (int k = 0; k < N_ACC; ++k)
            acc[k] += base[(uint64_t)b * N_ACC + k];
#pragma unroll
    for (int k = 0; k < N_ACC; ++k)
        red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < (unsigned)s)
#pragma unroll
            for (int k = 0; k < N_ACC; ++k)
                red[threadIdx.x][k] += red[threadIdx.x + s][k];
        __syncthreads();
    }
    if (threadIdx.x < N_ACC)
        rep_sums[(uint64_t)blockIdx.x * N_ACC + threadIdx.x] = red[0][threadIdx.x];
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

// Fixed-order sum of `rows` records of width w (w <= BLOCK): thread k sums column k.
__global__ __launch_bounds__(BLOCK) void reduce_rows_kernel(const double *__restrict__ partials,
                                                            uint32_t rows, uint32_t w,
                                                            double *__restrict__ out)
{
    if (threadIdx.x >= w)
        return;
    double t = 0.0;
    for (uint32_t r = 0; r < rows; ++r)
        t += partials[(uint64_t)r * w + threadIdx.x];
    out[threadIdx.x] = t;
}

// Digital shifts of the Sobol replicates: shift[r][d] = top 30 bits of word 0
// of Philox4x32-10(counter (d, r, 0, 1), key = seed).
__global__ void sobol_shift_kernel(uint64_t seed, uint32_t dims, uint32_t reps, uint32_t *out)
{
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= dims * reps)
        return;
    const uint32_t r = idx / dims, d = idx - r * dims;
    const U4 w = philox4x32_10(U4{d, r, 0u, 1u}, (uint32_t)seed, (uint32_t)(seed >> 32));
    out[idx] = w.x >> 2;
}

template <class R, int RNG, bool ASIAN, bool BUMPS, bool FT>
hipError_t launch_t(const PriceLaunch &L, hipStream_t s)
{
    const dim3 grid(L.blocks_per_rep, L.n_reps);
    const size_t smem = RNG == 1 ? (size_t)L.bridge_depth * 2 * BLOCK * sizeof(R) : 0;
    hipLaunchKernelGGL((price_kernel<R, RNG, ASIAN, BUMPS, FT>), grid, dim3(BLOCK), smem, s, L);
    return hipGetLastError();
}

template <class R, int RNG, bool ASIAN, bool BUMPS>
hipError_t launch_ft(const PriceLaunch &L, hipStream_t s)
{
    return L.scheme == 0 ? launch_t<R, RNG, ASIAN, BUMPS, true>(L, s)
                         : launch_t<R, RNG, ASIAN, BUMPS, false>(L, s);
}

template <class R, int RNG, bool ASIAN>
hipError_t launch_b(const PriceLaunch &L, hipStream_t s)
{
    return L.bumps ? launch_ft<R, RNG, ASIAN, true>(L, s) : launch_ft<R, RNG, ASIAN, false>(L, s);
}

template <class R, int RNG> hipError_t launch_a(const PriceLaunch &L, hipStream_t s)
{
    const bool asian = L.opt_type == 2 || L.opt_type == 3;
    return asian ? launch_b<R, RNG, true>(L, s) : launch_b<R, RNG, false>(L, s);
}

template <class R> hipError_t launch_r(const PriceLaunch &L, hipStream_t s)
{
    return L.rng == 0 ? launch_a<R, 0>(L, s) : launch_a<R, 1>(L, s);
}

} // namespace

hipError_t launch_sobol_shifts(uint64_t seed, uint32_t dims, uint32_t reps, uint32_t *out,
                               hipStream_t stream)
{
    const uint32_t n = dims * reps;
    hipLaunchKernelGGL(sobol_shift_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, seed, dims,
                       reps, out);
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
    hipLaunchKernelGGL(reduce_partials, dim3(L.n_reps), dim3(BLOCK), 0, stream, L.partials,
                       L.blocks_per_rep, rep_sums);
    return hipGetLastError();
}

} // namespace heston
