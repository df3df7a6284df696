// C ABI of libheston: argument checks, the per-request plan (step
// coefficients, fixing mask, Brownian-bridge walk), device scratch owned by a
// context, kernel launches on the context's stream, and the final estimates.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/heston.h"
#include "internal.hpp"
#include "runtime.hpp"

using namespace heston;

namespace heston {
namespace rt {

thread_local std::string g_last_error;

heston_status fail(heston_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

heston_status reserve(heston_ctx *c, DevBuf &b, size_t bytes)
{
    if (b.bytes >= bytes)
        return HESTON_OK;
    bytes = (bytes + 4095) & ~size_t(4095);
    const uint64_t after = c->in_use - b.bytes + bytes;
    if (c->budget && after > c->budget)
        return fail(HESTON_OVER_BUDGET, "device scratch of " + std::to_string(bytes) +
                                            " bytes exceeds the context budget");
    if (b.ptr) {
        (void)hipFree(b.ptr);
        c->in_use -= b.bytes;
        b.ptr = nullptr;
        b.bytes = 0;
    }
    HIP_TRY(hipMalloc(&b.ptr, bytes));
    b.bytes = bytes;
    b.gen = ++c->alloc_gen;
    c->in_use += bytes;
    return HESTON_OK;
}


bool finite_all(const heston_params *p)
{
    const double v[] = {p->S0, p->K, p->r, p->T, p->v0, p->kappa, p->theta, p->sigma, p->rho};
    for (double x : v)
        if (!std::isfinite(x))
            return false;
    return true;
}

heston_status check_params(const heston_params *p)
{
    if (!p)
        return fail(HESTON_INVALID_ARGUMENT, "params is NULL");
    if (!finite_all(p))
        return fail(HESTON_INVALID_ARGUMENT, "params contain NaN or Inf");
    if (!(p->S0 > 0) || !(p->K > 0) || !(p->T > 0))
        return fail(HESTON_INVALID_ARGUMENT, "need S0 > 0, K > 0, T > 0");
    if (!(p->v0 >= 0) || !(p->kappa > 0) || !(p->theta >= 0) || !(p->sigma >= 0))
        return fail(HESTON_INVALID_ARGUMENT, "need v0 >= 0, kappa > 0, theta >= 0, sigma >= 0");
    if (!(std::fabs(p->rho) <= 1))
        return fail(HESTON_INVALID_ARGUMENT, "need |rho| <= 1");
    return HESTON_OK;
}

StepCoef step_coef(const heston_params &p, double T, uint32_t N)
{
    StepCoef c;
    c.dt = T / (double)N;
    c.sqrt_dt = std::sqrt(c.dt);
    c.r_dt = p.r * c.dt;
    c.half_dt = 0.5 * c.dt;
    c.kappa_dt = p.kappa * c.dt;
    c.kappa_theta_dt = p.kappa * p.theta * c.dt;
    c.quarter_sigma2_dt = 0.25 * p.sigma * p.sigma * c.dt;
    return c;
}

// Brownian bridge on the unit grid 0..N: nodes are numbered in the first-in
// first-out bisection order (node 0 is B_N, then midpoints m = floor((l+r)/2)
// of intervals (l, r) with r - l >= 2, children (l, m) then (m, r) queued).
// The kernel walks the grid in time order: before step j it computes, for
// every pending midpoint between j and the smallest end-point already known,
// B_m = a B_j + b B_top + c z_node with a = (r-m)/(r-l), b = (m-l)/(r-l),
// c = sqrt((m-l)(r-m)/(r-l)), pushing each on a stack; then it pops B_{j+1}.
bool bridge_program(uint32_t N, BridgePlan &plan)
{
    std::vector<int32_t> node_of(N + 1, -1), left(N + 1, -1), right(N + 1, -1);
    node_of[N] = 0;
    int32_t k = 1;
    std::deque<std::pair<uint32_t, uint32_t>> q;
    q.emplace_back(0u, N);
    while (!q.empty()) {
        auto [l, r] = q.front();
        q.pop_front();
        if (r - l >= 2) {
            const uint32_t m = (l + r) / 2;
            node_of[m] = k++;
            left[m] = (int32_t)l;
            right[m] = (int32_t)r;
            q.emplace_back(l, m);
            q.emplace_back(m, r);
        }
    }
    plan.start.assign(N + 1, 0);
    plan.ops.clear();
    std::vector<uint32_t> stack{N};
    int depth = 1;
    for (uint32_t j = 0; j < N; ++j) {
        plan.start[j] = (int32_t)plan.ops.size();
        while (stack.back() > j + 1) {
            const uint32_t r = stack.back();
            const uint32_t m = (j + r) / 2;
            // The pending interval must be the bisection tree's (j, r).
            if (node_of[m] < 0 || left[m] != (int32_t)j || right[m] != (int32_t)r)
                return false;
            const double l = j, rr = r, mm = m;
            BridgeOp op;
            op.node = node_of[m];
            op.ad = (rr - mm) / (rr - l);
            op.bd = (mm - l) / (rr - l);
            op.cd = std::sqrt((mm - l) * (rr - mm) / (rr - l));
            op.a = (float)op.ad;
            op.b = (float)op.bd;
            op.c = (float)op.cd;
            plan.ops.push_back(op);
            stack.push_back(m);
            depth = std::max(depth, (int)stack.size());
        }
        if (stack.back() != j + 1)
            return false;
        stack.pop_back();
    }
    plan.start[N] = (int32_t)plan.ops.size();
    plan.depth = depth;
    return plan.ops.size() == (size_t)(N - 1);
}


// Device bitmask of the Asian fixing steps (bit j for step j), or null when
// every step fixes (or the option is European).
static heston_status upload_fix_bits(heston_ctx *c, const Request &q, const uint32_t **out)
{
    const heston_opts &o = q.o;
    *out = nullptr;
    if (q.type < 2 || !o.fixing_steps)
        return HESTON_OK;
    const size_t words = (q.n_steps + 1 + 31) / 32;
    std::vector<uint32_t> bits(words, 0u);
    for (uint32_t i = 0; i < o.n_fixings; ++i)
        bits[o.fixing_steps[i] >> 5] |= 1u << (o.fixing_steps[i] & 31u);
    heston_status st = reserve(c, c->fix_bits, words * 4);
    if (st != HESTON_OK)
        return st;
    HIP_TRY(hipMemcpyAsync(c->fix_bits.ptr, bits.data(), words * 4, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream)); // `bits` is released at return
    *out = (const uint32_t *)c->fix_bits.ptr;
    return HESTON_OK;
}

heston_status check_request(const Request &q)
{
    heston_status st = check_params(&q.p);
    if (st != HESTON_OK)
        return st;
    if (q.type < 0 || q.type > HESTON_GEO_ASIAN_PUT)
        return fail(HESTON_INVALID_ARGUMENT, "unknown option type");
    if (q.n_paths < 2)
        return fail(HESTON_INVALID_ARGUMENT, "need n_paths >= 2");
    if (q.n_steps < 1)
        return fail(HESTON_INVALID_ARGUMENT, "need n_steps >= 1");
    if (q.n_steps > (1u << 20))
        return fail(HESTON_UNSUPPORTED, "n_steps above 1<<20");
    const heston_opts &o = q.o;
    if (o.precision != HESTON_FP64 && o.precision != HESTON_FP32)
        return fail(HESTON_INVALID_ARGUMENT, "unknown precision");
    if (o.rng != HESTON_RNG_PHILOX && o.rng != HESTON_RNG_SOBOL_BRIDGE)
        return fail(HESTON_INVALID_ARGUMENT, "unknown rng");
    if (o.scheme < HESTON_FULL_TRUNCATION || o.scheme > HESTON_EXACT)
        return fail(HESTON_INVALID_ARGUMENT, "unknown scheme");
    if (o.scheme == HESTON_EXACT) {
        if (o.precision != HESTON_FP64)
            return fail(HESTON_UNSUPPORTED, "exact simulation runs in FP64");
        if (o.rng != HESTON_RNG_PHILOX)
            return fail(HESTON_UNSUPPORTED, "exact simulation draws Philox inputs only");
        if ((o.greeks & ~(uint32_t)HESTON_GREEKS_PATHWISE) != 0)
            return fail(HESTON_UNSUPPORTED, "exact simulation gives pathwise Greeks only");
        if (o.control_variate != HESTON_CONTROL_NONE)
            return fail(HESTON_UNSUPPORTED, "exact simulation takes no control variate");
        if (!(q.p.sigma > 0) || !(q.p.theta > 0))
            return fail(HESTON_INVALID_ARGUMENT, "exact simulation needs sigma > 0 and theta > 0");
        if (q.n_steps > HESTON_EXACT_MAX_STEPS)
            return fail(HESTON_UNSUPPORTED, "more exact steps than supported");
    }
    if (o.scheme == HESTON_QE) {
        if (o.rng != HESTON_RNG_PHILOX)
            return fail(HESTON_UNSUPPORTED, "the QE scheme draws Philox inputs only");
        if (!(q.p.sigma > 0) || !(q.p.theta > 0))
            return fail(HESTON_INVALID_ARGUMENT, "the QE scheme needs sigma > 0 and theta > 0");
    }
    if (o.greeks & ~7u)
        return fail(HESTON_INVALID_ARGUMENT, "unknown greeks bits");
    if ((o.greeks & HESTON_GREEKS_BUMP_PLAIN) && (o.greeks & HESTON_GREEKS_BUMP_FUSED))
        return fail(HESTON_INVALID_ARGUMENT, "BUMP_PLAIN and BUMP_FUSED are exclusive");
    if ((o.greeks & HESTON_GREEKS_BUMP_PLAIN) && o.rng != HESTON_RNG_PHILOX)
        return fail(HESTON_UNSUPPORTED, "plain bump-and-revalue needs Philox normals");
    if (o.greeks & (HESTON_GREEKS_BUMP_FUSED | HESTON_GREEKS_BUMP_PLAIN)) {
        const double b[] = {o.bump_S0_rel, o.bump_v0_rel, o.bump_r_abs, o.bump_T_abs};
        for (double x : b)
            if (!std::isfinite(x) || !(x > 0))
                return fail(HESTON_INVALID_ARGUMENT, "bump sizes must be finite and > 0");
        if (!(q.p.v0 > 0))
            return fail(HESTON_INVALID_ARGUMENT, "relative v0 bump needs v0 > 0");
        if (!(o.bump_S0_rel < 1) || !(o.bump_v0_rel < 1) || !(o.bump_T_abs < q.p.T))
            return fail(HESTON_INVALID_ARGUMENT, "bumps must keep S0, v0 and T positive");
        // The fused r bump of an arithmetic Asian sums e^{+-h t_i} over the
        // fixings by its Taylor series in h (through h^3 in FP64, h^2 in
        // FP32): h T is kept where the truncation stays below the parity bar
        // of the precision, (h T)^4 / 24 <= 4.2e-14 and (h T)^3 / 6 <= 4.5e-9.
        if ((o.greeks & HESTON_GREEKS_BUMP_FUSED) &&
            (q.type == HESTON_ASIAN_CALL || q.type == HESTON_ASIAN_PUT) &&
            !(o.bump_r_abs * q.p.T <= (o.precision == HESTON_FP64 ? 1e-3 : 3e-3)))
            return fail(HESTON_INVALID_ARGUMENT,
                        "fused r bump of an arithmetic Asian: bump_r_abs * T must be at most "
                        "1e-3 (FP64) or 3e-3 (FP32); use a smaller bump or plain bumps");
    }
    if (o.reserved != 0)
        return fail(HESTON_INVALID_ARGUMENT, "opts->reserved must be 0");
    if (o.control_variate != HESTON_CONTROL_NONE) {
        if (o.control_variate != HESTON_CONTROL_GEOMETRIC)
            return fail(HESTON_INVALID_ARGUMENT, "unknown control variate");
        if (q.type != HESTON_ASIAN_CALL && q.type != HESTON_ASIAN_PUT)
            return fail(HESTON_INVALID_ARGUMENT,
                        "the geometric control applies to arithmetic-Asian types");
        if (!(q.p.sigma > 0))
            return fail(HESTON_INVALID_ARGUMENT, "the geometric control needs sigma > 0");
        if ((o.fixing_steps ? o.n_fixings : q.n_steps) > HESTON_CONTROL_MAX_FIXINGS)
            return fail(HESTON_UNSUPPORTED, "more fixing dates than the geometric control takes");
        if (o.greeks & HESTON_GREEKS_BUMP_PLAIN)
            return fail(HESTON_UNSUPPORTED, "the control variate runs with the fused kernel only");
    }
    const bool asian = q.type >= 2;
    if (asian && o.fixing_steps) {
        if (o.n_fixings < 1)
            return fail(HESTON_INVALID_ARGUMENT, "n_fixings must be >= 1");
        for (uint32_t i = 0; i < o.n_fixings; ++i) {
            const uint32_t f = o.fixing_steps[i];
            if (f < 1 || f > q.n_steps || (i && f <= o.fixing_steps[i - 1]))
                return fail(HESTON_INVALID_ARGUMENT,
                            "fixing steps must be strictly increasing in [1, n_steps]");
        }
    }
    if (o.rng == HESTON_RNG_SOBOL_BRIDGE) {
        if (o.qmc_replicates < 1 || q.n_paths % o.qmc_replicates)
            return fail(HESTON_INVALID_ARGUMENT, "n_paths must be a multiple of qmc_replicates");
        if (q.n_paths / o.qmc_replicates > (1ull << 30))
            return fail(HESTON_UNSUPPORTED, "more than 2^30 points per replicate");
        if (!o.sobol_directions || o.sobol_dims < 2 * q.n_steps)
            return fail(HESTON_INVALID_ARGUMENT, "need sobol_directions for 2*n_steps dimensions");
        // the kernels map 30-bit coordinates to normals (the upper half by
        // complementing the 30 bits): wider direction numbers are rejected
        for (size_t k = 0; k < (size_t)2 * q.n_steps * 32; ++k)
            if (k % 32 < 30 && (o.sobol_directions[k] >> 30) != 0u)
                return fail(HESTON_INVALID_ARGUMENT, "sobol_directions must be 30-bit numbers");
        if (q.n_paths / o.qmc_replicates < 2)
            return fail(HESTON_INVALID_ARGUMENT, "need >= 2 points per replicate");
    }
    return HESTON_OK;
}

// The launch description of paths first .. first+count-1 of q from the request
// alone: model, scheme, time grids, bump sizes and fixing counts.  Device
// tables and buffers are left null.
void plan_launch(const Request &q, uint64_t first, uint64_t count, PriceLaunch &L)
{
    const heston_params &p = q.p;
    const heston_opts &o = q.o;
    std::memset(&L, 0, sizeof(L));
    L.S0 = p.S0; L.K = p.K; L.r = p.r; L.T = p.T; L.v0 = p.v0;
    L.kappa = p.kappa; L.theta = p.theta; L.sigma = p.sigma; L.rho = p.rho;
    L.rho_bar = std::sqrt(std::max(0.0, 1.0 - p.rho * p.rho));
    L.opt_type = q.type;
    // Euler is the Milstein kernel with the Milstein coefficient at zero.
    const bool euler = o.scheme == HESTON_EULER_FULL_TRUNCATION || o.scheme == HESTON_EULER_ABSORPTION;
    L.scheme = o.scheme == HESTON_EULER_FULL_TRUNCATION ? 0
               : o.scheme == HESTON_EULER_ABSORPTION    ? 1
               : o.scheme == HESTON_PARTIAL_TRUNCATION  ? 3
               : o.scheme == HESTON_REFLECTION          ? 3
                                                        : o.scheme;
    L.reflect = o.scheme == HESTON_REFLECTION;
    L.precision = o.precision;
    L.rng = o.rng;
    L.bumps = (o.greeks & HESTON_GREEKS_BUMP_FUSED) != 0;
    L.cv = o.control_variate == HESTON_CONTROL_GEOMETRIC;
    L.n_steps = q.n_steps;
    L.seed = q.seed;
    L.first_path = first;
    L.n_paths = count;
    L.wide_paths = first + count > (1ull << 32);
    L.base = step_coef(p, p.T, q.n_steps);
    if (euler)
        L.base.quarter_sigma2_dt = 0.0;
    if (L.bumps) {
        L.hS = o.bump_S0_rel * p.S0;
        L.hv = o.bump_v0_rel * p.v0;
        L.hr = o.bump_r_abs;
        L.hT = o.bump_T_abs;
        L.tup = step_coef(p, p.T + L.hT, q.n_steps);
        L.tdn = step_coef(p, p.T - L.hT, q.n_steps);
        if (euler)
            L.tup.quarter_sigma2_dt = L.tdn.quarter_sigma2_dt = 0.0;
    }
    const bool asian = q.type >= 2;
    L.n_fix = asian ? (o.fixing_steps ? o.n_fixings : q.n_steps) : 1;
    // sum of the fixing step indices: the fixing times sum to dt times it
    L.fix_step_sum = 0.0;
    if (o.fixing_steps)
        for (uint32_t i = 0; i < o.n_fixings; ++i)
            L.fix_step_sum += (double)o.fixing_steps[i];
    else
        L.fix_step_sum = 0.5 * (double)q.n_steps * ((double)q.n_steps + 1.0);
}

// Few FP64 paths with fused bumps (Philox, Milstein or Euler, European or
// arithmetic Asian, no control) take one scenario per lane: at most about one
// wave per SIMD, and a wave's work per step roughly halves (price_kernel SPLIT).
bool split_layout(const Request &q, const PriceLaunch &L, uint64_t count)
{
    return q.o.precision == HESTON_FP64 && L.rng == HESTON_RNG_PHILOX && L.bumps && !L.cv &&
           (L.scheme == 0 || L.scheme == 1) && q.type <= HESTON_ASIAN_PUT &&
           count <= (q.type >= HESTON_ASIAN_CALL ? SPLIT_MAX_PATHS_ASIAN : SPLIT_MAX_PATHS_EURO);
}
// Paths per block of the launch.
uint64_t paths_per_block(const PriceLaunch &L)
{
    return L.split ? (uint64_t)(BLOCK / 64) * SPLIT_PATHS_PER_WAVE : BLOCK;
}

// Builds the launch description of paths [first, first+count) of request q
// and uploads its tables into the context's scratch.  Does not launch.
// allow_split: the caller launches the path kernel for estimates only (no
// dumps or per-path payoffs), so the launch may take the split layout.
heston_status plan(heston_ctx *c, const Request &q, uint64_t first, uint64_t count, PriceLaunch &L,
                   bool allow_split = false)
{
    const heston_opts &o = q.o;
    plan_launch(q, first, count, L);
    const bool asian = q.type >= 2;
    const bool geo = q.type == HESTON_GEO_ASIAN_CALL || q.type == HESTON_GEO_ASIAN_PUT;
    {
        heston_status st = upload_fix_bits(c, q, &L.fix_bits);
        if (st != HESTON_OK)
            return st;
    }
    if (asian && !geo) {
        const size_t real = o.precision == HESTON_FP64 ? 8 : 4;
        heston_status st = reserve(c, c->step_w, (size_t)q.n_steps * STEP_WEIGHTS * real);
        if (st != HESTON_OK)
            return st;
        L.step_weights = c->step_w.ptr;
        HIP_TRY(launch_step_weights(L, c->step_w.ptr, c->stream));
    }
    uint64_t M;
    if (o.rng == HESTON_RNG_SOBOL_BRIDGE) {
        const uint32_t R = o.qmc_replicates, dims = 2 * q.n_steps;
        M = q.n_paths / R;
        L.rep0 = (uint32_t)(first / M);
        L.n_reps = (uint32_t)((first + count - 1) / M) - L.rep0 + 1;
        // The tables that do not depend on the seed (direction numbers,
        // bridge walk, the block-aligned walk's position tables and per-block
        // table) are rebuilt only when the step count or the direction numbers
        // change, or when their buffer has been reallocated; the seeded shifts
        // are drawn on every call.
        SobolTables &T = c->sobol;
        const uint32_t N = q.n_steps;
        const size_t dir_words = (size_t)dims * 32;
        if (!(T.n_steps == N && T.dirs.size() == dir_words &&
              std::memcmp(T.dirs.data(), o.sobol_directions, dir_words * 4) == 0)) {
            // the host tables are replaced: let copies still reading them finish
            HIP_TRY(hipStreamSynchronize(c->stream));
            T = SobolTables{};
            if (!bridge_program(N, T.bp))
                return fail(HESTON_DEVICE_ERROR, "internal: Brownian bridge walk inconsistent");
            T.n_steps = N;
            T.dirs.assign(o.sobol_directions, o.sobol_directions + dir_words);
        }
        const BridgePlan &bp = T.bp;
        heston_status st;
        if ((st = reserve(c, c->sobol_dirs, dir_words * 4)) != HESTON_OK ||
            (st = reserve(c, c->sobol_shift, (size_t)dims * R * 4)) != HESTON_OK ||
            (st = reserve(c, c->bridge_start, (N + 1) * 4)) != HESTON_OK ||
            (st = reserve(c, c->bridge_ops, std::max<size_t>(1, bp.ops.size()) * sizeof(BridgeOp))) !=
                HESTON_OK)
            return st;
        if (T.dirs_gen != c->sobol_dirs.gen) {
            HIP_TRY(hipMemcpyAsync(c->sobol_dirs.ptr, T.dirs.data(), dir_words * 4,
                                   hipMemcpyHostToDevice, c->stream));
            T.dirs_gen = c->sobol_dirs.gen;
        }
        // Blocks of 64 consecutive points share their Gray-code bits >= 6; when the
        // launch's waves are block-aligned, the XOR of those bits' direction numbers
        // is tabulated once per block and dimension; the XOR of the direction
        // numbers of the low six bits is tabulated once per node for each of their
        // 64 values; and the shifts and both tables are laid out in the order the
        // bridge walk consumes its nodes, so the kernel addresses them by walk
        // position instead of through each op's node index.  The tables are an
        // accelerator only: without room for them under the context budget (or in
        // device memory) the kernel combines the direction numbers itself.
        L.sobol_hi = nullptr;
        L.sobol_low = nullptr;
        const uint64_t n_blk = (M + 63) / 64, hi_bytes = n_blk * dims * 4;
        // the low-bit table [N+1][64][2] follows the [N][12] direction numbers it is built from
        const uint64_t low_bytes = (uint64_t)N * 48 + ((uint64_t)N + 1) * 512;
        const uint64_t extra = hi_bytes + (uint64_t)N * 4 + low_bytes;
        const uint64_t held = c->sobol_hi.bytes + c->sobol_perm.bytes + c->sobol_low.bytes;
        const bool fits = !c->budget || c->in_use - held + extra + 3 * 4096 <= c->budget;
        bool fast = M % 64 == 0 && (first % M) % 64 == 0 && hi_bytes <= SOBOL_HI_MAX_BYTES && fits;
        if (fast) {
            if ((st = reserve(c, c->sobol_hi, hi_bytes)) == HESTON_OK &&
                (st = reserve(c, c->sobol_perm, (size_t)N * 4)) == HESTON_OK)
                st = reserve(c, c->sobol_low, (size_t)low_bytes);
            if (st == HESTON_OUT_OF_MEMORY || st == HESTON_OVER_BUDGET) {
                g_last_error.clear();
                fast = false;
            } else if (st != HESTON_OK) {
                return st;
            }
        }
        if (fast) {
            if (T.node_of_pos.empty()) {
                T.node_of_pos.resize(N);
                T.node_of_pos[0] = 0;
                for (size_t k = 0; k < bp.ops.size(); ++k)
                    T.node_of_pos[k + 1] = bp.ops[k].node;
                T.dir12.resize((size_t)N * 12);
                for (uint32_t pos = 0; pos < N; ++pos)
                    for (uint32_t mm = 0; mm < 2; ++mm)
                        for (uint32_t b = 0; b < 6; ++b)
                            T.dir12[pos * 12 + mm * 6 + b] =
                                T.dirs[(size_t)(2 * T.node_of_pos[pos] + mm) * 32 + b];
            }
            if (T.perm_gen != c->sobol_perm.gen) {
                HIP_TRY(hipMemcpyAsync(c->sobol_perm.ptr, T.node_of_pos.data(), (size_t)N * 4,
                                       hipMemcpyHostToDevice, c->stream));
                T.perm_gen = c->sobol_perm.gen;
                T.hi_gen = 0; // the per-block table is ordered by this permutation
            }
            uint32_t *d12 = (uint32_t *)c->sobol_low.ptr, *low = d12 + (size_t)N * 12;
            if (T.low_gen != c->sobol_low.gen) {
                HIP_TRY(hipMemcpyAsync(d12, T.dir12.data(), (size_t)N * 48, hipMemcpyHostToDevice,
                                       c->stream));
                HIP_TRY(launch_sobol_low(d12, N, low, c->stream));
                T.low_gen = c->sobol_low.gen;
            }
            const int32_t *perm = (const int32_t *)c->sobol_perm.ptr;
            HIP_TRY(launch_sobol_shifts(q.seed, perm, dims, R, (uint32_t *)c->sobol_shift.ptr,
                                        c->stream));
            if (T.hi_gen != c->sobol_hi.gen || T.hi_blocks != n_blk) {
                HIP_TRY(launch_sobol_hi((const uint32_t *)c->sobol_dirs.ptr, perm, dims,
                                        (uint32_t)n_blk, (uint32_t *)c->sobol_hi.ptr, c->stream));
                T.hi_gen = c->sobol_hi.gen;
                T.hi_blocks = n_blk;
            }
            L.sobol_hi = (const uint32_t *)c->sobol_hi.ptr;
            L.sobol_low = low;
        } else {
            HIP_TRY(launch_sobol_shifts(q.seed, nullptr, dims, R, (uint32_t *)c->sobol_shift.ptr,
                                        c->stream));
        }
        if (T.start_gen != c->bridge_start.gen) {
            HIP_TRY(hipMemcpyAsync(c->bridge_start.ptr, bp.start.data(), (N + 1) * 4,
                                   hipMemcpyHostToDevice, c->stream));
            T.start_gen = c->bridge_start.gen;
        }
        if (!bp.ops.empty() && T.ops_gen != c->bridge_ops.gen) {
            HIP_TRY(hipMemcpyAsync(c->bridge_ops.ptr, bp.ops.data(), bp.ops.size() * sizeof(BridgeOp),
                                   hipMemcpyHostToDevice, c->stream));
            T.ops_gen = c->bridge_ops.gen;
        }
        L.sobol_dirs = (const uint32_t *)c->sobol_dirs.ptr;
        L.sobol_shift = (const uint32_t *)c->sobol_shift.ptr;
        L.bridge_start = (const int32_t *)c->bridge_start.ptr;
        L.bridge_ops = (const BridgeOp *)c->bridge_ops.ptr;
        L.bridge_root_scale = std::sqrt((double)q.n_steps);
        L.bridge_depth = bp.depth;
        if (bp.depth > MAX_BRIDGE_DEPTH)
            return fail(HESTON_UNSUPPORTED, "Brownian bridge deeper than supported");
    } else {
        M = first + count;
        L.rep0 = 0;
        L.n_reps = 1;
    }
    L.paths_per_rep = M;
    const uint64_t span = std::min<uint64_t>(count, M);
    L.split = allow_split && split_layout(q, L, count);
    const uint64_t per_block = paths_per_block(L);
    L.blocks_per_rep = (uint32_t)((span + per_block - 1) / per_block);
    if ((uint64_t)L.blocks_per_rep * per_block < span || L.blocks_per_rep > 0x7FFFFFFFu)
        return fail(HESTON_UNSUPPORTED, "too many paths for one launch");
    heston_status st;
    const size_t W = (size_t)L.acc_width();
    const size_t chunks = (L.blocks_per_rep + REDUCE_CHUNK - 1) / REDUCE_CHUNK; // first level
    if ((st = reserve(c, c->partials, (size_t)L.n_reps * L.blocks_per_rep * W * 8)) != HESTON_OK ||
        (st = reserve(c, c->rep_sums, (size_t)L.n_reps * W * 8)) != HESTON_OK ||
        (chunks > 1 &&
         (st = reserve(c, c->reduce_tmp, (size_t)L.n_reps * chunks * W * 8)) != HESTON_OK))
        return st;
    L.partials = (double *)c->partials.ptr;
    L.reduce_tmp = chunks > 1 ? (double *)c->reduce_tmp.ptr : nullptr;
    if (c->host_sums_bytes < (size_t)L.n_reps * W * 8) {
        if (c->host_sums)
            (void)hipHostFree(c->host_sums);
        c->host_sums = nullptr;
        c->host_sums_dev = nullptr;
        c->host_sums_bytes = 0;
        HIP_TRY(hipHostMalloc((void **)&c->host_sums, (size_t)L.n_reps * W * 8));
        HIP_TRY(hipHostGetDevicePointer((void **)&c->host_sums_dev, c->host_sums, 0));
        c->host_sums_bytes = (size_t)L.n_reps * W * 8;
    }
    return HESTON_OK;
}

heston_est est_from(double n, double s, double ss)
{
    const double m = s / n;
    double var = (ss - s * m) / (n - 1.0);
    if (var < 0)
        var = 0;
    return heston_est{m, std::sqrt(var / n)};
}

// Replicate estimates: mean of the R replicate means, SE = std of them / sqrt(R).
heston_est est_reps(const double *sums, uint32_t R, double M, int e, int W)
{
    double mean = 0;
    for (uint32_t r = 0; r < R; ++r)
        mean += sums[r * W + 2 * e] / M;
    mean /= R;
    double ss = 0;
    for (uint32_t r = 0; r < R; ++r) {
        const double d = sums[r * W + 2 * e] / M - mean;
        ss += d * d;
    }
    return heston_est{mean, R > 1 ? std::sqrt(ss / (R - 1.0) / R) : 0.0};
}

Request make_request(const heston_params *p, heston_option_type type, uint64_t n_paths,
                     uint32_t n_steps, uint64_t seed, const heston_opts *opts)
{
    Request q;
    q.p = p ? *p : heston_params{};
    q.type = (int)type;
    q.n_paths = n_paths;
    q.n_steps = n_steps;
    q.seed = seed;
    heston_default_opts(&q.o);
    if (opts)
        q.o = *opts;
    return q;
}

heston_ctx *default_ctx(heston_status &st)
{
    thread_local std::vector<heston_ctx *> per_device;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        st = fail(HESTON_DEVICE_ERROR, "no HIP device");
        return nullptr;
    }
    if ((int)per_device.size() <= dev)
        per_device.resize(dev + 1, nullptr);
    if (!per_device[dev]) {
        st = heston_ctx_create(dev, nullptr, 0, &per_device[dev]);
        if (st != HESTON_OK)
            return nullptr;
    }
    st = HESTON_OK;
    return per_device[dev];
}

double &param_ref(heston_params &p, int k)
{
    double *f[] = {&p.S0, &p.K, &p.r, &p.T, &p.v0, &p.kappa, &p.theta, &p.sigma, &p.rho};
    return *f[k];
}

// Plain bump-and-revalue: 1 + 2 nb independent launches writing per-path
// payoffs, then per-path differences reduced on the device.  base_sums
// (nullable, host N_ACC doubles) receives the base launch's estimator sums.
heston_status bump_revalue_impl(heston_ctx *c, const Request &q0, const heston_bump *bumps,
                                uint32_t nb, heston_est *price, heston_est *first,
                                heston_est *second, double *device_ms, double *base_sums)
{
    if (nb < 1 || nb > (uint32_t)MAX_BUMPS || !bumps)
        return fail(HESTON_INVALID_ARGUMENT, "need 1..8 bumps");
    if (q0.o.rng != HESTON_RNG_PHILOX)
        return fail(HESTON_UNSUPPORTED, "plain bump-and-revalue needs Philox normals");
    const uint64_t n = q0.n_paths;
    std::vector<Request> qs(1 + 2 * nb, q0);
    BumpScales sc;
    std::memset(&sc, 0, sizeof(sc));
    for (auto &q : qs)
        q.o.greeks = HESTON_GREEKS_PATHWISE;
    for (uint32_t b = 0; b < nb; ++b) {
        const heston_bump &bp = bumps[b];
        if (bp.param < 0 || bp.param > 8 || !std::isfinite(bp.size) || !(bp.size > 0))
            return fail(HESTON_INVALID_ARGUMENT, "bump " + std::to_string(b) + " is invalid");
        heston_params base = q0.p;
        const double h = bp.relative ? bp.size * std::fabs(param_ref(base, bp.param)) : bp.size;
        if (!(h > 0))
            return fail(HESTON_INVALID_ARGUMENT, "bump " + std::to_string(b) + " has size 0");
        param_ref(qs[1 + 2 * b].p, bp.param) += h;
        param_ref(qs[2 + 2 * b].p, bp.param) -= h;
        sc.first[b] = 1.0 / (2.0 * h);
        sc.second[b] = 1.0 / (h * h);
        for (int k = 1; k <= 2; ++k) {
            heston_status st = check_request(qs[k + 2 * b]);
            if (st != HESTON_OK)
                return fail(st, "bumped scenario " + std::to_string(b) + ": " + g_last_error);
        }
    }
    heston_status st;
    const size_t rows = qs.size();
    if ((st = reserve(c, c->pay, rows * n * 8)) != HESTON_OK)
        return st;
    double *pay = (double *)c->pay.ptr;
    HIP_TRY(hipEventRecord(c->ev0, c->stream));
    PriceLaunch L;
    for (size_t s = 0; s < rows; ++s) {
        if ((st = plan(c, qs[s], 0, n, L)) != HESTON_OK)
            return st;
        L.pay_out = pay + s * n;
        HIP_TRY(launch_paths(L, c->stream));
        if (s == 0 && base_sums) {
            HIP_TRY(launch_reduce(L, (double *)c->rep_sums.ptr, c->stream));
            HIP_TRY(hipMemcpyAsync(c->host_sums, c->rep_sums.ptr, N_ACC * 8, hipMemcpyDeviceToHost,
                                   c->stream));
        }
    }
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((n + BLOCK - 1) / BLOCK, 1024);
    if ((st = reserve(c, c->bump_partials, (size_t)blocks * BUMP_W * 8)) != HESTON_OK ||
        (st = reserve(c, c->bump_sums, BUMP_W * 8)) != HESTON_OK)
        return st;
    HIP_TRY(launch_bump_combine(pay, n, nb, sc, (double *)c->bump_partials.ptr, blocks, c->stream));
    HIP_TRY(hipEventRecord(c->ev1, c->stream));
    HIP_TRY(launch_reduce_rows((double *)c->bump_partials.ptr, blocks, BUMP_W,
                               (double *)c->bump_sums.ptr, c->stream));
    double sums[BUMP_W];
    HIP_TRY(hipMemcpyAsync(sums, c->bump_sums.ptr, sizeof(sums), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (base_sums)
        std::memcpy(base_sums, c->host_sums, N_ACC * 8);
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    const double dn = (double)n;
    if (price)
        *price = est_from(dn, sums[0], sums[1]);
    for (uint32_t b = 0; b < nb; ++b) {
        if (first)
            first[b] = est_from(dn, sums[2 + 4 * b], sums[3 + 4 * b]);
        if (second)
            second[b] = est_from(dn, sums[4 + 4 * b], sums[5 + 4 * b]);
    }
    if (device_ms)
        *device_ms = ms;
    return HESTON_OK;
}

heston_status check_adjoint(const Request &q, uint32_t every, const void *ckpt, uint64_t bytes)
{
    heston_status st = check_request(q);
    if (st != HESTON_OK)
        return st;
    if (q.o.rng != HESTON_RNG_PHILOX)
        return fail(HESTON_UNSUPPORTED, "adjoint sensitivities need Philox normals");
    if (q.o.scheme != HESTON_FULL_TRUNCATION && q.o.scheme != HESTON_ABSORPTION &&
        q.o.scheme != HESTON_QE)
        return fail(HESTON_UNSUPPORTED,
                    "adjoint sensitivities follow the Milstein scheme (full truncation or "
                    "absorption) or the QE scheme");
    if (q.o.control_variate != HESTON_CONTROL_NONE)
        return fail(HESTON_UNSUPPORTED, "adjoint calls take no control variate");
    if (q.type > HESTON_ASIAN_PUT)
        return fail(HESTON_UNSUPPORTED, "adjoint sensitivities cover European and arithmetic-Asian payoffs");
    if (!(std::fabs(q.p.rho) < 1))
        return fail(HESTON_INVALID_ARGUMENT, "adjoint needs |rho| < 1");
    if (every != 8 && every != 16)
        return fail(HESTON_INVALID_ARGUMENT, "checkpoint interval must be 8 or 16");
    if (!ckpt)
        return fail(HESTON_INVALID_ARGUMENT, "checkpoint buffer is NULL");
    const uint64_t need =
        ckpt_bytes(q.n_paths, q.n_steps, every, q.o.precision == HESTON_FP64 ? 8 : 4);
    if (bytes < need)
        return fail(HESTON_INVALID_ARGUMENT, "checkpoint buffer smaller than " +
                                                 std::to_string(need) + " bytes");
    return HESTON_OK;
}


// ---------------------------------------------------------------------------
// Fixed device scratch of heston_price_greeks_noalloc: one array per device,
// held until the process ends.  Host code never passes `scratch` itself (its
// name is a host-side stand-in); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) unsigned char scratch[HESTON_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
struct NoallocDevice {
    unsigned char *ptr = nullptr; // device address of `scratch` on this device
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};
static std::mutex g_noalloc_mu;
static NoallocDevice g_noalloc[NOALLOC_MAX_DEVICES];

// Set-up on the current device (first call only): the scratch address and
// the two timing events.
static heston_status noalloc_device(int dev, NoallocDevice **out)
{
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(HESTON_UNSUPPORTED, "device index above the no-allocation limit");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoallocDevice &d = g_noalloc[dev];
    if (!d.ptr) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!d.ev0)
            HIP_TRY(hipEventCreate(&d.ev0));
        if (!d.ev1)
            HIP_TRY(hipEventCreate(&d.ev1));
        d.ptr = (unsigned char *)p;
    }
    *out = &d;
    return HESTON_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// The fixing-date bitmask of q written to dev_bits (device, `words` words) in
// chunks staged through a small host array.
static heston_status noalloc_fix_bits(const Request &q, uint32_t *dev_bits, size_t words,
                                      hipStream_t stream)
{
    constexpr size_t CH = 1024;
    uint32_t chunk[CH];
    uint32_t i = 0; // next fixing step (the steps are strictly increasing)
    for (size_t w0 = 0; w0 < words; w0 += CH) {
        const size_t n = std::min(CH, words - w0);
        std::memset(chunk, 0, sizeof(chunk));
        for (; i < q.o.n_fixings && q.o.fixing_steps[i] < 32 * (w0 + n); ++i) {
            const uint32_t j = q.o.fixing_steps[i];
            chunk[(j >> 5) - w0] |= 1u << (j & 31u);
        }
        HIP_TRY(hipMemcpyAsync(dev_bits + w0, chunk, n * 4, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream)); // `chunk` is refilled next
    }
    return HESTON_OK;
}

} // namespace rt
} // namespace heston

using namespace heston::rt;

extern "C" {

heston_status heston_default_opts(heston_opts *o)
{
    if (!o)
        return fail(HESTON_INVALID_ARGUMENT, "opts is NULL");
    std::memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(heston_opts);
    o->precision = HESTON_FP64;
    o->rng = HESTON_RNG_PHILOX;
    o->scheme = HESTON_FULL_TRUNCATION;
    o->greeks = HESTON_GREEKS_PATHWISE | HESTON_GREEKS_BUMP_FUSED;
    o->qmc_replicates = 16;
    o->bump_S0_rel = 0.01;
    o->bump_v0_rel = 0.01;
    o->bump_r_abs = 1e-4;
    o->bump_T_abs = 1.0 / 365.0;
    return HESTON_OK;
}

heston_status heston_ctx_create(int device, void *hip_stream, uint64_t hbm_budget_bytes,
                                heston_ctx **out)
{
    if (!out)
        return fail(HESTON_INVALID_ARGUMENT, "out is NULL");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1)
        return fail(HESTON_DEVICE_ERROR, "no HIP device");
    if (device < 0 || device >= n)
        return fail(HESTON_INVALID_ARGUMENT, "device index out of range");
    DeviceGuard g(device);
    heston_ctx *c = new heston_ctx;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->budget = hbm_budget_bytes;
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        delete c;
        return fail(HESTON_DEVICE_ERROR, "hipEventCreate failed");
    }
    *out = c;
    return HESTON_OK;
}

heston_status heston_ctx_destroy(heston_ctx *c)
{
    if (!c)
        return fail(HESTON_INVALID_ARGUMENT, "ctx is NULL");
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (DevBuf *b : {&c->partials, &c->rep_sums, &c->fix_bits, &c->sobol_dirs, &c->sobol_shift, &c->sobol_hi, &c->sobol_perm, &c->sobol_low,
                      &c->bridge_start, &c->bridge_ops, &c->pay, &c->bump_partials,
                      &c->geo_buf, &c->geo_partials, &c->geo_steps, &c->exact_scratch,
                      &c->reduce_tmp,
                      &c->bump_sums, &c->step_w, &c->batch_opts, &c->batch_items, &c->batch_partials,
                      &c->batch_sums, &c->batch_counter, &c->batch_scratch})
        if (b->ptr)
            (void)hipFree(b->ptr);
    if (c->host_sums)
        (void)hipHostFree(c->host_sums);
    if (c->host_geo)
        (void)hipHostFree(c->host_geo);
    (void)hipEventDestroy(c->ev0);
    (void)hipEventDestroy(c->ev1);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
        (void)hipEventDestroy(c->fork);
        (void)hipEventDestroy(c->join);
    }
    delete c;
    return HESTON_OK;
}

// Positive nodes and weights of the 16-point Gauss-Legendre rule: Newton's
// method on the three-term recurrence of the Legendre polynomials, from the
// usual cosine first guesses; w = 2 / ((1 - x^2) P16'(x)^2).
static void gauss_legendre16(double x[8], double w[8])
{
    constexpr int n = 16;
    for (int i = 0; i < n / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            double p = 1.0, pm = 0.0;
            for (int k = 1; k <= n; ++k) {
                const double pk = ((2.0 * k - 1.0) * z * p - (k - 1.0) * pm) / k;
                pm = p;
                p = pk;
            }
            dp = n * (z * p - pm) / (z * z - 1.0);
            const double dz = p / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16)
                break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Inputs of the geometric control's device price: model, fixing dates (copied
// to the device when given explicitly), quadrature rule, buffers.
static heston_status geo_control_setup(heston_ctx *c, const Request &q, GeoControl &g)
{
    const heston_params &p = q.p;
    const heston_opts &o = q.o;
    std::memset(&g, 0, sizeof(g));
    g.lnS0 = std::log(p.S0);
    g.K = p.K;
    g.lnK = std::log(p.K);
    g.r = p.r;
    g.T = p.T;
    g.v0 = p.v0;
    g.kappa = p.kappa;
    g.theta = p.theta;
    g.sigma = p.sigma;
    g.rho = p.rho;
    g.dt = p.T / q.n_steps;
    g.n_fix = o.fixing_steps ? o.n_fixings : q.n_steps;
    heston_status st;
    if (o.fixing_steps) {
        if ((st = reserve(c, c->geo_steps, (size_t)o.n_fixings * 4)) != HESTON_OK)
            return st;
        HIP_TRY(hipMemcpyAsync(c->geo_steps.ptr, o.fixing_steps, (size_t)o.n_fixings * 4,
                               hipMemcpyHostToDevice, c->stream));
        g.steps = (const uint32_t *)c->geo_steps.ptr;
    }
    // First integration range: where a normal ln G with the variance of the
    // average of a Brownian motion of variance rate min(v0, theta) (the slower
    // decay of the two levels) has decayed, exp(-v^2 s^2 / 2) = e^-39, times 3
    // for the heavier tails of the Heston transform; a power of two in [64,
    // GEO_MAX_FIXED_RANGE].  If the transform has not decayed there, the
    // device search takes over.
    {
        const uint32_t n = g.n_fix;
        double mm = 0; // sum over i, j of min(t_i, t_j), times in increasing order
        for (uint32_t k = 0; k < n; ++k)
            mm += (o.fixing_steps ? (double)o.fixing_steps[k] : (double)(k + 1)) * g.dt *
                  (2.0 * (n - k) - 1.0);
        const double vmin = std::min(p.v0, p.theta) > 0 ? std::min(p.v0, p.theta)
                                                        : std::max(p.v0, p.theta);
        const double s2 = vmin * mm / ((double)n * n);
        const double v = s2 > 0 ? 3.0 * std::sqrt(78.0 / s2) : 1e300;
        uint32_t range = 64;
        while (range < GEO_MAX_FIXED_RANGE && range < v)
            range *= 2;
        g.v_max = range;
    }
    static const struct Rule {
        double x[8], w[8];
        Rule() { gauss_legendre16(x, w); }
    } rule;
    std::memcpy(g.gl_x, rule.x, sizeof(g.gl_x));
    std::memcpy(g.gl_w, rule.w, sizeof(g.gl_w));
    if ((st = reserve(c, c->geo_buf, GEO_BUF_DOUBLES * 8)) != HESTON_OK ||
        (st = reserve(c, c->geo_partials, (size_t)geo_node_blocks() * 8)) != HESTON_OK)
        return st;
    if (!c->host_geo)
        HIP_TRY(hipHostMalloc((void **)&c->host_geo, 2 * sizeof(double)));
    if (!c->side) {
        HIP_TRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&c->join, hipEventDisableTiming));
    }
    return HESTON_OK;
}

// Control-variate estimate from the replicate sums of a (arithmetic payoff),
// g (geometric payoff) and a - g: beta = Cov(a, g) / Var(g) over all paths,
// with Cov(a, g) = (Var(a) + Var(g) - Var(a - g)) / 2.
static void cv_combine(const double *s, const PriceLaunch &L, bool reps, uint64_t n_paths,
                       double mu, heston_result &r)
{
    const int W = N_ACC_CV;
    double Sa = 0, Saa = 0, Sg = 0, Sgg = 0, Sd = 0, Sdd = 0;
    for (uint32_t k = 0; k < L.n_reps; ++k) {
        const double *x = s + (size_t)k * W;
        Sa += x[2 * EST_PRICE];
        Saa += x[2 * EST_PRICE + 1];
        Sg += x[2 * EST_CV_GEO];
        Sgg += x[2 * EST_CV_GEO + 1];
        Sd += x[2 * EST_CV_DIFF];
        Sdd += x[2 * EST_CV_DIFF + 1];
    }
    const double n = (double)n_paths;
    auto var = [n](double S, double SS) { return (SS - S * (S / n)) / (n - 1.0); };
    const double va = var(Sa, Saa), vg = var(Sg, Sgg), vd = var(Sd, Sdd);
    const double cov = 0.5 * (va + vg - vd);
    const double beta = vg > 0 ? cov / vg : 0.0;
    heston_est e;
    if (!reps) {
        e.value = Sa / n - beta * (Sg / n - mu);
        e.std_err = std::sqrt(std::max(va - beta * cov, 0.0) / n);
    } else {
        const double M = (double)L.paths_per_rep;
        const uint32_t R = L.n_reps;
        double m = 0;
        for (uint32_t k = 0; k < R; ++k)
            m += s[(size_t)k * W + 2 * EST_PRICE] / M -
                 beta * (s[(size_t)k * W + 2 * EST_CV_GEO] / M - mu);
        m /= R;
        double ss = 0;
        for (uint32_t k = 0; k < R; ++k) {
            const double d = s[(size_t)k * W + 2 * EST_PRICE] / M -
                             beta * (s[(size_t)k * W + 2 * EST_CV_GEO] / M - mu) - m;
            ss += d * d;
        }
        e.value = m;
        e.std_err = R > 1 ? std::sqrt(ss / (R - 1.0) / R) : 0.0;
    }
    r.cv_price = e;
    r.cv_beta = beta;
    r.cv_mean = mu;
    r.valid_mask |= HESTON_VALID_CONTROL;
}

// Exact simulation of paths first .. first+count-1: sums[EXACT_REC] receives
// the FP64 estimator sums (price, pathwise Delta and Rho as (sum, sum of
// squares)) and, at N_ACC, the number of failed paths.
static heston_status run_exact(heston_ctx *c, const Request &q, uint64_t first, uint64_t count,
                               double *dump, double *sums, float *ms)
{
    const heston_params &p = q.p;
    ExactLaunch E;
    std::memset(&E, 0, sizeof(E));
    E.S0 = p.S0; E.K = p.K; E.r = p.r; E.T = p.T; E.v0 = p.v0;
    E.kappa = p.kappa; E.theta = p.theta; E.sigma = p.sigma; E.rho = p.rho;
    E.rho_bar = std::sqrt(std::max(0.0, 1.0 - p.rho * p.rho));
    E.D = p.T / q.n_steps;
    const double s2 = p.sigma * p.sigma;
    const double ek = std::exp(-p.kappa * E.D);
    E.ekD = ek;
    E.c = s2 * (1.0 - ek) / (4.0 * p.kappa);
    E.d = 4.0 * p.kappa * p.theta / s2;
    E.nu = 2.0 * p.kappa * p.theta / s2 - 1.0;
    E.kappa2 = p.kappa * p.kappa;
    E.two_sigma2 = 2.0 * s2;
    E.sigma2 = s2;
    E.inv_sigma2 = 1.0 / s2;
    E.t1_const = std::log(1.0 - ek) - std::log(p.kappa) + 0.5 * p.kappa * E.D;
    E.coth_k = p.kappa * (1.0 + ek) / (1.0 - ek);
    E.log_zk_scale = std::log(4.0 * p.kappa) - 0.5 * p.kappa * E.D - std::log(s2 * (1.0 - ek));
    E.log4_over_sigma2 = std::log(4.0 / s2);
    E.opt_type = q.type;
    E.n_steps = q.n_steps;
    E.n_fix = q.type >= 2 ? (q.o.fixing_steps ? q.o.n_fixings : q.n_steps) : 1;
    E.seed = q.seed;
    E.first_path = first;
    E.n_paths = count;
    E.n_lanes = (uint32_t)std::min<uint64_t>((count + BLOCK - 1) / BLOCK * BLOCK, EXACT_MAX_LANES);
    heston_status st;
    if ((st = upload_fix_bits(c, q, &E.fix_bits)) != HESTON_OK ||
        (st = reserve(c, c->exact_scratch, (size_t)EXACT_MAX_GRID * E.n_lanes * 8)) != HESTON_OK ||
        (st = reserve(c, c->partials, (size_t)(E.n_lanes / BLOCK) * EXACT_REC * 8)) != HESTON_OK ||
        (st = reserve(c, c->rep_sums, EXACT_REC * 8)) != HESTON_OK)
        return st;
    E.scratch = (double *)c->exact_scratch.ptr;
    E.partials = (double *)c->partials.ptr;
    E.dump = dump;
    HIP_TRY(hipEventRecord(c->ev0, c->stream));
    HIP_TRY(launch_exact(E, c->stream));
    HIP_TRY(hipEventRecord(c->ev1, c->stream));
    HIP_TRY(launch_reduce_rows(E.partials, E.n_lanes / BLOCK, EXACT_REC,
                               (double *)c->rep_sums.ptr, c->stream));
    HIP_TRY(hipMemcpyAsync(sums, c->rep_sums.ptr, EXACT_REC * 8, hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (ms)
        HIP_TRY(hipEventElapsedTime(ms, c->ev0, c->ev1));
    return HESTON_OK;
}

static heston_status price_greeks_impl(heston_ctx *c, const heston_params *params,
                                       heston_option_type type, uint64_t n_paths,
                                       uint32_t n_steps, uint64_t seed, const heston_opts *opts,
                                       heston_result *out)
{
    if (!c || !out)
        return fail(HESTON_INVALID_ARGUMENT, "ctx or out is NULL");
    if (opts && opts->struct_size != sizeof(heston_opts))
        return fail(HESTON_INVALID_ARGUMENT, "opts->struct_size does not match this library");
    const Request q = make_request(params, type, n_paths, n_steps, seed, opts);
    heston_status st = check_request(q);
    if (st != HESTON_OK)
        return st;
    DeviceGuard g(c->device);
    if (q.o.scheme == HESTON_EXACT) {
        double sums[EXACT_REC];
        float ms = 0;
        if ((st = run_exact(c, q, 0, n_paths, nullptr, sums, &ms)) != HESTON_OK)
            return st;
        if (sums[N_ACC] > 0)
            return fail(HESTON_UNSUPPORTED,
                        std::to_string((uint64_t)sums[N_ACC]) +
                            " paths left the exact sampler's range (Bessel series, grid length, "
                            "Poisson mean or gamma rejections)");
        heston_result r;
        std::memset(&r, 0, sizeof(r));
        r.price = est_from((double)n_paths, sums[0], sums[1]);
        r.pw_delta = est_from((double)n_paths, sums[2], sums[3]);
        r.pw_rho = est_from((double)n_paths, sums[4], sums[5]);
        r.n_paths = n_paths;
        r.valid_mask = HESTON_VALID_PRICE | HESTON_VALID_PATHWISE;
        r.device_ms = ms;
        *out = r;
        return HESTON_OK;
    }
    if (q.o.greeks & HESTON_GREEKS_BUMP_PLAIN) {
        // five Greeks from four central bumps, each scenario revalued on its own
        const heston_bump bumps[4] = {{HESTON_P_S0, 1, q.o.bump_S0_rel},
                                      {HESTON_P_V0, 1, q.o.bump_v0_rel},
                                      {HESTON_P_R, 0, q.o.bump_r_abs},
                                      {HESTON_P_T, 0, q.o.bump_T_abs}};
        heston_est price, first[4], second[4];
        double sums[N_ACC], ms = 0;
        if ((st = bump_revalue_impl(c, q, bumps, 4, &price, first, second, &ms, sums)) != HESTON_OK)
            return st;
        heston_result r;
        std::memset(&r, 0, sizeof(r));
        r.price = est_from((double)n_paths, sums[0], sums[1]);
        r.pw_delta = est_from((double)n_paths, sums[2], sums[3]);
        r.pw_rho = est_from((double)n_paths, sums[4], sums[5]);
        r.delta = first[0];
        r.gamma = second[0];
        r.vega = first[1];
        r.rho = first[2];
        r.theta = heston_est{-first[3].value, first[3].std_err};
        r.n_paths = n_paths;
        r.valid_mask = HESTON_VALID_PRICE | HESTON_VALID_PATHWISE | HESTON_VALID_BUMPS;
        r.device_ms = ms;
        *out = r;
        return HESTON_OK;
    }
    PriceLaunch L;
    if ((st = plan(c, q, 0, n_paths, L, true)) != HESTON_OK)
        return st;
    L.dump = nullptr;
    GeoControl gc;
    if (L.cv) {
        // the control's price (latency-bound, few waves) runs on the side
        // stream while the path kernel fills the device
        if ((st = geo_control_setup(c, q, gc)) != HESTON_OK)
            return st;
        HIP_TRY(hipEventRecord(c->fork, c->stream));
        HIP_TRY(hipStreamWaitEvent(c->side, c->fork, 0));
        HIP_TRY(launch_geo_price_fixed(gc, (double *)c->geo_partials.ptr,
                                       (double *)c->geo_buf.ptr, c->side));
        HIP_TRY(hipEventRecord(c->join, c->side));
    }
    HIP_TRY(hipEventRecord(c->ev0, c->stream));
    HIP_TRY(launch_paths(L, c->stream));
    HIP_TRY(hipEventRecord(c->ev1, c->stream));
    // the last reduction level writes the sums into the pinned host buffer
    // (no copy launch); the host reads them after the stream synchronises
    HIP_TRY(launch_reduce(L, c->host_sums_dev, c->stream));
    double *geo_out = c->host_geo; // pinned (set up with the control)
    if (L.cv) {
        HIP_TRY(hipStreamWaitEvent(c->stream, c->join, 0));
        HIP_TRY(hipMemcpyAsync(geo_out, (double *)c->geo_buf.ptr + GEO_OUT, 2 * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (L.cv && !(std::isfinite(geo_out[0]) && std::isfinite(geo_out[1]))) {
        // the transform had not decayed by the end of the fixed range: search
        HIP_TRY(launch_geo_price_search(gc, (double *)c->geo_partials.ptr,
                                        (double *)c->geo_buf.ptr, c->stream));
        HIP_TRY(hipMemcpyAsync(geo_out, (double *)c->geo_buf.ptr + GEO_OUT, 2 * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));

    heston_result r;
    std::memset(&r, 0, sizeof(r));
    const double *s = c->host_sums;
    heston_est *slot[N_EST] = {&r.price, &r.pw_delta, &r.pw_rho, &r.delta,
                               &r.gamma, &r.vega,     &r.rho,    &r.theta};
    const int n_est = L.bumps ? N_EST : EST_DELTA;
    for (int e = 0; e < n_est; ++e)
        *slot[e] = q.o.rng == HESTON_RNG_SOBOL_BRIDGE
                       ? est_reps(s, L.n_reps, (double)L.paths_per_rep, e, L.acc_width())
                       : est_from((double)n_paths, s[2 * e], s[2 * e + 1]);
    r.n_paths = n_paths;
    r.valid_mask = HESTON_VALID_PRICE | HESTON_VALID_PATHWISE | (L.bumps ? HESTON_VALID_BUMPS : 0u);
    r.device_ms = ms;
    if (L.cv) {
        const double mu = q.type == HESTON_ASIAN_CALL ? geo_out[0] : geo_out[1];
        if (!std::isfinite(mu))
            return fail(HESTON_UNSUPPORTED,
                        "the geometric control's transform has not decayed by v = 2^14");
        cv_combine(s, L, q.o.rng == HESTON_RNG_SOBOL_BRIDGE, n_paths, mu, r);
    }
    *out = r;
    return HESTON_OK;
}

heston_status heston_price_greeks_ex(heston_ctx *c, const heston_params *params,
                                     heston_option_type type, uint64_t n_paths, uint32_t n_steps,
                                     uint64_t seed, const heston_opts *opts, heston_result *out)
{
    const auto t0 = std::chrono::steady_clock::now();
    const heston_status st = price_greeks_impl(c, params, type, n_paths, n_steps, seed, opts, out);
    if (st == HESTON_OK)
        out->latency_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

heston_status heston_price_greeks(const heston_params *params, heston_option_type type,
                                  uint64_t n_paths, uint32_t n_steps, uint64_t seed,
                                  heston_result *out)
{
    heston_status st;
    heston_ctx *c = default_ctx(st);
    if (!c)
        return st;
    return heston_price_greeks_ex(c, params, type, n_paths, n_steps, seed, nullptr, out);
}

heston_status heston_dump_paths(heston_ctx *c, const heston_params *params,
                                heston_option_type type, uint64_t n_paths, uint32_t n_steps,
                                uint64_t seed, const heston_opts *opts, uint64_t first,
                                uint64_t count, double *out_dev)
{
    if (!c || !out_dev)
        return fail(HESTON_INVALID_ARGUMENT, "ctx or out_dev is NULL");
    if (opts && opts->struct_size != sizeof(heston_opts))
        return fail(HESTON_INVALID_ARGUMENT, "opts->struct_size does not match this library");
    const Request q = make_request(params, type, n_paths, n_steps, seed, opts);
    heston_status st = check_request(q);
    if (st != HESTON_OK)
        return st;
    if (count == 0)
        return HESTON_OK;
    if (q.o.rng == HESTON_RNG_SOBOL_BRIDGE && (first >= n_paths || count > n_paths - first))
        return fail(HESTON_INVALID_ARGUMENT, "dump range beyond n_paths of a Sobol request");
    if (first + count < first)
        return fail(HESTON_INVALID_ARGUMENT, "dump range overflows");
    DeviceGuard g(c->device);
    if (q.o.scheme == HESTON_EXACT) {
        double sums[EXACT_REC];
        return run_exact(c, q, first, count, out_dev, sums, nullptr);
    }
    PriceLaunch L;
    if ((st = plan(c, q, first, count, L)) != HESTON_OK)
        return st;
    L.dump = out_dev;
    HIP_TRY(launch_paths(L, c->stream));
    HIP_TRY(launch_reduce(L, (double *)c->rep_sums.ptr, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return HESTON_OK;
}

heston_status heston_bump_revalue(heston_ctx *c, const heston_params *params,
                                  heston_option_type type, uint64_t n_paths, uint32_t n_steps,
                                  uint64_t seed, const heston_opts *opts,
                                  const heston_bump *bumps, uint32_t n_bumps, heston_est *price,
                                  heston_est *first, heston_est *second, double *device_ms)
{
    if (!c)
        return fail(HESTON_INVALID_ARGUMENT, "ctx is NULL");
    if (opts && opts->struct_size != sizeof(heston_opts))
        return fail(HESTON_INVALID_ARGUMENT, "opts->struct_size does not match this library");
    Request q = make_request(params, type, n_paths, n_steps, seed, opts);
    q.o.greeks = HESTON_GREEKS_PATHWISE;
    heston_status st = check_request(q);
    if (st != HESTON_OK)
        return st;
    if (q.o.control_variate != HESTON_CONTROL_NONE)
        return fail(HESTON_UNSUPPORTED, "bump-and-revalue takes no control variate");
    DeviceGuard g(c->device);
    return bump_revalue_impl(c, q, bumps, n_bumps, price, first, second, device_ms, nullptr);
}

uint64_t heston_adjoint_ckpt_bytes(uint64_t n_paths, uint32_t n_steps, uint32_t every,
                                   int32_t precision)
{
    if (every == 0 || n_steps == 0 || (precision != HESTON_FP64 && precision != HESTON_FP32))
        return 0;
    return ckpt_bytes(n_paths, n_steps, every, precision == HESTON_FP64 ? 8 : 4);
}

heston_status heston_adjoint_forward(heston_ctx *c, const heston_params *params,
                                     heston_option_type type, uint64_t n_paths, uint32_t n_steps,
                                     uint64_t seed, const heston_opts *opts, uint32_t every,
                                     void *ckpt_dev, uint64_t ckpt_nbytes, heston_est *price,
                                     double *device_ms)
{
    if (!c || !price)
        return fail(HESTON_INVALID_ARGUMENT, "ctx or price is NULL");
    if (opts && opts->struct_size != sizeof(heston_opts))
        return fail(HESTON_INVALID_ARGUMENT, "opts->struct_size does not match this library");
    Request q = make_request(params, type, n_paths, n_steps, seed, opts);
    q.o.greeks = HESTON_GREEKS_PATHWISE;
    heston_status st = check_adjoint(q, every, ckpt_dev, ckpt_nbytes);
    if (st != HESTON_OK)
        return st;
    DeviceGuard g(c->device);
    PriceLaunch L;
    if ((st = plan(c, q, 0, n_paths, L)) != HESTON_OK)
        return st;
    L.ckpt = ckpt_dev;
    L.ckpt_every = every;
    HIP_TRY(hipEventRecord(c->ev0, c->stream));
    HIP_TRY(launch_adjoint_forward(L, c->stream));
    HIP_TRY(hipEventRecord(c->ev1, c->stream));
    HIP_TRY(launch_reduce(L, (double *)c->rep_sums.ptr, c->stream));
    HIP_TRY(hipMemcpyAsync(c->host_sums, c->rep_sums.ptr, N_ACC * 8, hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    *price = est_from((double)n_paths, c->host_sums[0], c->host_sums[1]);
    if (device_ms)
        *device_ms = ms;
    return HESTON_OK;
}

heston_status heston_adjoint_backward(heston_ctx *c, const heston_params *params,
                                      heston_option_type type, uint64_t n_paths,
                                      uint32_t n_steps, uint64_t seed, const heston_opts *opts,
                                      uint32_t every, const void *ckpt_dev, uint64_t ckpt_nbytes,
                                      double dprice, heston_est grads[7], double *per_path_dev,
                                      double *device_ms)
{
    if (!c || !grads)
        return fail(HESTON_INVALID_ARGUMENT, "ctx or grads is NULL");
    if (opts && opts->struct_size != sizeof(heston_opts))
        return fail(HESTON_INVALID_ARGUMENT, "opts->struct_size does not match this library");
    if (!std::isfinite(dprice))
        return fail(HESTON_INVALID_ARGUMENT, "dprice is not finite");
    Request q = make_request(params, type, n_paths, n_steps, seed, opts);
    q.o.greeks = HESTON_GREEKS_PATHWISE;
    heston_status st = check_adjoint(q, every, ckpt_dev, ckpt_nbytes);
    if (st != HESTON_OK)
        return st;
    DeviceGuard g(c->device);
    PriceLaunch L;
    if ((st = plan(c, q, 0, n_paths, L)) != HESTON_OK)
        return st;
    L.ckpt = const_cast<void *>(ckpt_dev);
    L.ckpt_every = every;
    HIP_TRY(hipEventRecord(c->ev0, c->stream));
    HIP_TRY(launch_adjoint(L, dprice, per_path_dev, c->stream));
    HIP_TRY(hipEventRecord(c->ev1, c->stream));
    HIP_TRY(launch_reduce(L, (double *)c->rep_sums.ptr, c->stream));
    HIP_TRY(hipMemcpyAsync(c->host_sums, c->rep_sums.ptr, N_ACC * 8, hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    for (int k = 0; k < 7; ++k)
        grads[k] = est_from((double)n_paths, c->host_sums[2 * (k + 1)], c->host_sums[2 * (k + 1) + 1]);
    if (device_ms)
        *device_ms = ms;
    return HESTON_OK;
}

heston_status heston_price_greeks_noalloc(const heston_params *params, heston_option_type type,
                                          uint64_t n_paths, uint32_t n_steps, uint64_t seed,
                                          const heston_opts *opts, void *hip_stream,
                                          heston_result *out)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!out)
        return fail(HESTON_INVALID_ARGUMENT, "out is NULL");
    if (opts && opts->struct_size != sizeof(heston_opts))
        return fail(HESTON_INVALID_ARGUMENT, "opts->struct_size does not match this library");
    const Request q = make_request(params, type, n_paths, n_steps, seed, opts);
    heston_status st = check_request(q);
    if (st != HESTON_OK)
        return st;
    if (q.o.rng != HESTON_RNG_PHILOX)
        return fail(HESTON_UNSUPPORTED, "the no-allocation call takes Philox normals only");
    if (q.o.scheme == HESTON_EXACT)
        return fail(HESTON_UNSUPPORTED, "the no-allocation call does not run exact simulation");
    if (q.o.greeks & HESTON_GREEKS_BUMP_PLAIN)
        return fail(HESTON_UNSUPPORTED, "the no-allocation call gives fused bumps only");
    if (q.o.control_variate != HESTON_CONTROL_NONE)
        return fail(HESTON_UNSUPPORTED, "the no-allocation call takes no control variate");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    NoallocDevice *d = nullptr;
    if ((st = noalloc_device(dev, &d)) != HESTON_OK)
        return st;
    hipStream_t stream = (hipStream_t)hip_stream;

    PriceLaunch L;
    plan_launch(q, 0, n_paths, L);
    L.rep0 = 0;
    L.n_reps = 1;
    L.paths_per_rep = n_paths;
    L.split = split_layout(q, L, n_paths); // as the context call lays it out
    const uint64_t per_block = paths_per_block(L);
    L.blocks_per_rep =
        (uint32_t)std::min<uint64_t>((n_paths + per_block - 1) / per_block, 0xFFFFFFFFu);
    // scratch layout: fixing bitmask, fixing weights, block partials,
    // first-level sums, estimator sums (each 256-byte aligned)
    const bool asian = q.type >= 2;
    const bool geo = q.type == HESTON_GEO_ASIAN_CALL || q.type == HESTON_GEO_ASIAN_PUT;
    const size_t W = (size_t)L.acc_width();
    const size_t words = (asian && q.o.fixing_steps) ? (q.n_steps + 1 + 31) / 32 : 0;
    const size_t weights =
        (asian && !geo) ? (size_t)q.n_steps * STEP_WEIGHTS * (q.o.precision == HESTON_FP64 ? 8 : 4) : 0;
    const size_t chunks = (L.blocks_per_rep + REDUCE_CHUNK - 1) / REDUCE_CHUNK;
    const size_t o_bits = 0, o_w = align256(o_bits + words * 4);
    const size_t o_part = align256(o_w + weights);
    const size_t o_tmp = align256(o_part + (size_t)L.blocks_per_rep * W * 8);
    const size_t o_sums = align256(o_tmp + (chunks > 1 ? chunks * W * 8 : 0));
    const size_t need = o_sums + W * 8;
    if ((uint64_t)L.blocks_per_rep * per_block < n_paths || need > HESTON_NOALLOC_SCRATCH_BYTES)
        return fail(HESTON_OVER_BUDGET,
                    "the request needs " + std::to_string(need) +
                        " bytes of device scratch, more than the no-allocation call's fixed " +
                        std::to_string((size_t)HESTON_NOALLOC_SCRATCH_BYTES));
    unsigned char *base = d->ptr;
    if (words) {
        if ((st = noalloc_fix_bits(q, (uint32_t *)(base + o_bits), words, stream)) != HESTON_OK)
            return st;
        L.fix_bits = (const uint32_t *)(base + o_bits);
    }
    if (weights) {
        L.step_weights = base + o_w;
        HIP_TRY(launch_step_weights(L, base + o_w, stream));
    }
    L.partials = (double *)(base + o_part);
    L.reduce_tmp = chunks > 1 ? (double *)(base + o_tmp) : nullptr;
    L.dump = nullptr;
    double *dev_sums = (double *)(base + o_sums);
    double sums[N_ACC];
    HIP_TRY(hipEventRecord(d->ev0, stream));
    HIP_TRY(launch_paths(L, stream));
    HIP_TRY(hipEventRecord(d->ev1, stream));
    HIP_TRY(launch_reduce(L, dev_sums, stream));
    HIP_TRY(hipMemcpyAsync(sums, dev_sums, W * 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, d->ev0, d->ev1));

    heston_result r;
    std::memset(&r, 0, sizeof(r));
    heston_est *slot[N_EST] = {&r.price, &r.pw_delta, &r.pw_rho, &r.delta,
                               &r.gamma, &r.vega,     &r.rho,    &r.theta};
    const int n_est = L.bumps ? N_EST : EST_DELTA;
    for (int e = 0; e < n_est; ++e)
        *slot[e] = est_from((double)n_paths, sums[2 * e], sums[2 * e + 1]);
    r.n_paths = n_paths;
    r.valid_mask = HESTON_VALID_PRICE | HESTON_VALID_PATHWISE | (L.bumps ? HESTON_VALID_BUMPS : 0u);
    r.device_ms = ms;
    r.latency_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = r;
    return HESTON_OK;
}

const char *heston_status_str(heston_status s)
{
    switch (s) {
    case HESTON_OK: return "ok";
    case HESTON_PENDING: return "pending";
    case HESTON_INVALID_ARGUMENT: return "invalid argument";
    case HESTON_OUT_OF_MEMORY: return "out of device memory";
    case HESTON_OVER_BUDGET: return "over the context's memory budget";
    case HESTON_DEVICE_ERROR: return "device error";
    case HESTON_UNSUPPORTED: return "unsupported";
    case HESTON_NOT_FOUND: return "not found";
    }
    return "unknown status";
}

const char *heston_last_error(void) { return g_last_error.c_str(); }

int heston_abi_version(void) { return HESTON_ABI_VERSION; }

} // extern "C"
