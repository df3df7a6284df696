// Host-side description of one pricing launch, shared by the C-ABI layer
// (api.hip) and the kernel launchers (price_kernel.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heston {

// Estimators reduced across paths, each as (sum, sum of squares) in FP64.
enum Estimator : int {
    EST_PRICE = 0,
    EST_PW_DELTA,
    EST_PW_RHO,
    EST_DELTA,
    EST_GAMMA,
    EST_VEGA,
    EST_RHO,
    EST_THETA,
    N_EST
};
constexpr int N_ACC = 2 * N_EST;   // doubles per partial record
// Records per block of the first level of a long reduction.
constexpr uint32_t REDUCE_CHUNK = 256;
// The arithmetic-Asian kernel with the geometric control adds two estimators:
// the geometric payoff g and the difference a - g of the two payoffs.
enum : int { EST_CV_GEO = N_EST, EST_CV_DIFF, N_EST_CV };
constexpr int N_ACC_CV = 2 * N_EST_CV;
constexpr int DUMP_WIDTH = 16;
constexpr int BLOCK = 256;         // threads per block of the path kernels
constexpr int MAX_BRIDGE_DEPTH = 24;
// Fourth Philox counter word of the QE scheme's per-step block.
constexpr uint32_t QE_COUNTER_TAG = 4u;
// Largest per-block Sobol table (ceil(M/64) x 2N words) built for a launch;
// above it the kernel combines the high direction numbers itself.
// Scenario-split layout of small FP64 bump launches (price_kernel SPLIT):
// paths per wave, and the largest launches it is used for, measured crossovers
// with the fused layout at 100 steps: about three waves per SIMD for European
// payoffs, eight for arithmetic Asians (whose fixings lengthen the fused step).
constexpr uint32_t SPLIT_PATHS_PER_WAVE = 12;
constexpr uint64_t SPLIT_MAX_PATHS_EURO = 36864;
constexpr uint64_t SPLIT_MAX_PATHS_ASIAN = 98304;
constexpr uint64_t SOBOL_HI_MAX_BYTES = 256ull << 20;
// Fixing weights per step j (fixing time t = (j+1) dt): e^{rt}, t e^{rt},
// t^2 e^{rt}, t^3 e^{rt} on the base grid, e^{rt} on the T + hT and T - hT grids.
constexpr int STEP_WEIGHTS = 8;

// Step coefficients of one time grid (dt = T/N of a scenario), computed once
// on the host in FP64.
struct StepCoef {
    double dt, sqrt_dt, r_dt, half_dt, kappa_dt, kappa_theta_dt, quarter_sigma2_dt;
};

// Brownian-bridge walk in time order (see bridge_program in api.hip).
struct BridgeOp {
    int32_t node;     // node index k: Sobol coordinates 2k (price) and 2k+1 (variance)
    float a, b, c;    // B_m = a B_cur + b B_top + c z_k   (float copy)
    double ad, bd, cd; // same in double
};

struct PriceLaunch {
    // model and contract
    double S0, K, r, T, v0, kappa, theta, sigma, rho, rho_bar;
    int opt_type;      // heston_option_type
    int scheme;        // kernel scheme: 0 full truncation, 1 absorption, 2 QE,
                       // 3 partial truncation or reflection (see `reflect`)
    bool reflect;      // scheme 3: reflection (else partial truncation)
    int precision;     // 0 fp64, 1 fp32
    int rng;           // 0 Philox, 1 Sobol + bridge
    bool bumps;        // fused bump scenarios
    bool split;        // one scenario per lane (price_kernel's SPLIT layout; blocks_per_rep
                       // then counts blocks of BLOCK / 64 * SPLIT_PATHS_PER_WAVE paths)
    bool cv;           // arithmetic Asian with the geometric control (records N_ACC_CV wide)
    uint32_t n_steps;
    uint32_t n_fix;                 // number of fixing dates
    double fix_step_sum;            // sum of the fixing step indices (fixing times / dt)
    const uint32_t *fix_bits;       // device bitmask over steps 1..N (bit j), or null = every step
    uint64_t seed;
    uint64_t first_path;            // first path handled by the launch
    uint64_t n_paths;               // paths in the launch
    uint64_t paths_per_rep;         // points per replicate (Sobol), n_paths for Philox
    bool wide_paths;                // some path index of the launch is >= 2^32
    uint32_t n_reps;                // replicates covered by the launch
    uint32_t rep0;                  // replicate of the launch's first path
    // bumps
    double hS, hv, hr, hT;
    StepCoef base, tup, tdn;        // grids of T, T + hT, T - hT
    // quasi-random
    const uint32_t *sobol_dirs;     // device [2N][32]
    const uint32_t *sobol_shift;    // device [R][2N] (position-ordered when sobol_low is set)
    const uint32_t *sobol_hi;       // device [ceil(M/64)][2N], position-ordered, or null: per
                                    // 64-point block, XOR of the direction numbers of Gray-code
                                    // bits >= 6
    const uint32_t *sobol_low;      // device [N+1][64][2] or null: per walk position and value
                                    // of a point's low six Gray-code bits, the XOR of the
                                    // selected direction numbers 0..5 of the node's two
                                    // dimensions (row N zero; set exactly when sobol_hi is)
    const int32_t *bridge_start;    // device [N+1]: ops of step j are [start[j], start[j+1])
    const BridgeOp *bridge_ops;     // device [N-1]
    double bridge_root_scale;       // sqrt(N)
    int bridge_depth;
    // outputs
    double *partials;               // device [n_reps][blocks_per_rep][acc_width()]
    double *reduce_tmp;             // device [n_reps][ceil(blocks_per_rep / REDUCE_CHUNK)]
                                    // [acc_width()] first-level sums, or null when
                                    // blocks_per_rep <= REDUCE_CHUNK
    uint32_t blocks_per_rep;
    double *dump;                   // device [n_paths][DUMP_WIDTH] or null
    double *pay_out;                // device [n_paths] discounted payoff per path, or null
    const void *step_weights;       // device [N][STEP_WEIGHTS] in the path precision (Asian)
    void *ckpt;                     // device checkpoint buffer (adjoint forward) or null
    uint32_t ckpt_every;            // steps between checkpoints

    // doubles per partial record
    __host__ __device__ int acc_width() const { return cv ? N_ACC_CV : N_ACC; }
};

// Exact simulation (exact_kernel.hip): Broadie-Kaya steps of length D over
// the n_steps grid, FP64.  Per-launch constants are computed on the host.
constexpr uint32_t EXACT_COUNTER_TAG = 5u;      // fourth Philox counter word, plus 256 k
constexpr int EXACT_MAX_GAMMA_ATTEMPTS = 64;
constexpr double EXACT_MAX_POISSON_MEAN = 700.0;
constexpr uint32_t EXACT_MAX_GRID = 16384;      // characteristic-function points per draw
constexpr uint32_t EXACT_MAX_LANES = 131072;    // resident lanes (two waves per SIMD:
                                                 // the kernel holds 244 VGPRs)
constexpr int EXACT_REC = N_ACC + 2;            // partial record: estimator sums, failures, pad
struct ExactLaunch {
    double S0, K, r, T, v0, kappa, theta, sigma, rho, rho_bar;
    double D;            // step length T / n_steps
    double nu;           // 2 kappa theta / sigma^2 - 1 (Bessel order)
    double d;            // 4 kappa theta / sigma^2 (degrees of freedom)
    double c;            // sigma^2 (1 - e^{-kappa D}) / (4 kappa)
    double ekD;          // e^{-kappa D}
    double kappa2, two_sigma2, sigma2, inv_sigma2;
    double t1_const;     // ln(1 - e^{-kappa D}) - ln kappa + kappa D / 2
    double coth_k;       // kappa (1 + e^{-kappa D}) / (1 - e^{-kappa D})
    double log_zk_scale; // ln(4 kappa e^{-kappa D/2} / (sigma^2 (1 - e^{-kappa D})))
    double log4_over_sigma2; // ln(4 / sigma^2)
    int opt_type;
    uint32_t n_steps, n_fix;
    const uint32_t *fix_bits; // device bitmask over steps 1..N, or null = every step
    uint64_t seed;
    uint64_t first_path, n_paths;
    uint32_t n_lanes;         // lanes of the launch; lane l takes paths l, l + n_lanes, ...
    double *scratch;          // device [EXACT_MAX_GRID][n_lanes]: Re Phi on the grid
    double *partials;         // device [blocks][EXACT_REC]
    double *dump;             // device [n_paths][DUMP_WIDTH] or null
};
hipError_t launch_exact(const ExactLaunch &L, hipStream_t stream);

// Semi-analytic price of the geometric-average control (geo_control.hip).
struct GeoControl {
    double lnS0, K, lnK, r, T, v0, kappa, theta, sigma, rho;
    double dt;                 // fixing time of step k is k dt
    const uint32_t *steps;     // fixing steps (device), or null = every step 1..n_fix
    uint32_t n_fix;
    uint32_t v_max;            // first integration range [0, v_max] (a power of two)
    double gl_x[8], gl_w[8];   // positive 16-point Gauss-Legendre nodes and weights
};

// Wave-uniform constants of one option's paths (single scenario).
struct PathConsts {
    StepCoef c;
    double S0, K, r, T, v0, rho, rho_bar, sigma, theta;
    uint64_t seed;
    const uint32_t *fix_bits; // null: every step is a fixing date (Asian)
    uint32_t n_steps, n_fix;
    int type;                 // heston_option_type
    uint32_t wide;            // some path index is >= 2^32
};

// Batched launches: one option (request) of a batch and the launch itself.
constexpr uint32_t BATCH_CHUNK = 1024;     // paths per work item (4 x BLOCK)
// An item runs as BATCH_UNITS units of BLOCK paths, each a unit of dynamic
// scheduling with its own partial record; an item's record is the sum of its
// units' records in unit order (ITEM_REC doubles per item).
constexpr uint32_t BATCH_UNITS = BATCH_CHUNK / BLOCK;
constexpr int ITEM_REC = (int)BATCH_UNITS * N_ACC;
constexpr int BATCH_CKPT_EVERY = 8;        // adjoint checkpoint interval in batches
struct BatchOption {
    PathConsts k;
    uint64_t n_paths;
    uint64_t chunk_base;      // chunk index of the option's first item in this launch
    double *partials;         // device: unit u of item first_item + i at partials + (i BATCH_UNITS + u) N_ACC
    uint32_t first_item, n_items;
    uint32_t adjoint; // 0: price + pathwise Delta/Rho; 1: price + 7 adjoint sensitivities
    uint32_t pad;
};
struct BatchLaunch {
    int precision, scheme;
    bool adjoint;                // the items in [item_begin, item_end) are adjoint items
    const BatchOption *opts;     // device [n_opts]
    uint32_t n_opts;
    const uint32_t *item_opt;    // device [n_items]
    uint32_t item_begin, item_end;
    uint32_t *counter;           // device, zero before the launch
    unsigned char *scratch;      // device [grid][scratch_per_block] (adjoint checkpoints)
    uint64_t scratch_per_block;
    uint32_t grid;
};
int batch_resident_blocks(int precision, int scheme, bool adjoint);
hipError_t launch_batch(const BatchLaunch &B, hipStream_t s);
// sums[o][N_ACC]: option o's unit records (at opts[o].partials) added in order.
hipError_t launch_batch_reduce(const BatchLaunch &B, double *sums, hipStream_t s);

// Checkpoint buffer of the adjoint, structure of arrays in the path state's
// precision R: for c = 0 .. n_ckpt-1 the state at step c*every, x then V, each
// [n_paths]; then the final log-price x_N and the fixing sum A = sum e^{x}
// (zero for a European), each [n_paths].
__host__ __device__ inline uint64_t ckpt_count(uint32_t n_steps, uint32_t every)
{
    return (n_steps + every - 1) / every;
}
inline uint64_t ckpt_bytes(uint64_t n_paths, uint32_t n_steps, uint32_t every, size_t real)
{
    return (2 * ckpt_count(n_steps, every) + 2) * n_paths * real;
}

// Adjoint forward: prices the request's paths and stores the checkpoints of
// L.ckpt every L.ckpt_every steps; block partials of (price, pathwise Delta,
// pathwise Rho) in L.partials as for launch_paths.
hipError_t launch_adjoint_forward(const PriceLaunch &L, hipStream_t stream);

// Adjoint sums: price and the derivatives of the discounted payoff with respect
// to (S0, v0, r, kappa, theta, sigma, rho), each as (sum, sum of squares).
enum AdjointOut : int { ADJ_PRICE = 0, ADJ_S0, ADJ_V0, ADJ_R, ADJ_KAPPA, ADJ_THETA, ADJ_SIGMA, ADJ_RHO };

// Launches the reverse sweep over the checkpoints written by the forward
// launch `L` (same request, L.ckpt set); block partials go to L.partials in the
// N_ACC layout of AdjointOut; per_path (nullable) receives [n_paths][8]
// (payoff and the seven derivatives) scaled by `seed_grad`.
hipError_t launch_adjoint(const PriceLaunch &L, double seed_grad, double *per_path,
                          hipStream_t stream);

// Plain bump-and-revalue: per-path central differences of n_bump pairs of
// payoff rows.  pay = [1 + 2 n_bump][n_paths] (row 0 the base scenario, rows
// 1+2b and 2+2b the up and down revaluations of bump b).  Each block writes a
// BUMP_W-double partial record: [0], [1] sum and sum of squares of the base
// payoff; then for bump b at 2 + 4b: sum and sum of squares of
// (up - down) * scale1[b], then of (up - 2 base + down) * scale2[b].
constexpr int MAX_BUMPS = 8;
constexpr int BUMP_W = 2 + 4 * MAX_BUMPS;
struct BumpScales {
    double first[MAX_BUMPS], second[MAX_BUMPS];
};
hipError_t launch_bump_combine(const double *pay, uint64_t n_paths, uint32_t n_bump,
                               const BumpScales &sc, double *partials, uint32_t blocks,
                               hipStream_t stream);
// Fixed-order sum of `rows` partial records of width w into out[w].
hipError_t launch_reduce_rows(const double *partials, uint32_t rows, uint32_t w, double *out,
                              hipStream_t stream);

// Launches the path kernel of `L` on `stream` (one partial record per block).
hipError_t launch_paths(const PriceLaunch &L, hipStream_t stream);
// Sums the partial records of each replicate, in a fixed order, into
// `rep_sums` (device [n_reps][L.acc_width()]).
hipError_t launch_reduce(const PriceLaunch &L, double *rep_sums, hipStream_t stream);

// Geometric-average control, in one device buffer `buf` of GEO_BUF_DOUBLES:
// [0, 2 GEO_BOUND_POINTS) the modulus bounds |M(1 + iv)| / v and K |M(iv)| / v
// at v = 2^k (M the transform of ln G; search only), then at GEO_OUT the
// discounted call and put prices of G, E[G], the Gil-Pelaez integral and the
// two bounds at the end of the fixed range.  The prices are NaN when the
// transform has not decayed by the end of the range (fixed: g.v_max, at most
// GEO_MAX_FIXED_RANGE; search: 2^14).  `partials` (device [geo_node_blocks()])
// holds one double per block of the node kernel.
constexpr int GEO_BOUND_POINTS = 15;
constexpr int GEO_OUT = 2 * GEO_BOUND_POINTS;
constexpr int GEO_BUF_DOUBLES = GEO_OUT + 6;
constexpr uint32_t GEO_MAX_FIXED_RANGE = 4096;
uint32_t geo_node_blocks();
hipError_t launch_geo_price_fixed(const GeoControl &g, double *partials, double *buf,
                                  hipStream_t stream);
hipError_t launch_geo_price_search(const GeoControl &g, double *partials, double *buf,
                                   hipStream_t stream);

// Fills the [N][STEP_WEIGHTS] fixing weights of `L` (its precision) at
// L.step_weights.
hipError_t launch_step_weights(const PriceLaunch &L, void *out, hipStream_t stream);

// Writes the [reps][dims] digital shifts of the Sobol replicates of `seed`.
// perm (device [N], nullable): node of each walk position; with it the tables
// are position-ordered (column 2 pos + m = dimension 2 perm[pos] + m).
hipError_t launch_sobol_hi(const uint32_t *dirs, const int32_t *perm, uint32_t dims, uint32_t n_blk,
                           uint32_t *out, hipStream_t stream);
hipError_t launch_sobol_shifts(uint64_t seed, const int32_t *perm, uint32_t dims, uint32_t reps,
                               uint32_t *out,
                               hipStream_t stream);
// Expands dir12 (device [N][12]: direction numbers 0..5 of the two dimensions
// of the node at each walk position) into the [N+1][64][2] low-bit table.
hipError_t launch_sobol_low(const uint32_t *dir12, uint32_t N, uint32_t *out, hipStream_t stream);

} // namespace heston
