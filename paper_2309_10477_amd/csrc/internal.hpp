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
constexpr int DUMP_WIDTH = 16;
constexpr int BLOCK = 256;         // threads per block of the path kernels
constexpr int MAX_BRIDGE_DEPTH = 24;

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
    int scheme;        // 0 full truncation, 1 absorption
    int precision;     // 0 fp64, 1 fp32
    int rng;           // 0 Philox, 1 Sobol + bridge
    bool bumps;        // fused bump scenarios
    uint32_t n_steps;
    uint32_t n_fix;                 // number of fixing dates
    const uint32_t *fix_bits;       // device bitmask over steps 1..N (bit j), or null = every step
    uint64_t seed;
    uint64_t first_path;            // first path handled by the launch
    uint64_t n_paths;               // paths in the launch
    uint64_t paths_per_rep;         // points per replicate (Sobol), n_paths for Philox
    uint32_t n_reps;                // replicates covered by the launch
    uint32_t rep0;                  // replicate of the launch's first path
    // bumps
    double hS, hv, hr, hT;
    StepCoef base, tup, tdn;        // grids of T, T + hT, T - hT
    // quasi-random
    const uint32_t *sobol_dirs;     // device [2N][32]
    const uint32_t *sobol_shift;    // device [R][2N]
    const int32_t *bridge_start;    // device [N+1]: ops of step j are [start[j], start[j+1])
    const BridgeOp *bridge_ops;     // device [N-1]
    double bridge_root_scale;       // sqrt(N)
    int bridge_depth;
    // outputs
    double *partials;               // device [n_reps][blocks_per_rep][N_ACC]
    uint32_t blocks_per_rep;
    double *dump;                   // device [n_paths][DUMP_WIDTH] or null
};

// Launches the path kernel of `L` on `stream` (one partial record per block).
hipError_t launch_paths(const PriceLaunch &L, hipStream_t stream);
// Sums the partial records of each replicate, in a fixed order, into
// `rep_sums` (device [n_reps][N_ACC]).
hipError_t launch_reduce(const PriceLaunch &L, double *rep_sums, hipStream_t stream);

// Writes the [reps][dims] digital shifts of the Sobol replicates of `seed`.
hipError_t launch_sobol_shifts(uint64_t seed, uint32_t dims, uint32_t reps, uint32_t *out,
                               hipStream_t stream);

} // namespace heston
