/*
 * heston.h -- C ABI of the MI355X (gfx950) Heston / Milstein Monte-Carlo
 * library (libheston.so).
 *
 * The library prices European and arithmetic-Asian calls and puts under the
 * Heston model (paper: "Heston Model for option pricing", eq. heston_eq) by
 * Monte Carlo over paths of the Milstein scheme (Background, algorithm
 * "Milstein approximation under Heston model"), with the Monte-Carlo
 * estimator of algorithm "Monte Carlo option pricing estimation", and returns
 * the Greeks: the pathwise Delta and Rho estimators of the section "Pathwise
 * method for greeks estimation" (eqs. euro_pw and asian_pw; the Asian Rho uses
 * the exact derivative of the discrete average, without the printed K T
 * factor), five central bump-and-revalue Greeks on common random numbers, and
 * reverse-mode (adjoint) sensitivities to the seven model inputs.
 *
 * Conventions shared by every call
 *   - Every call returns heston_status; outputs are written only on HESTON_OK.
 *   - Host structs and host arrays are owned by the caller and only read during
 *     the call.  Device pointers passed in are borrowed for the duration of the
 *     call and used on the context's stream.
 *   - No C++ exception crosses this boundary.  A NaN or infinite input gives
 *     HESTON_INVALID_ARGUMENT; heston_last_error() then describes the cause.
 *   - Valid model inputs: S0 > 0, K > 0, T > 0, v0 >= 0, kappa > 0, theta >= 0,
 *     sigma >= 0, |rho| <= 1 (|rho| < 1 for adjoint calls); n_paths >= 2,
 *     n_steps >= 1; fixing steps strictly increasing in [1, n_steps].
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key =
 *     (lo32 seed, hi32 seed) and counter = (step >> 1, lo32 path, hi32 path, 0);
 *     words 0,1 feed even steps and words 2,3 odd steps; uniforms
 *     ((w >> 9) + 1/2) 2^-23; normals by Box-Muller,
 *     Za = sqrt(-2 ln ua) cos(2 pi ub), Zb = sqrt(-2 ln ua) sin(2 pi ub);
 *     Z1 = Za drives the log-price, Z2 = rho Za + sqrt(1-rho^2) Zb the
 *     variance (algorithm "Generation of two correlated Normal random
 *     variables").  The same request gives bit-identical results every time.
 *   - A context is used by one host thread at a time.
 */
#ifndef HESTON_H
#define HESTON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HESTON_ABI_VERSION 3

/* Model and contract inputs (paper: Table "Heston model parameters"). */
typedef struct heston_params {
    double S0, K, r, T, v0, kappa, theta, sigma, rho;
} heston_params;

/* Payoffs (paper: Background, European and arithmetic-Asian payoffs; the
 * paper notes the average may also be geometric: G = exp(mean of ln S over the
 * fixing dates)).  Geometric averages are priced by the pricing calls only
 * (not by adjoint calls, batches or the server). */
typedef enum heston_option_type {
    HESTON_EURO_CALL = 0,
    HESTON_EURO_PUT = 1,
    HESTON_ASIAN_CALL = 2,
    HESTON_ASIAN_PUT = 3,
    HESTON_GEO_ASIAN_CALL = 4,
    HESTON_GEO_ASIAN_PUT = 5
} heston_option_type;

typedef enum heston_status {
    HESTON_OK = 0,
    HESTON_PENDING = 1,
    HESTON_INVALID_ARGUMENT = -1,
    HESTON_OUT_OF_MEMORY = -2,
    HESTON_OVER_BUDGET = -3,
    HESTON_DEVICE_ERROR = -4,
    HESTON_UNSUPPORTED = -5,
    HESTON_NOT_FOUND = -6
} heston_status;

/* Arithmetic of the per-path state.  Cross-path sums are always FP64. */
enum { HESTON_FP64 = 0, HESTON_FP32 = 1 };
/* Normals: Philox pseudo-random, or Sobol points through a Brownian bridge. */
enum { HESTON_RNG_PHILOX = 0, HESTON_RNG_SOBOL_BRIDGE = 1 };
/* Scheme.  Milstein with full truncation (max(V,0) in drift and diffusion,
 * unclamped V carried) or with the paper's absorption (V <- max(V,0) after
 * every step, algorithm "Milstein approximation under Heston model"); the
 * paper's Euler discretisation (section "Euler discretisation": the same steps
 * without the Milstein term sigma^2 dt (Z2^2 - 1) / 4) with either truncation;
 * Milstein with partial truncation or reflection (Lord, Koekkoek, van Dijk,
 * Quantitative Finance 10(2), 2010: in V' = f1(V) + kappa (theta - f2(V)) dt +
 * sigma sqrt(f3(V) dt) Z2 + the Milstein term, with f3 also in the log-price
 * step, partial truncation takes f1 = f2 = identity, f3 = max(., 0), and
 * reflection f1 = f2 = f3 = |.|; the carried V is reported); or
 * Andersen's quadratic-exponential scheme, which the paper names as future
 * work (L. Andersen, J. Computational Finance 11(3), 2008: the variance drawn
 * from a moment-matched squared normal or a point mass at zero with an
 * exponential tail, switching at psi = 3/2; the log-price step uses the start
 * and end variances with weights 1/2, no martingale correction).  QE needs
 * Philox inputs, sigma > 0 and theta > 0; its step j takes one Philox block
 * with counter (j, lo32 path, hi32 path, 4): Box-Muller of words 0, 1 for the
 * price and variance normals, word 2 for the exponential-branch uniform.
 * HESTON_EXACT is the paper's exact simulation (algorithm "Broadie and Kaya
 * exact simulation algorithm"): each of the n_steps steps of length T/n_steps
 * draws V_t from its non-central chi-square law given V_u, the integral of V
 * over the step by inverting its conditional characteristic function, and
 * ln S from both; no discretisation bias.  It runs in FP64 with Philox inputs
 * and pathwise Greeks only, needs sigma > 0 and theta > 0, and takes at most
 * HESTON_EXACT_MAX_STEPS steps; its inputs are laid out per (step, path) as
 * Philox blocks with counter (step, lo32 path, hi32 path, 5 + 256 k).  Paths
 * whose draws leave the sampler's numerical range (see exact_kernel.hip) make
 * the call fail with HESTON_UNSUPPORTED.  The context keeps a scratch array of
 * 128 KiB per resident lane (min(n_paths rounded up to 256, 131072) lanes: up
 * to 16 GiB), counted against its HBM budget.
 * Adjoint calls take the Milstein schemes with full truncation or absorption
 * and QE; so do batches and the server. */
enum {
    HESTON_FULL_TRUNCATION = 0,
    HESTON_ABSORPTION = 1,
    HESTON_QE = 2,
    HESTON_EULER_FULL_TRUNCATION = 3,
    HESTON_EULER_ABSORPTION = 4,
    HESTON_PARTIAL_TRUNCATION = 5,
    HESTON_REFLECTION = 6,
    HESTON_EXACT = 7
};
#define HESTON_EXACT_MAX_STEPS 4096
/* Greek estimators (bit mask). */
enum {
    HESTON_GREEKS_PATHWISE = 1u,   /* paper's pathwise Delta and Rho              */
    HESTON_GREEKS_BUMP_FUSED = 2u, /* 5 bump Greeks, one pass sharing the normals */
    HESTON_GREEKS_BUMP_PLAIN = 4u  /* 5 bump Greeks, 9 independent revaluations
                                      (exclusive with BUMP_FUSED)                */
};

/* Control variate of the price (heston_opts.control_variate).  GEOMETRIC
 * applies to arithmetic-Asian types: on the same paths the kernel also forms
 * the geometric-average payoff of the same kind and strike on the same fixing
 * dates (the paper notes that the average may be geometric), whose expectation
 * the library computes semi-analytically on the device (Heston is affine in
 * ln S: the transform of ln G follows from closed-form Riccati steps between
 * fixing dates, the price from Gil-Pelaez inversion by Gauss-Legendre panels).
 * The estimate is mean(a) - beta (mean(g) - E[g]) with beta = Cov(a, g) /
 * Var(g) from the same paths (Kemna and Vorst, J. Banking and Finance 14,
 * 1990); std_err = sqrt((Var(a) - beta Cov(a, g)) / n) (Philox), or the std
 * of the replicate estimates / sqrt(R) with the pooled beta (Sobol).
 * Requires sigma > 0 and at most HESTON_CONTROL_MAX_FIXINGS fixing dates;
 * not with HESTON_GREEKS_BUMP_PLAIN. */
enum { HESTON_CONTROL_NONE = 0, HESTON_CONTROL_GEOMETRIC = 1 };
#define HESTON_CONTROL_MAX_FIXINGS 8192

/* valid_mask bits of heston_result. */
enum {
    HESTON_VALID_PRICE = 1u,
    HESTON_VALID_PATHWISE = 2u,
    HESTON_VALID_BUMPS = 4u,
    HESTON_VALID_ADJOINT = 8u,
    HESTON_VALID_CONTROL = 16u
};

typedef struct heston_est {
    double value;   /* estimate                                             */
    double std_err; /* standard error: sample SE over paths (Philox), or the
                       std of the replicate estimates / sqrt(R) (Sobol)    */
} heston_est;

typedef struct heston_result {
    heston_est price;
    heston_est delta, gamma, vega, rho, theta; /* bump-and-revalue; vega = dP/dv0, theta = -dP/dT */
    heston_est pw_delta, pw_rho;               /* paper's pathwise estimators                  */
    heston_est adj[7]; /* adjoint dP/d(S0, v0, r, kappa, theta, sigma, rho) (batches, serving) */
    uint64_t n_paths;  /* paths the estimates use                                            */
    uint32_t valid_mask;
    uint32_t reserved;
    double device_ms; /* GPU time (HIP events): the path kernel of a pricing call, the
                         batched launch of a batch; for a served request the summed
                         durations of the launches that carried its work items (those
                         launches also carry other requests' items)                   */
    heston_est cv_price; /* price with the control variate (HESTON_VALID_CONTROL)       */
    double cv_beta;      /* fitted control coefficient beta                             */
    double cv_mean;      /* E of the discounted control payoff, computed on the device  */
    double latency_ms;   /* host wall time until the result was available: from entry
                            to return of a synchronous call (pricing, batch), from
                            heston_submit to completion of a served request            */
} heston_result;

typedef struct heston_opts {
    uint32_t struct_size; /* sizeof(heston_opts); set by heston_default_opts     */
    int32_t precision;    /* HESTON_FP64 (default) or HESTON_FP32                */
    int32_t rng;          /* HESTON_RNG_PHILOX (default) or HESTON_RNG_SOBOL_BRIDGE */
    int32_t scheme;       /* HESTON_FULL_TRUNCATION (default), HESTON_ABSORPTION, HESTON_QE,
                             HESTON_EULER_FULL_TRUNCATION, HESTON_EULER_ABSORPTION,
                             HESTON_PARTIAL_TRUNCATION, HESTON_REFLECTION or HESTON_EXACT */
    uint32_t greeks;      /* HESTON_GREEKS_* mask; default PATHWISE | BUMP_FUSED */
    uint32_t qmc_replicates; /* Sobol: R digitally shifted replicates; n_paths must
                                be a multiple of R (points per replicate = n_paths/R) */
    const uint32_t *sobol_directions; /* Sobol: host array [sobol_dims][32] of 30-bit
                                direction numbers v[d][b] (only b < 30 read; one
                                wider than 30 bits in the first 2 n_steps rows is
                                HESTON_INVALID_ARGUMENT), the
                                Joe-Kuo table in the layout of torch's SobolEngine
                                state; dimension 2k feeds bridge node k of the price
                                motion and 2k+1 that of the variance motion */
    uint32_t sobol_dims;      /* rows in sobol_directions; must be >= 2 n_steps  */
    const uint32_t *fixing_steps; /* Asian fixing steps (host, strictly increasing
                                in [1, n_steps]); NULL = every step; ignored for
                                European options, whose only date is n_steps    */
    uint32_t n_fixings;
    double bump_S0_rel; /* default 0.01   (h = bump_S0_rel * S0)      */
    double bump_v0_rel; /* default 0.01   (h = bump_v0_rel * v0)      */
    double bump_r_abs;  /* default 1e-4; with fused bumps of an arithmetic
                           Asian bump_r_abs * T <= 1e-3 (FP64) or 3e-3 (FP32):
                           its r-bumped averages come from a Taylor series in
                           the bump (else HESTON_INVALID_ARGUMENT)          */
    double bump_T_abs;  /* default 1/365; n_steps and the fixing step
                           indices stay fixed, so dt is rescaled      */
    int32_t control_variate; /* HESTON_CONTROL_NONE (default) or HESTON_CONTROL_GEOMETRIC */
    uint32_t reserved;       /* must be 0                                               */
} heston_opts;

typedef struct heston_ctx heston_ctx;

/* Fills *opts with the defaults above.  Returns HESTON_INVALID_ARGUMENT for NULL. */
heston_status heston_default_opts(heston_opts *opts);

/* Creates a context on HIP device `device`.  `hip_stream` (a hipStream_t, may
 * be NULL for the device's null stream) is borrowed: every kernel and copy of
 * the context runs on it, and the caller keeps it alive until
 * heston_ctx_destroy.  `hbm_budget_bytes` caps the device memory the context
 * allocates for itself (0 = no cap).  Errors: INVALID_ARGUMENT (bad device or
 * NULL out), DEVICE_ERROR. */
heston_status heston_ctx_create(int device, void *hip_stream, uint64_t hbm_budget_bytes,
                                heston_ctx **out);
heston_status heston_ctx_destroy(heston_ctx *ctx);

/* Price and Greeks of one option (paper: algorithm "Monte Carlo option
 * pricing estimation" over paths of algorithm "Milstein approximation under
 * Heston model").  Paths 0 .. n_paths-1 of the stream of `seed`.  Blocks until
 * the result is on the host.  `opts` may be NULL for the defaults.  Errors:
 * INVALID_ARGUMENT, UNSUPPORTED (n_steps above the kernel limit of 1<<20),
 * OUT_OF_MEMORY / OVER_BUDGET (scratch), DEVICE_ERROR. */
heston_status heston_price_greeks_ex(heston_ctx *ctx, const heston_params *params,
                                     heston_option_type type, uint64_t n_paths, uint32_t n_steps,
                                     uint64_t seed, const heston_opts *opts, heston_result *out);

/* heston_price_greeks_ex on a per-thread default context of the current HIP
 * device and its null stream, with the default options. */
heston_status heston_price_greeks(const heston_params *params, heston_option_type type,
                                  uint64_t n_paths, uint32_t n_steps, uint64_t seed,
                                  heston_result *out);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): heston_price_greeks_ex
 * without a context and without any device or pinned-host allocation.  The
 * call keeps its device scratch (fixing mask and weights, block partials,
 * reduction sums) in one fixed array of HESTON_NOALLOC_SCRATCH_BYTES per
 * device, held by the library until the process ends; the first call on a
 * device looks up that array's address and creates two timing events.
 * Kernels and copies run on `hip_stream` (a hipStream_t; NULL: the device's
 * null stream) of the current HIP device, and the call blocks until the
 * result is on the host.  Results are bitwise those of heston_price_greeks_ex
 * with the same arguments.  Calls that overlap on one device share the array
 * and race: serialise them.  Nothing in the array needs to start at zero.
 * Covers Philox normals, every Milstein/Euler/QE scheme flag, European and
 * Asian payoffs, pathwise Greeks and fused bumps.  Errors: INVALID_ARGUMENT,
 * UNSUPPORTED (Sobol normals, exact simulation, plain bumps, control
 * variate), OVER_BUDGET (the request's scratch exceeds the fixed size: about
 * 0.5 byte per path plus 64 bytes per step), DEVICE_ERROR. */
#define HESTON_NOALLOC_SCRATCH_BYTES (16u << 20)
heston_status heston_price_greeks_noalloc(const heston_params *params, heston_option_type type,
                                          uint64_t n_paths, uint32_t n_steps, uint64_t seed,
                                          const heston_opts *opts, void *hip_stream,
                                          heston_result *out);

/* Per-path records of paths first .. first+count-1 of the same request, for
 * parity checks: writes count x HESTON_DUMP_WIDTH doubles, row-major, to the
 * DEVICE buffer `out_dev` (caller-owned, at least count*HESTON_DUMP_WIDTH*8
 * bytes).  The records are produced by the pricing kernel itself.  Columns:
 *   0 S_T, 1 V_T (carried variance), 2 Sbar (Asian average: arithmetic or
 *     geometric by type; S_T for European),
 *   3 discounted payoff, 4 pathwise Delta, 5 pathwise Rho,
 *   6..13 discounted payoffs of the bumped scenarios S0+, S0-, v0+, v0-, r+,
 *         r-, T+, T- (NaN unless opts->greeks has BUMP_FUSED),
 *   14 ln(S_T/S0),
 *   15 with HESTON_CONTROL_GEOMETRIC the discounted control payoff (geometric
 *      average, same kind and strike); under HESTON_EXACT the integral of V
 *      over [0, T]; otherwise 0.
 * Under HESTON_EXACT a path outside the sampler's range has NaN in every
 * column. 
 * For Sobol requests `first + count` must not exceed n_paths. */
#define HESTON_DUMP_WIDTH 16
heston_status heston_dump_paths(heston_ctx *ctx, const heston_params *params,
                                heston_option_type type, uint64_t n_paths, uint32_t n_steps,
                                uint64_t seed, const heston_opts *opts, uint64_t first,
                                uint64_t count, double *out_dev);

/* ------------------------------------------------------------------------
 * Plain bump-and-revalue on common random numbers.
 *
 * Every scenario is an independent revaluation (a full launch that regenerates
 * the same Philox or Sobol normals): the base scenario, then for each bump b
 * the up and the down revaluation of one input.  Returns the base price, the
 * central first difference (P+ - P-) / (2h) and the second difference
 * (P+ - 2P + P-) / h^2 of every bump, each with the standard error of its
 * per-path difference.  A T bump keeps n_steps and the fixing step indices,
 * so dt is rescaled.  Up to 8 bumps; the per-path payoffs of all 1 + 2 n_bumps
 * scenarios are held on the device (8 bytes per path per scenario).  Errors:
 * INVALID_ARGUMENT (bad bump, a bumped input out of range), the pricing
 * call's errors. */
typedef enum heston_param {
    HESTON_P_S0 = 0, HESTON_P_K = 1, HESTON_P_R = 2, HESTON_P_T = 3, HESTON_P_V0 = 4,
    HESTON_P_KAPPA = 5, HESTON_P_THETA = 6, HESTON_P_SIGMA = 7, HESTON_P_RHO = 8
} heston_param;

typedef struct heston_bump {
    int32_t param;    /* heston_param                                        */
    int32_t relative; /* nonzero: h = size * |input|; zero: h = size          */
    double size;
} heston_bump;

#define HESTON_MAX_BUMPS 8
heston_status heston_bump_revalue(heston_ctx *ctx, const heston_params *params,
                                  heston_option_type type, uint64_t n_paths, uint32_t n_steps,
                                  uint64_t seed, const heston_opts *opts,
                                  const heston_bump *bumps, uint32_t n_bumps,
                                  heston_est *price, heston_est *first, heston_est *second,
                                  double *device_ms);

/* ------------------------------------------------------------------------
 * Adjoint (reverse-mode) sensitivities of the price to
 * theta = (S0, v0, r, kappa, theta, sigma, rho): the exact derivative of every
 * path's discounted payoff (pathwise method, section "Pathwise method for
 * greeks estimation", carried through every Milstein step, or through every
 * step of Andersen's QE scheme with its branch decisions held fixed), averaged
 * over paths.  Philox normals only; |rho| < 1.
 *
 * heston_adjoint_forward prices the option and writes the step states every
 * `every` steps (8 or 16) and the final state into the caller-owned DEVICE
 * buffer ckpt_dev of at least heston_adjoint_ckpt_bytes(...) bytes.
 * heston_adjoint_backward, called with the same request and the unchanged
 * buffer, recomputes each segment from its checkpoint with the same normals
 * and runs the reverse sweep; grads[k] = dprice * mean over paths of the
 * derivative, with its standard error.  per_path_dev (nullable, DEVICE,
 * [n_paths][8] doubles) receives each path's payoff and its seven derivatives
 * times dprice.  The buffer layout is private to the library.  Errors:
 * INVALID_ARGUMENT (bad request, every not 8 or 16, buffer too small),
 * UNSUPPORTED (Sobol normals, bump Greeks in opts are ignored), DEVICE_ERROR. */
uint64_t heston_adjoint_ckpt_bytes(uint64_t n_paths, uint32_t n_steps, uint32_t every,
                                   int32_t precision);
heston_status heston_adjoint_forward(heston_ctx *ctx, const heston_params *params,
                                     heston_option_type type, uint64_t n_paths, uint32_t n_steps,
                                     uint64_t seed, const heston_opts *opts, uint32_t every,
                                     void *ckpt_dev, uint64_t ckpt_bytes, heston_est *price,
                                     double *device_ms);
heston_status heston_adjoint_backward(heston_ctx *ctx, const heston_params *params,
                                      heston_option_type type, uint64_t n_paths,
                                      uint32_t n_steps, uint64_t seed, const heston_opts *opts,
                                      uint32_t every, const void *ckpt_dev, uint64_t ckpt_bytes,
                                      double dprice, heston_est grads[7], double *per_path_dev,
                                      double *device_ms);

/* ------------------------------------------------------------------------
 * Batched pricing: many options of different sizes in one persistent launch.
 *
 * A request names one option, its path count and step count, its own seed
 * (its paths are paths 0 .. n_paths-1 of that seed's stream, as for
 * heston_price_greeks_ex) and what it wants: the price with the pathwise
 * Delta/Rho, or the price with the seven adjoint sensitivities (then the
 * pathwise Delta/Rho equal the adjoint dS0/dr).  Asian requests fix at every
 * step.  Work is split into items of 1024 paths; each request's result sums
 * its items in item order, so it is bitwise the same whether it is priced
 * alone or in any batch. */
enum { HESTON_WANT_PATHWISE = 1u, HESTON_WANT_ADJOINT = 2u };

typedef struct heston_request {
    heston_params params;
    int32_t type;       /* heston_option_type                                   */
    uint32_t n_steps;
    uint64_t n_paths;   /* paths (serving: the cap)                             */
    uint64_t seed;
    uint32_t want;      /* HESTON_WANT_PATHWISE or HESTON_WANT_ADJOINT          */
    uint32_t reserved;
    double se_target;   /* serving: stop at the first item boundary where the
                           price SE <= se_target (0: run all n_paths)          */
} heston_request;

/* Prices reqs[0..n-1] (host array) into out[0..n-1] (host array).  opts
 * (nullable) supplies precision and scheme (HESTON_FULL_TRUNCATION,
 * HESTON_ABSORPTION or HESTON_QE; under QE the adjoint differentiates the
 * steps with their branches held fixed); Philox normals only; opts
 * fixing_steps must be NULL.  Blocks until done; device_ms (nullable) gets the
 * GPU time of the batched kernels.  Errors: INVALID_ARGUMENT (any request
 * invalid; nothing is priced), UNSUPPORTED, OVER_BUDGET / OUT_OF_MEMORY
 * (item records: 512 bytes per 1024 paths), DEVICE_ERROR. */
heston_status heston_price_batch(heston_ctx *ctx, const heston_request *reqs, uint32_t n,
                                 const heston_opts *opts, heston_result *out, double *device_ms);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of pricing requests.
 *
 * A server owns an engine thread and device memory on the context's device.
 * heston_submit enqueues a request and returns at once with a ticket.  The
 * engine admits queued requests while the server's device-memory budget and
 * request slots allow (a request holds 512 bytes per 1024-path item of its path
 * cap plus a 256-byte state), and repeatedly launches the batched kernel over
 * the next items of every admitted request, so requests that arrive while
 * others run join the next launch and their work overlaps on the device.
 * Each request's running sums live on the device and are extended item by
 * item, in item order, by a fold kernel that also applies the stopping rule:
 * the request completes at the first item boundary (at least two items) where
 * the price SE is <= se_target, or at its path cap.  Its result therefore
 * depends only on its own items and is bitwise the same however it was
 * batched.  Latency = completion seen by the engine - heston_submit call. */
typedef struct heston_server heston_server;

typedef struct heston_server_config {
    uint32_t struct_size;       /* sizeof(heston_server_config)                    */
    int32_t precision;          /* HESTON_FP32 (default) or HESTON_FP64            */
    int32_t scheme;             /* HESTON_FULL_TRUNCATION (default), ABSORPTION or
                                   QE                                             */
    uint32_t max_active;        /* admitted requests at once (default 4096)        */
    uint32_t max_steps;         /* largest n_steps accepted (default 2048)         */
    uint32_t reserved;
    uint64_t hbm_budget_bytes;  /* device memory for request state and launch
                                   buffers (default 8 GiB)                        */
    uint64_t launch_path_steps; /* work per launch (default 2^29 path-steps)      */
} heston_server_config;

typedef struct heston_server_stats {
    uint64_t submitted, admitted, completed, queued, active;
    uint64_t launches;
    double path_steps;          /* path-steps simulated (items launched)           */
    double busy_ms;             /* time with at least one launch on the device (the
                                   union of the launches' intervals; launches on
                                   the three slots' streams may overlap)          */
    double p50_ms, p99_ms, mean_ms, max_ms; /* latency of completed requests       */
    uint64_t pool_bytes;        /* device memory for request states (the budget
                                   minus adjoint scratch and launch buffers)     */
    uint64_t pool_free_bytes;
} heston_server_stats;

heston_status heston_server_default_config(heston_server_config *cfg);
/* Errors: INVALID_ARGUMENT, OVER_BUDGET (the budget cannot hold the launch
 * buffers), OUT_OF_MEMORY, DEVICE_ERROR. */
heston_status heston_server_create(heston_ctx *ctx, const heston_server_config *cfg,
                                   heston_server **out);
/* Stops the engine after the work in flight; pending requests are dropped. */
heston_status heston_server_destroy(heston_server *srv);
/* INVALID_ARGUMENT for a bad request (its want, params, n_steps > max_steps, or
 * a path cap whose state alone exceeds the budget). */
heston_status heston_submit(heston_server *srv, const heston_request *req, uint64_t *ticket);
/* HESTON_OK and *out when done (the ticket is then released), HESTON_PENDING
 * while queued or running, HESTON_NOT_FOUND for an unknown ticket. */
heston_status heston_poll(heston_server *srv, uint64_t ticket, heston_result *out);
/* Blocks until the ticket is done (or timeout_ms elapses: HESTON_PENDING). */
heston_status heston_wait(heston_server *srv, uint64_t ticket, double timeout_ms,
                          heston_result *out);
heston_status heston_server_get_stats(heston_server *srv, heston_server_stats *out);

/* Static description of a status code; never NULL. */
const char *heston_status_str(heston_status status);
/* Message of the last failed call on this host thread ("" if none). */
const char *heston_last_error(void);
/* HESTON_ABI_VERSION of the loaded library. */
int heston_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HESTON_H */
