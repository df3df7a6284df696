// Host runtime shared by the C-ABI files: the context, device scratch with a
// memory budget, argument checks and the per-request plan.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/heston.h"
#include "internal.hpp"

// A device buffer that only grows; its bytes count against the context budget.
// gen numbers its allocations (0: none), so that what was written into one
// allocation is not taken for the contents of a later one at the same address.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    uint64_t gen = 0;
};

// Brownian-bridge walk of an N-step grid (built on the host by bridge_program):
// the first op of each step and the ops in walk order.
struct BridgePlan {
    std::vector<int32_t> start; // N+1
    std::vector<heston::BridgeOp> ops; // N-1
    int depth = 1;
};

// The quasi-random tables that do not depend on the seed, kept from one Sobol
// call to the next: the bridge walk of n_steps, the direction numbers the
// device tables were built from (compared in full before any reuse), the
// position-ordered host tables of the block-aligned walk, and for each device
// table the allocation it was written into (its buffer's gen when written).
struct SobolTables {
    uint32_t n_steps = 0;
    std::vector<uint32_t> dirs; // [2 n_steps][32]
    BridgePlan bp;
    std::vector<int32_t> node_of_pos; // block-aligned walk: node at each position
    std::vector<uint32_t> dir12;      // block-aligned walk: [N][12] low direction numbers
    uint64_t dirs_gen = 0, start_gen = 0, ops_gen = 0; // sobol_dirs, bridge_start, bridge_ops
    uint64_t perm_gen = 0, low_gen = 0;                // sobol_perm, sobol_low
    uint64_t hi_gen = 0, hi_blocks = 0;                // sobol_hi and its 64-point blocks
};

struct heston_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t budget = 0; // 0 = unlimited
    uint64_t in_use = 0; // bytes held by the buffers below
    uint64_t alloc_gen = 0; // allocations made so far (DevBuf::gen)
    DevBuf partials, rep_sums, fix_bits, sobol_dirs, sobol_shift, sobol_hi, sobol_perm, sobol_low;
    DevBuf bridge_start, bridge_ops;
    DevBuf pay, bump_partials, bump_sums, step_w;
    DevBuf geo_buf, geo_partials, geo_steps; // geometric-average control
    DevBuf exact_scratch;                    // exact sampler: Re Phi per lane
    DevBuf reduce_tmp;                       // first-level sums of long reductions
    DevBuf batch_opts, batch_items, batch_partials, batch_sums, batch_counter, batch_scratch;
    double *host_sums = nullptr;     // pinned
    double *host_sums_dev = nullptr; // its device address: the estimate
                                     // reduction writes its sums straight there
    size_t host_sums_bytes = 0;
    double *host_geo = nullptr; // pinned: the geometric control's call and put prices
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // side stream (default priority, created on first use) on which the
    // geometric control's price runs beside the path kernel
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    SobolTables sobol; // seed-independent quasi-random tables on the device
};

namespace heston {
namespace rt {

// Records the message of a failed call for heston_last_error (per host thread).
heston_status fail(heston_status st, const std::string &msg);
extern thread_local std::string g_last_error;

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return ::heston::rt::fail(e_ == hipErrorOutOfMemory ? HESTON_OUT_OF_MEMORY            \
                                                                : HESTON_DEVICE_ERROR,           \
                                      std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

// Grows `b` to at least `bytes` (contents are not kept), within the budget.
heston_status reserve(heston_ctx *c, DevBuf &b, size_t bytes);

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev)
            (void)hipSetDevice(dev);
        else
            prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

struct Request {
    heston_params p;
    int type;
    uint64_t n_paths;
    uint32_t n_steps;
    uint64_t seed;
    heston_opts o;
};

heston_status check_params(const heston_params *p);
heston_status check_request(const Request &q);
StepCoef step_coef(const heston_params &p, double T, uint32_t N);
heston_est est_from(double n, double s, double ss);
Request make_request(const heston_params *p, heston_option_type type, uint64_t n_paths,
                     uint32_t n_steps, uint64_t seed, const heston_opts *opts);

} // namespace rt
} // namespace heston
