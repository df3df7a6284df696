// Host runtime shared by the C-ABI files: the context, device scratch with a
// memory budget, argument checks and the per-request plan.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/heston.h"
#include "internal.hpp"

// A device buffer that only grows; its bytes count against the context budget.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct heston_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t budget = 0; // 0 = unlimited
    uint64_t in_use = 0; // bytes held by the buffers below
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
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // side stream (default priority, created on first use) on which the
    // geometric control's price runs beside the path kernel
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
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
