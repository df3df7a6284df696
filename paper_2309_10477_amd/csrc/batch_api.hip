// heston_price_batch: the host side of the persistent batched kernel.
#include <hip/hip_runtime.h>

#include <chrono>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/heston.h"
#include "batch_plan.hpp"
#include "internal.hpp"
#include "runtime.hpp"

namespace heston {
namespace rt {

heston_status check_batch_request(const heston_request &r, const heston_opts &o, Request &q)
{
    q = make_request(&r.params, (heston_option_type)r.type, r.n_paths, r.n_steps, r.seed, &o);
    q.o.greeks = HESTON_GREEKS_PATHWISE;
    q.o.rng = HESTON_RNG_PHILOX;
    q.o.fixing_steps = nullptr;
    heston_status st = check_request(q);
    if (st != HESTON_OK)
        return st;
    if (r.type > HESTON_ASIAN_PUT)
        return fail(HESTON_UNSUPPORTED, "batches price European and arithmetic-Asian payoffs");
    if (r.want != HESTON_WANT_PATHWISE && r.want != HESTON_WANT_ADJOINT)
        return fail(HESTON_INVALID_ARGUMENT, "want must be WANT_PATHWISE or WANT_ADJOINT");
    if (r.want == HESTON_WANT_ADJOINT && !(std::fabs(r.params.rho) < 1))
        return fail(HESTON_INVALID_ARGUMENT, "adjoint needs |rho| < 1");
    if (!std::isfinite(r.se_target) || r.se_target < 0)
        return fail(HESTON_INVALID_ARGUMENT, "se_target must be finite and >= 0");
    return HESTON_OK;
}

BatchOption batch_option(const heston_request &r)
{
    BatchOption b;
    std::memset(&b, 0, sizeof(b));
    const heston_params &p = r.params;
    PathConsts &k = b.k;
    k.c = step_coef(p, p.T, r.n_steps);
    k.S0 = p.S0;
    k.K = p.K;
    k.r = p.r;
    k.T = p.T;
    k.v0 = p.v0;
    k.rho = p.rho;
    k.rho_bar = std::sqrt(std::max(0.0, 1.0 - p.rho * p.rho));
    k.sigma = p.sigma;
    k.theta = p.theta;
    k.seed = r.seed;
    k.fix_bits = nullptr;
    k.n_steps = r.n_steps;
    k.n_fix = r.type >= 2 ? r.n_steps : 1;
    k.type = r.type;
    k.wide = r.n_paths > (1ull << 32) ? 1u : 0u;
    b.n_paths = r.n_paths;
    b.adjoint = r.want == HESTON_WANT_ADJOINT ? 1u : 0u;
    return b;
}

void fill_result(const heston_request &r, uint64_t n_paths, const double *s, heston_result &out)
{
    std::memset(&out, 0, sizeof(out));
    const double n = (double)n_paths;
    out.price = est_from(n, s[0], s[1]);
    if (r.want == HESTON_WANT_ADJOINT) {
        for (int k = 0; k < 7; ++k)
            out.adj[k] = est_from(n, s[2 + 2 * k], s[3 + 2 * k]);
        out.pw_delta = out.adj[0];
        out.pw_rho = out.adj[2];
        out.valid_mask = HESTON_VALID_PRICE | HESTON_VALID_PATHWISE | HESTON_VALID_ADJOINT;
    } else {
        out.pw_delta = est_from(n, s[2], s[3]);
        out.pw_rho = est_from(n, s[4], s[5]);
        out.valid_mask = HESTON_VALID_PRICE | HESTON_VALID_PATHWISE;
    }
    out.n_paths = n_paths;
}

uint64_t adjoint_scratch_per_block(uint32_t max_steps, int precision)
{
    const size_t real = precision == HESTON_FP64 ? 8 : 4;
    return (2 * ckpt_count(max_steps, BATCH_CKPT_EVERY) + 2) * BLOCK * real;
}

heston_status run_batch(heston_ctx *c, BatchWork &w, int precision, int scheme, double *ms_out)
{
    const uint32_t n_opts = (uint32_t)w.opts.size();
    const uint32_t n_items = (uint32_t)w.item_opt.size();
    heston_status st;
    if ((st = reserve(c, c->batch_opts, n_opts * sizeof(BatchOption))) != HESTON_OK ||
        (st = reserve(c, c->batch_items, std::max<size_t>(n_items, 1) * 4)) != HESTON_OK ||
        (st = reserve(c, c->batch_counter, 16)) != HESTON_OK)
        return st;
    // unit records: the option's own slot array when given, else one shared array
    if (w.partials == nullptr) {
        if ((st = reserve(c, c->batch_partials, std::max<size_t>(n_items, 1) * ITEM_REC * 8)) !=
            HESTON_OK)
            return st;
        for (auto &o : w.opts)
            o.partials = (double *)c->batch_partials.ptr + (uint64_t)o.first_item * ITEM_REC;
    }
    int grid_price = 0, grid_adj = 0;
    if (w.n_price_items)
        grid_price = batch_resident_blocks(precision, scheme, false);
    if (w.n_items_total() > w.n_price_items)
        grid_adj = batch_resident_blocks(precision, scheme, true);
    if ((w.n_price_items && grid_price <= 0) || (w.n_items_total() > w.n_price_items && grid_adj <= 0))
        return fail(HESTON_DEVICE_ERROR, "occupancy query failed");
    const uint64_t per_block = adjoint_scratch_per_block(w.max_adj_steps, precision);
    if (grid_adj > 0 &&
        (st = reserve(c, c->batch_scratch, (size_t)grid_adj * per_block)) != HESTON_OK)
        return st;
    HIP_TRY(hipMemcpyAsync(c->batch_opts.ptr, w.opts.data(), n_opts * sizeof(BatchOption),
                           hipMemcpyHostToDevice, c->stream));
    if (n_items)
        HIP_TRY(hipMemcpyAsync(c->batch_items.ptr, w.item_opt.data(), n_items * 4,
                               hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(c->batch_counter.ptr, 0, 16, c->stream));
    BatchLaunch B;
    std::memset(&B, 0, sizeof(B));
    B.precision = precision;
    B.scheme = scheme;
    B.opts = (const BatchOption *)c->batch_opts.ptr;
    B.n_opts = n_opts;
    B.item_opt = (const uint32_t *)c->batch_items.ptr;
    HIP_TRY(hipEventRecord(c->ev0, c->stream));
    if (w.n_price_items) {
        B.adjoint = false;
        B.item_begin = 0;
        B.item_end = w.n_price_items;
        B.counter = (uint32_t *)c->batch_counter.ptr;
        B.grid = (uint32_t)std::min<uint64_t>(grid_price, (uint64_t)w.n_price_items * BATCH_UNITS);
        HIP_TRY(launch_batch(B, c->stream));
    }
    if (n_items > w.n_price_items) {
        B.adjoint = true;
        B.item_begin = w.n_price_items;
        B.item_end = n_items;
        B.counter = (uint32_t *)c->batch_counter.ptr + 1;
        B.scratch = (unsigned char *)c->batch_scratch.ptr;
        B.scratch_per_block = per_block;
        B.grid = (uint32_t)std::min<uint64_t>(grid_adj,
                                              (uint64_t)(n_items - w.n_price_items) * BATCH_UNITS);
        HIP_TRY(launch_batch(B, c->stream));
    }
    HIP_TRY(hipEventRecord(c->ev1, c->stream));
    float ms = 0;
    HIP_TRY(hipEventSynchronize(c->ev1));
    HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    if (ms_out)
        *ms_out = ms;
    return HESTON_OK;
}

// Orders requests (price-mode first, then adjoint; each by decreasing step
// count) and lays out their items: option j of the plan covers chunks
// [chunk_begin, chunk_begin + n_items) of request order[j].
void plan_batch(const std::vector<heston_request> &reqs, const std::vector<uint64_t> &chunk_begin,
                const std::vector<uint64_t> &chunk_count, BatchWork &w)
{
    const size_t n = reqs.size();
    w.order.resize(n);
    std::iota(w.order.begin(), w.order.end(), 0);
    std::stable_sort(w.order.begin(), w.order.end(), [&](size_t a, size_t b) {
        const bool aa = reqs[a].want == HESTON_WANT_ADJOINT, ab = reqs[b].want == HESTON_WANT_ADJOINT;
        if (aa != ab)
            return !aa;
        return reqs[a].n_steps > reqs[b].n_steps;
    });
    w.opts.clear();
    w.item_opt.clear();
    w.n_price_items = 0;
    w.max_adj_steps = 0;
    for (size_t j = 0; j < n; ++j) {
        const heston_request &r = reqs[w.order[j]];
        BatchOption b = batch_option(r);
        b.first_item = (uint32_t)w.item_opt.size();
        b.n_items = (uint32_t)chunk_count[w.order[j]];
        b.chunk_base = chunk_begin[w.order[j]];
        w.item_opt.insert(w.item_opt.end(), b.n_items, (uint32_t)j);
        if (b.adjoint)
            w.max_adj_steps = std::max(w.max_adj_steps, r.n_steps);
        else
            w.n_price_items += b.n_items;
        w.opts.push_back(b);
    }
}

} // namespace rt
} // namespace heston

using namespace heston;
using namespace heston::rt;

extern "C" heston_status heston_price_batch(heston_ctx *c, const heston_request *reqs, uint32_t n,
                                            const heston_opts *opts, heston_result *out,
                                            double *device_ms)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!c || !reqs || !out || n == 0)
        return fail(HESTON_INVALID_ARGUMENT, "ctx, reqs or out is NULL, or n is 0");
    if (opts && opts->struct_size != sizeof(heston_opts))
        return fail(HESTON_INVALID_ARGUMENT, "opts->struct_size does not match this library");
    heston_opts o;
    heston_default_opts(&o);
    if (opts)
        o = *opts;
    if (o.rng != HESTON_RNG_PHILOX)
        return fail(HESTON_UNSUPPORTED, "batches use Philox normals");
    if (o.scheme != HESTON_FULL_TRUNCATION && o.scheme != HESTON_ABSORPTION &&
        o.scheme != HESTON_QE)
        return fail(HESTON_UNSUPPORTED,
                    "batches use the Milstein scheme (full truncation or absorption) or QE");
    if (o.fixing_steps)
        return fail(HESTON_INVALID_ARGUMENT, "batched Asians fix at every step; fixing_steps must be NULL");
    if (o.control_variate != HESTON_CONTROL_NONE)
        return fail(HESTON_UNSUPPORTED, "batches take no control variate");
    std::vector<heston_request> rq(reqs, reqs + n);
    std::vector<uint64_t> begin(n, 0), count(n);
    uint64_t total = 0;
    for (uint32_t i = 0; i < n; ++i) {
        Request q;
        heston_status st = check_batch_request(rq[i], o, q);
        if (st != HESTON_OK)
            return fail(st, "request " + std::to_string(i) + ": " + g_last_error);
        count[i] = (rq[i].n_paths + BATCH_CHUNK - 1) / BATCH_CHUNK;
        total += count[i];
    }
    if (total >= (1ull << 32))
        return fail(HESTON_UNSUPPORTED, "more than 2^32 work items");
    DeviceGuard g(c->device);
    BatchWork w;
    plan_batch(rq, begin, count, w);
    double ms = 0;
    heston_status st = run_batch(c, w, o.precision, o.scheme, &ms);
    if (st != HESTON_OK)
        return st;
    if ((st = reserve(c, c->batch_sums, (size_t)n * N_ACC * 8)) != HESTON_OK)
        return st;
    BatchLaunch B;
    std::memset(&B, 0, sizeof(B));
    B.opts = (const BatchOption *)c->batch_opts.ptr;
    B.n_opts = n;
    HIP_TRY(launch_batch_reduce(B, (double *)c->batch_sums.ptr, c->stream));
    std::vector<double> sums((size_t)n * N_ACC);
    HIP_TRY(hipMemcpyAsync(sums.data(), c->batch_sums.ptr, sums.size() * 8, hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (uint32_t j = 0; j < n; ++j) {
        const size_t i = w.order[j];
        fill_result(rq[i], rq[i].n_paths, &sums[(size_t)j * N_ACC], out[i]);
        out[i].device_ms = ms;
    }
    const double wall =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (uint32_t i = 0; i < n; ++i)
        out[i].latency_ms = wall;
    if (device_ms)
        *device_ms = ms;
    return HESTON_OK;
}
