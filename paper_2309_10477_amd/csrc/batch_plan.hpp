// Host-side plan of a batched launch, shared by heston_price_batch and the
// serving loop.
#pragma once

#include <vector>

#include "../../include/heston.h"
#include "internal.hpp"
#include "runtime.hpp"

namespace heston {
namespace rt {

struct BatchWork {
    std::vector<BatchOption> opts;  // plan order: price-mode options first
    std::vector<uint32_t> item_opt; // option of each item
    std::vector<size_t> order;      // order[j] = caller index of plan option j
    uint32_t n_price_items = 0;     // items [0, n_price_items) are price-mode
    uint32_t max_adj_steps = 0;
    double *partials = nullptr;     // non-null: every opts[j].partials is already set
    uint32_t n_items_total() const { return (uint32_t)item_opt.size(); }
};

heston_status check_batch_request(const heston_request &r, const heston_opts &o, Request &q);
BatchOption batch_option(const heston_request &r);
void fill_result(const heston_request &r, uint64_t n_paths, const double *sums, heston_result &out);
uint64_t adjoint_scratch_per_block(uint32_t max_steps, int precision);
// Lays out chunks [chunk_begin[i], chunk_begin[i] + chunk_count[i]) of every request.
void plan_batch(const std::vector<heston_request> &reqs, const std::vector<uint64_t> &chunk_begin,
                const std::vector<uint64_t> &chunk_count, BatchWork &w);
// Uploads the plan and launches the batched kernels on the context stream;
// returns after they finish, with their GPU time in *ms.
heston_status run_batch(heston_ctx *c, BatchWork &w, int precision, int scheme, double *ms);

} // namespace rt
} // namespace heston
