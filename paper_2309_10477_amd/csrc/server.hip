// Serving: continuous batching of pricing requests over the batched kernel.
//
// Engine thread:
//   1. admit queued requests while request slots and the device-memory budget
//      allow; a request's device state is a 256-byte record of running sums
//      plus one 512-byte record per 1024-path item of its path cap (one
//      128-byte record per 256-path unit);
//   2. launch: take the next items of every schedulable admitted request
//      (a fair share of the per-launch work each), run the batched kernel over
//      them, then the fold kernel, which extends every request's running sums
//      item by item in item order and applies the stopping rule, and copies the
//      folded states back to pinned memory.  Each of the three launch slots
//      has its own stream and adjoint scratch, so a launch's kernels fill the
//      compute units that the previous launch's last items leave idle; the
//      folds run in launch order (each waits on the previous launch's fold),
//      so new requests join while earlier ones run and every request's sums
//      are extended in item order;
//   3. complete: when a launch's event has fired, requests whose state says
//      done get their result and latency recorded, and their memory is freed.
// A request with an SE target is scheduled up to the items its observed SE
// implies (16 before its first fold), in as many pipelined launches as its
// fair share spreads them over; each fold refines the estimate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/heston.h"
#include "admission.hpp"
#include "batch_plan.hpp"
#include "device_math.hpp"
#include "internal.hpp"
#include "runtime.hpp"

namespace heston {
namespace {

// Device-resident state of one request (256 bytes).
struct ReqState {
    double sums[N_ACC];   // running sums over items 0 .. folded-1
    uint64_t cap_paths;   // path cap
    double se_target;     // 0: run to the cap
    uint32_t folded;      // items folded so far
    uint32_t done;        // the stopping rule has fired
    uint32_t cap_items;
    uint32_t stop_items;  // items in the final result
    double pad[12];
};
static_assert(sizeof(ReqState) == 256, "ReqState is 256 bytes");

struct FoldTask {
    ReqState *state;
    const double *records; // the request's item records, item 0 first
    uint32_t upto;         // items written once this launch is done
    uint32_t out_index;    // where the folded state is copied for the host
    uint32_t first;        // the request's first launch: initialise its state
    uint32_t cap_items;
    uint64_t cap_paths;
    double se_target;
};

// Column k of item i's record: the sum of its unit records in unit order.
__device__ __forceinline__ double item_col(const double *records, uint32_t i, uint32_t k)
{
    const double *r = records + (uint64_t)i * ITEM_REC + k;
    double t = r[0];
#pragma unroll
    for (uint32_t u = 1; u < BATCH_UNITS; ++u)
        t += r[u * N_ACC];
    return t;
}

// One block per task, the new items taken FOLD_CHUNK at a time: each thread
// sums one item's unit records (in unit order) into LDS, then thread 0 walks
// the chunk's price sums in item order to find where the stopping rule fires,
// and thread k < N_ACC adds column k of the chunk's items up to there, in
// item order.  The additions are those of a sequential walk, in its order.
constexpr uint32_t FOLD_CHUNK = 64;

__global__ __launch_bounds__(FOLD_CHUNK) void fold_kernel(const FoldTask *__restrict__ tasks,
                                                          ReqState *__restrict__ out)
{
    __shared__ double s_item[FOLD_CHUNK][N_ACC];
    __shared__ uint32_t s_take;
    __shared__ uint32_t s_done;
    const FoldTask t = tasks[blockIdx.x];
    ReqState *st = t.state;
    const uint32_t tid = threadIdx.x;
    if (t.first) {
        double *raw = reinterpret_cast<double *>(st);
        if (tid < sizeof(ReqState) / 8)
            raw[tid] = 0.0;
        __syncthreads();
        if (tid == 0) {
            st->cap_paths = t.cap_paths;
            st->se_target = t.se_target;
            st->cap_items = t.cap_items;
        }
        __syncthreads();
    }
    if (!st->done) {
        const uint32_t from = st->folded;
        const uint64_t cap_paths = st->cap_paths;
        const uint32_t cap_items = st->cap_items;
        const double se_target = st->se_target;
        double acc = tid < N_ACC ? st->sums[tid] : 0.0;
        double s = st->sums[0], ss = st->sums[1];
        uint32_t stop = t.upto, done = 0;
        for (uint32_t base = from; base < t.upto; base += FOLD_CHUNK) {
            const uint32_t n = min(FOLD_CHUNK, t.upto - base);
            if (tid < n)
                for (uint32_t k = 0; k < N_ACC; ++k)
                    s_item[tid][k] = item_col(t.records, base + tid, k);
            __syncthreads();
            if (tid == 0) {
                uint32_t take = n, d = 0;
                for (uint32_t j = 0; j < n; ++j) {
                    const uint32_t i = base + j;
                    s += s_item[j][0];
                    ss += s_item[j][1];
                    const uint64_t paths = std::min<uint64_t>((uint64_t)(i + 1) * BATCH_CHUNK, cap_paths);
                    const double nn = (double)paths, m = s / nn;
                    const double var = paths > 1 ? fmax((ss - s * m) / (nn - 1.0), 0.0) : 0.0;
                    const bool se_ok = se_target > 0 && i + 1 >= 2 && sqrt(var / nn) <= se_target;
                    if (se_ok || i + 1 == cap_items) {
                        take = j + 1;
                        d = 1;
                        break;
                    }
                }
                s_take = take;
                s_done = d;
            }
            __syncthreads();
            const uint32_t take = s_take;
            if (tid < N_ACC)
                for (uint32_t j = 0; j < take; ++j)
                    acc += s_item[j][tid];
            done = s_done;
            __syncthreads(); // the chunk is read before the next one overwrites it
            if (done) {
                stop = base + take;
                break;
            }
        }
        if (tid < N_ACC)
            st->sums[tid] = acc;
        __syncthreads();
        if (tid == 0) {
            st->folded = stop;
            if (done) {
                st->done = 1;
                st->stop_items = stop;
            }
        }
    }
    __syncthreads();
    // copy the state out for the host (after the updates above)
    const double *src = reinterpret_cast<const double *>(st);
    double *dst = reinterpret_cast<double *>(out + t.out_index);
    if (threadIdx.x < sizeof(ReqState) / 8)
        dst[threadIdx.x] = src[threadIdx.x];
}

} // namespace
} // namespace heston

using namespace heston;
using namespace heston::rt;
using Clock = std::chrono::steady_clock;

namespace {

struct Req {
    heston_request r;
    uint64_t ticket;
    Clock::time_point t_submit;
    bool started = false;     // its device state has been initialised
    uint32_t cap_items = 0;
    uint32_t scheduled = 0;   // items launched so far (items [0, scheduled))
    uint32_t folded = 0;      // items folded (from the last completed launch)
    uint32_t target = 16;     // items the engine currently aims for
    uint32_t inflight = 0;    // launches holding items of this request
    double gpu_ms = 0;        // summed durations of the completed launches that held its items
    bool done = false;
    unsigned char *mem = nullptr; // state then item records, in the pool
    ReqState *state() const { return reinterpret_cast<ReqState *>(mem); }
    double *records() const { return reinterpret_cast<double *>(mem + sizeof(ReqState)); }
};

struct Launch {
    hipStream_t stream = nullptr;
    hipEvent_t fold_done = nullptr; // the fold of this slot's latest launch
    unsigned char *scratch = nullptr; // this slot's adjoint scratch
    DevBuf opts, items, counter, tasks, out;
    heston::BatchOption *h_opts = nullptr;
    uint32_t *h_items = nullptr;
    FoldTask *h_tasks = nullptr;
    ReqState *h_out = nullptr;
    size_t cap_opts = 0, cap_items = 0;
    hipEvent_t start = nullptr, end = nullptr;
    bool busy = false;
    std::vector<Req *> reqs;
    double path_steps = 0;
};

} // namespace

struct heston_server {
    heston_ctx *ctx = nullptr;
    heston_server_config cfg{};
    DevBuf pool_buf, scratch;
    uint64_t scratch_per_block = 0;
    uint32_t grid_price = 0, grid_adj = 0;
    Pool pool;
    std::vector<Launch> launches; // ring
    size_t next_launch = 0;
    std::deque<size_t> inflight;  // launch indices in launch order
    int last_fold = -1;           // slot of the latest launch (its fold orders the next)
    // busy time: the union of the launches' device intervals, accumulated per
    // busy period (from the first launch enqueued with none in flight to the
    // end of the last one completed)
    hipEvent_t span_start = nullptr;
    double busy_closed_ms = 0, busy_open_ms = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> queue;
    std::vector<Req *> active;
    std::unordered_map<uint64_t, Req *> tickets;
    std::unordered_map<uint64_t, heston_result> results;
    std::vector<double> latencies_ms;
    uint64_t next_ticket = 1;
    heston_server_stats stats{};
    std::atomic<bool> stop{false};
    std::thread engine;
    std::string engine_error;
};

namespace {

constexpr size_t N_SLOTS = 3; // launch slots, each with its own stream

// Waits for each slot's stream, then frees its buffers, events and stream.
void release_launches(heston_server *s)
{
    for (auto &L : s->launches) {
        if (L.stream)
            (void)hipStreamSynchronize(L.stream);
        for (DevBuf *b : {&L.opts, &L.items, &L.counter, &L.tasks, &L.out})
            if (b->ptr)
                (void)hipFree(b->ptr);
        if (L.h_opts) (void)hipHostFree(L.h_opts);
        if (L.h_items) (void)hipHostFree(L.h_items);
        if (L.h_tasks) (void)hipHostFree(L.h_tasks);
        if (L.h_out) (void)hipHostFree(L.h_out);
        if (L.start) (void)hipEventDestroy(L.start);
        if (L.end) (void)hipEventDestroy(L.end);
        if (L.fold_done) (void)hipEventDestroy(L.fold_done);
        if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    s->launches.clear();
}

heston_status alloc_host(void **p, size_t bytes)
{
    HIP_TRY(hipHostMalloc(p, bytes));
    return HESTON_OK;
}

// Server-owned device buffers (outside the context's accounting; the engine
// thread must not touch the context's state).
heston_status grow(DevBuf &b, size_t bytes)
{
    if (b.bytes >= bytes)
        return HESTON_OK;
    if (b.ptr)
        (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
    HIP_TRY(hipMalloc(&b.ptr, bytes));
    b.bytes = bytes;
    return HESTON_OK;
}

heston_status grow_launch(Launch &L, size_t n_opts, size_t n_items)
{
    heston_status st;
    if (n_opts > L.cap_opts) {
        const size_t cap = std::max(n_opts, 2 * L.cap_opts);
        if (L.h_opts) (void)hipHostFree(L.h_opts);
        if (L.h_tasks) (void)hipHostFree(L.h_tasks);
        if (L.h_out) (void)hipHostFree(L.h_out);
        L.h_opts = nullptr; L.h_tasks = nullptr; L.h_out = nullptr;
        if ((st = alloc_host((void **)&L.h_opts, cap * sizeof(heston::BatchOption))) != HESTON_OK ||
            (st = alloc_host((void **)&L.h_tasks, cap * sizeof(FoldTask))) != HESTON_OK ||
            (st = alloc_host((void **)&L.h_out, cap * sizeof(ReqState))) != HESTON_OK ||
            (st = grow(L.opts, cap * sizeof(heston::BatchOption))) != HESTON_OK ||
            (st = grow(L.tasks, cap * sizeof(FoldTask))) != HESTON_OK ||
            (st = grow(L.out, cap * sizeof(ReqState))) != HESTON_OK)
            return st;
        L.cap_opts = cap;
    }
    if (n_items > L.cap_items) {
        const size_t cap = std::max(n_items, 2 * L.cap_items);
        if (L.h_items) (void)hipHostFree(L.h_items);
        L.h_items = nullptr;
        if ((st = alloc_host((void **)&L.h_items, cap * 4)) != HESTON_OK ||
            (st = grow(L.items, cap * 4)) != HESTON_OK)
            return st;
        L.cap_items = cap;
    }
    return grow(L.counter, 16);
}

// Admission: queued requests move to the active set in arrival order while a
// slot and pool memory are available.
void admit(heston_server *s)
{
    s->stats.admitted += admit_in_order(
        s->queue, s->active, s->cfg.max_active, s->pool,
        [](const Req *q) { return sizeof(ReqState) + (uint64_t)q->cap_items * ITEM_REC * 8; },
        [](Req *q, unsigned char *m) { q->mem = m; });
}

// Items a request asks for in the next launch.  A request with an SE target
// asks for items up to its current estimate of the items it needs, also while
// earlier launches of it are in flight (launches are pipelined); the fold
// stops at the first item that meets the target, so items beyond it are
// computed and ignored, and the result does not depend on the scheduling.
uint32_t wanted_items(const Req *q)
{
    if (q->done || q->scheduled >= q->cap_items)
        return 0;
    const uint32_t goal = q->r.se_target > 0 ? std::min(q->target, q->cap_items) : q->cap_items;
    return goal > q->scheduled ? goal - q->scheduled : 0;
}

heston_status launch_next(heston_server *s, bool &launched)
{
    launched = false;
    Launch &L = s->launches[s->next_launch];
    if (L.busy)
        return HESTON_OK;
    std::vector<Req *> sel;
    std::vector<uint32_t> want;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        admit(s);
        for (Req *q : s->active) {
            const uint32_t w = wanted_items(q);
            if (w) {
                sel.push_back(q);
                want.push_back(w);
            }
        }
    }
    if (sel.empty())
        return HESTON_OK;
    // fair share of the launch's work, at least one item each
    const double share = (double)s->cfg.launch_path_steps / (double)sel.size();
    std::vector<heston_request> rq;
    std::vector<uint64_t> begin, count;
    double ps = 0;
    for (size_t i = 0; i < sel.size(); ++i) {
        const double per_item = (double)BATCH_CHUNK * sel[i]->r.n_steps;
        const uint32_t quota = (uint32_t)std::max(1.0, std::floor(share / per_item));
        const uint32_t k = std::min(want[i], quota);
        rq.push_back(sel[i]->r);
        begin.push_back(sel[i]->scheduled);
        count.push_back(k);
        ps += per_item * k;
    }
    BatchWork w;
    plan_batch(rq, begin, count, w);
    heston_status st = grow_launch(L, w.opts.size(), w.item_opt.size());
    if (st != HESTON_OK)
        return st;
    L.reqs.clear();
    for (size_t j = 0; j < w.opts.size(); ++j) {
        Req *q = sel[w.order[j]];
        heston::BatchOption &o = w.opts[j];
        o.partials = q->records() + (uint64_t)o.chunk_base * ITEM_REC;
        L.h_opts[j] = o;
        L.h_tasks[j] = FoldTask{q->state(), q->records(), (uint32_t)(o.chunk_base + o.n_items),
                                (uint32_t)j, q->started ? 0u : 1u, q->cap_items, q->r.n_paths,
                                q->r.se_target};
        q->started = true;
        L.reqs.push_back(q);
    }
    std::memcpy(L.h_items, w.item_opt.data(), w.item_opt.size() * 4);
    const uint32_t n_opts = (uint32_t)w.opts.size(), n_items = (uint32_t)w.item_opt.size();
    hipStream_t sm = L.stream;
    if (s->inflight.empty())
        HIP_TRY(hipEventRecord(s->span_start, sm));
    HIP_TRY(hipMemcpyAsync(L.opts.ptr, L.h_opts, n_opts * sizeof(heston::BatchOption),
                           hipMemcpyHostToDevice, sm));
    HIP_TRY(hipMemcpyAsync(L.items.ptr, L.h_items, n_items * 4, hipMemcpyHostToDevice, sm));
    HIP_TRY(hipMemcpyAsync(L.tasks.ptr, L.h_tasks, n_opts * sizeof(FoldTask),
                           hipMemcpyHostToDevice, sm));
    HIP_TRY(hipMemsetAsync(L.counter.ptr, 0, 16, sm));
    HIP_TRY(hipEventRecord(L.start, sm));
    BatchLaunch B;
    std::memset(&B, 0, sizeof(B));
    B.precision = s->cfg.precision;
    B.scheme = s->cfg.scheme;
    B.opts = (const heston::BatchOption *)L.opts.ptr;
    B.n_opts = n_opts;
    B.item_opt = (const uint32_t *)L.items.ptr;
    if (w.n_price_items) {
        B.adjoint = false;
        B.item_begin = 0;
        B.item_end = w.n_price_items;
        B.counter = (uint32_t *)L.counter.ptr;
        B.grid = std::min<uint32_t>(s->grid_price, w.n_price_items * BATCH_UNITS);
        HIP_TRY(launch_batch(B, sm));
    }
    if (n_items > w.n_price_items) {
        B.adjoint = true;
        B.item_begin = w.n_price_items;
        B.item_end = n_items;
        B.counter = (uint32_t *)L.counter.ptr + 1;
        B.scratch = L.scratch;
        B.scratch_per_block = s->scratch_per_block;
        B.grid = std::min<uint32_t>(s->grid_adj, (n_items - w.n_price_items) * BATCH_UNITS);
        HIP_TRY(launch_batch(B, sm));
    }
    if (s->last_fold >= 0)
        HIP_TRY(hipStreamWaitEvent(sm, s->launches[(size_t)s->last_fold].fold_done, 0));
    hipLaunchKernelGGL(fold_kernel, dim3(n_opts), dim3(64), 0, sm, (const FoldTask *)L.tasks.ptr,
                       (ReqState *)L.out.ptr);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(L.fold_done, sm));
    s->last_fold = (int)s->next_launch;
    HIP_TRY(hipMemcpyAsync(L.h_out, L.out.ptr, n_opts * sizeof(ReqState), hipMemcpyDeviceToHost,
                           sm));
    HIP_TRY(hipEventRecord(L.end, sm));
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (size_t j = 0; j < w.opts.size(); ++j) {
            Req *q = sel[w.order[j]];
            q->scheduled += w.opts[j].n_items;
            q->inflight++;
        }
        s->stats.launches++;
        s->stats.path_steps += ps;
    }
    L.path_steps = ps;
    L.busy = true;
    s->inflight.push_back(s->next_launch);
    s->next_launch = (s->next_launch + 1) % s->launches.size();
    launched = true;
    return HESTON_OK;
}

void finish(heston_server *s, Req *q, const ReqState &st)
{
    heston_result res;
    const uint64_t n_used = std::min<uint64_t>((uint64_t)st.stop_items * BATCH_CHUNK, q->r.n_paths);
    fill_result(q->r, n_used, st.sums, res);
    const double ms =
        std::chrono::duration<double, std::milli>(Clock::now() - q->t_submit).count();
    res.device_ms = q->gpu_ms;
    res.latency_ms = ms;
    s->results[q->ticket] = res;
    s->latencies_ms.push_back(ms);
    s->stats.completed++;
    q->done = true;
}

// Processes completed launches in order; returns true if any completed.
heston_status complete_ready(heston_server *s, bool block, bool &any)
{
    any = false;
    while (!s->inflight.empty()) {
        Launch &L = s->launches[s->inflight.front()];
        if (block) {
            HIP_TRY(hipEventSynchronize(L.end));
        } else {
            const hipError_t e = hipEventQuery(L.end);
            if (e == hipErrorNotReady)
                break;
            HIP_TRY(e);
        }
        block = false;
        float ms = 0, span = 0;
        (void)hipEventElapsedTime(&ms, L.start, L.end);
        (void)hipEventElapsedTime(&span, s->span_start, L.end);
        std::lock_guard<std::mutex> lk(s->mu);
        // launches complete in launch order; the busy period's extent so far
        s->busy_open_ms = std::max(s->busy_open_ms, (double)span);
        for (size_t j = 0; j < L.reqs.size(); ++j) {
            Req *q = L.reqs[j];
            const ReqState &st = L.h_out[j];
            q->inflight--;
            q->gpu_ms += ms;
            if (!q->done) {
                q->folded = st.folded;
                if (st.done) {
                    finish(s, q, st);
                } else if (q->r.se_target > 0 && st.folded > 0) {
                    // items needed for the target if the SE keeps falling as 1/sqrt(n)
                    const double n = (double)std::min<uint64_t>((uint64_t)st.folded * BATCH_CHUNK,
                                                               q->r.n_paths);
                    const double m = st.sums[0] / n;
                    const double var = std::max((st.sums[1] - st.sums[0] * m) / (n - 1.0), 0.0);
                    const double se = std::sqrt(var / n);
                    const double need = st.folded * (se * se) / (q->r.se_target * q->r.se_target);
                    q->target = (uint32_t)std::min<double>(q->cap_items,
                                                           std::max<double>(st.folded + 1,
                                                                            std::ceil(need * 1.05)));
                }
            }
        }
        // release finished requests no launch refers to any more
        for (size_t j = 0; j < L.reqs.size(); ++j) {
            Req *q = L.reqs[j];
            if (q->done && q->inflight == 0 && q->mem) {
                s->pool.release(q->mem);
                q->mem = nullptr;
                s->active.erase(std::find(s->active.begin(), s->active.end(), q));
                s->tickets.erase(q->ticket);
                delete q;
            }
        }
        L.busy = false;
        L.reqs.clear();
        s->inflight.pop_front();
        if (s->inflight.empty()) {
            s->busy_closed_ms += s->busy_open_ms;
            s->busy_open_ms = 0;
        }
        s->stats.busy_ms = s->busy_closed_ms + s->busy_open_ms;
        any = true;
    }
    if (any)
        s->cv_done.notify_all();
    return HESTON_OK;
}

void engine_main(heston_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    while (!s->stop.load()) {
        bool launched = false, completed = false;
        heston_status st = launch_next(s, launched);
        if (st == HESTON_OK)
            st = complete_ready(s, false, completed);
        if (st != HESTON_OK) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->engine_error = g_last_error;
            s->stop.store(true);
            s->cv_done.notify_all();
            break;
        }
        if (launched || completed)
            continue;
        if (!s->inflight.empty()) {
            // every launch slot busy or nothing new to launch: wait for the oldest
            const bool ring_full = s->inflight.size() == s->launches.size();
            if (ring_full) {
                complete_ready(s, true, completed);
                continue;
            }
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait_for(lk, std::chrono::microseconds(50));
            continue;
        }
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->queue.empty())
            s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    }
    // drain the launches in flight so no kernel outlives the engine
    bool any = false;
    while (!s->inflight.empty())
        if (complete_ready(s, true, any) != HESTON_OK)
            break;
}

} // namespace

extern "C" {

heston_status heston_server_default_config(heston_server_config *c)
{
    if (!c)
        return fail(HESTON_INVALID_ARGUMENT, "cfg is NULL");
    std::memset(c, 0, sizeof(*c));
    c->struct_size = sizeof(heston_server_config);
    c->precision = HESTON_FP32;
    c->scheme = HESTON_FULL_TRUNCATION;
    c->max_active = 4096;
    c->max_steps = 2048;
    c->hbm_budget_bytes = 8ull << 30;
    c->launch_path_steps = 1ull << 29;
    return HESTON_OK;
}

heston_status heston_server_create(heston_ctx *ctx, const heston_server_config *cfg,
                                   heston_server **out)
{
    if (!ctx || !out)
        return fail(HESTON_INVALID_ARGUMENT, "ctx or out is NULL");
    heston_server_config c;
    heston_server_default_config(&c);
    if (cfg) {
        if (cfg->struct_size != sizeof(heston_server_config))
            return fail(HESTON_INVALID_ARGUMENT, "cfg->struct_size does not match this library");
        c = *cfg;
    }
    if ((c.precision != HESTON_FP32 && c.precision != HESTON_FP64) ||
        (c.scheme != HESTON_FULL_TRUNCATION && c.scheme != HESTON_ABSORPTION &&
         c.scheme != HESTON_QE) || c.max_active == 0 ||
        c.max_steps == 0 || c.max_steps > (1u << 20) || c.launch_path_steps == 0)
        return fail(HESTON_INVALID_ARGUMENT, "invalid server configuration");
    DeviceGuard g(ctx->device);
    heston_server *s = new heston_server;
    s->ctx = ctx;
    s->cfg = c;
    auto bail = [&](heston_status st) {
        release_launches(s);
        if (s->span_start) (void)hipEventDestroy(s->span_start);
        if (s->pool_buf.ptr) (void)hipFree(s->pool_buf.ptr);
        if (s->scratch.ptr) (void)hipFree(s->scratch.ptr);
        delete s;
        return st;
    };
    s->launches.resize(N_SLOTS);
    for (auto &L : s->launches)
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&L.start) != hipSuccess || hipEventCreate(&L.end) != hipSuccess ||
            hipEventCreateWithFlags(&L.fold_done, hipEventDisableTiming) != hipSuccess)
            return bail(fail(HESTON_DEVICE_ERROR, "stream or event creation failed"));
    if (hipEventCreate(&s->span_start) != hipSuccess)
        return bail(fail(HESTON_DEVICE_ERROR, "hipEventCreate failed"));
    s->grid_price = batch_resident_blocks(c.precision, c.scheme, false);
    s->grid_adj = batch_resident_blocks(c.precision, c.scheme, true);
    if (s->grid_price == 0 || s->grid_adj == 0)
        return bail(fail(HESTON_DEVICE_ERROR, "occupancy query failed"));
    s->scratch_per_block = adjoint_scratch_per_block(c.max_steps, c.precision);
    const uint64_t slot_scratch = (uint64_t)s->grid_adj * s->scratch_per_block;
    const uint64_t scratch_bytes = N_SLOTS * slot_scratch;
    const uint64_t launch_bytes = 64ull << 20; // launch buffers, grown on demand
    if (c.hbm_budget_bytes < scratch_bytes + launch_bytes + 4096)
        return bail(fail(HESTON_OVER_BUDGET, "budget below the adjoint scratch (" +
                                                 std::to_string(scratch_bytes) +
                                                 " bytes) and the launch buffers"));
    const uint64_t pool_bytes = c.hbm_budget_bytes - scratch_bytes - launch_bytes;
    if (hipMalloc(&s->scratch.ptr, scratch_bytes) != hipSuccess ||
        hipMalloc(&s->pool_buf.ptr, pool_bytes) != hipSuccess)
        return bail(fail(HESTON_OUT_OF_MEMORY, "server memory"));
    s->scratch.bytes = scratch_bytes;
    s->pool_buf.bytes = pool_bytes;
    s->pool.init((unsigned char *)s->pool_buf.ptr, pool_bytes);
    for (size_t i = 0; i < s->launches.size(); ++i) {
        Launch &L = s->launches[i];
        L.scratch = (unsigned char *)s->scratch.ptr + i * slot_scratch;
        // sized for the usual launch up front: growing a buffer later frees the
        // old one, which waits for the whole device
        heston_status st = grow_launch(L, std::min<uint32_t>(c.max_active, 4096), 1u << 16);
        if (st != HESTON_OK)
            return bail(st);
    }
    s->engine = std::thread(engine_main, s);
    *out = s;
    return HESTON_OK;
}

heston_status heston_server_destroy(heston_server *s)
{
    if (!s)
        return fail(HESTON_INVALID_ARGUMENT, "server is NULL");
    s->stop.store(true);
    s->cv_work.notify_all();
    if (s->engine.joinable())
        s->engine.join();
    DeviceGuard g(s->ctx->device);
    release_launches(s);
    (void)hipEventDestroy(s->span_start);
    (void)hipFree(s->pool_buf.ptr);
    (void)hipFree(s->scratch.ptr);
    for (Req *q : s->queue)
        delete q;
    for (Req *q : s->active)
        delete q;
    delete s;
    return HESTON_OK;
}

heston_status heston_submit(heston_server *s, const heston_request *req, uint64_t *ticket)
{
    if (!s || !req || !ticket)
        return fail(HESTON_INVALID_ARGUMENT, "server, req or ticket is NULL");
    heston_opts o;
    heston_default_opts(&o);
    o.precision = s->cfg.precision;
    o.scheme = s->cfg.scheme;
    Request q;
    heston_status st = check_batch_request(*req, o, q);
    if (st != HESTON_OK)
        return st;
    if (req->n_steps > s->cfg.max_steps)
        return fail(HESTON_INVALID_ARGUMENT, "n_steps above the server's max_steps");
    const uint64_t items = (req->n_paths + BATCH_CHUNK - 1) / BATCH_CHUNK;
    if (items >= (1ull << 28) || sizeof(ReqState) + items * ITEM_REC * 8 > s->pool_buf.bytes)
        return fail(HESTON_INVALID_ARGUMENT, "path cap too large for the server's budget");
    Req *r = new Req;
    r->r = *req;
    r->cap_items = (uint32_t)items;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop.load()) {
            delete r;
            return fail(HESTON_DEVICE_ERROR, "server stopped: " + s->engine_error);
        }
        r->ticket = s->next_ticket++;
        s->queue.push_back(r);
        s->tickets[r->ticket] = r;
        s->stats.submitted++;
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return HESTON_OK;
}

heston_status heston_poll(heston_server *s, uint64_t ticket, heston_result *out)
{
    if (!s || !out)
        return fail(HESTON_INVALID_ARGUMENT, "server or out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it != s->results.end()) {
        *out = it->second;
        s->results.erase(it);
        return HESTON_OK;
    }
    if (s->tickets.count(ticket))
        return s->stop.load() ? fail(HESTON_DEVICE_ERROR, "server stopped: " + s->engine_error)
                              : HESTON_PENDING;
    return fail(HESTON_NOT_FOUND, "unknown ticket");
}

heston_status heston_wait(heston_server *s, uint64_t ticket, double timeout_ms, heston_result *out)
{
    if (!s || !out)
        return fail(HESTON_INVALID_ARGUMENT, "server or out is NULL");
    const auto deadline = Clock::now() + std::chrono::duration<double, std::milli>(timeout_ms);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        auto it = s->results.find(ticket);
        if (it != s->results.end()) {
            *out = it->second;
            s->results.erase(it);
            return HESTON_OK;
        }
        if (!s->tickets.count(ticket))
            return fail(HESTON_NOT_FOUND, "unknown ticket");
        if (s->stop.load())
            return fail(HESTON_DEVICE_ERROR, "server stopped: " + s->engine_error);
        if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout)
            return HESTON_PENDING;
    }
}

heston_status heston_server_get_stats(heston_server *s, heston_server_stats *out)
{
    if (!s || !out)
        return fail(HESTON_INVALID_ARGUMENT, "server or out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    heston_server_stats st = s->stats;
    st.queued = s->queue.size();
    st.active = s->active.size();
    st.pool_bytes = s->pool_buf.bytes;
    st.pool_free_bytes = s->pool.free_bytes();
    std::vector<double> l = s->latencies_ms;
    if (!l.empty()) {
        std::sort(l.begin(), l.end());
        auto pct = [&](double q) {
            const size_t i = (size_t)std::min<double>(l.size() - 1, std::ceil(q * l.size()) - 1);
            return l[i];
        };
        st.p50_ms = pct(0.50);
        st.p99_ms = pct(0.99);
        double sum = 0;
        for (double v : l)
            sum += v;
        st.mean_ms = sum / l.size();
        st.max_ms = l.back();
    }
    *out = st;
    return HESTON_OK;
}

} // extern "C"
