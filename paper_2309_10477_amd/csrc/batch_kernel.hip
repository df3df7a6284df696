// Persistent batched kernel: many options of different sizes in one launch.
//
// The work is a list of items; item g is chunk chunk_base[o] + (g - first_item[o])
// of option o = item_opt[g], i.e. paths [chunk * CHUNK, (chunk + 1) * CHUNK) of
// that option's own stream, run as BATCH_UNITS units of BLOCK paths.  A grid
// sized to the resident capacity of the chip pops unit indices from one device
// counter until the list is exhausted, so every workgroup ends when the
// counter passes the last unit.  Items are ordered by decreasing cost (longest
// step counts first), so the tail of the launch holds the cheapest units.
// Each unit writes one FP64 partial record; a second kernel sums every
// option's records in unit order.  The partial of a unit depends only on its
// own paths and the option's sum only on the unit order, so an option's result
// is bitwise the same alone or in any batch.
//
// Per item and path: the Milstein path of the paper's algorithm "Milstein
// approximation under Heston model" (or Andersen's QE step, the paper's Future
// Work) in R, payoff and pathwise estimators in FP64; in adjoint mode the
// path's forward pass also stores checkpoints in the workgroup's scratch slot
// and the reverse sweep follows immediately.
#include "device_math.hpp"
#include "internal.hpp"
#include "path_step.hpp"

namespace heston {
namespace {

// Runs unit `sub` of an item (its paths sub BLOCK .. sub BLOCK + BLOCK-1);
// the wave sums go to the LDS row red[wave].
// SC: 0 Milstein with full truncation, 1 with absorption, 2 QE.
template <class R, bool ASIAN, int SC, bool ADJ>
__device__ __forceinline__ void run_unit_paths(const BatchOption &op, uint64_t chunk, uint32_t sub,
                                               R *scratch, double (*red)[N_ACC])
{
    const uint32_t tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const uint64_t p = chunk * BATCH_CHUNK + (uint64_t)sub * BLOCK + tid;
    const bool active = p < op.n_paths;
    double out[8];
    if constexpr (ADJ) {
        R x, v, A, B;
        if constexpr (SC == 2) {
            forward_path_qe<R, ASIAN>(op.k, p, x, v, A, B, scratch, BLOCK, tid, BATCH_CKPT_EVERY);
            __threadfence_block();
            adjoint_path_qe<R, ASIAN, BATCH_CKPT_EVERY>(op.k, p, scratch, BLOCK, tid, out);
        } else {
            forward_path<R, ASIAN, SC == 0>(op.k, p, x, v, A, B, scratch, BLOCK, tid,
                                            BATCH_CKPT_EVERY);
            __threadfence_block();
            adjoint_path<R, ASIAN, SC == 0, BATCH_CKPT_EVERY>(op.k, p, scratch, BLOCK, tid, out);
        }
    } else {
        R x, v, A, B;
        if constexpr (SC == 2)
            forward_path_qe<R, ASIAN>(op.k, p, x, v, A, B, nullptr, 0, 0, 2);
        else
            forward_path<R, ASIAN, SC == 0>(op.k, p, x, v, A, B, nullptr, 0, 0, 2);
        path_estimators<ASIAN>(op.k, (double)x, (double)A, (double)B, out[0], out[1], out[2]);
#pragma unroll
        for (int e = 3; e < 8; ++e)
            out[e] = 0.0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const double y = active ? out[e] : 0.0;
        const double s1 = wave_sum(y);
        const double s2 = wave_sum(y * y);
        if (lane == 0) {
            red[wave][2 * e] = s1;
            red[wave][2 * e + 1] = s2;
        }
    }
}

// Adjoint units run the forward pass and the reverse sweep back to back; left
// to itself the single-precision kernel held up to 141 VGPRs (three waves per
// SIMD); bounded to four waves per SIMD it fits in 128 or fewer (114-115 for
// the Milstein schemes in the current build), without spills.
// The QE reverse sweep keeps more per step (Zs, the branch input) and would
// spill at four waves; it is bounded to three.
template <class R, int SC, bool ADJ> struct BatchWaves {
    static constexpr int value = (ADJ && sizeof(R) == 4) ? (SC == 2 ? 3 : 4) : 1;
};

template <class R, int SC, bool ADJ>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(BatchWaves<R, SC, ADJ>::value)))
void batch_kernel(const BatchOption *__restrict__ opts,
                                                      const uint32_t *__restrict__ item_opt,
                                                      uint32_t item_begin, uint32_t item_end,
                                                      uint32_t *counter,
                                                      unsigned char *scratch,
                                                      uint64_t scratch_per_block)
{
    __shared__ uint32_t s_unit;
    __shared__ double red[BLOCK / 64][N_ACC];
    R *my_scratch = reinterpret_cast<R *>(scratch + (uint64_t)blockIdx.x * scratch_per_block);
    const uint32_t n_units = (item_end - item_begin) * BATCH_UNITS;
    for (;;) {
        if (threadIdx.x == 0)
            s_unit = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t pos = __builtin_amdgcn_readfirstlane(s_unit);
        __syncthreads();
        if (pos >= n_units)
            break;
        const uint32_t g = item_begin + pos / BATCH_UNITS, sub = pos % BATCH_UNITS;
        const uint32_t o = __builtin_amdgcn_readfirstlane(item_opt[g]);
        const BatchOption &op = opts[o];
        const uint32_t i = g - op.first_item;
        const uint64_t chunk = op.chunk_base + i;
        if (op.k.type >= 2)
            run_unit_paths<R, true, SC, ADJ>(op, chunk, sub, my_scratch, red);
        else
            run_unit_paths<R, false, SC, ADJ>(op, chunk, sub, my_scratch, red);
        __syncthreads();
        if (threadIdx.x < N_ACC) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < BLOCK / 64; ++w)
                t += red[w][threadIdx.x];
            op.partials[((uint64_t)i * BATCH_UNITS + sub) * N_ACC + threadIdx.x] = t;
        }
    }
}

// Option o's sums: its unit records added in unit order.  Thread t owns
// column t % N_ACC and units u = t / N_ACC (mod BLOCK / N_ACC); the
// BLOCK / N_ACC per-column partials are then added in a fixed order.
__global__ __launch_bounds__(BLOCK) void batch_reduce_kernel(const BatchOption *__restrict__ opts,
                                                             double *__restrict__ sums)
{
    constexpr int LANES = BLOCK / N_ACC;
    __shared__ double red[LANES][N_ACC];
    const BatchOption &op = opts[blockIdx.x];
    const int col = threadIdx.x % N_ACC, slot = threadIdx.x / N_ACC;
    const uint64_t n_units = (uint64_t)op.n_items * BATCH_UNITS;
    double t = 0.0;
    for (uint64_t u = slot; u < n_units; u += LANES)
        t += op.partials[u * N_ACC + col];
    red[slot][col] = t;
    __syncthreads();
    if (threadIdx.x < N_ACC) {
        double s = 0.0;
        for (int k = 0; k < LANES; ++k)
            s += red[k][threadIdx.x];
        sums[(uint64_t)blockIdx.x * N_ACC + threadIdx.x] = s;
    }
}

template <class R, int SC, bool ADJ> int resident_blocks()
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<R, SC, ADJ>, BLOCK, 0) !=
            hipSuccess)
        return 0;
    return cus * (per_cu > 0 ? per_cu : 1);
}

template <class R, int SC, bool ADJ>
hipError_t launch_t(const BatchLaunch &B, hipStream_t s)
{
    hipLaunchKernelGGL((batch_kernel<R, SC, ADJ>), dim3(B.grid), dim3(BLOCK), 0, s, B.opts,
                       B.item_opt, B.item_begin, B.item_end, B.counter, B.scratch,
                       B.scratch_per_block);
    return hipGetLastError();
}

template <class R, int SC> int resident_sc(bool adj)
{
    return adj ? resident_blocks<R, SC, true>() : resident_blocks<R, SC, false>();
}

template <class R> int resident_r(int scheme, bool adj)
{
    return scheme == 0 ? resident_sc<R, 0>(adj) : scheme == 1 ? resident_sc<R, 1>(adj)
                                                              : resident_sc<R, 2>(adj);
}

template <class R, int SC> hipError_t launch_sc(const BatchLaunch &B, hipStream_t s)
{
    return B.adjoint ? launch_t<R, SC, true>(B, s) : launch_t<R, SC, false>(B, s);
}

template <class R> hipError_t launch_r(const BatchLaunch &B, hipStream_t s)
{
    return B.scheme == 0 ? launch_sc<R, 0>(B, s) : B.scheme == 1 ? launch_sc<R, 1>(B, s)
                                                                 : launch_sc<R, 2>(B, s);
}

} // namespace

// scheme: HESTON_FULL_TRUNCATION (0), HESTON_ABSORPTION (1) or HESTON_QE (2).
int batch_resident_blocks(int precision, int scheme, bool adjoint)
{
    return precision == 0 ? resident_r<double>(scheme, adjoint) : resident_r<float>(scheme, adjoint);
}

hipError_t launch_batch(const BatchLaunch &B, hipStream_t s)
{
    return B.precision == 0 ? launch_r<double>(B, s) : launch_r<float>(B, s);
}

hipError_t launch_batch_reduce(const BatchLaunch &B, double *sums, hipStream_t s)
{
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(B.n_opts), dim3(BLOCK), 0, s, B.opts, sums);
    return hipGetLastError();
}

} // namespace heston
