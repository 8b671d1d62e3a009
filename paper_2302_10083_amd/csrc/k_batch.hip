// Batched prime implicants: many independent functions in one persistent
// launch.
//
// The paper notes that independent executions of one Boolean circuit can be
// bit-sliced side by side (Sec. 4.2, batch bit-slicing).  Here the unit of
// batching is a whole function: each workgroup takes the next function from a
// ticket (largest first) and runs its entire pipeline on its own - low tiles
// from the truth table, the high-digit column pass, the final reduce, the
// bitmap and the ordered list - so workgroups never wait on each other and
// the launch can be captured in a graph.  Functions with up to 16 variables
// take this path (digits 13..16 form one register-resident group).
#include "launch.h"
#include "tile_ops.h"

namespace dqmc {

constexpr int kBatchThreads = 768;
constexpr uint32_t kTileL = 19683;  // words spanned by digits 4..12

// Column pass of a function with 13 <= n <= 16: the digits 13..n (GR of them)
// are merged, then reduced, in registers for state words l + 3^9 * c.  The
// column is processed in three chunks over its top digit: chunk 2 (top digit
// *) is the AND of chunks 0 and 1 on the binary inputs; every chunk is merged
// and reduced over the lower digits; then chunks 0 and 1 are reduced against
// chunk 2 (the order merge-top, merge-lower, reduce-lower, reduce-top).
template <int GR>
__device__ __forceinline__ void batch_column(uint32_t *state, uint32_t l)
{
    constexpr int CC = (int)pow3(GR - 1);  // combinations of the lower digits
    constexpr int BC = 1 << (GR - 1);
    if (l >= kTileL) return;
    uint32_t bin[2 * BC];
    static_for<2 * BC>([&](auto bi) {
        constexpr int b = decltype(bi)::value;
        constexpr int c = [] {
            int cc = 0, p = 1;
            for (int r = 0; r < GR; ++r, p *= 3) cc += ((b >> r) & 1) * p;
            return cc;
        }();
        bin[b] = (state + (uint64_t)kTileL * c)[l];
    });
    auto chunk = [&](uint32_t(&y)[CC], auto ki) {
        constexpr int k = decltype(ki)::value;
        static_for<CC>([&](auto ji) {
            constexpr int j = decltype(ji)::value;
            if constexpr (all_binary(j, GR - 1)) {
                constexpr int b = bin_index(j, GR - 1);
                if constexpr (k < 2) y[j] = bin[b + BC * k];
                else y[j] = bin[b] & bin[b + BC];
            } else {
                y[j] = 0u;
            }
        });
        reg_merge<GR - 1>(y);
        reg_reduce<GR - 1>(y);
    };
    uint32_t y2[CC];
    chunk(y2, std::integral_constant<int, 2>{});
    static_for<CC>([&](auto ji) {
        constexpr int j = decltype(ji)::value;
        (state + (uint64_t)kTileL * (j + 2 * CC))[l] = y2[j];
    });
    static_for<2>([&](auto ki) {
        constexpr int k = decltype(ki)::value;
        uint32_t y[CC];
        chunk(y, ki);
        static_for<CC>([&](auto ji) {
            constexpr int j = decltype(ji)::value;
            (state + (uint64_t)kTileL * (j + k * CC))[l] = y[j] & ~y2[j];
        });
    });
}

// Make this workgroup's state writes visible to its own later reads by other
// threads (through L1/L2) before the next phase starts.
__device__ __forceinline__ void phase_barrier()
{
    __threadfence();
    __syncthreads();
}

__device__ void batch_job(const BatchJob &j, uint32_t *t, uint64_t *sh)
{
    const int n = j.n;
    if (n <= 12) {
        const int lw = n <= 3 ? 0 : n - 3;
        const uint32_t tw = (uint32_t)pow3(lw);
        tile_from_tt(t, j.tt, n, lw, tw, 0);
        lds_all_digits<true>(t, tw, lw);
        for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) t[w] = inword_reduce(t[w]);
        __syncthreads();
        lds_all_digits<false>(t, tw, lw);
        for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) j.state[w] = t[w];
        const uint64_t total = tile_list(t, tw, n, 0, j.list, j.cap, 0, sh);
        if (threadIdx.x == 0) *j.count = total;
        return;
    }
    const int H = n - 12;
    const uint32_t tw = kTileL;
    // 1. tiles with binary digits 13..n: load and merge digits 1..12
    for (uint64_t bh = 0; bh < (1ull << H); ++bh) {
        tile_from_tt(t, j.tt, n, 9, tw, bh);
        lds_all_digits<true>(t, tw, 9);
        uint64_t tile = 0;
        for (int q = 0; q < H; ++q)
            if ((bh >> q) & 1) tile += pow3(q);
        uint32_t *dst = j.state + tile * tw;
        for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) dst[w] = t[w];
        __syncthreads();
    }
    phase_barrier();
    // 2. digits 13..n: merge, then reduce
    for (uint32_t l0 = 0; l0 < kTileL; l0 += blockDim.x) {
        const uint32_t l = l0 + threadIdx.x;
        switch (H) {
        case 1: batch_column<1>(j.state, l); break;
        case 2: batch_column<2>(j.state, l); break;
        case 3: batch_column<3>(j.state, l); break;
        default: batch_column<4>(j.state, l); break;
        }
    }
    phase_barrier();
    // 3. every tile: reduce digits 1..12, write the primes, list them in order
    uint64_t run = 0;
    const uint64_t ntiles = pow3(H);
    for (uint64_t tile = 0; tile < ntiles; ++tile) {
        uint32_t *src = j.state + tile * tw;
        load_tile<true, kBatchThreads>(t, src, tw);
        __syncthreads();
        lds_all_digits<false>(t, tw, 9);
        store_tile<kBatchThreads>(src, t, tw);
        run += tile_list(t, tw, n, tile * tw, j.list, j.cap, run, sh);
        __syncthreads();
    }
    if (threadIdx.x == 0) *j.count = run;
}

__global__ __launch_bounds__(kBatchThreads) void batch_kernel(const BatchJob *jobs, const uint32_t *order,
                                                              uint32_t njobs, uint32_t *ticket)
{
    extern __shared__ uint32_t t[];
    __shared__ uint64_t sh[kBatchThreads / 64];
    __shared__ uint32_t item;
    for (;;) {
        if (threadIdx.x == 0) item = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t k = item;
        __syncthreads();
        if (k >= njobs) break;
        batch_job(jobs[order[k]], t, sh);
        __syncthreads();
    }
}

hipError_t batch_setup()
{
    return hipFuncSetAttribute((const void *)batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kTileL * sizeof(uint32_t)));
}

hipError_t launch_batch(const BatchJob *jobs, const uint32_t *order, uint32_t njobs, uint32_t *ticket,
                        uint32_t grid, hipStream_t s)
{
    hipError_t e = launch_fill_u32(ticket, 1, 0, s);
    if (e != hipSuccess) return e;
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(kBatchThreads), kTileL * sizeof(uint32_t), s, jobs, order,
                       njobs, ticket);
    return hipGetLastError();
}

}  // namespace dqmc
