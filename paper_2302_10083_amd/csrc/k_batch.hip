// Batched prime implicants: many independent functions per launch.
//
// The paper notes that independent executions of one Boolean circuit can be
// bit-sliced side by side (Sec. 4.2, batch bit-slicing).  Here the unit of
// batching is a whole function:
//  - functions with up to 12 variables fit one LDS tile: in one persistent
//    launch each workgroup takes the next function from a ticket (largest
//    first) and runs its entire pipeline on its own;
//  - functions with 13..16 variables run tile-parallel: five launches shared
//    by all of them (tiles of the truth table, the column of digits 13..n in
//    registers, the final reduce of every tile with its summary, the per-
//    function scan of the tile counts, the ordered list), each launch a flat
//    range of work items over all the functions.
// No workgroup ever waits on another, and every launch can be captured in a
// graph.
#include "launch.h"
#include "tile_ops.h"

namespace dqmc {

constexpr int kBatchThreads = 768;
constexpr uint32_t kTileL = kTileWords;  // words spanned by digits 1..12

// Column pass of a function with 13 <= n <= 16: the digits 13..n (GR of them)
// are merged, then reduced, in registers for state words l + kTileL * c.  The
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

// A whole function with n <= 12 in one LDS tile.
__device__ void batch_job(const BatchJob &j, uint32_t *t, uint64_t *sh)
{
    const int n = j.n;
    const int lw = n <= 5 ? 0 : n - 5;
    const uint32_t tw = kBlockWords * (uint32_t)pow3(lw);
    tile_from_tt(t, j.tt, n, lw, tw, 0);
    lds_all_digits<true>(t, tw, lw);
    lds_inblock_reduce(t, tw);
    lds_all_digits<false>(t, tw, lw);
    for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) j.state[w] = t[w];
    const uint64_t total = tile_list(t, tw, 0, j.list, j.cap, 0, sh);
    if (threadIdx.x == 0) *j.count = total;
}

// Two workgroups per CU (the LDS tile allows two; registers are held to 80).
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(6)))
void batch_kernel(const BatchJob *jobs, const uint32_t *order, uint32_t njobs, uint32_t *ticket)
{
    extern __shared__ __align__(16) uint32_t t[];
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

// --- tile-parallel path (13 <= n <= 16) -------------------------------------

constexpr uint32_t kColThreads = 256;
constexpr uint32_t kColBlocks = (kTileL + kColThreads - 1) / kColThreads;  // per function

// 1. Tiles whose digits 13..n are binary: from the truth table, merged over
//    digits 1..12, to the state.
__global__ __launch_bounds__(kBatchThreads) void tb_merge_tt_kernel(TileBatch b)
{
    extern __shared__ __align__(16) uint32_t t[];
    const uint32_t item = blockIdx.x;
    const TileJob &j = b.jobs[b.bin_job[item]];
    const uint64_t bh = item - j.first_bin;
    tile_from_tt(t, j.tt, j.n, 7, kTileL, bh);
    lds_all_digits<true>(t, kTileL, 7);
    uint64_t tile = 0;
    for (int q = 0; q < j.n - 12; ++q)
        if ((bh >> q) & 1) tile += pow3(q);
    uint32_t *dst = j.state + tile * kTileL;
    for (uint32_t w = threadIdx.x; w < kTileL; w += blockDim.x) dst[w] = t[w];
}

// 2. Digits 13..n of every column l (merge, then reduce, in registers).
__global__ __launch_bounds__(kColThreads) __attribute__((amdgpu_waves_per_eu(5))) void tb_column_kernel(TileBatch b)
{
    // consecutive column blocks of a function on one XCD, whose L2 then
    // holds the 128-byte lines they share (the 8192-function batch: 6.8 ->
    // 6.0 ms as a replayed graph, 6.81 -> 6.62 ms launched directly)
    const uint32_t bid = (uint32_t)xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t jid = bid / kColBlocks;
    const uint32_t l = (bid % kColBlocks) * kColThreads + threadIdx.x;
    const TileJob &j = b.jobs[jid];
    switch (j.n - 12) {
    case 1: batch_column<1>(j.state, l); break;
    case 2: batch_column<2>(j.state, l); break;
    case 3: batch_column<3>(j.state, l); break;
    default: batch_column<4>(j.state, l); break;
    }
}

// 3. Every tile: reduce digits 1..12 (the prime bitmap) and its summary.
__global__ __launch_bounds__(768) void tb_reduce_kernel(TileBatch b)
{
    extern __shared__ __align__(16) uint32_t t[];
    __shared__ uint32_t red[2 * kMapWords + 1];  // the upper half is unused here
    const uint32_t tile = blockIdx.x;
    const TileJob &j = b.jobs[b.tile_job[tile]];
    reduce_full_tile<false>(t, j.state + (uint64_t)(tile - j.first_tile) * kTileL, b.counts + tile,
                     b.chunkmap + (uint64_t)tile * kMapWords, red);
}

// 4. One wavefront per function: exclusive scan of its tile counts into list
//    offsets, and its prime count.
__global__ __launch_bounds__(256) void tb_scan_kernel(TileBatch b)
{
    const uint32_t jid = blockIdx.x * 4 + threadIdx.x / 64;
    if (jid >= b.njobs) return;
    const TileJob &j = b.jobs[jid];
    const uint32_t nt = (uint32_t)pow3(j.n - 12), lane = lane_id();
    uint64_t run = 0;
    for (uint32_t base = 0; base < nt; base += 64) {
        const uint32_t k = base + lane;
        const uint32_t c = k < nt ? b.counts[j.first_tile + k] : 0u;
        const uint32_t inc = wave_inclusive_scan32(c);
        if (k < nt) b.offs[j.first_tile + k] = run + (inc - c);
        run += __shfl(inc, 63, 64);
    }
    if (lane == 0) *j.count = run;
}

// 5. One wavefront per tile: its primes, in order, into its function's list.
__global__ __launch_bounds__(256) void tb_list_kernel(TileBatch b)
{
    __shared__ uint16_t nzs[4][kTileChunks];
    const uint32_t tile = blockIdx.x * 4 + threadIdx.x / 64;
    if (tile >= b.ntiles) return;
    const TileJob &j = b.jobs[b.tile_job[tile]];
    const uint32_t c = b.counts[tile];
    const uint64_t off = b.offs[tile];
    if (j.list == nullptr || c == 0 || off >= j.cap) return;
    const uint64_t local = tile - j.first_tile;
    list_tile(j.state + local * kTileL, kTileL, local * kTileL, off, b.chunkmap + (uint64_t)tile * kMapWords, j.list,
              j.cap, nzs[threadIdx.x / 64]);
}

hipError_t launch_tile_batch(const TileBatch &b, hipStream_t s)
{
    if (b.njobs == 0) return hipSuccess;
    const size_t lds = kTileL * sizeof(uint32_t);
    hipLaunchKernelGGL(tb_merge_tt_kernel, dim3(b.nbin), dim3(kBatchThreads), lds, s, b);
    hipLaunchKernelGGL(tb_column_kernel, dim3(b.njobs * kColBlocks), dim3(kColThreads), 0, s, b);
    hipLaunchKernelGGL(tb_reduce_kernel, dim3(b.ntiles), dim3(768), lds, s, b);
    hipLaunchKernelGGL(tb_scan_kernel, dim3((b.njobs + 3) / 4), dim3(256), 0, s, b);
    hipLaunchKernelGGL(tb_list_kernel, dim3((b.ntiles + 3) / 4), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t batch_setup()
{
    const int lds = (int)(kTileL * sizeof(uint32_t));
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds)) !=
        hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)tb_merge_tt_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 lds)) != hipSuccess)
        return e;
    return hipFuncSetAttribute((const void *)tb_reduce_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
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
