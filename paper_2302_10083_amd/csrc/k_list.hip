// Output step of Alg. 4: every set bit of the prime bitmap, as increasing
// cube indices.  The bitmap pass leaves a summary per low tile (its number of
// set bits and which 64-word chunks are non-zero); a scan turns the counts
// into list offsets, and the list pass reads only the non-zero chunks.
#include "launch.h"
#include "h5.h"
#include "tile_ops.h"

namespace dqmc {

// Tile counts -> exclusive list offsets, in two launches: per-block sums of
// kScanBlock counts, then every block adds up the sums of the blocks before
// it and scans its own counts.
constexpr int kScanThreads = 1024;
constexpr int kScanPerThread = 8;
constexpr int kScanBlock = kScanThreads * kScanPerThread;

__global__ __launch_bounds__(kScanThreads) void block_sums_kernel(const uint32_t *counts, uint64_t ntiles,
                                                                  uint64_t *sums)
{
    __shared__ uint64_t wsum[kScanThreads / 64];
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanBlock;
    uint64_t c = 0;
    for (int j = 0; j < kScanPerThread; ++j) {
        const uint64_t t = b0 + (uint64_t)j * kScanThreads + threadIdx.x;
        c += t < ntiles ? counts[t] : 0u;
    }
    c = wave_sum(c);
    if (lane_id() == 0) wsum[threadIdx.x / 64] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t all = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) all += wsum[w];
        sums[blockIdx.x] = all;
    }
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const uint32_t *counts, uint64_t ntiles,
                                                                  const uint64_t *sums, uint64_t nblocks,
                                                                  uint64_t *offs, uint64_t *total,
                                                                  const uint64_t *base_in)
{
    __shared__ uint64_t wsum[kScanThreads / 64];
    __shared__ uint64_t base_sh;
    const uint32_t wv = threadIdx.x / 64, lane = lane_id();
    // sum of the blocks before this one (and of all blocks, for the total)
    uint64_t before = 0, all = 0;
    for (uint64_t b = threadIdx.x; b < nblocks; b += kScanThreads) {
        before += b < blockIdx.x ? sums[b] : 0;
        all += sums[b];
    }
    before = wave_sum(before);
    all = wave_sum(all);
    if (lane == 0) wsum[wv] = before;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t x = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) x += wsum[w];
        base_sh = x;
    }
    __syncthreads();
    const uint64_t b0 = base_in != nullptr ? *base_in : 0ull;
    const uint64_t base = b0 + base_sh;
    __syncthreads();
    if (lane == 0) wsum[wv] = all;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0 && total != nullptr) {
        uint64_t x = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) x += wsum[w];
        *total = b0 + x;
    }
    __syncthreads();
    // this thread's kScanPerThread consecutive counts
    const uint64_t t0 = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanPerThread;
    uint32_t v[kScanPerThread];
    uint64_t mine = 0;
    for (int j = 0; j < kScanPerThread; ++j) {
        v[j] = t0 + j < ntiles ? counts[t0 + j] : 0u;
        mine += v[j];
    }
    const uint64_t incl = wave_inclusive_scan(mine);
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint64_t run = base + incl - mine;
    for (uint32_t w = 0; w < wv; ++w) run += wsum[w];
    for (int j = 0; j < kScanPerThread; ++j) {
        if (t0 + j < ntiles) offs[t0 + j] = run;
        run += v[j];
    }
}

hipError_t launch_scan_counts(const uint32_t *counts, uint64_t ntiles, uint64_t *offs, uint64_t *count,
                              uint64_t *sums, hipStream_t s, const uint64_t *base)
{
    const uint64_t nb = (ntiles + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(block_sums_kernel, dim3((uint32_t)nb), dim3(kScanThreads), 0, s, counts, ntiles, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_apply_kernel, dim3((uint32_t)nb), dim3(kScanThreads), 0, s, counts, ntiles, sums, nb,
                       offs, count, base);
    return hipGetLastError();
}

uint64_t scan_scratch_words(uint64_t ntiles) { return (ntiles + kScanBlock - 1) / kScanBlock; }

struct ListArgs {
    const uint32_t *state;
    const uint32_t *counts;
    const uint32_t *chunkmap;
    const uint64_t *offs;
    uint64_t *list;
    uint64_t cap;
    uint64_t ntiles;
    uint64_t rho0;
    uint32_t tw;
    uint32_t ts;
    int n;
};

constexpr int kListThreads = 256;

// One wavefront per tile (grid-stride over tiles).
__global__ __launch_bounds__(kListThreads) void list_kernel(ListArgs a)
{
    constexpr int NW = kListThreads / 64;
    __shared__ uint16_t nzs[NW][kTileChunks];
    __shared__ uint64_t stage[NW][kListStage];
    const uint32_t wv = threadIdx.x / 64;
    const uint64_t nwaves = (uint64_t)gridDim.x * NW;
    for (uint64_t tile = (uint64_t)blockIdx.x * NW + wv; tile < a.ntiles; tile += nwaves) {
        const uint32_t c = a.counts[tile];
        const uint64_t off = a.offs[tile];
        if (c == 0 || off >= a.cap) continue;
        list_tile(a.state + tile * a.ts, a.tw, tile * a.tw, off, a.chunkmap + tile * kMapWords, a.list, a.cap, nzs[wv],
                  stage[wv], a.rho0);
    }
}

hipError_t launch_list(int n, const uint32_t *state, uint32_t tw, uint32_t ts, uint64_t ntiles, const uint32_t *counts,
                       const uint32_t *chunkmap, const uint64_t *offs, uint64_t *list, uint64_t cap, hipStream_t s,
                       uint64_t rho0)
{
    ListArgs a{state, counts, chunkmap, offs, list, cap, ntiles, rho0, tw, ts, n};
    // workgroups of four tile-waves, at most 32768 (grid-stride beyond): at
    // n = 24 the pass took 1.66 ms with 8192, 1.51 ms with 32768 and 1.57 ms
    // with one workgroup per four tiles
    const uint64_t waves = (ntiles + 3) / 4;
    uint64_t g = waves < 32768 ? waves : 32768;
    hipLaunchKernelGGL(list_kernel, dim3((uint32_t)(g == 0 ? 1 : g)), dim3(kListThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace dqmc
