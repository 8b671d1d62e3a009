// Batched prime implicants: many independent functions from a
// device-resident job array.
//
// The paper notes that independent executions of one Boolean circuit can be
// bit-sliced side by side (Sec. 4.2, batch bit-slicing).  Here the unit of
// batching is a whole function, and the job table lives on the device, so the
// host knows neither the jobs' sizes nor their number of tiles:
//  - a planner (one workgroup) checks every job, writes its status, sorts the
//    valid jobs by n (largest first, stable) and lays out the work items of
//    every pass, bin by bin (all jobs with the same n in a row);
//  - five launches then work through the items, one item (or one per
//    wavefront) per workgroup; their grids are exact when the host knows the
//    jobs' sizes (a plan, the server) and bounds otherwise:
//      1. the whole-function items (n <= 12: the whole pipeline in one LDS
//         tile, largest first) and the truth-table tiles of the jobs with
//         13 <= n <= 16 (the tiles with binary digits 13..n, merged over
//         digits 1..12);
//      2. the columns of digits 13..n (merge, then reduce, in registers);
//      3. every tile's reduce of digits 1..12 with its summary;
//      4. per job, the scan of its tile counts and its prime count;
//      5. the ordered list, one wavefront per tile.
// The items of one launch are independent, and the launch boundaries order
// the passes of a job: no workgroup waits on another, nothing is allocated,
// and nothing waits on the host, so the launches can be captured in a graph.
#include "dqmc.h"
#include "launch.h"
#include "tile_ops.h"

namespace dqmc {

constexpr uint32_t kTileL = kTileWords;  // words spanned by digits 1..12
constexpr uint32_t kSlot = kTileStride;  // words between tiles in a state (the tile and its padding)
constexpr uint32_t kColThreads = 256;
constexpr uint32_t kColBlocks = (kSlot + kColThreads - 1) / kColThreads;  // column items per job

// Work-item segments (one per pass).
enum BatchSeg : uint32_t {
    kSegWhole = 0,   // n <= 12: the whole function in one tile
    kSegMerge = 1,   // tiles with binary digits 13..n: truth table -> merged digits 1..12
    kSegColumn = 2,  // kColThreads columns: merge and reduce digits 13..n
    kSegReduce = 3,  // tiles: reduce digits 1..12, tile summary
    kSegScan = 4,    // per job: scan of the tile counts, the prime count
    kSegList = 5,    // tiles: the ordered list
    kSegs = 6,
};

// Header words (written by the planner, read with scalar loads by the launches).
constexpr int kHSegSize = 8;                 // [kSegs] items per segment
constexpr int kHHist = 16;                   // [17] valid jobs per n
constexpr int kHBinStart = kHHist + 17;      // [17] first position of n in `order`
constexpr int kHTileBase = kHBinStart + 17;  // [17] first tile of the jobs of n
constexpr int kHSegBin = kHTileBase + 17;    // [kSegs][17] first item of n in a segment
constexpr int kHMismatch = kHSegBin + kSegs * 17;  // 1: the jobs' sizes differ from the plan's
constexpr int kHWords = kHMismatch + 1;
static_assert(kHWords <= kBatchHdrWords, "batch header");

__host__ __device__ constexpr uint32_t pow3u(int k) { return (uint32_t)pow3(k); }

// Work items of one job with n variables in segment `seg`.
__host__ __device__ inline uint32_t seg_items(int n, uint32_t seg)
{
    if (n <= kBatchWholeMaxN) return seg == kSegWhole ? 1u : 0u;
    const int h = n - kBatchWholeMaxN;
    switch (seg) {
    case kSegMerge: return 1u << h;
    case kSegColumn: return kColBlocks;
    case kSegReduce:
    case kSegList: return pow3u(h);
    case kSegScan: return 1u;
    default: return 0u;
    }
}

__device__ inline bool job_valid(const dqmc_job &j)
{
    const uintptr_t tt = (uintptr_t)j.tt, st = (uintptr_t)j.state, ct = (uintptr_t)j.count, li = (uintptr_t)j.list;
    return j.n >= 0 && j.n <= kBatchMaxN && tt != 0 && st != 0 && ct != 0 && tt % 4 == 0 && st % 16 == 0 &&
           ct % 8 == 0 && li % 8 == 0;
}

// ---------------------------------------------------------------------------
// Planner: one workgroup of 1024 threads.

constexpr int kPlanThreads = 1024;
constexpr int kPlanWaves = kPlanThreads / 64;

__global__ __launch_bounds__(kPlanThreads) void batch_plan_kernel(dqmc_job *jobs, uint32_t njobs, BatchScratch s,
                                                                  BatchExpect ex)
{
    __shared__ uint32_t hist[17], running[17], binstart[17];
    __shared__ uint32_t wc[kPlanWaves][17];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wv = tid / 64;
    if (tid < 17) {
        hist[tid] = 0;
        running[tid] = 0;
    }
    __syncthreads();
    // 1. check every job; histogram of the valid ones by n
    for (uint32_t j = tid; j < njobs; j += kPlanThreads) {
        const bool ok = job_valid(jobs[j]);
        jobs[j].status = ok ? DQMC_OK : DQMC_EINVAL;
        if (ok) atomicAdd(&hist[jobs[j].n], 1u);
    }
    __syncthreads();
    // 2. bins by n descending, tile bases, the items of every segment.  A
    //    plan's launches are sized for the jobs it was made for: if their
    //    sizes differ now, nothing runs and every job is rejected.
    __shared__ uint32_t mismatch;
    if (tid == 0) {
        uint32_t *h = s.hdr;
        uint32_t mis = 0;
        for (int n = 0; n <= kBatchMaxN && ex.exact; ++n) mis |= hist[n] != ex.hist[n] ? 1u : 0u;
        mismatch = mis;
        h[kHMismatch] = mis;
        if (mis)
            for (int n = 0; n <= kBatchMaxN; ++n) hist[n] = 0;
        uint32_t pos = 0, tiles = 0;
        for (int n = kBatchMaxN; n >= 0; --n) {
            binstart[n] = pos;
            h[kHHist + n] = hist[n];
            h[kHBinStart + n] = pos;
            h[kHTileBase + n] = tiles;
            pos += hist[n];
            if (n > kBatchWholeMaxN) tiles += hist[n] * pow3u(n - kBatchWholeMaxN);
        }
        for (uint32_t seg = 0; seg < kSegs; ++seg) {
            uint32_t in = 0;
            for (int n = kBatchMaxN; n >= 0; --n) {
                h[kHSegBin + seg * 17 + n] = in;
                in += hist[n] * seg_items(n, seg);
            }
            h[kHSegSize + seg] = in;
        }
    }
    __syncthreads();
    if (mismatch) {
        for (uint32_t j = tid; j < njobs; j += kPlanThreads) jobs[j].status = DQMC_EINVAL;
        return;
    }
    // 3. stable rank of every valid job within its n: the order
    for (uint32_t c0 = 0; c0 < njobs; c0 += kPlanThreads) {
        const uint32_t j = c0 + tid;
        int v = 17;  // no bin
        if (j < njobs && jobs[j].status == DQMC_OK) v = jobs[j].n;
        uint32_t rank = 0;
        for (int u = 0; u <= kBatchMaxN; ++u) {
            const uint64_t m = __ballot(v == u);
            if (v == u) rank = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) wc[wv][u] = (uint32_t)__popcll(m);
        }
        __syncthreads();
        if (v <= kBatchMaxN) {
            uint32_t before = running[v];
            for (uint32_t w = 0; w < wv; ++w) before += wc[w][v];
            s.order[binstart[v] + before + rank] = j;
        }
        __syncthreads();
        if (tid <= (uint32_t)kBatchMaxN) {
            uint32_t add = 0;
            for (int w = 0; w < kPlanWaves; ++w) add += wc[w][tid];
            running[tid] += add;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Work items.

struct Item {
    uint32_t n;    // variables of the job
    uint32_t pos;  // position of the job in `order`
    uint32_t idx;  // index of the item within the job's items of this segment
};

// Item `rel` of segment `seg`.  The result is the same for every thread of a
// workgroup (or of a wavefront, for the per-wave items) and is kept in
// scalar registers.
__device__ inline Item decode(const uint32_t *hl, uint32_t seg, uint32_t rel)
{
    Item it{0, 0, 0};
    for (int m = kBatchMaxN; m >= 0; --m) {
        const uint32_t b0 = hl[kHSegBin + seg * 17 + m], per = seg_items(m, seg);
        if (per != 0 && rel >= b0 && rel - b0 < hl[kHHist + m] * per) {
            it.n = (uint32_t)m;
            it.idx = (rel - b0) % per;
            it.pos = hl[kHBinStart + m] + (rel - b0) / per;
        }
    }
    it.n = __builtin_amdgcn_readfirstlane(it.n);
    it.idx = __builtin_amdgcn_readfirstlane(it.idx);
    it.pos = __builtin_amdgcn_readfirstlane(it.pos);
    return it;
}

// First tile (in the batch's summary arrays) of the item's job.
__device__ inline uint32_t first_tile(const uint32_t *hl, const Item &it)
{
    return hl[kHTileBase + it.n] + (it.pos - hl[kHBinStart + it.n]) * pow3u((int)it.n - kBatchWholeMaxN);
}

// A whole function with n <= 12 in one LDS tile.
__device__ void whole_job(const dqmc_job &j, uint32_t *t, uint64_t *sh)
{
    const int n = j.n;
    const int lw = n <= 5 ? 0 : n - 5;
    const uint32_t tw = kBlockWords * pow3u(lw);
    tile_from_tt(t, j.tt, n, lw, tw, 0);
    lds_all_digits<true>(t, tw, lw);
    lds_inblock_reduce(t, tw);
    lds_all_digits<false>(t, tw, lw);
    for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) j.state[w] = t[w];
    const uint64_t cap = j.list != nullptr ? j.list_cap : 0;
    const uint64_t total = tile_list(t, tw, 0, j.list, cap, 0, sh);
    if (threadIdx.x == 0) *j.count = total;
}

// The tile with binary digits 13..n of value idx: from the truth table,
// merged over digits 1..12, to its place in the state.
__device__ void merge_tile(const dqmc_job &j, uint32_t idx, uint32_t *t)
{
    const int h = j.n - kBatchWholeMaxN;
    tile_from_tt(t, j.tt, j.n, 7, kTileL, idx);
    lds_all_digits<true>(t, kTileL, 7);
    uint32_t tile = 0;
    for (int q = 0; q < h; ++q)
        if ((idx >> q) & 1u) tile += pow3u(q);
    uint32_t *dst = j.state + (uint64_t)tile * kSlot;
    for (uint32_t w = threadIdx.x; w < kSlot; w += blockDim.x) dst[w] = w < kTileL ? t[w] : 0u;
}

// Column pass of a function with 13 <= n <= 16: the digits 13..n (GR of them)
// are merged, then reduced, in registers for state words l + kSlot * c (l runs
// over the whole slot: the padding words are 0 in every binary tile and stay
// 0).  The column is processed in three chunks over its top digit: chunk 2
// (top digit *) is the AND of chunks 0 and 1 on the binary inputs; every chunk
// is merged and reduced over the lower digits; then chunks 0 and 1 are reduced
// against chunk 2 (the order merge-top, merge-lower, reduce-lower, reduce-top).
template <int GR>
__device__ __forceinline__ void batch_column(uint32_t *state, uint32_t l)
{
    constexpr int CC = (int)pow3(GR - 1);  // combinations of the lower digits
    constexpr int BC = 1 << (GR - 1);
    if (l >= kSlot) return;
    uint32_t bin[2 * BC];
    static_for<2 * BC>([&](auto bi) {
        constexpr int b = decltype(bi)::value;
        constexpr int c = [] {
            int cc = 0, p = 1;
            for (int r = 0; r < GR; ++r, p *= 3) cc += ((b >> r) & 1) * p;
            return cc;
        }();
        bin[b] = (state + (uint64_t)kSlot * c)[l];
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
        (state + (uint64_t)kSlot * (j + 2 * CC))[l] = y2[j];
    });
    static_for<2>([&](auto ki) {
        constexpr int k = decltype(ki)::value;
        uint32_t y[CC];
        chunk(y, ki);
        static_for<CC>([&](auto ji) {
            constexpr int j = decltype(ji)::value;
            (state + (uint64_t)kSlot * (j + k * CC))[l] = y[j] & ~y2[j];
        });
    });
}

// ---------------------------------------------------------------------------
// The five launches.

// 1. Whole functions and truth-table tiles, one item per workgroup (grid: the
//    items, or a bound on them; workgroups past the items exit).
//    `whole_first`: the whole-function items (largest first) come before the
//    tiles, else after them.  Two workgroups per CU (two LDS tiles fit);
//    registers held to 80.
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(6)))
void batch_tt_kernel(const dqmc_job *jobs, BatchScratch s, int whole_first)
{
    const uint32_t *__restrict__ hl = s.hdr;
    const uint32_t segA = whole_first ? kSegWhole : kSegMerge, segB = whole_first ? kSegMerge : kSegWhole;
    const uint32_t na = hl[kHSegSize + segA], nall = na + hl[kHSegSize + segB];
    const uint32_t tk = blockIdx.x;
    if (tk >= nall) return;
    extern __shared__ __align__(16) uint32_t t[];
    __shared__ uint64_t sh[kBatchThreads / 64];
    const uint32_t seg = tk < na ? segA : segB;
    const Item it = decode(hl, seg, tk < na ? tk : tk - na);
    const dqmc_job j = jobs[s.order[it.pos]];
    if (seg == kSegWhole) whole_job(j, t, sh);
    else merge_tile(j, it.idx, t);
}

// 2. Columns: kColThreads consecutive columns l of one job per workgroup.
//    The jobs with 13..16 variables hold the first T positions of the order
//    (largest n first).  Job q goes to XCD q mod 8 (workgroups are dealt to
//    the XCDs round-robin), so that the kColBlocks column blocks of a job
//    share one L2 (neighbouring blocks share 128-byte lines) while every XCD
//    gets an even mix of sizes.  The grid is 8 * kColBlocks * ceil(T / 8)
//    workgroups (or a bound on it); those past the jobs exit.
__global__ __launch_bounds__(kColThreads) __attribute__((amdgpu_waves_per_eu(4)))
void batch_col_kernel(const dqmc_job *jobs, BatchScratch s)
{
    const uint32_t T = s.hdr[kHSegSize + kSegColumn] / kColBlocks;
    const uint32_t x = blockIdx.x % 8, slot = blockIdx.x / 8;
    const uint32_t q = x + 8 * (slot / kColBlocks), blk = slot % kColBlocks;
    if (q >= T) return;
    const dqmc_job j = jobs[s.order[q]];
    const uint32_t l = blk * kColThreads + threadIdx.x;
    switch (j.n - kBatchWholeMaxN) {
    case 1: batch_column<1>(j.state, l); break;
    case 2: batch_column<2>(j.state, l); break;
    case 3: batch_column<3>(j.state, l); break;
    default: batch_column<4>(j.state, l); break;
    }
}

// 3. Every tile: reduce digits 1..12 (the prime bitmap) and its summary, one
//    tile per workgroup (grid: a bound on the tiles).
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(6)))
void batch_reduce_kernel(const dqmc_job *jobs, BatchScratch s)
{
    const uint32_t *__restrict__ hl = s.hdr;
    const uint32_t nitems = hl[kHSegSize + kSegReduce];
    if (blockIdx.x >= nitems) return;
    extern __shared__ __align__(16) uint32_t t[];
    __shared__ uint32_t red[kRedWords];
    const Item it = decode(hl, kSegReduce, blockIdx.x);
    const uint32_t tile = first_tile(hl, it) + it.idx;
    reduce_full_tile(t, jobs[s.order[it.pos]].state + (uint64_t)it.idx * kSlot, s.counts + tile,
                            s.chunkmap + (uint64_t)tile * kMapWords, red);
}

// 4. One wavefront per job: exclusive scan of its tile counts into list
//    offsets, and its prime count.
__global__ __launch_bounds__(256) void batch_scan_kernel(const dqmc_job *jobs, BatchScratch s)
{
    const uint32_t *__restrict__ hl = s.hdr;
    const uint32_t nitems = hl[kHSegSize + kSegScan], lane = lane_id();
    for (uint32_t i = blockIdx.x * 4 + threadIdx.x / 64; i < nitems; i += gridDim.x * 4) {
        const Item it = decode(hl, kSegScan, i);
        const uint32_t t0 = first_tile(hl, it), nt = pow3u((int)it.n - kBatchWholeMaxN);
        uint64_t run = 0;
        for (uint32_t base = 0; base < nt; base += 64) {
            const uint32_t k = base + lane;
            const uint32_t c = k < nt ? s.counts[t0 + k] : 0u;
            const uint32_t inc = wave_inclusive_scan32(c);
            if (k < nt) s.offs[t0 + k] = run + (inc - c);
            run += __shfl(inc, 63, 64);
        }
        if (lane == 0) *jobs[s.order[it.pos]].count = run;
    }
}

// 5. One wavefront per tile: its primes, in order, into its job's list (grid:
//    a bound on the tiles, four per workgroup).
__global__ __launch_bounds__(256) void batch_list_kernel(const dqmc_job *jobs, BatchScratch s)
{
    const uint32_t *__restrict__ hl = s.hdr;
    const uint32_t nitems = hl[kHSegSize + kSegList];
    if (blockIdx.x * 4 >= nitems) return;
    __shared__ uint16_t nzs[4][kTileChunks];
    __shared__ uint64_t stage[4][kListStage];
    const uint32_t wv = threadIdx.x / 64, i = blockIdx.x * 4 + wv;
    if (i >= nitems) return;
    const Item it = decode(hl, kSegList, i);
    const dqmc_job j = jobs[s.order[it.pos]];
    const uint32_t tile = first_tile(hl, it) + it.idx;
    const uint32_t c = s.counts[tile];
    const uint64_t off = s.offs[tile];
    const uint64_t cap = j.list != nullptr ? j.list_cap : 0;
    if (c == 0 || off >= cap) return;
    list_tile(j.state + (uint64_t)it.idx * kSlot, kTileL, (uint64_t)it.idx * kTileL, off,
              s.chunkmap + (uint64_t)tile * kMapWords, j.list, cap, nzs[wv], stage[wv]);
}

uint64_t batch_scratch_bytes(uint32_t cap)
{
    auto a = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
    const uint64_t tiles = 81ull * cap;
    return a(4ull * kBatchHdrWords) + a(4ull * cap) + a(4ull * tiles) + a(4ull * kMapWords * tiles) + a(8ull * tiles);
}

BatchScratch batch_scratch_at(void *base, uint32_t cap)
{
    auto a = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
    const uint64_t tiles = 81ull * cap;
    uint8_t *p = (uint8_t *)base;
    BatchScratch s{};
    s.hdr = (uint32_t *)p;
    p += a(4ull * kBatchHdrWords);
    s.order = (uint32_t *)p;
    p += a(4ull * cap);
    s.counts = (uint32_t *)p;
    p += a(4ull * tiles);
    s.chunkmap = (uint32_t *)p;
    p += a(4ull * kMapWords * tiles);
    s.offs = (uint64_t *)p;
    s.cap = cap;
    return s;
}

// Dynamic LDS that caps the column launch at `cap` workgroups per CU (0: no
// cap beyond its registers, which allow four).
static size_t col_cap_pad(int cap)
{
    return cap <= 0 ? 0 : (size_t)(kLdsPerCu / (uint32_t)cap - 1024);
}

static int g_ncu = 256;

hipError_t batch_setup()
{
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        g_ncu = ncu;
    const int lds = (int)(kTileL * sizeof(uint32_t));
    hipError_t e = hipFuncSetAttribute((const void *)batch_tt_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)batch_col_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)col_cap_pad(1));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)batch_reduce_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kReduceTileBytes + kBlockListBytes));
}

hipError_t launch_batch(void *jobs, uint32_t njobs, const BatchScratch &s, int col_cap, int mode, hipStream_t st,
                        const BatchExpect *ex)
{
    if (njobs > s.cap || mode < 0 || mode >= kBatchModes || col_cap < 0 || col_cap > kBatchMaxColCap)
        return hipErrorInvalidValue;
    dqmc_job *j = (dqmc_job *)jobs;
    const size_t lds = kTileL * sizeof(uint32_t);
    const uint32_t ncu = (uint32_t)g_ncu;
    BatchExpect e{};
    // the grids of the one-item-per-workgroup launches: exact when the jobs'
    // sizes are known, else bounds (at most 3^4 tiles and kColBlocks column
    // blocks per job; the workgroups past the items exit at once)
    uint64_t first = 17ull * njobs, tiled = njobs, ntiles = 81ull * njobs;
    if (ex != nullptr && ex->exact) {
        e = *ex;
        first = tiled = ntiles = 0;
        for (int n = 0; n <= kBatchMaxN; ++n) {
            first += (uint64_t)e.hist[n] * (seg_items(n, kSegWhole) + seg_items(n, kSegMerge));
            if (n > kBatchWholeMaxN) tiled += e.hist[n];
            ntiles += (uint64_t)e.hist[n] * seg_items(n, kSegReduce);
        }
    }
    const uint64_t ncol = 8ull * kColBlocks * ((tiled + 7) / 8);
    auto g = [](uint64_t x) { return dim3((uint32_t)(x > 0 ? x : 1)); };
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanThreads), 0, st, j, njobs, s, e);
    hipLaunchKernelGGL(batch_tt_kernel, g(first), dim3(kBatchThreads), lds, st, j, s, mode == 0 ? 1 : 0);
    hipLaunchKernelGGL(batch_col_kernel, g(ncol), dim3(kColThreads), col_cap_pad(col_cap), st, j, s);
    hipLaunchKernelGGL(batch_reduce_kernel, g(ntiles), dim3(kBatchThreads), kReduceTileBytes + kBlockListBytes, st, j, s);
    hipLaunchKernelGGL(batch_scan_kernel, dim3(ncu), dim3(256), 0, st, j, s);
    hipLaunchKernelGGL(batch_list_kernel, g((ntiles + 3) / 4), dim3(256), 0, st, j, s);
    return hipGetLastError();
}

hipError_t launch_batch_plan(void *jobs, uint32_t njobs, const BatchScratch &s, hipStream_t st)
{
    if (njobs > s.cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanThreads), 0, st, (dqmc_job *)jobs, njobs, s,
                       BatchExpect{});
    return hipGetLastError();
}

void batch_expect_from_header(const uint32_t *hdr_host, BatchExpect *ex)
{
    ex->exact = 1;
    for (int n = 0; n <= kBatchMaxN; ++n) ex->hist[n] = hdr_host[kHHist + n];
}

uint32_t batch_header_words() { return (uint32_t)kHWords; }

}  // namespace dqmc
