// Low tile kernels: the in-block digits 1..5 and the block digits 6..12 of
// one tile of 3^min(n,12) cubes, processed in LDS.
//
// Alg. 4 loads the support into the state, then applies the Merge transform
// per dimension (top layer over whole blocks, bottom layer inside a block),
// then Reduce, then scans the state for the output list.  Here a tile is the
// unit of on-chip work: digits 1..5 use the shift-and-mask form of the bottom
// layer on a 256-bit block held in eight registers (Sec. 4.2, masks mu_i),
// digits 6..12 use the top-layer triple indexing of Sec. 4.2 (eq. indexes) on
// LDS words, three digits at a time in registers.  Digits above 12 are
// handled by the column passes (k_col.hip).
#include "launch.h"
#include "tile_ops.h"

namespace dqmc {

// Summary of an LDS tile for the list pass: its number of set bits and the
// bitmap of its non-zero 64-word chunks.
__device__ __forceinline__ void tile_summary(const uint32_t *t, const LowArgs &a, uint64_t tile, uint32_t *red)
{
    const uint32_t nw = blockDim.x / 64, wv = threadIdx.x / 64, lane = lane_id();
    if (threadIdx.x < kMapWords + 1) red[threadIdx.x] = 0;
    __syncthreads();
    uint32_t c = 0;
    for (uint32_t k = wv; k < (uint32_t)kTileChunks; k += nw) {
        const uint32_t w = k * kChunkWords + lane;
        const uint32_t v = w < a.tw ? t[w] : 0u;
        c += __popc(v);
        if (__ballot(v != 0u) != 0 && lane == 0) atomicOr(&red[1 + k / 32], 1u << (k % 32));
    }
    c = wave_sum32(c);
    if (lane == 0) atomicAdd(&red[0], c);
    __syncthreads();
    if (threadIdx.x == 0) a.counts[tile] = red[0];
    if (threadIdx.x < kMapWords) a.chunkmap[tile * kMapWords + threadIdx.x] = red[1 + threadIdx.x];
}

template <int MODE>
__host__ __device__ constexpr int low_threads()
{
    // the tile passes over HBM-resident states use one run of three blocks
    // per thread on the way in (729 runs in a full tile) and one 27-word
    // column per thread in the LDS rounds (648 columns)
    return (MODE == kLowReduceCount || MODE == kLowCount) ? 768 : kLowThreads;
}

// Two workgroups per CU (the LDS tile allows two): registers held to 80.
template <int MODE>
__global__ __launch_bounds__(low_threads<MODE>()) __attribute__((amdgpu_waves_per_eu(6))) void low_kernel(LowArgs a)
{
    constexpr int THREADS = low_threads<MODE>();
    extern __shared__ __align__(16) uint32_t dyn[];
    __shared__ uint64_t sh[THREADS / 64];
    uint32_t *t = dyn;

    if constexpr (MODE == kLowMergeTT || MODE == kLowPrimesTT) {
        // tile with binary digits 13..n given by the bits of blockIdx.x
        const uint64_t bh = blockIdx.x;
        tile_from_tt(t, a.tt, a.n, a.lw, a.tw, bh, a.flip);
        lds_all_digits<true>(t, a.tw, a.lw);
        uint64_t tile = 0;
        for (int j = 0, nh = a.n - 12; j < nh; ++j)
            if ((bh >> j) & 1) tile += pow3(j);
        if constexpr (MODE == kLowMergeTT) {
            // the whole slot: the tile and its zero padding
            uint32_t *dst = a.state + tile * a.ts;
            for (uint32_t w = threadIdx.x; w < a.ts; w += blockDim.x) dst[w] = w < a.tw ? t[w] : 0u;
        } else {
            lds_inblock_reduce(t, a.tw);
            lds_all_digits<false>(t, a.tw, a.lw);
            // the state (a.ts >= a.tw words: a tile slot with its padding
            // when the state is a third of a split state)
            for (uint32_t w = threadIdx.x; w < a.ts; w += blockDim.x) a.state[w] = w < a.tw ? t[w] : 0u;
            const uint64_t total = tile_list(t, a.tw, 0, a.list, a.cap, 0, sh);
            if (threadIdx.x == 0 && a.count != nullptr) *a.count = total;
        }
    } else {
        __shared__ uint32_t red[kRedWords];
        // Consecutive tiles on one XCD, as in the column passes (n = 24, the
        // final reduce: 16.6 -> 14.6 ms against round-robin tiles).  Every
        // tile here is a full read of equal cost; the list pass and the batch
        // kernels, whose work per tile varies, keep round-robin tiles.
        const uint64_t tile = xcd_remap(blockIdx.x, gridDim.x);
        const uint32_t *src = a.state + tile * a.ts;
        if constexpr (MODE == kLowReduceCount) {
            // always a full tile here (n > 12)
            if (a.tile_flags != nullptr) {
                // one tile per workgroup (more, with the flags of all read
                // first, was slower: a tile's run loads then wait for the
                // previous tile's stores, vmcnt retiring in order)
                const uint32_t *fw = a.tile_flags + tile * kMapWords;
                // the flag words of this wavefront's 64 runs (chunks 24 w .. 24 w + 23)
                const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
                const uint32_t k0 = 24 * wv / 32, k1 = (24 * wv + 23) / 32;
                const uint32_t f0 = k0 < (uint32_t)kMapWords ? fw[k0] : 0u;
                const uint32_t f1 = k1 < (uint32_t)kMapWords ? fw[k1] : 0u;
                reduce_full_tile<true>(t, a.state + tile * a.ts, a.counts + tile, a.chunkmap + tile * kMapWords, red,
                                       fw, f0, f1);
                return;
            }
            reduce_full_tile<true>(t, a.state + tile * a.ts, a.counts + tile, a.chunkmap + tile * kMapWords, red);
            return;
        } else {
            load_tile<THREADS>(t, src, a.tw);
            __syncthreads();
        }
        tile_summary(t, a, tile, red);
    }
}

static size_t low_lds_bytes(int mode, uint32_t tw)
{
    // the final reduce holds the tile with padded rows, then the list of its
    // non-zero blocks
    return mode == kLowReduceCount ? (size_t)kReduceTileBytes + kBlockListBytes : (size_t)tw * 4;
}

hipError_t low_setup()
{
    const int bytes = (int)low_lds_bytes(kLowMergeTT, kTileWords);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)low_kernel<kLowMergeTT>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)low_kernel<kLowPrimesTT>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)low_kernel<kLowReduceCount>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)low_lds_bytes(kLowReduceCount, kTileWords))) != hipSuccess)
        return e;
    return hipFuncSetAttribute((const void *)low_kernel<kLowCount>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_low(int mode, const LowArgs &a, uint64_t nblocks, hipStream_t s)
{
    const size_t lds = low_lds_bytes(mode, a.tw);
    const dim3 grid((uint32_t)nblocks);
    switch (mode) {
    case kLowMergeTT:
        hipLaunchKernelGGL(low_kernel<kLowMergeTT>, grid, dim3(low_threads<kLowMergeTT>()), lds, s, a);
        break;
    case kLowPrimesTT:
        hipLaunchKernelGGL(low_kernel<kLowPrimesTT>, grid, dim3(low_threads<kLowPrimesTT>()), lds, s, a);
        break;
    case kLowReduceCount:
        hipLaunchKernelGGL(low_kernel<kLowReduceCount>, grid, dim3(low_threads<kLowReduceCount>()), lds, s, a);
        break;
    case kLowCount:
        hipLaunchKernelGGL(low_kernel<kLowCount>, grid, dim3(low_threads<kLowCount>()), lds, s, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace dqmc
