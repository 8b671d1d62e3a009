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
    // per thread on the way in (729 runs in a full tile)
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
                reduce_full_tile(t, a.state + tile * a.ts, a.counts + tile, a.chunkmap + tile * kMapWords, red,
                                       fw, f0, f1);
                return;
            }
            reduce_full_tile(t, a.state + tile * a.ts, a.counts + tile, a.chunkmap + tile * kMapWords, red);
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
    // the final reduce holds the tile, then the list of its
    // non-zero blocks
    return mode == kLowReduceCount ? (size_t)kReduceTileBytes + kBlockListBytes : (size_t)tw * 4;
}

// The tiles the compact kernel deferred, as the full-tile kernel reduces
// them (a kernel of its own: the loop would cost the full-tile kernel its
// registers).  Grid-stride over the list; the count is uniform, so every
// wavefront leaves the loop together.
__global__ __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(6))) void low_deferred_kernel(LowArgs a)
{
    extern __shared__ __align__(16) uint32_t dyn[];
    __shared__ uint32_t red[kRedWords];
    const uint32_t nd = a.deferred[0];
    for (uint32_t i = blockIdx.x; i < nd; i += gridDim.x) {
        if (i != blockIdx.x) __syncthreads();  // the previous tile's LDS is free
        const uint64_t tl = a.deferred[1 + i];
        const uint32_t *fw = a.tile_flags + tl * kMapWords;
        const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
        const uint32_t k0 = 24 * wv / 32, k1 = (24 * wv + 23) / 32;
        const uint32_t f0 = k0 < (uint32_t)kMapWords ? fw[k0] : 0u;
        const uint32_t f1 = k1 < (uint32_t)kMapWords ? fw[k1] : 0u;
        reduce_full_tile(dyn, a.state + tl * a.ts, a.counts + tl, a.chunkmap + tl * kMapWords, red, fw, f0, f1);
    }
}

// Final reduce of a full tile with chunk flags, holding in LDS only the blocks
// that are non-zero after digit 6 (a mostly zero tile needs a fraction of the
// 70 KB): kCompactSlots slots of one block, a uint16 slot per block of the
// tile (kNoSlot: the block is zero) and a uint16 block per slot, 39.2 KB, so
// that four workgroups of 512 threads share a CU (the full tile allows two;
// the pass waits on its loads and stores, and one workgroup per CU took 1.7x
// as long as two).  Thread q loads runs q and q + 512.  The arithmetic is the
// full-tile kernel's: digit 6 on the way in, then digits 1..5 and 7..12 in one
// step on the listed blocks, and the stores of the chunks non-zero as loaded.
// A tile with more non-zero blocks than slots is left untouched and appended
// to a.deferred for the full-tile kernel.
constexpr int kCompactThreads = 512;
constexpr uint32_t kCompactWaves = kCompactThreads / 64;
static_assert(2 * kCompactThreads >= (int)kTileTriples, "two runs per thread at most");
constexpr uint32_t kCompactSlots = 1024;
constexpr int kSlotsPerThread = (int)((kCompactSlots + kCompactThreads - 1) / kCompactThreads);  // 2
constexpr uint32_t kNoSlot = 0xFFFFu;
constexpr uint32_t kSlotMapBytes = (kTileBlocks * 2 + 15) / 16 * 16;  // 4384
constexpr uint32_t kCompactLds = kSlotMapBytes + kCompactSlots * 2 + kCompactSlots * 32;

__global__ __launch_bounds__(kCompactThreads) __attribute__((amdgpu_waves_per_eu(8))) void low_compact_kernel(LowArgs a)
{
    extern __shared__ __align__(16) uint32_t dyn[];
    uint16_t *slot_of = reinterpret_cast<uint16_t *>(dyn);
    uint16_t *block_of = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(dyn) + kSlotMapBytes);
    uint4 *slots = reinterpret_cast<uint4 *>(reinterpret_cast<char *>(dyn) + kSlotMapBytes + kCompactSlots * 2);
    __shared__ uint32_t red[kRedWords];
    uint32_t *innz = red + kMapWords + 1;
    uint32_t *nlist = red + kRedWords - 1;

    const uint64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    uint32_t *src = a.state + tile * a.ts;
    const uint32_t *fw = a.tile_flags + tile * kMapWords;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = lane_id();

    // run q + T h (T threads) if it touches a flagged chunk (wavefront w's
    // runs cover the 24 chunks from 24 (T h / 64 + w)); run q + T is loaded
    // once run q is in LDS, which keeps one run in registers
    TileRun r;
    auto fetch = [&](uint32_t h) {
        const uint32_t q = threadIdx.x + h * kCompactThreads;
        const uint32_t cw0 = 24 * (kCompactWaves * h + wv), k0 = cw0 / 32, k1 = (cw0 + 23) / 32;
        const uint32_t f0 = k0 < (uint32_t)kMapWords ? fw[k0] : 0u;
        const uint32_t f1 = k1 < (uint32_t)kMapWords ? fw[k1] : 0u;
        const uint32_t c0 = 24 * q / kChunkWords, c1 = (24 * q + 23) / kChunkWords;
        const uint32_t g0 = c0 / 32 == k0 ? f0 : f1, g1 = c1 / 32 == k0 ? f0 : f1;
        const bool need = q < kTileTriples && (((g0 >> (c0 % 32)) | (g1 >> (c1 % 32))) & 1u);
        if (need) load_run(r, src, q);
        else static_for<6>([&](auto ki) { r.u[decltype(ki)::value] = make_uint4(0u, 0u, 0u, 0u); });
    };
    fetch(0);
    // the summary, the slot count and the block -> slot map start empty
    if (threadIdx.x < kRedWords) red[threadIdx.x] = 0;
    for (uint32_t i = threadIdx.x; i < kSlotMapBytes / 4; i += kCompactThreads) dyn[i] = 0xFFFFFFFFu;
    __syncthreads();
    // digit 6 across each run's blocks; the blocks left non-zero take slots
    static_for<2>([&](auto hi) {
        constexpr uint32_t h = decltype(hi)::value;
        const uint32_t q = threadIdx.x + h * kCompactThreads;
        if (h == 1 && 64 * wv + kCompactThreads < kTileTriples) fetch(1);  // wavefronts with a second run
        uint32_t b[3][kBlockWords];
        uint32_t nzb = 0;
        if (q < kTileTriples) {
            unpack_run(r, b[0], b[1], b[2]);
            mark_run_chunks(b[0], b[1], b[2], q, innz);
            uint32_t o[3] = {0u, 0u, 0u};
            static_for<kBlockWords>([&](auto wi) {
                constexpr int w = decltype(wi)::value;
                b[0][w] &= ~b[2][w];
                b[1][w] &= ~b[2][w];
                o[0] |= b[0][w];
                o[1] |= b[1][w];
                o[2] |= b[2][w];
            });
            nzb = (o[0] != 0u ? 1u : 0u) | (o[1] != 0u ? 2u : 0u) | (o[2] != 0u ? 4u : 0u);
        }
        const uint64_t m0 = __ballot(nzb & 1u), m1 = __ballot(nzb & 2u), m2 = __ballot(nzb & 4u);
        const uint32_t n0 = (uint32_t)__popcll(m0), n1 = (uint32_t)__popcll(m1), n2 = (uint32_t)__popcll(m2);
        if (n0 + n1 + n2 != 0) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(nlist, n0 + n1 + n2);
            base = __shfl(base, 0, 64);
            const uint64_t lt = (1ull << lane) - 1ull;  // lanes below this one
            const uint32_t at[3] = {base + (uint32_t)__popcll(m0 & lt), base + n0 + (uint32_t)__popcll(m1 & lt),
                                    base + n0 + n1 + (uint32_t)__popcll(m2 & lt)};
            static_for<3>([&](auto ki) {
                constexpr uint32_t k = decltype(ki)::value;
                if (((nzb >> k) & 1u) && at[k] < kCompactSlots) {
                    slots[2 * at[k]] = make_uint4(b[k][0], b[k][1], b[k][2], b[k][3]);
                    slots[2 * at[k] + 1] = make_uint4(b[k][4], b[k][5], b[k][6], b[k][7]);
                    block_of[at[k]] = (uint16_t)(3 * q + k);
                    slot_of[3 * q + k] = (uint16_t)at[k];
                }
            });
        }
    });
    __syncthreads();
    const uint32_t nb = *nlist;
    if (nb > kCompactSlots) {
        // too dense for the slots: the full-tile kernel takes it as loaded
        if (threadIdx.x == 0) a.deferred[1 + atomicAdd(&a.deferred[0], 1u)] = (uint32_t)tile;
        return;
    }
    // digits 1..5 and 7..12 in one step (see reduce_block_list)
    uint32_t res[kSlotsPerThread][kBlockWords];
    static_for<kSlotsPerThread>([&](auto hi) {
        constexpr uint32_t h = decltype(hi)::value;
        const uint32_t sl = threadIdx.x + h * kCompactThreads;
        if (sl < nb) {
            const uint4 lo = slots[2 * sl], up = slots[2 * sl + 1];
            uint32_t v[kBlockWords] = {lo.x, lo.y, lo.z, lo.w, up.x, up.y, up.z, up.w};
            uint32_t kill[kBlockWords] = {};
            const uint32_t blk = block_of[sl];
            uint32_t rest = blk / 3;  // digits 7..12 of the block index
            static_for<6>([&](auto di) {
                constexpr uint32_t p = (uint32_t)pow3(decltype(di)::value + 1);
                const uint32_t d = rest % 3;
                rest /= 3;
                if (d != 2u) {
                    const uint32_t ns = slot_of[blk + (2u - d) * p];
                    if (ns != kNoSlot) {
                        const uint4 nl = slots[2 * ns], nu = slots[2 * ns + 1];
                        kill[0] |= nl.x; kill[1] |= nl.y; kill[2] |= nl.z; kill[3] |= nl.w;
                        kill[4] |= nu.x; kill[5] |= nu.y; kill[6] |= nu.z; kill[7] |= nu.w;
                    }
                }
            });
            block_reduce(v);
            static_for<kBlockWords>([&](auto wi) {
                constexpr int w = decltype(wi)::value;
                res[h][w] = v[w] & ~kill[w];
            });
        }
    });
    lds_barrier();  // every read of the digit-6 values is done
    static_for<kSlotsPerThread>([&](auto hi) {
        constexpr uint32_t h = decltype(hi)::value;
        const uint32_t sl = threadIdx.x + h * kCompactThreads;
        if (sl < nb) {
            slots[2 * sl] = make_uint4(res[h][0], res[h][1], res[h][2], res[h][3]);
            slots[2 * sl + 1] = make_uint4(res[h][4], res[h][5], res[h][6], res[h][7]);
        }
    });
    __syncthreads();
    // the chunks non-zero as loaded back to HBM, one 256-byte store each;
    // wavefront w takes chunks kPer w .. kPer w + kPer - 1
    constexpr uint32_t kPer = (kTileChunks + kCompactWaves - 1) / kCompactWaves;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(src, 0, (int)(kTileWords * 4), kRawBufferWord3);
    const uint32_t *words = reinterpret_cast<const uint32_t *>(slots);
    const uint32_t kb = wv * kPer, ke = kb + kPer < (uint32_t)kTileChunks ? kb + kPer : (uint32_t)kTileChunks;
    uint32_t cnt = 0;
    for (uint32_t base = kb; base < ke; base += 32) {
        const uint32_t lo = base / 32;
        const uint64_t win = ((uint64_t)(lo + 1 < (uint32_t)kMapWords ? innz[lo + 1] : 0u) << 32) | innz[lo];
        uint32_t bits = (uint32_t)(win >> (base % 32));
        if (ke - base < 32) bits &= (1u << (ke - base)) - 1u;
        bits = __builtin_amdgcn_readfirstlane(bits);
        while (bits != 0u) {
            const uint32_t k = base + (uint32_t)__builtin_ctz(bits);
            bits &= bits - 1u;
            const uint32_t w = k * kChunkWords + lane;
            const bool in = w < kTileWords;  // the last chunk holds 24 words
            const uint32_t ns = in ? (uint32_t)slot_of[w / kBlockWords] : kNoSlot;
            const uint32_t v = ns != kNoSlot ? words[ns * kBlockWords + w % kBlockWords] : 0u;
            cnt += __popc(v);
            if (__ballot(v != 0u) != 0 && lane == 0) atomicOr(&red[1 + k / 32], 1u << (k % 32));
            __builtin_amdgcn_raw_buffer_store_b32(v, rs, in ? (int)(4 * w) : 0x40000000, 0, 0);
        }
    }
    cnt = wave_sum32(cnt);
    if (lane == 0 && cnt != 0) atomicAdd(&red[0], cnt);
    __syncthreads();
    if (threadIdx.x == 0) a.counts[tile] = red[0];
    if (threadIdx.x < kMapWords) a.chunkmap[tile * kMapWords + threadIdx.x] = red[1 + threadIdx.x];
}

// workgroups of the full-tile kernel over the deferred tiles: two per CU
constexpr uint32_t kDeferredGrid = 512;

hipError_t launch_low_compact(const LowArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(low_compact_kernel, dim3((uint32_t)a.ntiles), dim3(kCompactThreads), kCompactLds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(low_deferred_kernel, dim3(kDeferredGrid), dim3(low_threads<kLowReduceCount>()),
                       low_lds_bytes(kLowReduceCount, kTileWords), s, a);
    return hipGetLastError();
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
    if ((e = hipFuncSetAttribute((const void *)low_compact_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kCompactLds)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)low_deferred_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
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
