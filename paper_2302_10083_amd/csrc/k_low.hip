// Low tile kernels: the in-word digits 1..3 and the word digits 4..12 of one
// tile of 3^min(n,12) cubes, processed in LDS.
//
// Alg. 4 loads the support into the state, then applies the Merge transform
// per dimension (top layer over whole blocks, bottom layer inside a block),
// then Reduce, then scans the state for the output list.  Here a tile is the
// unit of on-chip work: digits 1..3 use the in-word shift-and-mask form of the
// bottom layer (Sec. 4.2, masks mu_i), digits 4..12 use the top-layer triple
// indexing of Sec. 4.2 (eq. indexes) on LDS words, three digits at a time in
// registers.  Digits above 12 are handled by the column passes (k_col.hip).
#include "launch.h"
#include "t27.h"

namespace dqmc {

// Apply Merge (MERGE) or Reduce to the K tile digits j..j+K-1 (stride s = 3^j
// words) of every column of the tile.
template <int K, bool MERGE>
__device__ __forceinline__ void lds_group(uint32_t *t, uint32_t tw, uint32_t s)
{
    constexpr int C = (int)pow3(K);
    const uint32_t ncols = tw / C;
    for (uint32_t q = threadIdx.x; q < ncols; q += blockDim.x) {
        const uint32_t lo = q % s, hi = q / s;
        uint32_t *col = t + lo + hi * s * C;
        uint32_t x[C];
        if constexpr (MERGE) {
            static_for<C>([&](auto ci) {
                constexpr int c = decltype(ci)::value;
                x[c] = all_binary(c, K) ? col[c * s] : 0u;
            });
            reg_merge<K>(x);
            static_for<C>([&](auto ci) {
                constexpr int c = decltype(ci)::value;
                if constexpr (!all_binary(c, K)) col[c * s] = x[c];
            });
        } else {
            static_for<C>([&](auto ci) {
                constexpr int c = decltype(ci)::value;
                x[c] = col[c * s];
            });
            reg_reduce<K>(x);
            static_for<C - 1>([&](auto ci) {
                constexpr int c = decltype(ci)::value;
                col[c * s] = x[c];
            });
        }
    }
}

template <bool MERGE>
__device__ __forceinline__ void lds_all_digits(uint32_t *t, uint32_t tw, int lw)
{
    uint32_t s = 1;
    for (int j = 0; j < lw;) {
        const int k = lw - j >= 3 ? 3 : lw - j;
        if (k == 3) lds_group<3, MERGE>(t, tw, s);
        else if (k == 2) lds_group<2, MERGE>(t, tw, s);
        else lds_group<1, MERGE>(t, tw, s);
        __syncthreads();
        s *= (uint32_t)pow3(k);
        j += k;
    }
}

// Fill the tile from the truth table: the word of every cube group whose word
// digits are all binary gets the merged in-word pattern of its 8 minterms;
// every other word starts at 0 (Alg. 4, "Load input").
__device__ __forceinline__ void load_tile_from_tt(uint32_t *t, uint32_t *lut, const LowArgs &a, uint64_t bh)
{
    lut[threadIdx.x] = inword_merge(expand_byte(threadIdx.x));  // blockDim == 256
    for (uint32_t w = threadIdx.x; w < a.tw; w += blockDim.x) t[w] = 0;
    __syncthreads();
    const uint32_t nb = 1u << a.lw;
    const uint32_t bytemask = a.n >= 3 ? 0xFFu : ((1u << (1u << a.n)) - 1u);
    for (uint32_t xm = threadIdx.x; xm < nb; xm += blockDim.x) {
        const uint64_t bi = (bh << a.lw) + xm;  // byte index = x >> 3
        const uint32_t byte = (a.tt[bi >> 2] >> ((bi & 3) * 8)) & bytemask;
        uint32_t w = 0, p = 1;
        for (int j = 0; j < a.lw; ++j, p *= 3) w += ((xm >> j) & 1u) * p;
        t[w] = lut[byte];
    }
    __syncthreads();
}

// Ordered compaction of the set bits of a single-tile state (n <= 12) into
// the list, and the total count.
__device__ __forceinline__ void single_tile_extract(const uint32_t *t, const LowArgs &a, uint64_t *sh)
{
    const uint32_t nw = blockDim.x / 64, wv = threadIdx.x / 64, lane = lane_id();
    const uint32_t seg = (a.tw + nw - 1) / nw;
    const uint32_t s0 = min(a.tw, wv * seg), s1 = min(a.tw, s0 + seg);
    uint32_t c = 0;
    for (uint32_t w = s0 + lane; w < s1; w += 64) c += __popc(t[w]);
    c = wave_sum32(c);
    if (lane == 0) sh[wv] = c;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (uint32_t w = 0; w < nw; ++w) {
        before += w < wv ? sh[w] : 0;
        total += sh[w];
    }
    if (threadIdx.x == 0 && a.count != nullptr) *a.count = total;
    if (a.list == nullptr) return;
    uint64_t run = before;
    const bool words = a.n >= 3;
    for (uint32_t r0 = s0; r0 < s1 && run < a.cap; r0 += 64) {
        const uint32_t w = r0 + lane;
        uint32_t v = w < s1 ? t[w] : 0u;
        if (__ballot(v != 0u) == 0) continue;  // nothing to list in these 64 words
        const uint32_t cc = __popc(v);
        const uint32_t incl = wave_inclusive_scan32(cc);
        uint64_t pos = run + (incl - cc);
        const uint64_t rbase = words ? 27ull * w : 0ull;
        while (v != 0u && pos < a.cap) {
            const uint32_t b = __builtin_ctz(v);
            v &= v - 1u;
            a.list[pos++] = rbase + b;
        }
        run += __shfl(incl, 63, 64);
    }
}

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

constexpr uint32_t kMaxTileWords = 19683;  // 3^9

template <int MODE>
__host__ __device__ constexpr int low_threads()
{
    // the tile passes over HBM-resident states use one 27-word column per
    // thread per LDS round (729 columns in a full tile)
    return (MODE == kLowReduceCount || MODE == kLowCount) ? 768 : kLowThreads;
}

// Copy a tile from HBM into LDS (optionally applying the in-word Reduce),
// with every load of a thread issued before the first LDS store.
template <bool REDUCE, int THREADS>
__device__ __forceinline__ void load_tile(uint32_t *t, const uint32_t *src, uint32_t tw)
{
    constexpr int U = (kMaxTileWords + THREADS - 1) / THREADS;
    uint32_t v[U];
    static_for<U>([&](auto ui) {
        constexpr int u = decltype(ui)::value;
        const uint32_t w = threadIdx.x + u * THREADS;
        v[u] = w < tw ? __builtin_nontemporal_load(src + w) : 0u;
    });
    static_for<U>([&](auto ui) {
        constexpr int u = decltype(ui)::value;
        const uint32_t w = threadIdx.x + u * THREADS;
        if (w < tw) t[w] = REDUCE ? inword_reduce(v[u]) : v[u];
    });
}

template <int THREADS>
__device__ __forceinline__ void store_tile(uint32_t *dst, const uint32_t *t, uint32_t tw)
{
    constexpr int U = (kMaxTileWords + THREADS - 1) / THREADS;
    uint32_t v[U];
    static_for<U>([&](auto ui) {
        constexpr int u = decltype(ui)::value;
        const uint32_t w = threadIdx.x + u * THREADS;
        v[u] = w < tw ? t[w] : 0u;
    });
    static_for<U>([&](auto ui) {
        constexpr int u = decltype(ui)::value;
        const uint32_t w = threadIdx.x + u * THREADS;
        if (w < tw) __builtin_nontemporal_store(v[u], dst + w);
    });
}

// Last Reduce round of a full tile (digits 10..12, stride 729 words): thread q
// owns column q, reduces it, and writes it to HBM (the prime bitmap);
// consecutive threads write consecutive words.  It also builds the tile
// summary in `red` (zeroed before): red[0] = set bits, red[1..] = map of the
// non-zero 64-word chunks.
__device__ __forceinline__ void last_round_to_hbm(uint32_t *t, uint32_t *dst, uint32_t *red)
{
    constexpr uint32_t S = 729;
    const uint32_t q = threadIdx.x;
    uint32_t c = 0;
    if (q < S) {
        uint32_t x[27];
        static_for<27>([&](auto ci) {
            constexpr int k = decltype(ci)::value;
            x[k] = t[q + k * S];
        });
        reg_reduce<3>(x);
        static_for<27>([&](auto ci) {
            constexpr int k = decltype(ci)::value;
            __builtin_nontemporal_store(x[k], dst + q + k * S);
            c += __popc(x[k]);
            if (x[k] != 0u) {
                const uint32_t chunk = (q + k * S) / kChunkWords;
                atomicOr(&red[1 + chunk / 32], 1u << (chunk % 32));
            }
        });
    }
    c = wave_sum32(c);
    if (lane_id() == 0 && c != 0) atomicAdd(&red[0], c);
}

template <int MODE>
__global__ __launch_bounds__(low_threads<MODE>()) void low_kernel(LowArgs a)
{
    constexpr int THREADS = low_threads<MODE>();
    extern __shared__ uint32_t dyn[];
    __shared__ uint64_t sh[THREADS / 64];
    uint32_t *t = dyn;

    if constexpr (MODE == kLowMergeTT || MODE == kLowPrimesTT) {
        // tile with binary digits 13..n given by the bits of blockIdx.x
        const uint64_t bh = blockIdx.x;
        load_tile_from_tt(t, dyn + a.tw, a, bh);
        lds_all_digits<true>(t, a.tw, a.lw);
        uint64_t tile = 0;
        for (int j = 0, nh = a.n - 12; j < nh; ++j)
            if ((bh >> j) & 1) tile += pow3(j);
        if constexpr (MODE == kLowMergeTT) {
            uint32_t *dst = a.state + tile * a.tw;
            for (uint32_t w = threadIdx.x; w < a.tw; w += blockDim.x) dst[w] = t[w];
        } else {
            for (uint32_t w = threadIdx.x; w < a.tw; w += blockDim.x) t[w] = inword_reduce(t[w]);
            __syncthreads();
            lds_all_digits<false>(t, a.tw, a.lw);
            for (uint32_t w = threadIdx.x; w < a.tw; w += blockDim.x) a.state[w] = t[w];
            single_tile_extract(t, a, sh);
        }
    } else {
        __shared__ uint32_t red[kMapWords + 1];
        const uint64_t tile = blockIdx.x;
        const uint32_t *src = a.state + tile * a.tw;
        if constexpr (MODE == kLowReduceCount) {
            // always a full tile here (n > 12): digits 4..6, 7..9 in LDS,
            // digits 10..12 in the last round, straight to HBM
            if (threadIdx.x < kMapWords + 1) red[threadIdx.x] = 0;
            load_tile<true, THREADS>(t, src, a.tw);
            __syncthreads();
            lds_group<3, false>(t, a.tw, 1);
            __syncthreads();
            lds_group<3, false>(t, a.tw, 27);
            __syncthreads();
            last_round_to_hbm(t, a.state + tile * a.tw, red);
            __syncthreads();
            if (threadIdx.x == 0) a.counts[tile] = red[0];
            if (threadIdx.x < kMapWords) a.chunkmap[tile * kMapWords + threadIdx.x] = red[1 + threadIdx.x];
            return;
        } else {
            load_tile<false, THREADS>(t, src, a.tw);
            __syncthreads();
        }
        tile_summary(t, a, tile, red);
    }
}

static size_t low_lds_bytes(int mode, uint32_t tw)
{
    return (size_t)tw * 4 + ((mode == kLowMergeTT || mode == kLowPrimesTT) ? 256 * 4 : 0);
}

hipError_t low_setup()
{
    const int bytes = (int)low_lds_bytes(kLowMergeTT, (uint32_t)pow3(9));
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)low_kernel<kLowMergeTT>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)low_kernel<kLowPrimesTT>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)low_kernel<kLowReduceCount>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess)
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
