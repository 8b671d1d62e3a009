// Device building blocks for LDS tiles of the block state (shared by the tile
// kernels and the batch kernels).
//
// A tile is the set of cubes with fixed digits 13..n: 3^lw consecutive blocks
// (lw = min(n-5, 7)), i.e. 8 * 3^lw state words, with digits 1..5 inside each
// block and digits 6..5+lw across blocks (Sec. 4.2: bottom layer in a block,
// top layer across blocks).  Across-block digits act on whole words: digit
// i >= 6 pairs words at distance 8 * 3^(i-6).
#pragma once

#include "h5.h"
#include "launch.h"

namespace dqmc {

constexpr uint32_t kMaxTileWords = kTileWords;  // 17496
constexpr uint32_t kTileTriples = kTileBlocks / 3;  // 729 runs of digit 6 = 0, 1, *

// Apply Merge (MERGE) or Reduce to the K tile digits of every column of the
// tile, the first of them at word stride s.
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
            uint32_t any = 0;
            static_for<C>([&](auto ci) {
                constexpr int c = decltype(ci)::value;
                x[c] = col[c * s];
                any |= x[c];
            });
            // a Reduce only clears bits: columns that are zero in the whole
            // wavefront stay as they are (most of a prime bitmap is zero)
            if (__ballot(any != 0u) == 0) continue;
            reg_reduce<K>(x);
            static_for<C - 1>([&](auto ci) {
                constexpr int c = decltype(ci)::value;
                col[c * s] = x[c];
            });
        }
    }
}

// All lw across-block digits of a tile (word strides 8, 24, ...), three per
// round.
template <bool MERGE>
__device__ __forceinline__ void lds_all_digits(uint32_t *t, uint32_t tw, int lw)
{
    uint32_t s = kBlockWords;
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

// Reduce of the in-block digits 1..5 of every block of an LDS tile.
__device__ __forceinline__ void lds_inblock_reduce(uint32_t *t, uint32_t tw)
{
    for (uint32_t b = threadIdx.x; b < tw / kBlockWords; b += blockDim.x) {
        uint32_t v[kBlockWords];
        static_for<kBlockWords>([&](auto wi) { v[decltype(wi)::value] = t[b * kBlockWords + decltype(wi)::value]; });
        block_reduce(v);
        static_for<kBlockWords>([&](auto wi) { t[b * kBlockWords + decltype(wi)::value] = v[decltype(wi)::value]; });
    }
    __syncthreads();
}

// Fill a tile from the truth table (Alg. 4, "Load input"): the block of
// every group of 32 minterms (block digits all binary) gets those minterms
// placed at their cubes and merged over digits 1..5; every other block starts
// at 0.  `bh` is the binary value of digits 13..n (the tile's high digits).
// The truth-table words are XORed with `flip` first (~0u: the complement).
__device__ __forceinline__ void tile_from_tt(uint32_t *t, const uint32_t *tt, int n, int lw, uint32_t tw, uint64_t bh,
                                             uint32_t flip = 0u)
{
    for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) t[w] = 0;
    __syncthreads();
    const uint32_t nb = 1u << lw;
    const uint32_t wordmask = n >= 5 ? ~0u : ((1u << (1u << n)) - 1u);
    for (uint32_t xm = threadIdx.x; xm < nb; xm += blockDim.x) {
        const uint64_t wi = (bh << lw) + xm;  // truth-table word = x >> 5
        uint32_t v[kBlockWords];
        block_from_tt((tt[wi] ^ flip) & wordmask, v);
        block_merge(v);
        uint32_t b = 0, p = 1;
        for (int j = 0; j < lw; ++j, p *= 3) b += ((xm >> j) & 1u) * p;
        static_for<kBlockWords>([&](auto wi2) { t[b * kBlockWords + decltype(wi2)::value] = v[decltype(wi2)::value]; });
    }
    __syncthreads();
}

// Ordered compaction of the set bits of an LDS tile whose first word is
// state word `wbase`: writes cube indices base + (rank) into list (entries at
// or past cap are dropped) and returns the tile's number of set bits (every
// thread).  `sh` holds blockDim/64 words.
__device__ __forceinline__ uint64_t tile_list(const uint32_t *t, uint32_t tw, uint64_t wbase, uint64_t *list,
                                              uint64_t cap, uint64_t base, uint64_t *sh)
{
    const uint32_t nw = blockDim.x / 64, wv = threadIdx.x / 64, lane = lane_id();
    const uint32_t seg = (tw + nw - 1) / nw;
    const uint32_t s0 = min(tw, wv * seg), s1 = min(tw, s0 + seg);
    uint32_t c = 0;
    for (uint32_t w = s0 + lane; w < s1; w += 64) c += __popc(t[w]);
    c = wave_sum32(c);
    __syncthreads();  // sh may still be read by the previous call
    if (lane == 0) sh[wv] = c;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (uint32_t w = 0; w < nw; ++w) {
        before += w < wv ? sh[w] : 0;
        total += sh[w];
    }
    if (list == nullptr) return total;
    uint64_t run = base + before;
    for (uint32_t r0 = s0; r0 < s1 && run < cap; r0 += 64) {
        const uint32_t w = r0 + lane;
        uint32_t v = w < s1 ? t[w] : 0u;
        if (__ballot(v != 0u) == 0) continue;  // nothing to list in these 64 words
        const uint32_t cc = __popc(v);
        const uint32_t incl = wave_inclusive_scan32(cc);
        uint64_t pos = run + (incl - cc);
        const uint64_t rbase = rho_of_word(wbase + w);
        while (v != 0u && pos < cap) {
            const uint32_t b = __builtin_ctz(v);
            v &= v - 1u;
            list[pos++] = rbase + b;
        }
        run += __shfl(incl, 63, 64);
    }
    return total;
}

// Copy a tile from HBM into LDS, with every load of a thread issued before
// the first LDS store.
template <int THREADS>
__device__ __forceinline__ void load_tile(uint32_t *t, const uint32_t *src, uint32_t tw)
{
    constexpr int U = (kMaxTileWords + THREADS - 1) / THREADS;
    uint32_t v[U];
    // (src + u * THREADS) is uniform: one scalar base per step, one lane offset
    static_for<U>([&](auto ui) {
        constexpr int u = decltype(ui)::value;
        const uint32_t *su = src + u * THREADS;
        v[u] = threadIdx.x + u * THREADS < tw ? su[threadIdx.x] : 0u;
    });
    static_for<U>([&](auto ui) {
        constexpr int u = decltype(ui)::value;
        if (threadIdx.x + u * THREADS < tw) t[threadIdx.x + u * THREADS] = v[u];
    });
}

// Last Reduce round of a full tile (digits 10..12, word stride 648): thread q
// owns column q, reduces it, and writes it to HBM (the prime bitmap);
// consecutive threads write consecutive words.  It also builds the tile
// summary in `red` (zeroed before): red[0] = set bits, red[1..] = map of the
// non-zero 64-word chunks.  The tile is reduced in place in HBM and a Reduce
// only clears bits, so a wavefront's 64-word store is skipped when every
// 64-word chunk it overlaps was zero as loaded (`innz`): those words are zero
// already.
template <bool SKIP_ZERO>
__device__ __forceinline__ void last_round_to_hbm(uint32_t *t, uint32_t *dst, uint32_t *red, const uint32_t *innz)
{
    constexpr uint32_t S = kTileWords / 27;  // 648
    const uint32_t q = threadIdx.x;
    uint32_t c = 0;
    if (q < S) {
        uint32_t x[27], any = 0;
        static_for<27>([&](auto ci) {
            constexpr int k = decltype(ci)::value;
            x[k] = t[q + k * S];
            any |= x[k];
        });
        if (__ballot(any != 0u) != 0) reg_reduce<3>(x);  // zero columns stay zero
        const uint32_t q0 = q & ~63u;  // first column of this wavefront
        const uint32_t q1 = q0 + 63u < S ? q0 + 63u : S - 1u;
        static_for<27>([&](auto ci) {
            constexpr int k = decltype(ci)::value;
            const uint32_t c0 = (q0 + k * S) / kChunkWords, c1 = (q1 + k * S) / kChunkWords;
            if (!SKIP_ZERO || (((innz[c0 / 32] >> (c0 % 32)) | (innz[c1 / 32] >> (c1 % 32))) & 1u)) dst[q + k * S] = x[k];
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

// Final Reduce of a full tile in HBM (kTileWords words at `tile`, 16-byte
// aligned; 768 threads): thread q < 729 loads the three blocks of run q
// (digit 6 = 0, 1, *; 96 contiguous bytes) and reduces digit 6 across them
// and digits 1..5 inside each block on the way into LDS; digits 7..9 are
// reduced in LDS; digits 10..12 in the last round straight back to HBM (the
// prime bitmap).  It also writes the tile summary: *count = its set bits,
// map[0..kMapWords) = its non-zero 64-word chunks.  `red` is
// 2 * kMapWords + 1 words of LDS.  SKIP_ZERO leaves out the stores of chunks
// that were zero as loaded (see last_round_to_hbm); it pays where most of the
// tile is zero (a single large function) and costs more than it saves on the
// small tiles of a batch.
template <bool SKIP_ZERO>
__device__ __forceinline__ void reduce_full_tile(uint32_t *t, uint32_t *tile, uint32_t *count, uint32_t *map,
                                                 uint32_t *red)
{
    // red[kMapWords + 1 ..] holds the input-chunk flags
    uint32_t *innz = red + kMapWords + 1;
    if (threadIdx.x < 2 * kMapWords + 1) red[threadIdx.x] = 0;
    if constexpr (SKIP_ZERO) __syncthreads();  // flags zeroed before they are set
    const uint32_t q = threadIdx.x;
    if (q < kTileTriples) {
        uint32_t b0[kBlockWords], b1[kBlockWords], b2[kBlockWords];
        const uint4 *src = reinterpret_cast<const uint4 *>(tile + 24 * q);
        const uint4 u0 = src[0], u1 = src[1], u2 = src[2], u3 = src[3], u4 = src[4], u5 = src[5];
        b0[0] = u0.x; b0[1] = u0.y; b0[2] = u0.z; b0[3] = u0.w;
        b0[4] = u1.x; b0[5] = u1.y; b0[6] = u1.z; b0[7] = u1.w;
        b1[0] = u2.x; b1[1] = u2.y; b1[2] = u2.z; b1[3] = u2.w;
        b1[4] = u3.x; b1[5] = u3.y; b1[6] = u3.z; b1[7] = u3.w;
        b2[0] = u4.x; b2[1] = u4.y; b2[2] = u4.z; b2[3] = u4.w;
        b2[4] = u5.x; b2[5] = u5.y; b2[6] = u5.z; b2[7] = u5.w;
        if constexpr (SKIP_ZERO) {
            // words 24q .. 24q+23 lie in at most two 64-word chunks
            const uint32_t w0 = 24 * q, c0 = w0 / kChunkWords, c1 = (w0 + 23) / kChunkWords;
            const uint32_t split = (c0 + 1) * kChunkWords - w0;  // words of the run in chunk c0
            uint32_t nz0 = 0, nz1 = 0;
            static_for<kBlockWords>([&](auto wi) {
                constexpr uint32_t w = decltype(wi)::value;
                nz0 |= (w < split ? b0[w] : 0u) | (w + 8 < split ? b1[w] : 0u) | (w + 16 < split ? b2[w] : 0u);
                nz1 |= (w < split ? 0u : b0[w]) | (w + 8 < split ? 0u : b1[w]) | (w + 16 < split ? 0u : b2[w]);
            });
            if (nz0 != 0u) atomicOr(&innz[c0 / 32], 1u << (c0 % 32));
            if (nz1 != 0u) atomicOr(&innz[c1 / 32], 1u << (c1 % 32));
        }
        // digit 6 first (the order of the reduced dimensions is free): the
        // runs with digit 6 = 0 or 1 lose what the * run holds; then digits
        // 1..5 inside each block, one block at a time.  A wavefront whose
        // runs are all zero (most of a prime bitmap) skips the arithmetic.
        uint4 *dst = reinterpret_cast<uint4 *>(t + 24 * q);
        auto put = [&](const uint32_t(&b)[kBlockWords], int k) {
            dst[2 * k] = make_uint4(b[0], b[1], b[2], b[3]);
            dst[2 * k + 1] = make_uint4(b[4], b[5], b[6], b[7]);
        };
        uint32_t any = 0;
        static_for<kBlockWords>([&](auto wi) {
            constexpr int w = decltype(wi)::value;
            any |= b0[w] | b1[w] | b2[w];
        });
        if (__ballot(any != 0u) != 0) {
            static_for<kBlockWords>([&](auto wi) {
                constexpr int w = decltype(wi)::value;
                b0[w] &= ~b2[w];
                b1[w] &= ~b2[w];
            });
            block_reduce(b0);
            put(b0, 0);
            block_reduce(b1);
            put(b1, 1);
            block_reduce(b2);
            put(b2, 2);
        } else {
            put(b0, 0);
            put(b1, 1);
            put(b2, 2);
        }
    }
    __syncthreads();
    lds_group<3, false>(t, kMaxTileWords, 3 * kBlockWords);  // digits 7..9
    __syncthreads();
    last_round_to_hbm<SKIP_ZERO>(t, tile, red, innz);  // digits 10..12
    __syncthreads();
    if (threadIdx.x == 0) *count = red[0];
    if (threadIdx.x < kMapWords) map[threadIdx.x] = red[1 + threadIdx.x];
}

// Ordered list of the set bits of one tile of a bitmap in HBM, by one
// wavefront: the tile's non-zero chunks (bit k of map = chunk k, from the
// tile summary) are listed in order, their words are loaded kListBatch chunks
// at a time, and each chunk's set bits are written at `off` plus the running
// count (word-major, then bit) as cube indices rho0 + rho_of_word(wbase +
// word) + bit.  Entries at or past cap are dropped.  nz holds kTileChunks
// entries private to the wave.
constexpr int kListBatch = 16;  // chunks whose words are loaded together

__device__ __forceinline__ void list_tile(const uint32_t *src, uint32_t tw, uint64_t wbase, uint64_t off,
                                          const uint32_t *map, uint64_t *list, uint64_t cap, uint16_t *nz,
                                          uint64_t rho0 = 0)
{
    const uint32_t lane = lane_id();
    const uint32_t mw = lane < (uint32_t)kMapWords ? map[lane] : 0u;
    const uint32_t pc = __popc(mw);
    const uint32_t incl = wave_inclusive_scan32(pc);
    const uint32_t m = __shfl(incl, 63, 64);
    uint32_t pos = incl - pc, bits = mw;
    while (bits != 0u) {
        const uint32_t b = __builtin_ctz(bits);
        bits &= bits - 1u;
        nz[pos++] = (uint16_t)(lane * 32 + b);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint64_t run = off;
    for (uint32_t r0 = 0; r0 < m && run < cap; r0 += kListBatch) {
        uint32_t v[kListBatch];
        static_for<kListBatch>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const uint32_t w = (r0 + i < m) ? (uint32_t)nz[r0 + i] * kChunkWords + lane : tw;
            v[i] = w < tw ? src[w] : 0u;
        });
        static_for<kListBatch>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            if (r0 + i < m) {
                uint32_t x = v[i];
                const uint32_t cc = __popc(x);
                const uint32_t inc = wave_inclusive_scan32(cc);
                uint64_t p = run + (inc - cc);
                const uint64_t w = (uint64_t)nz[r0 + i] * kChunkWords + lane;
                const uint64_t rbase = rho0 + rho_of_word(wbase + w);
                while (x != 0u && p < cap) {
                    const uint32_t b = __builtin_ctz(x);
                    x &= x - 1u;
                    list[p++] = rbase + b;
                }
                run += __shfl(inc, 63, 64);
            }
        });
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();  // nz is reused by the wave's next tile
}

}  // namespace dqmc
