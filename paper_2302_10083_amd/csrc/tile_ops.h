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
// LDS words of a tile's reduce bookkeeping: set-bit count, map of non-zero
// chunks, map of chunks non-zero as loaded, length of the non-zero block list
constexpr uint32_t kRedWords = 2 * kMapWords + 2;
// LDS of the final reduce of a full tile: its kTileWords words in order, then
// the list of its non-zero blocks (uint16).
constexpr uint32_t kBlockListBytes = (kTileBlocks * 2 + 15) / 16 * 16;
constexpr uint32_t kReduceTileBytes = kTileWords * 4;

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

// Word 3 of a raw buffer resource on CDNA (gfx9 family): DATA_FORMAT = 4
// (32 bit) in bits 15..18, every other field 0.
constexpr int kRawBufferWord3 = 0x00020000;

// Run q of a full tile (q < 729): its three blocks with digit 6 = 0, 1, *,
// 96 contiguous bytes of the tile in HBM (16-byte aligned).
struct TileRun {
    uint4 u[6];
};

__device__ __forceinline__ void load_run(TileRun &r, const uint32_t *tile, uint32_t q)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(tile + 24 * q);
    static_for<6>([&](auto ki) { r.u[decltype(ki)::value] = src[decltype(ki)::value]; });
}

// Run q as three blocks b[0..2] of eight words.
__device__ __forceinline__ void unpack_run(const TileRun &r, uint32_t (&b0)[kBlockWords], uint32_t (&b1)[kBlockWords],
                                           uint32_t (&b2)[kBlockWords])
{
    static_for<2>([&](auto hi) {
        constexpr int h = decltype(hi)::value;
        b0[4 * h] = r.u[h].x; b0[4 * h + 1] = r.u[h].y; b0[4 * h + 2] = r.u[h].z; b0[4 * h + 3] = r.u[h].w;
        b1[4 * h] = r.u[2 + h].x; b1[4 * h + 1] = r.u[2 + h].y; b1[4 * h + 2] = r.u[2 + h].z;
        b1[4 * h + 3] = r.u[2 + h].w;
        b2[4 * h] = r.u[4 + h].x; b2[4 * h + 1] = r.u[4 + h].y; b2[4 * h + 2] = r.u[4 + h].z;
        b2[4 * h + 3] = r.u[4 + h].w;
    });
}

// Marks in `innz` the 64-word chunks in which run q holds a non-zero word.
// The run's 24 words start at word 24q; 24q mod 64 repeats with period 8 in
// q, and only runs with q mod 8 = 2 (blocks 0, 1 | 2) and q mod 8 = 5 (block
// 0 | 1, 2) cross a chunk boundary, between two blocks.
__device__ __forceinline__ void mark_run_chunks(const uint32_t (&b0)[kBlockWords], const uint32_t (&b1)[kBlockWords],
                                                const uint32_t (&b2)[kBlockWords], uint32_t q, uint32_t *innz)
{
    uint32_t r0 = 0, r1 = 0, r2 = 0;
    static_for<kBlockWords>([&](auto wi) {
        constexpr uint32_t w = decltype(wi)::value;
        r0 |= b0[w];
        r1 |= b1[w];
        r2 |= b2[w];
    });
    const uint32_t m8 = q % 8;
    const uint32_t in0 = m8 == 2 ? (r0 | r1) : m8 == 5 ? r0 : (r0 | r1 | r2);
    const uint32_t in1 = m8 == 2 ? r2 : m8 == 5 ? (r1 | r2) : 0u;
    const uint32_t c0 = 24 * q / kChunkWords;
    if (in0 != 0u) atomicOr(&innz[c0 / 32], 1u << (c0 % 32));
    if (in1 != 0u) atomicOr(&innz[(c0 + 1) / 32], 1u << ((c0 + 1) % 32));
}

// Block blk of an LDS tile.
__device__ __forceinline__ void put_block(uint32_t *t, uint32_t blk, const uint32_t (&b)[kBlockWords])
{
    uint4 *dst = reinterpret_cast<uint4 *>(t + kBlockWords * blk);
    dst[0] = make_uint4(b[0], b[1], b[2], b[3]);
    dst[1] = make_uint4(b[4], b[5], b[6], b[7]);
}

// Block blk of an LDS tile, into registers.
__device__ __forceinline__ void get_block(const uint32_t *t, uint32_t blk, uint32_t (&b)[kBlockWords])
{
    const uint4 *src = reinterpret_cast<const uint4 *>(t + kBlockWords * blk);
    const uint4 lo = src[0], hi = src[1];
    b[0] = lo.x; b[1] = lo.y; b[2] = lo.z; b[3] = lo.w;
    b[4] = hi.x; b[5] = hi.y; b[6] = hi.z; b[7] = hi.w;
}

// Blocks per thread in the block-list reduce: 768 threads cover the 2187
// blocks of a tile in three.
constexpr int kListSlots = 3;

// Reduce of digits 1..5 and 7..12 on the blocks of the list (those non-zero
// after digit 6; the others stay zero) as one step (reading 7 of the design
// notes: a group of dimensions reduced at once, against the values the
// previous groups left, gives the same primes as one dimension after
// another): block b keeps its in-block reduce (Sec. 4.2, digits 1..5) less
// what its * neighbours along digits 7..12 hold, all read as digit 6 left
// them.  Reads and writes are split by a barrier; every thread calls it.
__device__ __forceinline__ void reduce_block_list(uint32_t *t, const uint16_t *blist, uint32_t nb)
{
    uint32_t res[kListSlots][kBlockWords];
    uint32_t blk[kListSlots];
    static_for<kListSlots>([&](auto si) {
        constexpr int sl = decltype(si)::value;
        const uint32_t i = threadIdx.x + sl * blockDim.x;
        blk[sl] = i < nb ? (uint32_t)blist[i] : 0u;
        if (i < nb) {
            uint32_t v[kBlockWords], kill[kBlockWords] = {};
            get_block(t, blk[sl], v);
            uint32_t rest = blk[sl] / 3;  // digits 7..12 of the block index
            static_for<6>([&](auto di) {
                constexpr uint32_t p = (uint32_t)pow3(decltype(di)::value + 1);
                const uint32_t d = rest % 3;
                rest /= 3;
                if (d != 2u) {
                    uint32_t u[kBlockWords];
                    get_block(t, blk[sl] + (2u - d) * p, u);
                    static_for<kBlockWords>([&](auto wi) { kill[decltype(wi)::value] |= u[decltype(wi)::value]; });
                }
            });
            block_reduce(v);
            static_for<kBlockWords>([&](auto wi) {
                constexpr int w = decltype(wi)::value;
                res[sl][w] = v[w] & ~kill[w];
            });
        }
    });
    lds_barrier();  // every read of the digit-6 values is done
    static_for<kListSlots>([&](auto si) {
        constexpr int sl = decltype(si)::value;
        if (threadIdx.x + sl * blockDim.x < nb) put_block(t, blk[sl], res[sl]);
    });
}

// The tile's chunks that were non-zero as loaded (`innz`), stored from the
// LDS tile to HBM at dst (the other chunks were zero there and stay
// zero), with the tile summary in red: red[0] += set bits, red[1 + k / 32]
// bit k for the chunks non-zero now.  Wavefront w takes chunks 23 w .. 23 w +
// 22 (12 wavefronts); lane j holds word j of a chunk, so each store is one
// 256-byte segment.
__device__ __forceinline__ void store_marked_chunks(const uint32_t *t, uint32_t *dst, uint32_t *red,
                                                    const uint32_t *innz)
{
    constexpr uint32_t kPer = (kTileChunks + 11) / 12;  // 23
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = lane_id();
    const uint32_t k0 = wv * kPer;
    if (k0 >= (uint32_t)kTileChunks) return;
    const uint32_t a0 = __builtin_amdgcn_readfirstlane(innz[k0 / 32]);
    const uint32_t a1 = k0 / 32 + 1 < (uint32_t)kMapWords ? __builtin_amdgcn_readfirstlane(innz[k0 / 32 + 1]) : 0u;
    const uint32_t nk = (uint32_t)kTileChunks - k0 < kPer ? (uint32_t)kTileChunks - k0 : kPer;
    // bit i: chunk k0 + i is marked
    uint32_t bits = (uint32_t)((((uint64_t)a1 << 32) | a0) >> (k0 % 32)) & ((1u << nk) - 1u);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(dst, 0, (int)(kTileWords * 4), kRawBufferWord3);
    uint32_t c = 0;
    while (bits != 0u) {
        const uint32_t k = k0 + (uint32_t)__builtin_ctz(bits);
        bits &= bits - 1u;
        const uint32_t w = k * kChunkWords + lane;
        const bool in = w < kTileWords;  // the last chunk holds 24 words
        const uint32_t v = in ? t[w] : 0u;
        c += __popc(v);
        if (__ballot(v != 0u) != 0 && lane == 0) atomicOr(&red[1 + k / 32], 1u << (k % 32));
        __builtin_amdgcn_raw_buffer_store_b32(v, rs, in ? (int)(4 * w) : 0x40000000, 0, 0);
    }
    c = wave_sum32(c);
    if (lane == 0 && c != 0) atomicAdd(&red[0], c);
}

// Reduce of digit 6 across the three blocks of run q into the LDS tile, the
// chunk flags of the run as loaded (unless MARK is false: given), and the
// run's blocks that are non-zero after it appended to `blist` (length
// *nlist).  Every thread of the workgroup calls it (ballots); threads without
// a run pass has_run = false.
template <bool MARK>
__device__ __forceinline__ void run_digit6_to_lds(uint32_t *t, const TileRun &r, uint32_t q, bool has_run,
                                                  uint32_t *innz, uint16_t *blist, uint32_t *nlist)
{
    uint32_t nzb = 0;  // bit k: block 3q + k is non-zero
    if (has_run) {
        uint32_t b0[kBlockWords], b1[kBlockWords], b2[kBlockWords];
        unpack_run(r, b0, b1, b2);
        if constexpr (MARK) mark_run_chunks(b0, b1, b2, q, innz);
        uint32_t o0 = 0, o1 = 0, o2 = 0;
        static_for<kBlockWords>([&](auto wi) {
            constexpr int w = decltype(wi)::value;
            b0[w] &= ~b2[w];
            b1[w] &= ~b2[w];
            o0 |= b0[w];
            o1 |= b1[w];
            o2 |= b2[w];
        });
        put_block(t, 3 * q, b0);
        put_block(t, 3 * q + 1, b1);
        put_block(t, 3 * q + 2, b2);
        nzb = (o0 != 0u ? 1u : 0u) | (o1 != 0u ? 2u : 0u) | (o2 != 0u ? 4u : 0u);
    }
    const uint64_t m0 = __ballot(nzb & 1u), m1 = __ballot(nzb & 2u), m2 = __ballot(nzb & 4u);
    const uint32_t c0 = (uint32_t)__popcll(m0), c1 = (uint32_t)__popcll(m1), c2 = (uint32_t)__popcll(m2);
    if (c0 + c1 + c2 == 0) return;
    uint32_t base = 0;
    const uint32_t lane = lane_id();
    if (lane == 0) base = atomicAdd(nlist, c0 + c1 + c2);
    base = __shfl(base, 0, 64);
    const uint64_t lt = (1ull << lane) - 1ull;  // lanes below this one
    if (nzb & 1u) blist[base + (uint32_t)__popcll(m0 & lt)] = (uint16_t)(3 * q);
    if (nzb & 2u) blist[base + c0 + (uint32_t)__popcll(m1 & lt)] = (uint16_t)(3 * q + 1);
    if (nzb & 4u) blist[base + c0 + c1 + (uint32_t)__popcll(m2 & lt)] = (uint16_t)(3 * q + 2);
}

// Final Reduce of a full tile in HBM (kTileWords words at `tile`, 16-byte
// aligned; 768 threads; kReduceTileBytes + kBlockListBytes of LDS at t):
// thread q < 729 loads run q and digit 6
// is reduced on the way into LDS.  The blocks non-zero after it are listed;
// each gets digits 1..5 and 7..12 in one step (reduce_block_list), and only
// the chunks non-zero as loaded are stored (store_marked_chunks): a Reduce
// only clears bits, so the others are zero in HBM already.  It also writes
// the tile summary: *count = its set bits, map[0..kMapWords) = its non-zero
// 64-word chunks.  `red` is kRedWords words of LDS.
// `flags` (kMapWords words, or nullptr) marks the chunks that may hold a set
// bit: the others are zero in HBM, so their runs are not loaded.  f0, f1 are
// the words 24 w / 32 and (24 w + 23) / 32 of the flags for the calling
// wavefront w (its 64 runs cover chunks 24 w .. 24 w + 23), loaded ahead by
// the caller.
__device__ __forceinline__ void reduce_full_tile(uint32_t *t, uint32_t *tile, uint32_t *count, uint32_t *map,
                                                 uint32_t *red, const uint32_t *flags = nullptr, uint32_t f0 = 0u,
                                                 uint32_t f1 = 0u)
{
    uint32_t *innz = red + kMapWords + 1;
    if (threadIdx.x < kRedWords) red[threadIdx.x] = 0;
    const uint32_t q = threadIdx.x;
    uint16_t *blist = reinterpret_cast<uint16_t *>(t + kTileWords);
    uint32_t *nlist = red + kRedWords - 1;
    TileRun r;
    if (flags != nullptr) {
        const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
        const uint32_t k0 = 24 * wv / 32;
        const uint32_t c0 = 24 * q / kChunkWords, c1 = (24 * q + 23) / kChunkWords;
        const uint32_t g0 = c0 / 32 == k0 ? f0 : f1, g1 = c1 / 32 == k0 ? f0 : f1;
        const bool need = q < kTileTriples && (((g0 >> (c0 % 32)) | (g1 >> (c1 % 32))) & 1u);
        if (need) load_run(r, tile, q);
        else static_for<6>([&](auto ki) { r.u[decltype(ki)::value] = make_uint4(0u, 0u, 0u, 0u); });
        __syncthreads();  // flags and list length zeroed before they are set
        // the chunks non-zero as loaded (a subset of the flagged ones):
        // only those are stored
        run_digit6_to_lds<true>(t, r, q, q < kTileTriples, innz, blist, nlist);
    } else {
        __syncthreads();  // flags and list length zeroed before they are set
        if (q < kTileTriples) load_run(r, tile, q);
        run_digit6_to_lds<true>(t, r, q, q < kTileTriples, innz, blist, nlist);
    }
    __syncthreads();
    reduce_block_list(t, blist, *nlist);
    __syncthreads();
    store_marked_chunks(t, tile, red, innz);
    __syncthreads();
    if (threadIdx.x == 0) *count = red[0];
    if (threadIdx.x < kMapWords) map[threadIdx.x] = red[1 + threadIdx.x];
}

// Entries of a wavefront's list staging buffer in LDS (see list_tile).
constexpr uint32_t kListStage = 512;

// Ordered list of the set bits of one tile of a bitmap in HBM, by one
// wavefront: the tile's non-zero chunks (bit k of map = chunk k, from the
// tile summary) are listed in order, and taken sixteen at a time: lane l
// holds words 16 (l mod 4) .. 16 (l mod 4) + 15 of the (l / 4)-th chunk of
// the batch, so lane order is word order.  One wave scan of the lanes' bit
// counts places every lane's bits, as cube indices rho0 +
// rho_of_word(wbase + word) + bit (wbase a multiple of 8), at `off` plus the
// running count.  They go through `stage` (kListStage entries private to the
// wave) in list order, so that the wave writes the batch's entries to HBM as
// consecutive 8-byte words (lanes writing their own bits would scatter every
// store over up to 64 lines); a batch's entries past kListStage are written
// directly.  Entries at or past cap are dropped.  nz holds kTileChunks
// entries private to the wave.
__device__ __forceinline__ void list_tile(const uint32_t *src, uint32_t tw, uint64_t wbase, uint64_t off,
                                          const uint32_t *map, uint64_t *list, uint64_t cap, uint16_t *nz,
                                          uint64_t *stage, uint64_t rho0 = 0)
{
    constexpr int kSpan = 16;  // words per lane
    const uint32_t lane = lane_id();
    const uint32_t mw = lane < (uint32_t)kMapWords ? map[lane] : 0u;
    const uint32_t pc = __popc(mw);
    const uint32_t incl0 = wave_inclusive_scan32(pc);
    const uint32_t m = __shfl(incl0, 63, 64);
    uint32_t pos0 = incl0 - pc, bits = mw;
    while (bits != 0u) {
        const uint32_t b = __builtin_ctz(bits);
        bits &= bits - 1u;
        nz[pos0++] = (uint16_t)(lane * 32 + b);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint32_t slot = lane / 4, qw = (lane % 4) * kSpan;
    uint64_t run = off;
    for (uint32_t r0 = 0; r0 < m && run < cap; r0 += 64 / 4) {
        uint32_t v[kSpan];
        uint32_t w0 = 0;
        static_for<kSpan>([&](auto ji) { v[decltype(ji)::value] = 0u; });
        if (r0 + slot < m) {
            w0 = (uint32_t)nz[r0 + slot] * kChunkWords + qw;
            if (w0 + kSpan <= tw) {
                const uint4 *p = reinterpret_cast<const uint4 *>(src + w0);  // 64-byte aligned
                static_for<kSpan / 4>([&](auto ki) {
                    constexpr int k = decltype(ki)::value;
                    const uint4 u = p[k];
                    v[4 * k] = u.x;
                    v[4 * k + 1] = u.y;
                    v[4 * k + 2] = u.z;
                    v[4 * k + 3] = u.w;
                });
            } else {
                // the tile's last chunk is partial
                static_for<kSpan>([&](auto ji) {
                    constexpr int j = decltype(ji)::value;
                    v[j] = w0 + j < tw ? src[w0 + j] : 0u;
                });
            }
        }
        uint32_t cnt = 0;
        static_for<kSpan>([&](auto ji) { cnt += __popc(v[decltype(ji)::value]); });
        const uint32_t incl = wave_inclusive_scan32(cnt);
        const uint32_t nb = __shfl(incl, 63, 64);  // the batch's entries
        uint32_t at = incl - cnt;                   // this lane's first, in the batch
        const uint64_t rb = rho0 + rho_of_word(wbase + w0);  // w0 is a multiple of 8
        static_for<kSpan>([&](auto ji) {
            constexpr int j = decltype(ji)::value;
            uint32_t x = v[j];
            const uint64_t rj = rb + (uint64_t)(kBlockCubes * (j / 8) + 32 * (j % 8));
            while (x != 0u) {
                const uint32_t b = __builtin_ctz(x);
                x &= x - 1u;
                if (at < kListStage) stage[at] = rj + b;
                else if (run + at < cap) list[run + at] = rj + b;
                ++at;
            }
        });
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint32_t ns = nb < kListStage ? nb : kListStage;
        for (uint32_t i = lane; i < ns; i += 64)
            if (run + i < cap) list[run + i] = stage[i];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();  // the stage is rewritten by the next batch
        run += nb;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();  // nz is reused by the wave's next tile
}

}  // namespace dqmc
