// Column passes: Merge / Reduce over a group of high digits (digit >= 13).
//
// These are the top-layer dimensions of Sec. 4.2: for digit i the triples
// are blocks at distance 3^(i-6) (eq. indexes), i.e. words at distance
// 8 * 3^(i-6), processed as a batch bit-slice over the 32 bit positions of a
// word at once.  Instead of one memory sweep per digit (Alg. 4), a pass takes
// a group of G = GR + GW consecutive digits g0.. and applies all of them
// while the data is on chip:
//
//   word index  w = l + L * (cr + 3^GR * (cw + 3^GW * o)),   L = 8 * 3^(g0-6)
//
// l (the word in a block and digits 6..g0-1) runs over consecutive words, one
// per lane, so every access of a wavefront is 64 consecutive words; cr (GR
// digits) indexes a lane's registers; cw (GW digits) is the wavefront within
// the workgroup; o is the combination of the digits above the group.  Digits
// of cr are transformed in registers, digits of cw through LDS.
#include "col_common.h"
#include "launch.h"
#include "h5.h"

namespace dqmc {

// Bit b set: binary wave combination b (bit r = digit r) is covered by the
// wave combination cw, i.e. agrees with it on every binary digit.
template <int GW>
__device__ __forceinline__ uint32_t binary_cover(int cw)
{
    uint32_t cover = 0;
    for (int b = 0; b < (1 << GW); ++b) {
        bool ok = true;
        int cc = cw;
        for (int r = 0; r < GW; ++r, cc /= 3) {
            const int d = cc % 3, bit = (b >> r) & 1;
            if (d != 2 && d != bit) ok = false;
        }
        cover |= ok ? (1u << b) : 0u;
    }
    return cover;
}

// The binary wave combinations in `cover` (a non-empty set of 2^s of them) as
// K LDS word offsets of their first exchange row (plus the lane), listed
// cyclically when fewer than K: AND being idempotent, a wavefront then reads
// K rows per register row at offsets fixed for the whole pass, with no
// per-row test of the cover (which the compiler turns into a branch and a
// wait for each LDS read).
template <int K, int BW>
__device__ __forceinline__ void cover_bases(uint32_t cover, uint32_t stride, uint32_t lane, uint32_t (&va)[K])
{
    const uint32_t m = (uint32_t)__builtin_popcount(cover);  // a power of two
    static_for<K>([&](auto ki) {
        const uint32_t want = (uint32_t)decltype(ki)::value & (m - 1u);
        uint32_t pick = 0, seen = 0;
        for (int b = 0; b < BW; ++b) {
            const bool on = (cover >> b) & 1u;
            pick = (on && seen == want) ? (uint32_t)b : pick;
            seen += on ? 1u : 0u;
        }
        va[decltype(ki)::value] = pick * stride + lane;
    });
}

// x &= ~M(w) on all 3^GR register rows, where w is the wave combination whose
// covered binary waves are `cover`: its binary rows are the AND of theirs (in
// xch, as the merge step left them) and its other rows follow by register
// merges.  Built one third of the top register digit at a time (top digit 0,
// 1, then * = the AND of the two) to hold 2 * 3^(GR-1) extra registers
// instead of 3^GR.  w differs from this wave in one binary digit, so it
// covers at most 2^(GW-1) binary waves.
template <int GR, int GW>
__device__ __forceinline__ void reduce_by_sibling(uint32_t (&x)[pow3(GR)], const uint32_t *xch, uint32_t cover,
                                                  uint32_t lane)
{
    constexpr int CL = (int)pow3(GR - 1);
    constexpr int BR = 1 << GR, BL = 1 << (GR - 1);
    constexpr int K = 1 << (GW - 1);
    uint32_t va[K];
    cover_bases<K, 1 << GW>(cover, BR * 64, lane, va);
    uint32_t y0[CL], y1[CL];
    static_for<CL>([&](auto ci) {
        constexpr int c = decltype(ci)::value;
        if constexpr (all_binary(c, GR - 1)) {
            uint32_t a0 = ~0u, a1 = ~0u;
            static_for<K>([&](auto ki) {
                a0 &= xch[va[decltype(ki)::value] + bin_index(c, GR - 1) * 64];
                a1 &= xch[va[decltype(ki)::value] + (BL + bin_index(c, GR - 1)) * 64];
            });
            y0[c] = a0;
            y1[c] = a1;
        }
    });
    reg_merge<GR - 1>(y0);
    reg_merge<GR - 1>(y1);
    static_for<CL>([&](auto ci) {
        constexpr int c = decltype(ci)::value;
        x[c] &= ~y0[c];
        x[c + CL] &= ~y1[c];
        x[c + 2 * CL] &= ~(y0[c] & y1[c]);
    });
}

// The reduce-only mode holds two workgroups of 3^GW waves per CU (its LDS
// exchange allows two), so its registers are capped for five waves per SIMD.
template <int GR, int GW, int MODE>
__global__ __launch_bounds__(col_threads<GW>())
__attribute__((amdgpu_waves_per_eu(MODE == kColReduce && GW == 2 ? 5 : 1))) void col_kernel(ColArgs a)
{
    constexpr int CR = (int)pow3(GR);
    constexpr int CW = (int)pow3(GW);
    constexpr int BR = 1 << GR;
    constexpr int BW = 1 << GW;
    constexpr int LANES = GW == 0 ? 256 : 64;
    constexpr bool NEED_MERGE = MODE != kColReduce;
    constexpr bool NEED_REDUCE = MODE != kColMerge;
    // LDS: merge exchange of binary waves' binary combos; the reduce-only
    // mode exchanges the star waves' full columns
    constexpr int XM = GW > 0 ? BW * BR * 64 : 1;
    // (one wave digit per round: the 3^(GW-1) waves whose digit r is *)
    constexpr int XR = (GW > 0 && !NEED_MERGE) ? (int)pow3(GW - 1) * CR * 64 : 1;
    constexpr int XSZ = XM > XR ? XM : XR;
    __shared__ uint32_t xch[XSZ];
    // merge+reduce with row flags: the block's 729 row bits
    constexpr bool WRITE_FLAGS = MODE == kColMergeReduce && GR == 4 && GW == 2;
    __shared__ uint32_t fl[WRITE_FLAGS ? kFlagWords : 1];
    if (WRITE_FLAGS && threadIdx.x < kFlagWords) fl[threadIdx.x] = 0u;  // ordered by the merge's barrier

    // grids stay below 2^32 workgroups: 32-bit division
    const uint32_t logical = (uint32_t)xcd_remap(blockIdx.x, a.nblocks), nlb = (uint32_t)a.nlb;
    const uint32_t lb = logical % nlb, ob = logical / nlb;
    uint64_t o = ob;
    if (a.outer_binary) {
        o = 0;
        uint64_t p = 1;
        for (uint64_t b = ob; b != 0; b >>= 1, p *= 3) o += (b & 1) * p;
    }
    // cw is uniform per wavefront; readfirstlane lets the row bases live in
    // scalar registers so that each access is (scalar base + lane offset)
    const int cw = GW == 0 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const uint32_t lane = GW == 0 ? threadIdx.x : (threadIdx.x & 63);
    const uint64_t L = a.L;
    uint64_t l64 = (uint64_t)lb * LANES + lane;
    bool active = l64 < L;
    if constexpr (GR == 4 && GW == 2) {
        if (a.slot_blocks != 0) {  // blocks cut per tile slot
            const uint32_t w = (lb % a.slot_blocks) * LANES + lane;
            l64 = (uint64_t)kTileStride * (lb / a.slot_blocks) + w;
            active = w < kTileStride;
        }
    }
    const uint32_t l = (uint32_t)l64;  // L < 2^32: plans keep g0 <= 24
    const uint32_t l4 = 4 * l;          // byte offset in a row (rows of the lanes' blocks are below 2^32 bytes)
    uint32_t *rows = a.state + L * (uint64_t)CR * ((uint64_t)cw + (uint64_t)CW * o);

    uint32_t x[CR];
    uint32_t live_pre[(CR + 31) / 32] = {};  // reduce mode with row flags: rows that may hold a bit
    bool cw_binary = true;
    if constexpr (GW > 0) {
        int c = cw;
        for (int r = 0; r < GW; ++r, c /= 3) cw_binary = cw_binary && (c % 3 != 2);
    }

    if constexpr (NEED_MERGE) {
        // 1. binary cubes of the group come from earlier passes
        static_for<CR>([&](auto ci) { x[decltype(ci)::value] = 0u; });
        if (cw_binary && active) {
            global_u32 *row = (global_u32 *)rows;
            static_for<CR>([&](auto ci) {
                constexpr int c = decltype(ci)::value;
                if constexpr (all_binary(c, GR)) x[c] = row_word(row, l4);
                row = next_row(row, L);
            });
        }
        // 2. wave digits: u = s AND t across wavefronts (on binary cr only)
        if constexpr (GW > 0) {
            if (cw_binary) {
                int bs = 0;
                {
                    int c = cw, p = 1;
                    for (int r = 0; r < GW; ++r, c /= 3, p <<= 1) bs += (c % 3) * p;
                }
                static_for<CR>([&](auto ci) {
                    constexpr int c = decltype(ci)::value;
                    if constexpr (all_binary(c, GR)) xch[(bs * BR + bin_index(c, GR)) * 64 + lane] = x[c];
                });
            }
            __syncthreads();
            if (!cw_binary) {
                // AND over the binary wave combinations covered by cw
                uint32_t va[BW];
                cover_bases<BW, BW>(binary_cover<GW>(cw), BR * 64, lane, va);
                static_for<CR>([&](auto ci) {
                    constexpr int c = decltype(ci)::value;
                    if constexpr (all_binary(c, GR)) {
                        uint32_t acc = ~0u;
                        static_for<BW>([&](auto ki) { acc &= xch[va[decltype(ki)::value] + bin_index(c, GR) * 64]; });
                        x[c] = acc;
                    }
                });
            }
        }
        // 3. register digits
        reg_merge<GR>(x);
        if constexpr (MODE == kColMerge) {
            // one branch per wave kind, none per row: per-row conditions on
            // cw_binary let the compiler merge stores of different rows into
            // one indexed load, which moves x to scratch memory
            global_u32 *row = (global_u32 *)rows;
            if (active && cw_binary) {
                static_for<CR>([&](auto ci) {
                    constexpr int c = decltype(ci)::value;
                    if constexpr (!all_binary(c, GR)) row_word(row, l4) = x[c];
                    row = next_row(row, L);
                });
            } else if (active) {
                static_for<CR>([&](auto ci) {
                    row_word(row, l4) = x[decltype(ci)::value];
                    row = next_row(row, L);
                });
            }
            return;
        }
    } else {
        // rows to load: all, or those the top group's pass flagged (the
        // others are zero in memory)
        uint32_t rf[3] = {~0u, ~0u, ~0u};
        if constexpr (GR == 4 && GW == 2) {
            if (a.flags != nullptr) {
                const uint32_t *fb = a.flags + (uint64_t)logical * kFlagWords;
                const uint32_t b0 = (uint32_t)(CR * cw), w0 = b0 / 32, sh = b0 % 32;
                uint32_t w[4];
                static_for<4>([&](auto ki) {
                    constexpr uint32_t k = decltype(ki)::value;
                    w[k] = w0 + k < kFlagWords ? fb[w0 + k] : 0u;
                });
                rf[0] = __builtin_amdgcn_alignbit(w[1], w[0], sh);
                rf[1] = __builtin_amdgcn_alignbit(w[2], w[1], sh);
                rf[2] = __builtin_amdgcn_alignbit(w[3], w[2], sh) & ((1u << (CR - 64)) - 1u);
            }
        }
        static_for<CR>([&](auto ci) { x[decltype(ci)::value] = 0u; });
        if (active) {
            global_u32 *row = (global_u32 *)rows;
            static_for<CR>([&](auto ci) {
                constexpr int c = decltype(ci)::value;
                if ((rf[c / 32] >> (c % 32)) & 1u) x[c] = row_word(row, l4);
                row = next_row(row, L);
            });
        }
        if constexpr (GR == 4 && GW == 2) {
            // with flags, the rows that may hold a bit are the flagged ones
            if (a.flags != nullptr) {
                live_pre[0] = rf[0];
                live_pre[1] = rf[1];
                live_pre[2] = rf[2];
            }
        }
    }
    // Reduce-only mode works in place and only clears bits: a row whose 64
    // words are all zero as loaded stays zero and is not stored again.
    uint32_t live[(CR + 31) / 32] = {};
    bool have_live = false;
    if constexpr (!NEED_MERGE && GR == 4 && GW == 2) {
        if (a.flags != nullptr) {
            static_for<(CR + 31) / 32>([&](auto ki) { live[decltype(ki)::value] = live_pre[decltype(ki)::value]; });
            have_live = true;
        }
    }
    if (!NEED_MERGE && !have_live) {
        static_for<CR>([&](auto ci) {
            constexpr int c = decltype(ci)::value;
            // packed now (a scalar word): otherwise the 81 ballots stay
            // live in scalar registers until the stores and spill
            live[c / 32] = __builtin_amdgcn_readfirstlane(live[c / 32] |
                                                          (__ballot(x[c] != 0u) != 0 ? 1u << (c % 32) : 0u));
            asm volatile("" : "+s"(live[c / 32]));
        });
    }

    if constexpr (NEED_REDUCE) {
        // 4. wave digits first, all against the star neighbours' values
        //    before any of this group's reduces (same as doing those
        //    dimensions one after another)
        if constexpr (GW > 0 && NEED_MERGE) {
            // Right after the merge x holds M itself.  By the merge identity
            // the star neighbour along wave digit r has M(self) AND M(sib),
            // sib being this wave with digit r flipped, so on any x <= M(self)
            // x AND NOT M(star) = x AND NOT M(sib).  The sibling's merged rows
            // follow from the binary rows still in xch: no second exchange
            // and no barrier before the stores.
            int cc = cw, p = 1;
            for (int r = 0; r < GW; ++r, cc /= 3, p *= 3) {
                const int d = cc % 3;
                if (d == 2) continue;
                static_assert(GR >= 1, "the sibling reduce splits the top register digit");
                const int sib = d == 0 ? cw + p : cw - p;
                reduce_by_sibling<GR, GW>(x, xch, binary_cover<GW>(sib), lane);
            }
        } else if constexpr (GW > 0) {
            // Reduce only: one wave digit per round.  The waves whose digit r
            // is * put their rows in LDS, the others clear what their star
            // neighbour holds.  Later rounds see the values earlier rounds
            // left (the dimensions reduced one after another, Alg. 3).
            int p = 1;
            for (int r = 0; r < GW; ++r, p *= 3) {
                const int d = (cw / p) % 3;
                // index of this wave among those with the same digits except r
                const int other = (cw / (p * 3)) * p + cw % p;
                if (r > 0) __syncthreads();  // the previous round's readers are done
                if (d == 2) {
                    static_for<CR>([&](auto ci) {
                        constexpr int c = decltype(ci)::value;
                        xch[(other * CR + c) * 64 + lane] = x[c];
                    });
                }
                __syncthreads();
                if (d != 2) {
                    static_for<CR>([&](auto ci) {
                        constexpr int c = decltype(ci)::value;
                        x[c] &= ~xch[(other * CR + c) * 64 + lane];
                    });
                }
            }
        }
        // 5. register digits, one after another
        reg_reduce<GR>(x);
        if (active) {
            const bool cw_allstar = (GW == 0) || (cw == CW - 1);
            global_u32 *row = (global_u32 *)rows;
            static_for<CR>([&](auto ci) {
                constexpr int c = decltype(ci)::value;
                if (MODE == kColMergeReduce || (!(cw_allstar && c == CR - 1) && ((live[c / 32] >> (c % 32)) & 1u)))
                    row_word(row, l4) = x[c];
                row = next_row(row, L);
            });
        }
        if constexpr (WRITE_FLAGS) {
            if (a.flags != nullptr) {
                // a bit per row with a set bit: this wave's rows c + 81 cw (a
                // bit per 32-word half would spare the reduce pass loads of
                // odd slots, but its bookkeeping cost the top pass more)
                uint32_t f[3] = {0u, 0u, 0u};
                static_for<CR>([&](auto ci) {
                    constexpr int c = decltype(ci)::value;
                    f[c / 32] = __builtin_amdgcn_readfirstlane(f[c / 32] |
                                                               (__ballot(x[c] != 0u) != 0 ? 1u << (c % 32) : 0u));
                    asm volatile("" : "+s"(f[c / 32]));
                });
                for (uint32_t i = lane; i < (uint32_t)CR; i += 64) {
                    const uint32_t fw = i < 32 ? f[0] : i < 64 ? f[1] : f[2];
                    if ((fw >> (i % 32)) & 1u) {
                        const uint32_t b = (uint32_t)(CR * cw) + i;
                        atomicOr(&fl[b / 32], 1u << (b % 32));
                    }
                }
                lds_barrier();
                if (threadIdx.x < kFlagWords) a.flags[(uint64_t)logical * kFlagWords + threadIdx.x] = fl[threadIdx.x];
            }
        }
    }
}

int col_lanes_per_block(int gw) { return gw == 0 ? 256 : 64; }

// Row flags of the top group's pass into the order of the reduce of digits
// 13..18 (n = 24, both groups of six digits).  An item is (ob, lb, wc): the
// reduce pass's outer combinations o = 32 ob .. 32 ob + 31, its column block
// lb, and its rows c = 32 wc .. 32 wc + 31.  Lane i of the item's 32 reads the
// top pass's flag word of its block (c, lb) for c = 32 wc + i (bits over o);
// 32 ballots transpose the 32 x 32 bits, and lane j writes the word of
// o = 32 ob + j (bits over c).  Two items per wavefront.
constexpr uint64_t kFlagItems = (uint64_t)kFlagWords * kFlagLowBlocks * kFlagWords;

__global__ __launch_bounds__(256) void flag_transpose_kernel(const uint32_t *top, uint32_t *low)
{
    const uint64_t item = ((uint64_t)blockIdx.x * 256 + threadIdx.x) / 32;
    const uint32_t i = threadIdx.x % 32;
    const bool valid = item < kFlagItems;
    const uint32_t wc = (uint32_t)(item % kFlagWords), lb = (uint32_t)(item / kFlagWords % kFlagLowBlocks);
    const uint32_t ob = (uint32_t)(item / (kFlagWords * kFlagLowBlocks));
    const uint32_t c = 32 * wc + i;
    uint32_t a = 0u;
    if (valid && c < 729u) a = top[((uint64_t)c * kFlagLowBlocks + lb) * kFlagWords + ob];
    const bool hi = (threadIdx.x % 64) >= 32;
    uint32_t out = 0u;
    for (uint32_t j = 0; j < 32; ++j) {
        const uint64_t m = __ballot((a >> j) & 1u);
        const uint32_t half = hi ? (uint32_t)(m >> 32) : (uint32_t)m;
        out = i == j ? half : out;
    }
    const uint32_t o = 32 * ob + i;
    if (valid && o < 729u) low[((uint64_t)o * kFlagLowBlocks + lb) * kFlagWords + wc] = out;
}

// The reduce pass's row flags, block (o, lb) holding a bit per slot c, as
// chunk flags of tile c + 729 o (bit lb).  An item is (o, cb, lw): slots
// c = 32 cb .. 32 cb + 31 and chunks lb = 32 lw .. 32 lw + 31; lane i reads
// the word of block (o, 32 lw + i), 32 ballots transpose, lane j writes word
// lw of tile 32 cb + j + 729 o.  Two items per wavefront.
constexpr uint64_t kTileFlagItems = 729ull * kFlagWords * kMapWords;

__global__ __launch_bounds__(256) void tile_flags_kernel(const uint32_t *low, uint32_t *tiles, uint32_t *deferred)
{
    // the final reduce's list of deferred tiles starts empty
    if (deferred != nullptr && blockIdx.x == 0 && threadIdx.x == 0) deferred[0] = 0u;
    const uint64_t item = ((uint64_t)blockIdx.x * 256 + threadIdx.x) / 32;
    const uint32_t i = threadIdx.x % 32;
    const bool valid = item < kTileFlagItems;
    const uint32_t lw = (uint32_t)(item % kMapWords), cb = (uint32_t)(item / kMapWords % kFlagWords);
    const uint32_t o = (uint32_t)(item / (kMapWords * kFlagWords));
    const uint32_t lb = 32 * lw + i;
    const uint32_t a = (valid && lb < kFlagLowBlocks) ? low[((uint64_t)o * kFlagLowBlocks + lb) * kFlagWords + cb] : 0u;
    const bool hi = (threadIdx.x % 64) >= 32;
    uint32_t out = 0u;
    for (uint32_t j = 0; j < 32; ++j) {
        const uint64_t m = __ballot((a >> j) & 1u);
        const uint32_t half = hi ? (uint32_t)(m >> 32) : (uint32_t)m;
        out = i == j ? half : out;
    }
    const uint32_t c = 32 * cb + i;
    if (valid && c < 729u) tiles[((uint64_t)o * 729 + c) * kMapWords + lw] = out;
}

hipError_t launch_tile_flags(const uint32_t *low, uint32_t *tiles, uint32_t *deferred, hipStream_t s)
{
    const uint64_t threads = kTileFlagItems * 32;
    hipLaunchKernelGGL(tile_flags_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s, low, tiles,
                       deferred);
    return hipGetLastError();
}

// Bytes of the flagged passes, from the flags: rows of the reduce of digits
// 13..18 (256 bytes, 128 in the last column block, whose upper 32 lanes lie
// past the slot), and per tile the runs of the final reduce that touch a
// flagged chunk (the same test as the kernels) and the flagged chunks.
__global__ __launch_bounds__(256) void flag_units_kernel(const uint32_t *low, const uint32_t *tiles,
                                                         unsigned long long *units)
{
    constexpr uint64_t nlow = 729ull * kFlagLowBlocks * kFlagWords;
    constexpr uint64_t ntiles = 531441;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long rows = 0, runs = 0, stores = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nlow; i += stride) {
        const uint32_t lb = (uint32_t)(i / kFlagWords % kFlagLowBlocks);
        rows += (unsigned long long)__popc(low[i]) * (lb + 1 == kFlagLowBlocks ? 128u : 256u);
    }
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += stride) {
        uint32_t f[kMapWords];
        static_for<kMapWords>([&](auto ki) { f[decltype(ki)::value] = tiles[t * kMapWords + decltype(ki)::value]; });
        auto bit = [&](uint32_t c) {
            uint32_t w = 0;
            static_for<kMapWords>([&](auto ki) { w = c / 32 == (uint32_t)decltype(ki)::value ? f[decltype(ki)::value] : w; });
            return (w >> (c % 32)) & 1u;
        };
        for (uint32_t q = 0; q < 729; ++q) runs += (bit(24 * q / 64) | bit((24 * q + 23) / 64)) ? 96u : 0u;
        // the final reduce stores the chunks non-zero as loaded, a subset of
        // the flagged ones (the last chunk holds 24 words)
        for (uint32_t k = 0; k < (uint32_t)kTileChunks; ++k)
            stores += bit(k) ? (k + 1 == (uint32_t)kTileChunks ? 96u : 256u) : 0u;
    }
    rows = wave_sum(rows);
    runs = wave_sum(runs);
    stores = wave_sum(stores);
    if (lane_id() == 0) {
        atomicAdd(&units[0], rows);
        atomicAdd(&units[1], runs);
        atomicAdd(&units[2], stores);
    }
}

hipError_t launch_flag_units(const uint32_t *low, const uint32_t *tiles, unsigned long long *units, hipStream_t s)
{
    hipLaunchKernelGGL(flag_units_kernel, dim3(2048), dim3(256), 0, s, low, tiles, units);
    return hipGetLastError();
}

hipError_t launch_flag_transpose(const uint32_t *top, uint32_t *low, hipStream_t s)
{
    const uint64_t threads = kFlagItems * 32;
    hipLaunchKernelGGL(flag_transpose_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s, top, low);
    return hipGetLastError();
}

// Dynamic LDS of the merge and merge+reduce passes with two wave digits: one
// workgroup per CU (n = 24: the top group's merge 14.1 -> 9.0 ms, the first
// group's 1.15 -> 0.80 ms).  The reduce-only mode holds one workgroup per CU
// through its own LDS exchange already.
static size_t g_merge42_pad = 0, g_mr42_pad = 0;

template <int GR, int GW>
static hipError_t launch_col_gw(int mode, const ColArgs &a, hipStream_t s)
{
    const dim3 grid((uint32_t)a.nblocks), block(col_threads<GW>());
    const size_t merge_pad = (GR == 4 && GW == 2) ? g_merge42_pad : 0;
    const size_t mr_pad = (GR == 4 && GW == 2) ? g_mr42_pad : 0;
    switch (mode) {
    case kColMerge: hipLaunchKernelGGL((col_kernel<GR, GW, kColMerge>), grid, block, merge_pad, s, a); break;
    case kColMergeReduce: hipLaunchKernelGGL((col_kernel<GR, GW, kColMergeReduce>), grid, block, mr_pad, s, a); break;
    case kColReduce: hipLaunchKernelGGL((col_kernel<GR, GW, kColReduce>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_col(int gr, int gw, int mode, const ColArgs &a, hipStream_t s)
{
    // groups with at most one wave digit use the chunked kernel (k_col_chunk.hip)
    if (gw <= 1) return launch_col_chunked(gr, gw, mode, a, s);
#define DQMC_COL(R, W) \
    if (gr == R && gw == W) return launch_col_gw<R, W>(mode, a, s);
    DQMC_COL(4, 2)
#undef DQMC_COL
    return hipErrorInvalidValue;
}

hipError_t col_setup()
{
    hipError_t e = occupancy_cap((const void *)col_kernel<4, 2, kColMerge>, 1, &g_merge42_pad);
    if (e == hipSuccess) e = occupancy_cap((const void *)col_kernel<4, 2, kColMergeReduce>, 1, &g_mr42_pad);
    if (e != hipSuccess) return e;
    return chunk_setup();
}

}  // namespace dqmc
