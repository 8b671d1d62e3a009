// Column passes, chunked form: the same Merge / Reduce passes over a group of
// high digits as k_col.hip (index layout and LDS exchange described there),
// with each lane's column processed in three chunks over its top register
// digit, so that 27 rows are in flight instead of 81.
#include "col_common.h"
#include "launch.h"
#include "h5.h"

namespace dqmc {

// The same passes with the column processed in three chunks over its top
// register digit (27 rows in flight instead of 81): used for groups with at
// most one wave digit, where it needs far fewer registers (n = 25, without
// occupancy caps: the merge of digits 18..21 in 6.5 ms instead of 9.3 ms).
// With two wave digits the whole-column kernel of k_col.hip is faster
// (n = 24: 10.3 ms against 12.8 ms for the top group), so it keeps those
// groups.
template <int GR, int GW, int MODE>
__global__ __launch_bounds__(col_threads<GW>()) void col_chunk_kernel(ColArgs a)
{
    constexpr int CR = (int)pow3(GR);
    constexpr int CW = (int)pow3(GW);
    constexpr int BR = 1 << GR;
    constexpr int BW = 1 << GW;
    // A column is processed in three chunks over its top register digit:
    // chunk k holds the CC combinations of the lower GR-1 register digits with
    // the top digit equal to k (register combination j + CC * k).
    constexpr int CC = (int)pow3(GR - 1);
    constexpr int BC = 1 << (GR - 1);
    constexpr int LANES = GW == 0 ? 256 : 64;
    constexpr bool NEED_MERGE = MODE != kColReduce;
    constexpr bool NEED_REDUCE = MODE != kColMerge;
    // LDS: binary waves' binary inputs (merge), star waves' chunk (reduce)
    constexpr int XM = GW > 0 ? BW * BR * 64 : 1;
    constexpr int XR = (GW > 0 && NEED_REDUCE) ? (CW - BW) * CC * 64 : 1;
    constexpr int XSZ = XM > XR ? XM : XR;
    __shared__ uint32_t xch[XSZ];

    const uint64_t logical = xcd_remap(blockIdx.x, a.nblocks);
    // grids stay below 2^32 workgroups: 32-bit division
    const uint32_t lb = (uint32_t)logical % (uint32_t)a.nlb, ob = (uint32_t)logical / (uint32_t)a.nlb;
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
    const uint64_t l64 = (uint64_t)lb * LANES + lane;
    const bool active = l64 < L;
    const uint32_t l = (uint32_t)l64;  // L < 2^32: plans keep g0 <= 24
    const uint32_t l4 = 4 * l;          // byte offset in a row
    uint32_t *rows = a.state + L * (uint64_t)CR * ((uint64_t)cw + (uint64_t)CW * o);
    // first row of chunk k (register combinations CC k .. CC k + CC - 1)
    auto chunk_rows = [&](int k) { return (global_u32 *)(rows + (uint64_t)(CC * k) * L); };

    bool cw_binary = true;
    if constexpr (GW > 0) {
        int c = cw;
        for (int r = 0; r < GW; ++r, c /= 3) cw_binary = cw_binary && (c % 3 != 2);
    }
    const bool cw_allstar = (GW == 0) || (cw == CW - 1);

    // binary inputs of the group (merge modes), by binary register index
    uint32_t bin[NEED_MERGE ? BR : 1];
    if constexpr (NEED_MERGE) {
        static_for<BR>([&](auto bi) {
            constexpr int b = decltype(bi)::value;
            constexpr int c = [] {  // register combination of binary index b
                int cc = 0, p = 1;
                for (int r = 0; r < GR; ++r, p *= 3) cc += ((b >> r) & 1) * p;
                return cc;
            }();
            bin[b] = (cw_binary && active) ? row_word((global_u32 *)(rows + (uint64_t)c * L), l4) : 0u;
        });
        // wave digits: u = s AND t across wavefronts, on the binary inputs
        if constexpr (GW > 0) {
            if (cw_binary) {
                int bs = 0;
                {
                    int c = cw, p = 1;
                    for (int r = 0; r < GW; ++r, c /= 3, p <<= 1) bs += (c % 3) * p;
                }
                static_for<BR>([&](auto bi) {
                    constexpr int b = decltype(bi)::value;
                    xch[(bs * BR + b) * 64 + lane] = bin[b];
                });
            }
            lds_barrier();
            if (!cw_binary) {
                uint32_t cover = 0;  // bit w set: binary wave w is covered by cw
                for (int w = 0; w < BW; ++w) {
                    bool ok = true;
                    int cc = cw;
                    for (int r = 0; r < GW; ++r, cc /= 3) {
                        const int d = cc % 3, bit = (w >> r) & 1;
                        if (d != 2 && d != bit) ok = false;
                    }
                    cover |= ok ? (1u << w) : 0u;
                }
                static_for<BR>([&](auto bi) {
                    constexpr int b = decltype(bi)::value;
                    uint32_t acc = ~0u;
                    for (int w = 0; w < BW; ++w)
                        if ((cover >> w) & 1u) acc &= xch[(w * BR + b) * 64 + lane];
                    bin[b] = acc;
                });
            }
        }
    }

    // Implicants of chunk k from the binary inputs: the top register digit
    // is merged first (chunk 2 = chunk 0 AND chunk 1 on binary inputs), then
    // the lower register digits.
    auto merged_chunk = [&](uint32_t(&y)[CC], auto ki) {
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
    };
    auto load_chunk = [&](uint32_t(&y)[CC], auto ki) {
        constexpr int k = decltype(ki)::value;
        static_for<CC>([&](auto ji) { y[decltype(ji)::value] = 0u; });
        if (!active) return;
        global_u32 *row = chunk_rows(k);
        static_for<CC>([&](auto ji) {
            y[decltype(ji)::value] = row_word(row, l4);
            row = next_row(row, L);
        });
    };
    // Wave digits of the group: every binary wave digit kills with the star
    // neighbour's value from before this group's reduces.
    auto wave_kill = [&](uint32_t(&y)[CC], bool sync_before) {
        if constexpr (GW > 0) {
            if (sync_before) lds_barrier();  // xch reuse
            if (!cw_binary) {
                const int ss = star_slot<GW>(cw);
                static_for<CC>([&](auto ji) {
                    constexpr int j = decltype(ji)::value;
                    xch[(ss * CC + j) * 64 + lane] = y[j];
                });
            }
            lds_barrier();
            int cc = cw, p = 1;
            for (int r = 0; r < GW; ++r, cc /= 3, p *= 3) {
                const int d = cc % 3;
                if (d == 2) continue;
                const int ss = star_slot<GW>(cw + (2 - d) * p);  // star neighbour in digit r
                static_for<CC>([&](auto ji) {
                    constexpr int j = decltype(ji)::value;
                    y[j] &= ~xch[(ss * CC + j) * 64 + lane];
                });
            }
        }
    };
    auto store_chunk = [&](const uint32_t(&y)[CC], auto ki, bool skip_binary, bool skip_allstar) {
        constexpr int k = decltype(ki)::value;
        if (!active) return;
        global_u32 *row = chunk_rows(k);
        static_for<CC>([&](auto ji) {
            constexpr int j = decltype(ji)::value;
            const bool bin_combo = k < 2 && all_binary(j, GR - 1);
            const bool star_combo = k == 2 && j == CC - 1;
            if (!(skip_binary && bin_combo) && !(skip_allstar && star_combo)) row_word(row, l4) = y[j];
            row = next_row(row, L);
        });
    };
    constexpr std::integral_constant<int, 0> K0{};
    constexpr std::integral_constant<int, 1> K1{};
    constexpr std::integral_constant<int, 2> K2{};

    if constexpr (MODE == kColMerge) {
        // write every combination with a * (binary ones hold the inputs)
        uint32_t y[CC];
        merged_chunk(y, K0);
        store_chunk(y, K0, cw_binary, false);
        merged_chunk(y, K1);
        store_chunk(y, K1, cw_binary, false);
        merged_chunk(y, K2);
        store_chunk(y, K2, false, false);
    } else {
        // Reduce in the order: wave digits, lower register digits, top
        // register digit.  Chunk 2 (top digit *) first; it is kept for the
        // top-digit kill of chunks 0 and 1.
        const bool skip_allstar = MODE == kColReduce && cw_allstar;
        uint32_t y2[CC];
        if constexpr (NEED_MERGE) merged_chunk(y2, K2);
        else load_chunk(y2, K2);
        wave_kill(y2, NEED_MERGE);
        reg_reduce<GR - 1>(y2);
        store_chunk(y2, K2, false, skip_allstar);
        static_for<2>([&](auto ki) {
            uint32_t y[CC];
            if constexpr (NEED_MERGE) merged_chunk(y, ki);
            else load_chunk(y, ki);
            wave_kill(y, true);
            reg_reduce<GR - 1>(y);
            static_for<CC>([&](auto ji) {
                constexpr int j = decltype(ji)::value;
                y[j] &= ~y2[j];
            });
            store_chunk(y, ki, false, false);
        });
    }
}

// Dynamic LDS per mode for the four-register-digit groups (the large ones),
// set by chunk_setup to cap the workgroups per CU.  Measured at n = 25
// (state 125.5 GB): with no wave digit, two workgroups per CU (merge+reduce
// of digits 22..25 37.4 -> 28.6 ms, reduce of 18..21 45.7 -> 42.9 ms, merge
// of 18..21 6.5 -> 5.1 ms); with one wave digit, two per CU for the merge
// modes (1.41 -> 0.99 ms for digits 13..17) and three for the reduce
// (44.9 -> 43.1 ms).
static size_t g_pad40[3] = {0, 0, 0};
static size_t g_pad41[3] = {0, 0, 0};

template <int GR, int GW>
static hipError_t launch_chunk_gw(int mode, const ColArgs &a, hipStream_t s)
{
    const dim3 grid((uint32_t)a.nblocks), block(col_threads<GW>());
    const size_t pad = GR != 4 ? 0 : GW == 0 ? g_pad40[mode] : g_pad41[mode];
    switch (mode) {
    case kColMerge: hipLaunchKernelGGL((col_chunk_kernel<GR, GW, kColMerge>), grid, block, pad, s, a); break;
    case kColMergeReduce: hipLaunchKernelGGL((col_chunk_kernel<GR, GW, kColMergeReduce>), grid, block, pad, s, a); break;
    case kColReduce: hipLaunchKernelGGL((col_chunk_kernel<GR, GW, kColReduce>), grid, block, pad, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t chunk_setup()
{
    const struct {
        const void *k;
        int wgs;
        size_t *pad;
    } caps[] = {
        {(const void *)col_chunk_kernel<4, 0, kColMerge>, 2, &g_pad40[kColMerge]},
        {(const void *)col_chunk_kernel<4, 0, kColMergeReduce>, 2, &g_pad40[kColMergeReduce]},
        {(const void *)col_chunk_kernel<4, 0, kColReduce>, 2, &g_pad40[kColReduce]},
        {(const void *)col_chunk_kernel<4, 1, kColMerge>, 2, &g_pad41[kColMerge]},
        {(const void *)col_chunk_kernel<4, 1, kColMergeReduce>, 2, &g_pad41[kColMergeReduce]},
        {(const void *)col_chunk_kernel<4, 1, kColReduce>, 3, &g_pad41[kColReduce]},
    };
    for (const auto &c : caps) {
        const hipError_t e = occupancy_cap(c.k, c.wgs, c.pad);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_col_chunked(int gr, int gw, int mode, const ColArgs &a, hipStream_t s)
{
#define DQMC_COLC(R, W) \
    if (gr == R && gw == W) return launch_chunk_gw<R, W>(mode, a, s);
    DQMC_COLC(1, 0)
    DQMC_COLC(2, 0)
    DQMC_COLC(3, 0)
    DQMC_COLC(4, 0)
    DQMC_COLC(4, 1)
#undef DQMC_COLC
    return hipErrorInvalidValue;
}

}  // namespace dqmc
