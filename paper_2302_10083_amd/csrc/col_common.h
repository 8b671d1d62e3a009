// Helpers shared by the two forms of the column passes (k_col.hip,
// k_col_chunk.hip).
#pragma once

#include "h5.h"

namespace dqmc {

// Position of wave combination cw among the non-binary combinations.
template <int GW>
__device__ __forceinline__ int star_slot(int cw)
{
    int k = 0;
    for (int c = 0; c < cw; ++c) {
        int q = c;
        bool b = true;
        for (int r = 0; r < GW; ++r, q /= 3) b = b && (q % 3 != 2);
        k += b ? 0 : 1;
    }
    return k;
}

// The next row of a column: rows are L words apart, and a column's rows are
// visited in order, so each costs one 64-bit scalar add.  The empty asm keeps
// the compiler from rewriting the chain into products c * L (a 64-bit
// multiply of a runtime value per row).
// The walk runs on a global-address-space pointer, so that the accesses stay
// global loads and stores (scalar base + lane offset), not flat ones.
typedef __attribute__((address_space(1))) uint32_t global_u32;

__device__ __forceinline__ global_u32 *next_row(global_u32 *row, uint64_t L)
{
    row += L;
    asm volatile("" : "+s"(row));
    return row;
}

// Word of a row at byte offset off (32 bits: scalar base + lane offset).
__device__ __forceinline__ global_u32 &row_word(global_u32 *row, uint32_t off)
{
    return *(global_u32 *)((__attribute__((address_space(1))) char *)row + off);
}

template <int GW>
__host__ __device__ constexpr int col_threads()
{
    return GW == 0 ? 256 : 64 * (int)pow3(GW);
}

// Occupancy caps.  A column pass writes 256-byte row segments that start at
// multiples of 8 * 3^(g0-6) words, off the 128-byte lines, so the lines at their
// edges are shared with the neighbouring blocks.  Stores of that shape run
// faster with few workgroups per CU (a store-only probe on MI355X: 4.9 TB/s
// at one workgroup per CU, 2.6 TB/s at full occupancy), and so do several of
// the passes, with fewer workgroups than registers and LDS would allow.  A
// launch enforces its cap by asking for unused dynamic LDS: at most `wgs`
// workgroups of (static + dynamic) LDS fit in the 160 KB of a CU.
inline size_t lds_bytes_for_cap(int wgs)
{
    return wgs <= 1 ? 88 * 1024 : wgs == 2 ? 64 * 1024 : 48 * 1024;
}

// Dynamic LDS that caps `kernel` at `wgs` workgroups per CU (0: no cap),
// with the kernel's dynamic-LDS limit raised to match.
inline hipError_t occupancy_cap(const void *kernel, int wgs, size_t *pad)
{
    *pad = 0;
    if (wgs <= 0) return hipSuccess;
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, kernel);
    if (e != hipSuccess) return e;
    const size_t want = lds_bytes_for_cap(wgs);
    if (fa.sharedSizeBytes >= want) return hipSuccess;
    *pad = want - fa.sharedSizeBytes;
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)*pad);
}

}  // namespace dqmc
