// Helpers shared by the two forms of the column passes (k_col.hip,
// k_col_chunk.hip).
#pragma once

#include "t27.h"

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

template <int GW>
__host__ __device__ constexpr int col_threads()
{
    return GW == 0 ? 256 : 64 * (int)pow3(GW);
}

}  // namespace dqmc
