// Kernels of the sliced path: functions with more variables than one state
// can hold, cut along their top t variables.
//
// For a cube a over the top t variables (each digit 0, 1 or *), let f_a be
// the function of the lower m = n - t variables that is the AND of f over the
// minterms of a.  A cube (s, a) is an implicant of f exactly when s is an
// implicant of f_a, so the Merge transform of Sec. 4.1 restricted to slice a
// is the whole MergeAll of f_a.  In the one-step form of ReduceAll (Sec. 4.1,
// Lemma) the low digits give the primes of f_a, and a top digit j with a_j
// binary removes (s, a) when (s, a[j <- *]) is an implicant.  So
//     O(f)[s, a] = O(f_a)[s] AND NOT OR_{j: a_j binary} M(f_{a[j <- *]})[s],
// which needs two slice-sized states at a time: O(f_a) and one M.
#include <algorithm>

#include "launch.h"
#include "h5.h"

namespace dqmc {

// Truth table of f_a: `fixed` holds the top-variable bits where a is 1,
// `stars` the bits where a is *.  flip is XORed into the input words first
// (the complement mode).
__global__ __launch_bounds__(256) void slice_tt_kernel(const uint32_t *tt, int m, uint32_t fixed, uint32_t stars,
                                                       uint32_t flip, uint32_t *out)
{
    if (m >= 5) {
        const uint64_t words = 1ull << (m - 5);
        const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
        for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += step) {
            uint32_t acc = ~0u, sub = 0u;
            do {  // every subset of the * bits
                acc &= tt[((uint64_t)(fixed | sub) << (m - 5)) + w] ^ flip;
                sub = (sub - stars) & stars;
            } while (sub != 0u);
            out[w] = acc;
        }
    } else if (blockIdx.x == 0 && threadIdx.x == 0) {
        uint32_t o = 0u;
        for (uint32_t x = 0; x < (1u << m); ++x) {
            uint32_t b = 1u, sub = 0u;
            do {
                const uint64_t X = x + ((uint64_t)(fixed | sub) << m);
                b &= ((tt[X >> 5] ^ flip) >> (X & 31)) & 1u;
                sub = (sub - stars) & stars;
            } while (sub != 0u);
            o |= b << x;
        }
        out[0] = o;
    }
}

hipError_t launch_slice_tt(const uint32_t *tt, int m, uint32_t fixed, uint32_t stars, uint32_t flip, uint32_t *out,
                           hipStream_t s)
{
    const uint64_t words = m >= 5 ? (1ull << (m - 5)) : 1;
    const uint64_t blocks = std::min<uint64_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(slice_tt_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, tt, m, fixed, stars, flip, out);
    return hipGetLastError();
}

// o &= ~mask on the chunks that the tile summary marks non-zero, and a new
// summary (count and chunk map) of the result.  One workgroup per tile; the
// chunks outside the map are zero in o and are not read.  The marked chunks
// are listed first, so that each wavefront can keep kAndNotBatch of them
// (two loads each) in flight.
constexpr int kAndNotThreads = 256;
constexpr int kAndNotBatch = 8;

__global__ __launch_bounds__(kAndNotThreads) void andnot_map_kernel(uint32_t *o, const uint32_t *mask,
                                                                     uint32_t *counts, uint32_t *chunkmap, uint32_t tw,
                                                                     uint32_t ts)
{
    constexpr uint32_t NW = kAndNotThreads / 64;
    __shared__ uint32_t red[kMapWords + 1];
    __shared__ uint16_t nz[kTileChunks];
    __shared__ uint32_t nnz;
    const uint64_t tile = blockIdx.x;
    if (counts[tile] == 0u) return;  // nothing set, and the map is already empty
    const uint32_t wv = threadIdx.x / 64, lane = lane_id();
    if (threadIdx.x < (uint32_t)kMapWords + 1) red[threadIdx.x] = 0u;
    if (wv == 0) {
        const uint32_t mw = lane < (uint32_t)kMapWords ? chunkmap[tile * kMapWords + lane] : 0u;
        const uint32_t pc = __popc(mw);
        const uint32_t incl = wave_inclusive_scan32(pc);
        uint32_t pos = incl - pc, bits = mw;
        while (bits != 0u) {
            const uint32_t b = __builtin_ctz(bits);
            bits &= bits - 1u;
            nz[pos++] = (uint16_t)(lane * 32 + b);
        }
        if (lane == 63) nnz = incl;
    }
    __syncthreads();
    const uint32_t total = nnz;
    uint32_t *ot = o + tile * ts;
    const uint32_t *mt = mask + tile * ts;
    uint32_t c = 0;
    for (uint32_t r0 = wv * kAndNotBatch; r0 < total; r0 += NW * kAndNotBatch) {
        uint32_t ov[kAndNotBatch], mv[kAndNotBatch];
        static_for<kAndNotBatch>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const uint32_t w = r0 + i < total ? (uint32_t)nz[r0 + i] * kChunkWords + lane : tw;
            ov[i] = w < tw ? ot[w] : 0u;
            mv[i] = w < tw ? mt[w] : 0u;
        });
        static_for<kAndNotBatch>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            if (r0 + i < total) {
                const uint32_t k = nz[r0 + i];
                const uint32_t w = k * kChunkWords + lane;
                const uint32_t x = ov[i] & ~mv[i];
                if (x != ov[i]) ot[w] = x;  // only words with a set bit of o
                c += __popc(x);
                if (__ballot(x != 0u) != 0 && lane == 0) atomicOr(&red[1 + (k >> 5)], 1u << (k & 31));
            }
        });
    }
    c = wave_sum32(c);
    if (lane == 0) atomicAdd(&red[0], c);
    __syncthreads();
    if (threadIdx.x == 0) counts[tile] = red[0];
    if (threadIdx.x < (uint32_t)kMapWords) chunkmap[tile * kMapWords + threadIdx.x] = red[1 + threadIdx.x];
}

hipError_t launch_andnot_map(uint32_t *o, const uint32_t *mask, uint32_t *counts, uint32_t *chunkmap, uint64_t ntiles,
                             uint32_t tw, uint32_t ts, hipStream_t s)
{
    hipLaunchKernelGGL(andnot_map_kernel, dim3((uint32_t)ntiles), dim3(kAndNotThreads), 0, s, o, mask, counts,
                       chunkmap, tw, ts);
    return hipGetLastError();
}

}  // namespace dqmc
