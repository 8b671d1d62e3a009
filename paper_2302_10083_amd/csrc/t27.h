// T27 state layout and the per-dimension Merge/Reduce transforms on it.
//
// A state is the indicator of a set of ternary cubes (Sec. 4.1, "State
// representation").  Cube rho (Sec. 4.2, notation rho: digit i of rho is the
// symbol s_i, with * = 2) lives in 32-bit word rho / 27, bit rho % 27.  So the
// three lowest ternary digits are inside a word ("bottom layer" of Sec. 4.2
// with h = 3 and 27 of 32 bits used) and digit i >= 4 moves the word index by
// 3^(i-4) ("top layer").  Word bits 27..31 are always 0.  For n < 3 the state
// is one word holding bits 0..3^n-1.
//
// Merge (Sec. 4.1, Def. of Merge) for dimension i maps the triple of cubes
// (s, t, u) with s_i = 0, t_i = 1, u_i = * and equal elsewhere to
// (s, t, u OR (s AND t)).  When every dimension is merged exactly once,
// starting from the indicator of the support, u is still 0 when its own
// dimension is merged, so the step is u = s AND t.
// Reduce (Sec. 4.1, Def. of Reduce) maps it to (s AND NOT u, t AND NOT u, u).
// Both may be applied dimension by dimension in any order (Sec. 4.1, the
// proposition equating Alg. 2 and Alg. 3, and the reordering used for the
// fused bottom layers in Sec. 6), merges first, then reduces.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace dqmc {

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0..N-1, so that
// register arrays are only ever indexed by constants.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}

template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Bits of a word whose in-word digit 1 / 2 / 3 is 0 (the masks mu_i of
// Sec. 4.2 for h = 3).
constexpr uint32_t kMu1 = 0x1249249u;
constexpr uint32_t kMu2 = 0x1C0E07u;
constexpr uint32_t kMu3 = 0x1FFu;

__host__ __device__ constexpr uint64_t pow3(int k)
{
    uint64_t r = 1;
    for (int i = 0; i < k; ++i) r *= 3;
    return r;
}

__host__ __device__ constexpr int tdigit(int c, int r)
{
    return (int)((uint64_t)c / pow3(r) % 3);
}

// True if no digit of combination c (base 3, k digits) equals 2.
__host__ __device__ constexpr bool all_binary(int c, int k)
{
    for (int r = 0; r < k; ++r)
        if (tdigit(c, r) == 2) return false;
    return true;
}

// True if digits r+1..k-1 of c are all binary.
__host__ __device__ constexpr bool binary_above(int c, int r, int k)
{
    for (int q = r + 1; q < k; ++q)
        if (tdigit(c, q) == 2) return false;
    return true;
}

// Binary index sum_r digit_r 2^r of an all-binary combination c.
__host__ __device__ constexpr int bin_index(int c, int k)
{
    int b = 0;
    for (int r = 0; r < k; ++r) b |= tdigit(c, r) << r;
    return b;
}

// Merge of the three in-word dimensions on a word whose set bits are all at
// cubes without * in those digits.
__device__ __forceinline__ uint32_t inword_merge(uint32_t v)
{
    v |= ((v & (v >> 1)) & kMu1) << 2;
    v |= ((v & (v >> 3)) & kMu2) << 6;
    v |= ((v & (v >> 9)) & kMu3) << 18;
    return v;
}

// Reduce of the three in-word dimensions (in place, one after the other).
__device__ __forceinline__ uint32_t inword_reduce(uint32_t v)
{
    uint32_t k;
    k = (v >> 2) & kMu1;
    v &= ~(k | (k << 1));
    k = (v >> 6) & kMu2;
    v &= ~(k | (k << 3));
    k = (v >> 18) & kMu3;
    v &= ~(k | (k << 9));
    return v;
}

// Truth-table byte (f at x = 8m + j, j = x_1 + 2 x_2 + 4 x_3) placed at the
// T27 positions x_1 + 3 x_2 + 9 x_3 of the cubes without * in digits 1..3.
__device__ __forceinline__ uint32_t expand_byte(uint32_t byte)
{
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        v |= ((byte >> j) & 1u) << ((j & 1) + 3 * ((j >> 1) & 1) + 9 * ((j >> 2) & 1));
    return v;
}

// Merge of K dimensions on a register column x[c], c = sum_r digit_r 3^r,
// where x[c] = 0 for every c with a digit 2.  Dimension r is merged on the
// combinations whose higher digits are still binary; the others are filled
// when their own higher dimension is merged.
template <int K>
__device__ __forceinline__ void reg_merge(uint32_t (&x)[pow3(K)])
{
    static_for<K>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        static_for<(int)pow3(K)>([&](auto ci) {
            constexpr int c = decltype(ci)::value;
            if constexpr (tdigit(c, r) == 2 && binary_above(c, r, K))
                x[c] = x[c - 2 * (int)pow3(r)] & x[c - (int)pow3(r)];
        });
    });
}

// Reduce of K dimensions on a register column, one dimension after another.
template <int K>
__device__ __forceinline__ void reg_reduce(uint32_t (&x)[pow3(K)])
{
    static_for<K>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        static_for<(int)pow3(K)>([&](auto ci) {
            constexpr int c = decltype(ci)::value;
            constexpr int d = tdigit(c, r);
            if constexpr (d != 2) x[c] &= ~x[c + (2 - d) * (int)pow3(r)];
        });
    });
}

// ---------------------------------------------------------------------------
// wavefront helpers (64 lanes)

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// orders global memory, which makes every wave wait for all of its
// outstanding global loads and stores first; where a barrier only guards LDS
// that wait would expose the latency of stores issued just before it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint64_t wave_inclusive_scan(uint64_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t o = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += o;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan32(uint32_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += o;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Block index -> logical tile with consecutive logical tiles on one XCD.
// Workgroups are dispatched round-robin over the 8 XCDs; keeping neighbouring
// tiles on one XCD lets its L2 absorb the 128-byte lines they share.
__device__ __forceinline__ uint64_t xcd_remap(uint64_t b, uint64_t nb)
{
    constexpr uint64_t X = 8;
    const uint64_t q = nb / X, rem = nb % X;
    const uint64_t xcd = b % X, slot = b / X;
    return (xcd < rem) ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

}  // namespace dqmc
