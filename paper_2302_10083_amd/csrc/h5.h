// Block state layout ("H5") and the per-dimension Merge/Reduce transforms on
// it.
//
// A state is the indicator of a set of ternary cubes (Sec. 4.1, "State
// representation").  Cube rho (Sec. 4.2, notation rho: digit i of rho is the
// symbol s_i, with * = 2) lives in 256-bit block rho / 243, at bit
// p = rho % 243 of the block; a block is 8 consecutive uint32 words and bit p
// is bit p % 32 of its word p / 32.  So the five lowest ternary digits are
// inside a block (the bottom layer of Sec. 4.2 with h = 5: 243 of 256 bits
// used, the paper's own AVX2 choice), and digit i >= 6 moves the block index
// by 3^(i-6), i.e. the logical word index by 8 * 3^(i-6) (the top layer).
// Bits 243..255 of a block (bits 19..31 of its last word) are always 0.  For
// n < 5 the state is one block holding bits 0..3^n-1.  For n > 12 the blocks
// of each value of digits 13..n (a tile of 3^7 blocks) sit in a slot of
// kTileStride words whose last 8 words are 0, so digit i >= 13 moves the word
// index by kTileStride * 3^(i-13).  Memory order is rho order.
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

constexpr int kBlockWords = 8;     // uint32 words per block
constexpr int kBlockCubes = 243;   // cubes per block (3^5)
constexpr int kBlockDigits = 5;    // digits inside a block

// Word w of the mask mu_i (Sec. 4.2) for the in-block digit i (0-based):
// bits p = 32 w + b < 243 whose digit i is 0.
__host__ __device__ constexpr uint32_t block_mu(int i, int w)
{
    uint32_t m = 0;
    for (int b = 0; b < 32; ++b) {
        const uint64_t p = 32u * (uint32_t)w + (uint32_t)b;
        if (p < (uint64_t)kBlockCubes && (p / pow3(i)) % 3 == 0) m |= 1u << b;
    }
    return m;
}

// 256-bit shifts of a block held in 8 registers (word 0 = bits 0..31).
template <int K>
__device__ __forceinline__ void block_shr(const uint32_t (&v)[kBlockWords], uint32_t (&o)[kBlockWords])
{
    constexpr int q = K / 32, r = K % 32;
    static_for<kBlockWords>([&](auto wi) {
        constexpr int w = decltype(wi)::value;
        if constexpr (w + q >= kBlockWords) o[w] = 0u;
        else if constexpr (r == 0) o[w] = v[w + q];
        else if constexpr (w + q + 1 >= kBlockWords) o[w] = v[w + q] >> r;
        else o[w] = __builtin_amdgcn_alignbit(v[w + q + 1], v[w + q], (uint32_t)r);
    });
}

template <int K>
__device__ __forceinline__ void block_shl(const uint32_t (&v)[kBlockWords], uint32_t (&o)[kBlockWords])
{
    constexpr int q = K / 32, r = K % 32;
    static_for<kBlockWords>([&](auto wi) {
        constexpr int w = decltype(wi)::value;
        if constexpr (w - q < 0) o[w] = 0u;
        else if constexpr (r == 0) o[w] = v[w - q];
        else if constexpr (w - q - 1 < 0) o[w] = v[w - q] << r;
        else o[w] = __builtin_amdgcn_alignbit(v[w - q], v[w - q - 1], (uint32_t)(32 - r));
    });
}

// Merge of the five in-block dimensions on a block whose set bits are all at
// cubes without * in those digits: u = s AND t, with s at bit p (digit i of p
// is 0), t at p + 3^i and u at p + 2 * 3^i.
__device__ __forceinline__ void block_merge(uint32_t (&v)[kBlockWords])
{
    static_for<kBlockDigits>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        constexpr int S = (int)pow3(i);
        uint32_t a[kBlockWords], b[kBlockWords];
        block_shr<S>(v, a);
        static_for<kBlockWords>([&](auto wi) {
            constexpr int w = decltype(wi)::value;
            a[w] &= v[w] & block_mu(i, w);
        });
        block_shl<2 * S>(a, b);
        static_for<kBlockWords>([&](auto wi) {
            constexpr int w = decltype(wi)::value;
            v[w] |= b[w];
        });
    });
}

// Reduce of the five in-block dimensions (in place, one after the other).
__device__ __forceinline__ void block_reduce(uint32_t (&v)[kBlockWords])
{
    static_for<kBlockDigits>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        constexpr int S = (int)pow3(i);
        uint32_t a[kBlockWords], b[kBlockWords];
        block_shr<2 * S>(v, a);  // the * cube's bit, at its digit-0 sibling
        static_for<kBlockWords>([&](auto wi) {
            constexpr int w = decltype(wi)::value;
            a[w] &= block_mu(i, w);
        });
        block_shl<S>(a, b);  // and at its digit-1 sibling
        static_for<kBlockWords>([&](auto wi) {
            constexpr int w = decltype(wi)::value;
            v[w] &= ~(a[w] | b[w]);
        });
    });
}

// Cube position x_1 + 3 x_2 + 9 x_3 + 27 x_4 + 81 x_5 of the minterm
// j = x_1 + 2 x_2 + 4 x_3 + 8 x_4 + 16 x_5 inside a block.
__host__ __device__ constexpr int block_pos(int j)
{
    int p = 0;
    for (int r = 0; r < kBlockDigits; ++r) p += ((j >> r) & 1) * (int)pow3(r);
    return p;
}

// Truth-table word (f at x = 32 m + j) placed at the positions of its 32
// minterms in a block (the cubes without * in digits 1..5).
__device__ __forceinline__ void block_from_tt(uint32_t x, uint32_t (&v)[kBlockWords])
{
    static_for<kBlockWords>([&](auto wi) { v[decltype(wi)::value] = 0u; });
    static_for<32>([&](auto ji) {
        constexpr int j = decltype(ji)::value;
        constexpr int p = block_pos(j);
        v[p / 32] |= ((x >> j) & 1u) << (p % 32);
    });
}

// Cube index of bit 0 of state word `w` (word w % 8 of block w / 8).
__host__ __device__ __forceinline__ uint64_t rho_of_word(uint64_t w)
{
    return (uint64_t)kBlockCubes * (w >> 3) + 32u * (uint32_t)(w & 7u);
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

// Number of digits of combination c (base 3, k digits) that are 2 (*).
__host__ __device__ constexpr int star_count(int c, int k)
{
    int s = 0;
    for (int r = 0; r < k; ++r) s += tdigit(c, r) == 2 ? 1 : 0;
    return s;
}

// Reduce of K dimensions on a register column in one step (the Lemma of
// Sec. 4.1 applied to the K dimensions): combination c loses every bit that
// one of its star neighbours c[r <- *] (r over the digits of c that are not
// *) holds at the start.  Combinations are visited by increasing number of
// stars, so a neighbour (one star more) still holds its starting value when
// it is read.  On a column that is M with some other dimensions already
// reduced, this equals reducing the K dimensions one after another: a bit
// that a neighbour lost to one of those other dimensions is lost by c to the
// same dimension (the larger cube contains c's extension).  Two neighbours
// fold into one three-input bit operation.
template <int K>
__device__ __forceinline__ void reg_reduce(uint32_t (&x)[pow3(K)])
{
    static_for<K>([&](auto si) {
        constexpr int s = decltype(si)::value;
        static_for<(int)pow3(K)>([&](auto ci) {
            constexpr int c = decltype(ci)::value;
            if constexpr (star_count(c, K) == s) {
                uint32_t kill = 0u;
                static_for<K>([&](auto ri) {
                    constexpr int r = decltype(ri)::value;
                    constexpr int d = tdigit(c, r);
                    if constexpr (d != 2) kill |= x[c + (2 - d) * (int)pow3(r)];
                });
                x[c] &= ~kill;
            }
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
