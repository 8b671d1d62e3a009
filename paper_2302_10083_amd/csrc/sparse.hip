// Sparse path: the classic level-by-level Quine-McCluskey algorithm with the
// optimisations of Sec. 5 (Alg. 1 driven by hash-based neighbour search).
//
// A cube is a 2n-bit key, two bits per variable in string order (variable
// x_{i+1} at bits 2i, 2i+1): 00 = 0, 01 = 1, 10 = * (Sec. 5, bit-based
// representation).  Level w holds every implicant with w stars, as a compact
// list (for sequential sweeps) and an open-addressing hash set with linear
// probing (for neighbour lookups).  Step w:
//   1. generation: an implicant c of level w-1 whose first star is at
//      position f is merged only on positions p < f where c_p = 0, with its
//      partner c[p <- 1] looked up in the set; u = c[p <- *] is appended to
//      level w.  Every implicant of level w arises exactly once this way (at
//      its first star), so the list needs no deduplication (Sec. 5, avoiding
//      repeated implicant generation);
//   2. the hash set of level w is built from the list;
//   3. marking: for every u of level w and every star q of u, both halves
//      u[q <- 0] and u[q <- 1] get the redundant control bit in the set of
//      level w-1 (the extra pass over the new implicants of Sec. 5);
//   4. the unmarked entries of level w-1 are its prime implicants
//      (Sec. 5, two-stage custom hash set: elements are marked, never removed).
// The primes are finally converted to cube indices rho and sorted (a radix
// sort of their own, below), so the output is the same list as the dense
// path's.
#include <stdio.h>

#include <algorithm>
#include <vector>

#include "api_types.h"
#include "dqmc.h"
#include "h5.h"
#include "launch.h"

namespace dqmc {

constexpr uint64_t kEmpty = ~0ull;          // never a key: 11 is not a symbol
constexpr uint64_t kRedundant = 1ull << 63;  // control bit of a stored key
constexpr int kSpThreads = 256;

// Slot hash of a key: the "Mix01" variant of the MurmurHash3 64-bit finaliser
// (shifts 31, 27, 33 and the two multipliers of D. Stafford, "Better Bit
// Mixing - Improving on MurmurHash3's 64-bit Finalizer", 2011).
__device__ __forceinline__ uint64_t sp_hash(uint64_t k)
{
    k = (k ^ (k >> 31)) * 0x7FB5D329728EA185ULL;
    k = (k ^ (k >> 27)) * 0x81DADEF4BC2DD44DULL;
    return k ^ (k >> 33);
}

// Minterm x (n <= 31 bits) -> key with pair 0b0v at each position.
__device__ __forceinline__ uint64_t sp_spread(uint64_t x)
{
    x &= 0xFFFFFFFFull;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

__device__ __forceinline__ bool sp_find(const uint64_t *table, uint64_t mask, uint64_t key, uint64_t *slot)
{
    uint64_t h = sp_hash(key) & mask;
    for (;;) {
        const uint64_t v = table[h];
        if (v == kEmpty) return false;
        if ((v & ~kRedundant) == key) {
            *slot = h;
            return true;
        }
        h = (h + 1) & mask;
    }
}

// Space for `mine` entries per thread, reserved with one atomic per
// workgroup: returns this thread's first position.  Every thread of the
// workgroup must call it (loops have workgroup-uniform trip counts).
__device__ __forceinline__ uint64_t block_reserve(uint32_t mine, unsigned long long *counter)
{
    __shared__ uint32_t wsum[kSpThreads / 64];
    __shared__ unsigned long long bbase;
    const uint32_t wv = threadIdx.x / 64, lane = lane_id();
    const uint32_t incl = wave_inclusive_scan32(mine);
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int k = 0; k < kSpThreads / 64; ++k) tot += wsum[k];
        bbase = tot ? atomicAdd(counter, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    uint64_t off = bbase + (incl - mine);
    for (uint32_t k = 0; k < wv; ++k) off += wsum[k];
    __syncthreads();  // wsum / bbase are reused by the next call
    return off;
}

__device__ __forceinline__ void sp_put(uint64_t *out, uint64_t pos, uint64_t cap, uint64_t value,
                                       unsigned int *overflow)
{
    if (pos < cap) out[pos] = value;
    else atomicOr(overflow, 1u);
}

// Level 0: the support as keys.
__global__ __launch_bounds__(kSpThreads) void sp_minterms_kernel(const uint32_t *tt, int n, uint64_t *out,
                                                                 unsigned long long *counter, uint64_t cap,
                                                                 unsigned int *overflow)
{
    const uint64_t nmin = 1ull << n;
    const uint64_t nwords = (nmin + 31) / 32;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t total = (nwords + kSpThreads - 1) / kSpThreads * kSpThreads;  // workgroup-uniform trips
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total; w += stride) {
        uint32_t bits = w < nwords ? tt[w] : 0u;
        if (n < 5) bits &= (uint32_t)((1ull << nmin) - 1ull);
        uint64_t pos = block_reserve((uint32_t)__popc(bits), counter);
        while (bits != 0u) {
            const uint32_t b = __builtin_ctz(bits);
            bits &= bits - 1u;
            sp_put(out, pos++, cap, sp_spread(w * 32 + b), overflow);
        }
    }
}

__global__ __launch_bounds__(kSpThreads) void sp_fill_kernel(uint64_t *p, uint64_t count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = kEmpty;
}

__global__ __launch_bounds__(kSpThreads) void sp_insert_kernel(const uint64_t *keys, uint64_t count,
                                                               uint64_t *table, uint64_t mask)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t key = keys[i];
        uint64_t h = sp_hash(key) & mask;
        for (;;) {
            const unsigned long long old =
                atomicCAS((unsigned long long *)&table[h], (unsigned long long)kEmpty, (unsigned long long)key);
            if (old == kEmpty || old == key) break;
            h = (h + 1) & mask;
        }
    }
}

// Step 1: implicants of level w from the list of level w-1 (one thread per
// implicant).
__global__ __launch_bounds__(kSpThreads) void sp_generate_kernel(const uint64_t *prev, uint64_t count,
                                                                 const uint64_t *table, uint64_t mask, int n,
                                                                 uint64_t *out, unsigned long long *counter,
                                                                 uint64_t cap, unsigned int *overflow)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t total = (count + kSpThreads - 1) / kSpThreads * kSpThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const bool live = i < count;
        const uint64_t c = live ? prev[i] : 0ull;
        // first star: lowest position whose pair has its high bit set
        const uint64_t stars = c & 0xAAAAAAAAAAAAAAAAull;
        const int f = live ? (stars == 0 ? n : (__builtin_ctzll(stars) >> 1)) : 0;
        uint32_t takes = 0;
        for (int p = 0; p < f; ++p) {
            uint64_t slot;
            if (((c >> (2 * p)) & 3ull) == 0ull && sp_find(table, mask, c | (1ull << (2 * p)), &slot)) {
                takes |= 1u << p;
                // the pair of u's first star is marked here (the partner's
                // slot is at hand); sp_mark_kernel covers the other stars
                atomicOr((unsigned long long *)&table[slot], (unsigned long long)kRedundant);
            }
        }
        if (takes != 0u) {
            uint64_t slot;
            if (sp_find(table, mask, c, &slot))
                atomicOr((unsigned long long *)&table[slot], (unsigned long long)kRedundant);
        }
        uint64_t pos = block_reserve((uint32_t)__popc(takes), counter);
        while (takes != 0u) {
            const int p = __builtin_ctz(takes);
            takes &= takes - 1u;
            sp_put(out, pos++, cap, c | (2ull << (2 * p)), overflow);
        }
    }
}

// Step 3: both halves of every star of every new implicant are redundant
// (the first star's pair was marked during generation).
__global__ __launch_bounds__(kSpThreads) void sp_mark_kernel(const uint64_t *cur, uint64_t count, uint64_t *table,
                                                             uint64_t mask, unsigned int *missing)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t u = cur[i];
        uint64_t stars = u & 0xAAAAAAAAAAAAAAAAull;
        stars &= stars - 1ull;  // all but the first star
        while (stars != 0) {
            const int q = __builtin_ctzll(stars) >> 1;
            stars &= stars - 1ull;
            const uint64_t h0 = u & ~(3ull << (2 * q)), h1 = h0 | (1ull << (2 * q));
            uint64_t s0, s1;
            if (sp_find(table, mask, h0, &s0)) atomicOr((unsigned long long *)&table[s0], (unsigned long long)kRedundant);
            else atomicOr(missing, 1u);
            if (sp_find(table, mask, h1, &s1)) atomicOr((unsigned long long *)&table[s1], (unsigned long long)kRedundant);
            else atomicOr(missing, 1u);
        }
    }
}

// Step 4: unmarked entries of a level's set are prime.  Each thread looks at
// kCollect slots (a workgroup covers kCollect * 256 consecutive slots, loads
// coalesced) per reservation.
constexpr int kCollect = 8;

__global__ __launch_bounds__(kSpThreads) void sp_collect_kernel(const uint64_t *table, uint64_t size, uint64_t *out,
                                                                unsigned long long *counter, uint64_t cap,
                                                                unsigned int *overflow)
{
    constexpr uint64_t kSpan = (uint64_t)kCollect * kSpThreads;
    const uint64_t stride = (uint64_t)gridDim.x * kSpan;
    for (uint64_t b0 = (uint64_t)blockIdx.x * kSpan; b0 < size; b0 += stride) {
        uint64_t v[kCollect];
        uint32_t mine = 0;
        static_for<kCollect>([&](auto ji) {
            constexpr int j = decltype(ji)::value;
            const uint64_t i = b0 + (uint64_t)j * kSpThreads + threadIdx.x;
            v[j] = i < size ? table[i] : kEmpty;
            mine += (v[j] != kEmpty && (v[j] & kRedundant) == 0ull) ? 1u : 0u;
        });
        uint64_t pos = block_reserve(mine, counter);
        static_for<kCollect>([&](auto ji) {
            constexpr int j = decltype(ji)::value;
            if (v[j] != kEmpty && (v[j] & kRedundant) == 0ull) sp_put(out, pos++, cap, v[j], overflow);
        });
    }
}

// key -> rho = sum 3^i * symbol_i
__global__ __launch_bounds__(kSpThreads) void sp_to_rho_kernel(uint64_t *keys, uint64_t count, int n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t k = keys[i];
        uint64_t r = 0;
        for (int p = n - 1; p >= 0; --p) r = r * 3 + ((k >> (2 * p)) & 3ull);
        keys[i] = r;
    }
}

// LSD radix sort of 64-bit keys on their low end_bit bits, 8 bits per pass.
// A pass counts the digits of every tile of kSortTile consecutive keys
// (sort_hist_kernel, counts stored digit-major: all tiles' counts of digit 0,
// then of digit 1, ...), scans the counts into output offsets with the
// library's count scan, and moves every key to its digit's offset plus its
// rank among the equal digits before it in the tile (sort_scatter_kernel).
// Keys of equal digit keep their order, so after the passes over digits of
// increasing weight the keys are sorted.
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;                                 // keys per thread and tile
constexpr uint64_t kSortTile = kSortThreads * kSortRounds;    // 2048 keys
constexpr int kSortBins = 256;
static_assert(kSortBins == kSortThreads, "one bin per thread");

__global__ __launch_bounds__(kSortThreads) void sort_hist_kernel(const uint64_t *keys, uint64_t n, int shift,
                                                                 uint32_t *counts, uint64_t ntiles)
{
    __shared__ uint32_t h[kSortBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * kSortTile;
    for (int j = 0; j < kSortRounds; ++j) {
        const uint64_t i = t0 + (uint64_t)j * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Keys are taken in index order: round j, then wavefront, then lane.  In a
// round, a lane's rank among the lanes of its wavefront with the same digit
// comes from eight ballots (one per digit bit); the wavefronts' counts per
// digit go through LDS.
__global__ __launch_bounds__(kSortThreads) void sort_scatter_kernel(const uint64_t *keys, uint64_t *out, uint64_t n,
                                                                    int shift, const uint64_t *offs, uint64_t ntiles)
{
    constexpr int W = kSortThreads / 64;
    __shared__ uint64_t base[kSortBins];  // next output position of each digit
    __shared__ uint32_t wc[W][kSortBins];  // this round: keys per wavefront and digit
    const uint32_t wv = threadIdx.x / 64, lane = lane_id();
    base[threadIdx.x] = offs[(uint64_t)threadIdx.x * ntiles + blockIdx.x];
    const uint64_t t0 = (uint64_t)blockIdx.x * kSortTile;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int j = 0; j < kSortRounds; ++j) {
        for (int w = 0; w < W; ++w) wc[w][threadIdx.x] = 0;
        __syncthreads();
        const uint64_t i = t0 + (uint64_t)j * kSortThreads + threadIdx.x;
        const bool live = i < n;
        const uint64_t k = live ? keys[i] : 0ull;
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        uint64_t peers = __ballot(live);
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        if (live && rank == 0) wc[wv][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (live) {
            uint64_t pos = base[d] + rank;
            for (uint32_t w = 0; w < wv; ++w) pos += wc[w][d];
            out[pos] = k;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < W; ++w) add += wc[w][threadIdx.x];
        base[threadIdx.x] += add;
    }
}

// Scratch of sort_keys for n keys: the digit counts, their offsets and the
// scan's block sums, each 256-byte aligned.
static uint64_t sort_scratch_bytes(uint64_t n)
{
    auto a = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
    const uint64_t nt = (n + kSortTile - 1) / kSortTile, m = (uint64_t)kSortBins * nt;
    return a(4 * m) + a(8 * m) + a(8 * scan_scratch_words(m));
}

// Sorts keys[0..n) on bits 0..end_bit-1, using tmp (n keys) and `scratch`
// (sort_scratch_bytes(n), 256-byte aligned); returns the buffer that holds
// the sorted keys (keys or tmp), or nullptr on a launch error.
static uint64_t *sort_keys(uint64_t *keys, uint64_t *tmp, uint64_t n, int end_bit, void *scratch, hipStream_t s)
{
    auto a = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
    const uint64_t nt = (n + kSortTile - 1) / kSortTile, m = (uint64_t)kSortBins * nt;
    uint32_t *counts = (uint32_t *)scratch;
    uint64_t *offs = (uint64_t *)((uint8_t *)scratch + a(4 * m));
    uint64_t *sums = (uint64_t *)((uint8_t *)scratch + a(4 * m) + a(8 * m));
    uint64_t *src = keys, *dst = tmp;
    for (int shift = 0; shift < end_bit; shift += 8) {
        hipLaunchKernelGGL(sort_hist_kernel, dim3((uint32_t)nt), dim3(kSortThreads), 0, s, src, n, shift, counts, nt);
        if (hipGetLastError() != hipSuccess) return nullptr;
        if (launch_scan_counts(counts, m, offs, nullptr, sums, s, nullptr) != hipSuccess) return nullptr;
        hipLaunchKernelGGL(sort_scatter_kernel, dim3((uint32_t)nt), dim3(kSortThreads), 0, s, src, dst, n, shift, offs,
                           nt);
        if (hipGetLastError() != hipSuccess) return nullptr;
        std::swap(src, dst);
    }
    return src;
}

static uint32_t sp_grid(uint64_t items)
{
    uint64_t g = (items + kSpThreads - 1) / kSpThreads;
    if (g > 16384) g = 16384;
    return (uint32_t)(g == 0 ? 1 : g);
}

static uint64_t pow2_at_least(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace dqmc

using namespace dqmc;

namespace {

// Device counters of one call: [0] level count, [1] prime count,
// [2] overflow flag, [3] missing-half flag (an internal error).
struct SpCounters {
    unsigned long long level;
    unsigned long long primes;
    unsigned int overflow;
    unsigned int missing;
};

int sp_fail(dqmc_ctx *ctx, int code, const char *msg)
{
    snprintf(ctx->err, sizeof(ctx->err), "%s", msg);
    return code;
}

}  // namespace

extern "C" {

uint64_t dqmc_sparse_workspace_bytes(int n, uint64_t max_level, uint64_t max_primes)
{
    if (n < 0 || n > DQMC_SPARSE_MAX_N) return 0;
    // dqmc_sparse_primes splits what follows its 4 KiB of counters and
    // alignment 3/8 : 3/8 : 1/4 into the two level regions (a list entry and
    // at most four set slots per implicant, 40 bytes) and the prime region
    // (keys and the sort's second buffer, 16 bytes per prime); the sort's
    // counts and offsets reuse the level regions.
    const uint64_t lv = std::max<uint64_t>(max_level, 1), np = std::max<uint64_t>(max_primes, 1);
    const uint64_t for_levels = (40 * lv + 1024) * 8 / 3 + 8;
    const uint64_t for_primes = (16 * np + 1024) * 4 + 8;
    const uint64_t for_sort = (sort_scratch_bytes(np) + 1024) * 4 / 3 + 8;
    return 4096 + std::max(for_levels, std::max(for_primes, for_sort));
}

int dqmc_sparse_primes(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint64_t *d_list, uint64_t list_cap,
                       uint64_t *d_count, void *d_work, uint64_t work_bytes, uint64_t *h_need, void *stream)
{
    if (ctx == nullptr) return DQMC_EINVAL;
    ctx->err[0] = 0;
    if (n < 0 || n > DQMC_SPARSE_MAX_N) return sp_fail(ctx, DQMC_EINVAL, "sparse path needs 0 <= n <= 31");
    if (d_tt == nullptr || d_count == nullptr || d_work == nullptr)
        return sp_fail(ctx, DQMC_EINVAL, "NULL truth table, count or workspace");
    if (((uintptr_t)d_tt & 3) || ((uintptr_t)d_count & 7) || ((uintptr_t)d_list & 7) || ((uintptr_t)d_work & 255))
        return sp_fail(ctx, DQMC_EINVAL, "misaligned buffer (workspace: 256 bytes)");
    if (hipSetDevice(ctx->device) != hipSuccess) return sp_fail(ctx, DQMC_EDEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    if (h_need) h_need[0] = h_need[1] = 0;
    // workspace: counters | level A (list, set) | level B (list, set) | primes
    // (keys) | sorted primes | sort scratch, with the level regions and the
    // prime region sized from what is left: 3/8 each level, 1/4 primes
    uint8_t *base = (uint8_t *)d_work;
    const uint64_t avail = work_bytes > 4096 ? work_bytes - 4096 : 0;
    SpCounters *cnt = (SpCounters *)base;
    uint8_t *p = base + 256;
    const uint64_t region = (avail * 3 / 8) & ~uint64_t(255);
    uint8_t *levA = p, *levB = p + region;
    uint8_t *prim = p + 2 * region;
    const uint64_t prim_bytes = (avail - 2 * region) & ~uint64_t(255);
    const uint64_t prim_cap = prim_bytes / 16;  // keys + sorted copy
    uint64_t *pkeys = (uint64_t *)prim, *psorted = pkeys + prim_cap;
    if (region < 1024 || prim_cap < 1) return sp_fail(ctx, DQMC_ENOMEM, "workspace too small");
    // a level region holds its list (lcap entries, rounded up to 256 bytes)
    // and a set of pow2 >= 2m <= 4m slots: at most 8 + 32 bytes per entry
    const uint64_t lcap = (region - 256) / 40;
    auto hip_ok = [&](hipError_t e) { return e == hipSuccess; };
    SpCounters h{};
    auto read_counters = [&]() {
        return hip_ok(hipMemcpyAsync(&h, cnt, sizeof(SpCounters), hipMemcpyDeviceToHost, s)) &&
               hip_ok(hipStreamSynchronize(s));
    };
    auto clear_counters = [&](bool keep_primes) {
        SpCounters z{};
        if (keep_primes) z.primes = h.primes;
        return hip_ok(hipMemcpyAsync(cnt, &z, sizeof(SpCounters), hipMemcpyHostToDevice, s)) &&
               hip_ok(hipStreamSynchronize(s));
    };
    if (!clear_counters(false)) return sp_fail(ctx, DQMC_EDEVICE, "counter upload failed");
    // level 0: the support
    uint64_t *L0 = (uint64_t *)levA;
    hipLaunchKernelGGL(sp_minterms_kernel, dim3(sp_grid(((1ull << n) + 31) / 32)), dim3(kSpThreads), 0, s, d_tt, n,
                       L0, &cnt->level, lcap, &cnt->overflow);
    if (!hip_ok(hipGetLastError()) || !read_counters()) return sp_fail(ctx, DQMC_EDEVICE, "level 0 failed");
    uint64_t need_level = h.level, need_primes = 0;
    if (h.overflow) {
        if (h_need) h_need[0] = need_level;
        return sp_fail(ctx, DQMC_ENOMEM, "workspace too small for level 0");
    }
    uint64_t m_prev = h.level;
    uint8_t *cur = levA, *nxt = levB;
    auto build_set = [&](uint8_t *reg, uint64_t m, uint64_t **list, uint64_t **set, uint64_t *size) {
        *list = (uint64_t *)reg;
        *size = pow2_at_least(2 * std::max<uint64_t>(m, 1));
        *set = (uint64_t *)(reg + ((8 * lcap + 255) & ~uint64_t(255)));
        hipLaunchKernelGGL(sp_fill_kernel, dim3(sp_grid(*size)), dim3(kSpThreads), 0, s, *set, *size);
        hipLaunchKernelGGL(sp_insert_kernel, dim3(sp_grid(m)), dim3(kSpThreads), 0, s, *list, m, *set, *size - 1);
        return hip_ok(hipGetLastError());
    };
    uint64_t *list_prev, *set_prev, size_prev;
    if (!build_set(cur, m_prev, &list_prev, &set_prev, &size_prev))
        return sp_fail(ctx, DQMC_EDEVICE, "set construction failed");
    if (!clear_counters(false)) return sp_fail(ctx, DQMC_EDEVICE, "counter upload failed");
    for (int w = 1; m_prev > 0; ++w) {
        uint64_t m = 0;
        uint64_t *list_cur = nullptr, *set_cur = nullptr, size_cur = 0;
        if (w <= n) {
            hipLaunchKernelGGL(sp_generate_kernel, dim3(sp_grid(m_prev)), dim3(kSpThreads), 0, s, list_prev, m_prev,
                               set_prev, size_prev - 1, n, (uint64_t *)nxt, &cnt->level, lcap, &cnt->overflow);
            if (!hip_ok(hipGetLastError()) || !read_counters())
                return sp_fail(ctx, DQMC_EDEVICE, "generation failed");
            need_level = std::max<uint64_t>(need_level, h.level);
            if (h.overflow) {
                if (h_need) h_need[0] = need_level;
                return sp_fail(ctx, DQMC_ENOMEM, "workspace too small for a level");
            }
            m = h.level;
            if (m > 0) {
                if (!build_set(nxt, m, &list_cur, &set_cur, &size_cur))
                    return sp_fail(ctx, DQMC_EDEVICE, "set construction failed");
                if (w >= 2)
                    hipLaunchKernelGGL(sp_mark_kernel, dim3(sp_grid(m)), dim3(kSpThreads), 0, s, list_cur, m,
                                       set_prev, size_prev - 1, &cnt->missing);
            }
        }
        hipLaunchKernelGGL(sp_collect_kernel, dim3(sp_grid((size_prev + kCollect - 1) / kCollect)), dim3(kSpThreads), 0,
                           s, set_prev, size_prev,
                           pkeys, &cnt->primes, prim_cap, &cnt->overflow);
        if (!hip_ok(hipGetLastError()) || !read_counters()) return sp_fail(ctx, DQMC_EDEVICE, "collection failed");
        need_primes = h.primes;
        if (h.missing) return sp_fail(ctx, DQMC_EDEVICE, "internal error: a merged half is missing");
        if (h.overflow) {
            if (h_need) {
                h_need[0] = need_level;
                h_need[1] = need_primes;
            }
            return sp_fail(ctx, DQMC_ENOMEM, "workspace too small for the primes");
        }
        // next level: reset the level counter, keep the prime count
        h.level = 0;
        if (!clear_counters(true)) return sp_fail(ctx, DQMC_EDEVICE, "counter upload failed");
        std::swap(cur, nxt);
        list_prev = list_cur;
        set_prev = set_cur;
        size_prev = size_cur;
        m_prev = m;
    }
    const uint64_t np = h.primes;
    if (h_need) {
        h_need[0] = need_level;
        h_need[1] = np;
    }
    // rho order
    if (np > 0) {
        hipLaunchKernelGGL(sp_to_rho_kernel, dim3(sp_grid(np)), dim3(kSpThreads), 0, s, pkeys, np, n);
        int end_bit = 1;  // rho < 3^n
        {
            uint64_t top = 1;
            for (int i = 0; i < n; ++i) top *= 3;
            while (end_bit < 64 && (1ull << end_bit) < top) ++end_bit;
        }
        // the sort's counts and offsets reuse the level regions (free by now)
        if (sort_scratch_bytes(np) > 2 * region) return sp_fail(ctx, DQMC_ENOMEM, "workspace too small for the sort");
        const uint64_t *sorted = sort_keys(pkeys, psorted, np, end_bit, (void *)levA, s);
        if (sorted == nullptr) return sp_fail(ctx, DQMC_EDEVICE, "sort failed");
        const uint64_t k = std::min(np, d_list ? list_cap : 0);
        if (k > 0 && !hip_ok(hipMemcpyAsync(d_list, sorted, k * 8, hipMemcpyDeviceToDevice, s)))
            return sp_fail(ctx, DQMC_EDEVICE, "list copy failed");
    }
    uint64_t npv = np;
    if (!hip_ok(hipMemcpyAsync(d_count, &npv, 8, hipMemcpyHostToDevice, s)) || !hip_ok(hipStreamSynchronize(s)))
        return sp_fail(ctx, DQMC_EDEVICE, "count upload failed");
    return DQMC_OK;
}

}  // extern "C"
