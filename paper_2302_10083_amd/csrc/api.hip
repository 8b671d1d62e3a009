// C ABI of libdqmc (declared in include/dqmc.h): argument checks, the pass
// plan for a given n, and the launch sequence.
//
// Pass plan for n > 12 (Alg. 4 with dimensions grouped; any order of the
// Merge dimensions, then any order of the Reduce dimensions, gives the same
// result - Sec. 4.1, and Sec. 6 fuses bottom Merge and Reduce layers):
//   1. low tiles from the truth table: merge digits 1..12 (only tiles whose
//      digits 13..n are binary hold data at that point);
//   2. column passes merging the high digit groups G_1 .. G_{k-1};
//   3. the top group G_k: merge and reduce in one pass;
//   4. column passes reducing G_{k-1} .. G_1;
//   5. low tiles: reduce digits 1..12, write O, extract the list.
// For n <= 12 one workgroup does everything in LDS.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <cmath>
#include <vector>

#include "api_types.h"
#include "dqmc.h"  // include/dqmc.h (the public C ABI)
#include "launch.h"
#include "h5.h"

using namespace dqmc;


namespace {

constexpr int kLowDigits = 12;  // digits 1..12 live in one low tile
// n at which dqmc_primes splits the top digit by default: its three
// 24-variable slices take the two-group plan, which moves fewer bytes per
// cube than any plan for 25 digits
constexpr int kSplitDefaultN = 25;

struct Group {
    int g0;  // first digit (1-based)
    int gr;  // digits in registers
    int gw;  // digits across wavefronts
    int size() const { return gr + gw; }
};

constexpr int kMaxGroup = 6;  // 4 digits in registers + 2 across wavefronts

// Default plan: as few groups as possible, sizes as equal as possible.
std::vector<int> default_sizes(int n)
{
    std::vector<int> out;
    const int H = n - kLowDigits;
    if (H <= 0) return out;
    const int k = (H + kMaxGroup - 1) / kMaxGroup;
    for (int j = 0; j < k; ++j) out.push_back(H / k + (j < H % k ? 1 : 0));
    return out;
}

std::vector<Group> groups_of(const std::vector<int> &sizes)
{
    std::vector<Group> out;
    int g0 = kLowDigits + 1;
    for (int s : sizes) {
        const int gr = s < 4 ? s : 4;
        out.push_back({g0, gr, s - gr});
        g0 += s;
    }
    return out;
}

std::vector<int> plan_sizes(const dqmc_ctx *ctx, int n)
{
    if (ctx != nullptr && n >= 0 && n <= DQMC_MAX_N && ctx->plan_len[n] > 0)
        return std::vector<int>(ctx->plan[n], ctx->plan[n] + ctx->plan_len[n]);
    return default_sizes(n);
}

uint64_t pow2u(int k) { return 1ull << k; }

int fail(dqmc_ctx *ctx, int code, const char *fmt, const char *detail)
{
    if (ctx) snprintf(ctx->err, sizeof(ctx->err), fmt, detail);
    return code;
}

#define DQMC_HIP(ctx, call)                                                                   \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail((ctx), DQMC_EDEVICE, "HIP error: %s", hipGetErrorString(e_)); \
    } while (0)

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

int check_common(dqmc_ctx *ctx, int n)
{
    if (ctx == nullptr) return DQMC_EINVAL;
    ctx->err[0] = 0;
    if (n < 0 || n > DQMC_MAX_N) {
        char buf[64];
        snprintf(buf, sizeof(buf), "%d", n);
        return fail(ctx, DQMC_EINVAL, "n = %s is outside [0, 25]", buf);
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DQMC_EDEVICE, "%s", "hipSetDevice failed");
    return DQMC_OK;
}

// Words of a state: 3^(n-5) blocks of 8 words up to n = 12 (one tile), then
// 3^(n-12) tile slots of kTileStride words.
uint64_t state_words_of(int n)
{
    if (n > kLowDigits) return (uint64_t)kTileStride * pow3(n - kLowDigits);
    return kBlockWords * pow3(n > 5 ? n - 5 : 0);
}

double state_bytes(int n) { return 4.0 * (double)state_words_of(n); }

// States are read in 16-byte pieces (the final low pass loads a run of three
// blocks per thread as four-word vectors).
constexpr size_t kStateAlign = 16;
double tt_bytes(int n) { return n <= 5 ? 4.0 : (double)(1ull << (n - 3)); }

// Enqueue one kernel pass; with profiling on, bracket it with events.
template <typename F>
int run_pass(dqmc_ctx *ctx, hipStream_t s, const char *name, int n, double model_bytes, int list_bpp, F &&launch)
{
    int k = -1;
    if (ctx->prof && ctx->nrec < DQMC_MAX_RECORDS) {
        k = ctx->nrec++;
        dqmc_pass_record &r = ctx->rec[k];
        snprintf(r.pass, sizeof(r.pass), "%s", name);
        r.n = n;
        r.list_bytes_per_prime = list_bpp;
        r.ms = 0.f;
        r.model_bytes = model_bytes;
        DQMC_HIP(ctx, hipEventRecord(ctx->ev[2 * k], s));
    }
    DQMC_HIP(ctx, launch());
    if (k >= 0) DQMC_HIP(ctx, hipEventRecord(ctx->ev[2 * k + 1], s));
    return DQMC_OK;
}

LowArgs low_args(dqmc_ctx *ctx, int n)
{
    LowArgs a{};
    a.n = n;
    a.lw = n <= 5 ? 0 : (n - 5 < 7 ? n - 5 : 7);
    a.tw = kBlockWords * (uint32_t)pow3(a.lw);
    a.ts = n > kLowDigits ? kTileStride : a.tw;
    a.ntiles = n <= kLowDigits ? 1 : pow3(n - kLowDigits);
    a.counts = ctx->counts;
    a.chunkmap = ctx->chunkmap;
    a.cap = 0;
    return a;
}

ColArgs col_args(uint32_t *state, int n, const Group &g, bool outer_binary)
{
    ColArgs c{};
    c.state = state;
    c.L = (uint64_t)kTileStride * pow3(g.g0 - kLowDigits - 1);
    const uint64_t lanes = (uint64_t)col_lanes_per_block(g.gw);
    c.nlb = (c.L + lanes - 1) / lanes;
    const int od = n - (g.g0 + g.size() - 1);
    c.outer_binary = outer_binary ? 1 : 0;
    c.nouter = outer_binary ? pow2u(od) : pow3(od);
    c.nblocks = c.nlb * c.nouter;
    return c;
}

// Row flags between the top group's merge+reduce and the reduce of the group
// below it: n = 24 with the plan [6, 6] (both column passes of 729 rows per
// block), when the context has the flag buffers.
bool use_row_flags(const dqmc_ctx *ctx, int n, const std::vector<Group> &gs)
{
    return ctx->flags_top != nullptr && ctx->flags_low != nullptr && ctx->flags_tile != nullptr && n == 24 &&
           gs.size() == 2 && gs[0].gr == 4 &&
           gs[0].gw == 2 && gs[1].gr == 4 && gs[1].gw == 2;
}

// Steps 1-2 (and the top group's merge when reduce == false).
int enqueue_merge(dqmc_ctx *ctx, int n, const uint32_t *tt, uint32_t flip, uint32_t *state, bool fuse_top_reduce,
                  hipStream_t s)
{
    LowArgs a = low_args(ctx, n);
    a.tt = tt;
    a.flip = flip;
    a.state = state;
    const double S = state_bytes(n);
    const double binfrac_high = std::pow(2.0 / 3.0, n - kLowDigits);
    int rc = run_pass(ctx, s, "low_merge_tt", n, tt_bytes(n) + S * binfrac_high, 0,
                      [&] { return launch_low(kLowMergeTT, a, pow2u(n - kLowDigits), s); });
    if (rc != DQMC_OK) return rc;
    const std::vector<Group> gs = groups_of(plan_sizes(ctx, n));
    for (size_t j = 0; j < gs.size(); ++j) {
        const bool top = j + 1 == gs.size();
        const int mode = (top && fuse_top_reduce) ? kColMergeReduce : kColMerge;
        ColArgs c = col_args(state, n, gs[j], true);
        if (mode == kColMergeReduce && use_row_flags(ctx, n, gs)) {
            // slot-aligned blocks (the reduce pass's), so the flags carry over exactly
            c.flags = ctx->flags_top;
            c.slot_blocks = (uint32_t)kFlagLowBlocks;
            c.nlb = kFlagTopBlocks;  // n = 24: no outer digits
            c.nblocks = c.nlb * c.nouter;
        }
        const int od = n - (gs[j].g0 + gs[j].size() - 1);
        const double fo = std::pow(2.0 / 3.0, od), fg = std::pow(2.0 / 3.0, gs[j].size());
        const double bytes = mode == kColMerge ? S * fo * (fg + (1.0 - fg)) : S * fo * (fg + 1.0);
        char name[40];
        snprintf(name, sizeof(name), "%s_g%d_%d", mode == kColMerge ? "col_merge" : "col_merge_reduce", gs[j].g0,
                 gs[j].size());
        rc = run_pass(ctx, s, name, n, bytes, 0, [&] { return launch_col(gs[j].gr, gs[j].gw, mode, c, s); });
        if (rc != DQMC_OK) return rc;
    }
    return DQMC_OK;
}

// The low-tile pass that ends a prime bitmap: reduce of digits 1..12 with the
// tile summaries, or the summaries alone.
int enqueue_summary(dqmc_ctx *ctx, int n, int mode, uint32_t *state, hipStream_t s, uint64_t tile0 = 0,
                    const uint32_t *tile_flags = nullptr)
{
    LowArgs a = low_args(ctx, n);
    a.state = state;
    a.tile_flags = tile_flags;
    a.counts += tile0;  // the summaries of a slice start at tile0 of a larger state
    a.chunkmap += tile0 * kMapWords;
    const double S = state_bytes(n);
    const bool reduce = mode == kLowReduceCount;
    // with chunk flags: the compact kernel, then the tiles it deferred
    const bool compact = reduce && tile_flags != nullptr && ctx->deferred != nullptr && n > kLowDigits;
    if (compact) a.deferred = ctx->deferred;
    return run_pass(ctx, s, reduce ? "low_reduce_count" : "low_count", n,
                    (reduce ? 2 * S : S) + a.ntiles * 4.0 * (1 + kMapWords), 0,
                    [&] { return compact ? launch_low_compact(a, s) : launch_low(mode, a, a.ntiles, s); });
}

// Scan of the tile counts (starting at *base when base is given) and the
// list pass (cube indices offset by rho0).
int enqueue_scan_list(dqmc_ctx *ctx, int n, const uint32_t *state, uint64_t *list, uint64_t cap, uint64_t *count,
                      const uint64_t *base, uint64_t rho0, hipStream_t s)
{
    const LowArgs a = low_args(ctx, n);
    int rc = run_pass(ctx, s, "scan_counts", n, a.ntiles * 12.0, 0, [&] {
        return launch_scan_counts(ctx->counts, a.ntiles, ctx->offs, count, ctx->sums, s, base);
    });
    if (rc != DQMC_OK || list == nullptr) return rc;
    // the list pass reads the summaries and the non-zero chunks (data
    // dependent, so only the summaries are in the model) and writes 8 bytes
    // per listed prime
    return run_pass(ctx, s, "list", n, a.ntiles * 4.0 * (3 + kMapWords), 8, [&] {
        return launch_list(n, state, a.tw, a.ts, a.ntiles, ctx->counts, ctx->chunkmap, ctx->offs, list, cap, s, rho0);
    });
}

// Final low-tile pass (reduce or plain count), scan of the tile counts, and
// the list pass.
int enqueue_extract_tiles(dqmc_ctx *ctx, int n, int mode, uint32_t *state, uint64_t *list, uint64_t cap,
                          uint64_t *count, hipStream_t s, const uint32_t *tile_flags = nullptr)
{
    const int rc = enqueue_summary(ctx, n, mode, state, s, 0, tile_flags);
    if (rc != DQMC_OK) return rc;
    return enqueue_scan_list(ctx, n, state, list, cap, count, nullptr, 0, s);
}

// Steps 1-4 for n > 12: merges, the top group's merge and reduce, and the
// reduces of the other high groups (the low digits are reduced by the
// summary pass).
// *tile_flags (may be NULL): chunk flags for the final reduce, or nullptr.
int enqueue_reduce_high(dqmc_ctx *ctx, int n, const uint32_t *tt, uint32_t flip, uint32_t *state, hipStream_t s,
                        const uint32_t **tile_flags = nullptr)
{
    if (tile_flags != nullptr) *tile_flags = nullptr;
    int rc = enqueue_merge(ctx, n, tt, flip, state, true, s);
    if (rc != DQMC_OK) return rc;
    const std::vector<Group> gs = groups_of(plan_sizes(ctx, n));
    const bool flags = use_row_flags(ctx, n, gs);
    if (n == 24) ctx->flags_used = flags && tile_flags != nullptr;
    if (flags) {
        // 18 MB read, 18 MB written
        rc = run_pass(ctx, s, "flag_transpose", n, 8.0 * 729 * kFlagLowBlocks * kFlagWords, 0,
                      [&] { return launch_flag_transpose(ctx->flags_top, ctx->flags_low, s); });
        if (rc != DQMC_OK) return rc;
    }
    for (int j = (int)gs.size() - 2; j >= 0; --j) {
        ColArgs c = col_args(state, n, gs[j], false);
        if (flags && j == 0) c.flags = ctx->flags_low;
        const double S = state_bytes(n);
        char name[40];
        snprintf(name, sizeof(name), "col_reduce_g%d_%d", gs[j].g0, gs[j].size());
        rc = run_pass(ctx, s, name, n, S * (2.0 - std::pow(3.0, -gs[j].size())), 0,
                      [&] { return launch_col(gs[j].gr, gs[j].gw, kColReduce, c, s); });
        if (rc != DQMC_OK) return rc;
    }
    if (flags && tile_flags != nullptr) {
        // the reduce pass's row flags as chunk flags of the tiles (18 MB
        // read, 19 MB written)
        rc = run_pass(ctx, s, "tile_flags", n, 4.0 * 729 * kFlagLowBlocks * kFlagWords + 4.0 * pow3(12) * kMapWords,
                      0, [&] { return launch_tile_flags(ctx->flags_low, ctx->flags_tile, ctx->deferred, s); });
        if (rc != DQMC_OK) return rc;
        *tile_flags = ctx->flags_tile;
    }
    return DQMC_OK;
}

// Slices of a function along its top variables (the sliced path and the
// top-digit split) run the passes of an m-variable function on a restricted
// truth table.  The tile summaries of the slice go to tiles tile0.. of the
// context's summary arrays.

int enqueue_split_state(dqmc_ctx *ctx, int n, const uint32_t *tt, uint32_t flip, uint32_t *state, uint64_t tile0,
                        hipStream_t s);
bool use_split(const dqmc_ctx *ctx, int n);

// The low-pass arguments of an m-variable slice state; `slot`: the state is a
// tile slot of a larger state (a third of a split of m + 1 = 13 variables),
// written whole, its padding zero.
LowArgs slice_low_args(dqmc_ctx *ctx, int m, bool slot)
{
    LowArgs a = low_args(ctx, m);
    if (slot) a.ts = kTileStride;
    return a;
}

// Primes of the m-variable function `tt` into `state`, with the summaries;
// by the top-digit split where it is on for m, except inside a split (one
// level only: the thirds' truth tables share one buffer).
int enqueue_slice_primes(dqmc_ctx *ctx, int m, const uint32_t *tt, uint32_t *state, uint64_t tile0, hipStream_t s,
                         bool allow_split = true, bool slot = false)
{
    if (allow_split && use_split(ctx, m)) return enqueue_split_state(ctx, m, tt, 0u, state, tile0, s);
    if (m <= kLowDigits) {
        LowArgs a = slice_low_args(ctx, m, slot);
        a.tt = tt;
        a.state = state;
        const int rc = run_pass(ctx, s, "low_primes_tt", m, tt_bytes(m) + state_bytes(m), 0,
                                [&] { return launch_low(kLowPrimesTT, a, 1, s); });
        return rc != DQMC_OK ? rc : enqueue_summary(ctx, m, kLowCount, state, s, tile0);
    }
    const uint32_t *tf = nullptr;
    const int rc = enqueue_reduce_high(ctx, m, tt, 0u, state, s, &tf);
    return rc != DQMC_OK ? rc : enqueue_summary(ctx, m, kLowReduceCount, state, s, tile0, tf);
}

// Implicants of the m-variable function `tt` into `state`.
int enqueue_slice_implicants(dqmc_ctx *ctx, int m, const uint32_t *tt, uint32_t *state, hipStream_t s,
                             bool slot = false)
{
    if (m <= kLowDigits) {
        LowArgs a = slice_low_args(ctx, m, slot);
        a.tt = tt;
        a.state = state;
        return run_pass(ctx, s, "low_merge_tt", m, tt_bytes(m) + state_bytes(m), 0,
                        [&] { return launch_low(kLowMergeTT, a, 1, s); });
    }
    return enqueue_merge(ctx, m, tt, 0u, state, false, s);
}

// o &= ~mask on the marked chunks of a slice, with new summaries.
int enqueue_slice_filter(dqmc_ctx *ctx, int m, uint32_t *o, const uint32_t *mask, uint64_t tile0, hipStream_t s)
{
    const LowArgs la = low_args(ctx, m);
    // data dependent (only the marked chunks are read); the model counts the
    // summaries
    return run_pass(ctx, s, "andnot_map", m, la.ntiles * 8.0 * (1 + kMapWords), 0, [&] {
        return launch_andnot_map(o, mask, ctx->counts + tile0, ctx->chunkmap + tile0 * kMapWords, la.ntiles, la.tw, la.ts,
                                 s);
    });
}

// The truth table of slice (fixed, stars) of the top variables into `out`
// (a context buffer: slice_tt for the sliced path, split_tt for the split).
int enqueue_slice_tt(dqmc_ctx *ctx, int m, const uint32_t *tt, uint32_t fixed, uint32_t stars, uint32_t flip,
                     uint32_t *out, hipStream_t s)
{
    const double sub = (double)(1u << __builtin_popcount(stars));
    return run_pass(ctx, s, "slice_tt", m, tt_bytes(m) * (sub + 1.0), 0,
                    [&] { return launch_slice_tt(tt, m, fixed, stars, flip, out, s); });
}

// Top-digit split (n > 12): the state of n variables is three consecutive
// slice states of m = n - 1 variables (digit n = 0, 1, *), and its tiles are
// the slices' tiles in order.  Slices 0 and 1 are their functions' primes
// minus the implicants of f_* = f_0 AND f_1 (the star neighbour of both, held
// meanwhile in the * third); the * slice is the primes of f_*.  This writes
// the state and the tile summaries from tile0 on; the thirds' truth tables go
// to the context's split_tt, so that `tt` may be the sliced path's slice_tt.
int enqueue_split_state(dqmc_ctx *ctx, int n, const uint32_t *tt, uint32_t flip, uint32_t *state, uint64_t tile0,
                        hipStream_t s)
{
    const int m = n - 1;
    // a third is 3^(m-12) tile slots (one slot, with its padding, at m = 12)
    const uint64_t third = (uint64_t)kTileStride * pow3(m - kLowDigits), tiles = low_args(ctx, m).ntiles;
    uint32_t *star = state + 2 * third;
    int rc = enqueue_slice_tt(ctx, m, tt, 0u, 1u, flip, ctx->split_tt, s);
    if (rc == DQMC_OK) rc = enqueue_slice_implicants(ctx, m, ctx->split_tt, star, s, true);
    for (uint32_t a = 0; a < 3 && rc == DQMC_OK; ++a) {
        uint32_t *o = state + a * third;
        const uint64_t t0 = tile0 + a * tiles;
        rc = enqueue_slice_tt(ctx, m, tt, a == 1 ? 1u : 0u, a == 2 ? 1u : 0u, flip, ctx->split_tt, s);
        if (rc == DQMC_OK) rc = enqueue_slice_primes(ctx, m, ctx->split_tt, o, t0, s, false, true);
        if (rc == DQMC_OK && a < 2) rc = enqueue_slice_filter(ctx, m, o, star, t0, s);
    }
    return rc;
}

// dqmc_primes by the split: the split state, then one scan and list over all
// tiles.
int enqueue_primes_split(dqmc_ctx *ctx, int n, const uint32_t *tt, uint32_t flip, uint32_t *state, uint64_t *list,
                         uint64_t cap, uint64_t *count, hipStream_t s)
{
    const int rc = enqueue_split_state(ctx, n, tt, flip, state, 0, s);
    return rc != DQMC_OK ? rc : enqueue_scan_list(ctx, n, state, list, cap, count, nullptr, 0, s);
}

bool use_split(const dqmc_ctx *ctx, int n)
{
    if (n <= kLowDigits || n > DQMC_MAX_N) return false;
    if (ctx->split[n] >= 0) return ctx->split[n] == 1;
    return n == kSplitDefaultN;
}

// A cube on the top t variables of the sliced path: bits where it is 1, and
// bits where it is *.
struct SliceKey {
    uint32_t fixed;
    uint32_t stars;
    bool operator==(const SliceKey &o) const { return fixed == o.fixed && stars == o.stars; }
    uint64_t code() const { return (uint64_t)fixed | ((uint64_t)stars << 32); }
};

// Slice idx (its digits in base 3, * = 2) as a key.
SliceKey slice_key(uint64_t idx, int t)
{
    SliceKey k{0u, 0u};
    for (int j = 0; j < t; ++j, idx /= 3) {
        if (idx % 3 == 1) k.fixed |= 1u << j;
        if (idx % 3 == 2) k.stars |= 1u << j;
    }
    return k;
}

// The slices a[j <- *] for the binary digits j of slice idx.
std::vector<SliceKey> star_neighbours(uint64_t idx, int t)
{
    const SliceKey a = slice_key(idx, t);
    std::vector<SliceKey> out;
    for (int j = 0; j < t; ++j)
        if (((a.stars >> j) & 1u) == 0u) out.push_back(SliceKey{a.fixed & ~(1u << j), a.stars | (1u << j)});
    return out;
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed device scratch of dqmc_primes_noalloc: the per-tile summaries (set-bit
// count and non-zero chunk map), the list offsets and the scan's block sums of
// one function of at most kNoAllocMaxN variables.  Each device holds its own
// copy for the life of the process.  In host code `scratch` names a host-side
// stand-in: its device address comes from hipGetSymbolAddress, once per
// device (noalloc_scratch below), and only that address is ever used.
namespace {
constexpr int kNoAllocMaxN = 24;
constexpr uint64_t kNoAllocTiles = pow3(kNoAllocMaxN - kLowDigits);
constexpr uint64_t kNoAllocSums = (kNoAllocTiles + 8191) / 8192 + 1;  // >= scan_scratch_words(tiles)
// layout in uint64 words: offs | sums | counts (u32) | chunkmap (u32)
constexpr uint64_t kNoAllocWords = kNoAllocTiles + kNoAllocSums + (kNoAllocTiles * (1 + kMapWords) + 1) / 2;
constexpr int kNoAllocMaxDevices = 64;
}  // namespace

static __device__ __align__(256) uint64_t scratch[kNoAllocWords];

namespace {
std::mutex g_noalloc_mu;
uint64_t *g_noalloc_ptr[kNoAllocMaxDevices];  // device address of `scratch`, per device

// The device address of this device's scratch (the current device), with the
// kernels' launch attributes set, on the first call on the device.  Returns
// nullptr on a HIP error.
uint64_t *noalloc_scratch(int dev)
{
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[dev] != nullptr) return g_noalloc_ptr[dev];
    if (scan_scratch_words(kNoAllocTiles) > kNoAllocSums) return nullptr;
    if (low_setup() != hipSuccess || col_setup() != hipSuccess) return nullptr;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return nullptr;
    g_noalloc_ptr[dev] = (uint64_t *)p;
    return g_noalloc_ptr[dev];
}
}  // namespace

extern "C" {

uint64_t dqmc_num_cubes(int n) { return (n < 0 || n > DQMC_MAX_N) ? 0 : pow3(n); }
uint64_t dqmc_tt_words(int n) { return (n < 0 || n > DQMC_MAX_N) ? 0 : (n <= 5 ? 1 : (1ull << (n - 5))); }
uint64_t dqmc_state_words(int n) { return (n < 0 || n > DQMC_MAX_N) ? 0 : state_words_of(n); }
uint64_t dqmc_dense_words(int n) { return (n < 0 || n > DQMC_MAX_N) ? 0 : (pow3(n) + 63) / 64; }

int dqmc_create(int device, dqmc_ctx **out)
{
    if (out == nullptr) return DQMC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return DQMC_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return DQMC_EDEVICE;
    if (low_setup() != hipSuccess || col_setup() != hipSuccess || batch_setup() != hipSuccess) return DQMC_EDEVICE;
    dqmc_ctx *c = new dqmc_ctx();
    c->device = device;
    if (hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->ncu <= 0)
        c->ncu = 256;
    c->tiles_cap = pow3(DQMC_MAX_N - kLowDigits);
    c->counts = nullptr;
    c->chunkmap = nullptr;
    c->offs = nullptr;
    c->sums = nullptr;
    c->slice_tt = nullptr;
    c->split_tt = nullptr;
    c->run = nullptr;
    c->flags_top = nullptr;
    c->flags_low = nullptr;
    c->flags_tile = nullptr;
    c->deferred = nullptr;
    c->flags_used = false;
    c->batch_mem = nullptr;
    c->batch_cap = 0;
    c->err[0] = 0;
    c->prof = false;
    c->events_made = false;
    c->nrec = 0;
    for (int i = 0; i <= DQMC_MAX_N; ++i) {
        c->plan_len[i] = 0;
        c->split[i] = -1;
    }
    if (hipMalloc((void **)&c->counts, c->tiles_cap * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&c->chunkmap, c->tiles_cap * kMapWords * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&c->offs, c->tiles_cap * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void **)&c->sums, scan_scratch_words(c->tiles_cap) * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void **)&c->slice_tt, dqmc_tt_words(DQMC_MAX_N) * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&c->split_tt, dqmc_tt_words(DQMC_MAX_N - 1) * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&c->run, 2 * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void **)&c->flags_top, kFlagTopBlocks * kFlagWords * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&c->flags_low, 729 * kFlagLowBlocks * kFlagWords * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&c->flags_tile, pow3(12) * kMapWords * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&c->deferred, (pow3(12) + 1) * sizeof(uint32_t)) != hipSuccess) {
        dqmc_destroy(c);
        return DQMC_ENOMEM;
    }
    *out = c;
    return DQMC_OK;
}

void dqmc_destroy(dqmc_ctx *ctx)
{
    if (ctx == nullptr) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->events_made)
        for (int i = 0; i < 2 * DQMC_MAX_RECORDS; ++i) (void)hipEventDestroy(ctx->ev[i]);
    if (ctx->counts) (void)hipFree(ctx->counts);
    if (ctx->chunkmap) (void)hipFree(ctx->chunkmap);
    if (ctx->offs) (void)hipFree(ctx->offs);
    if (ctx->sums) (void)hipFree(ctx->sums);
    if (ctx->slice_tt) (void)hipFree(ctx->slice_tt);
    if (ctx->split_tt) (void)hipFree(ctx->split_tt);
    if (ctx->run) (void)hipFree(ctx->run);
    if (ctx->flags_top) (void)hipFree(ctx->flags_top);
    if (ctx->flags_low) (void)hipFree(ctx->flags_low);
    if (ctx->flags_tile) (void)hipFree(ctx->flags_tile);
    if (ctx->deferred) (void)hipFree(ctx->deferred);
    if (ctx->batch_mem) (void)hipFree(ctx->batch_mem);
    delete ctx;
}

const char *dqmc_last_error(const dqmc_ctx *ctx) { return ctx ? ctx->err : "no context"; }

int dqmc_implicants(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint32_t *d_state, void *stream)
{
    return dqmc_implicants_ex(ctx, n, d_tt, 0u, d_state, stream);
}

int dqmc_implicants_ex(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint32_t flags, uint32_t *d_state, void *stream)
{
    int rc = check_common(ctx, n);
    if (rc != DQMC_OK) return rc;
    if ((flags & ~(uint32_t)DQMC_NEGATE) != 0u) return fail(ctx, DQMC_EINVAL, "%s", "unknown flag bits");
    const uint32_t flip = (flags & DQMC_NEGATE) ? ~0u : 0u;
    if (d_tt == nullptr || d_state == nullptr) return fail(ctx, DQMC_EINVAL, "%s", "NULL truth table or state");
    if (!aligned(d_tt, 4) || !aligned(d_state, kStateAlign)) return fail(ctx, DQMC_EINVAL, "%s", "misaligned buffer");
    hipStream_t s = (hipStream_t)stream;
    if (n <= kLowDigits) {
        LowArgs a = low_args(ctx, n);
        a.tt = d_tt;
        a.flip = flip;
        a.state = d_state;
        return run_pass(ctx, s, "low_merge_tt", n, tt_bytes(n) + state_bytes(n), 0,
                        [&] { return launch_low(kLowMergeTT, a, 1, s); });
    }
    return enqueue_merge(ctx, n, d_tt, flip, d_state, false, s);
}

int dqmc_primes(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint32_t *d_state, uint64_t *d_list,
                uint64_t list_cap, uint64_t *d_count, void *stream)
{
    return dqmc_primes_ex(ctx, n, d_tt, 0u, d_state, d_list, list_cap, d_count, stream);
}

int dqmc_primes_ex(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint32_t flags, uint32_t *d_state, uint64_t *d_list,
                   uint64_t list_cap, uint64_t *d_count, void *stream)
{
    int rc = check_common(ctx, n);
    if (rc != DQMC_OK) return rc;
    if ((flags & ~(uint32_t)DQMC_NEGATE) != 0u) return fail(ctx, DQMC_EINVAL, "%s", "unknown flag bits");
    const uint32_t flip = (flags & DQMC_NEGATE) ? ~0u : 0u;
    if (d_tt == nullptr || d_state == nullptr || d_count == nullptr)
        return fail(ctx, DQMC_EINVAL, "%s", "NULL truth table, state or count");
    if (!aligned(d_tt, 4) || !aligned(d_state, kStateAlign) || !aligned(d_count, 8) || !aligned(d_list, 8))
        return fail(ctx, DQMC_EINVAL, "%s", "misaligned buffer");
    hipStream_t s = (hipStream_t)stream;
    if (n <= kLowDigits) {
        LowArgs a = low_args(ctx, n);
        a.tt = d_tt;
        a.flip = flip;
        a.state = d_state;
        a.list = d_list;
        a.cap = d_list ? list_cap : 0;
        a.count = d_count;
        return run_pass(ctx, s, "low_primes_tt", n, tt_bytes(n) + state_bytes(n), d_list ? 8 : 0,
                        [&] { return launch_low(kLowPrimesTT, a, 1, s); });
    }
    if (use_split(ctx, n)) return enqueue_primes_split(ctx, n, d_tt, flip, d_state, d_list, list_cap, d_count, s);
    const uint32_t *tf = nullptr;
    rc = enqueue_reduce_high(ctx, n, d_tt, flip, d_state, s, &tf);
    if (rc != DQMC_OK) return rc;
    return enqueue_extract_tiles(ctx, n, kLowReduceCount, d_state, d_list, list_cap, d_count, s, tf);
}

int dqmc_primes_noalloc(int n, const uint32_t *d_tt, uint32_t *d_state, uint64_t *d_list, uint64_t list_cap,
                        uint64_t *d_count, void *stream)
{
    if (n < 0 || n > DQMC_MAX_N) return DQMC_EINVAL;
    if (n > kNoAllocMaxN) return DQMC_ESCRATCH;
    if (d_tt == nullptr || d_state == nullptr || d_count == nullptr) return DQMC_EINVAL;
    if (!aligned(d_tt, 4) || !aligned(d_state, kStateAlign) || !aligned(d_count, 8) || !aligned(d_list, 8))
        return DQMC_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) return DQMC_EDEVICE;
    uint64_t *p = noalloc_scratch(dev);
    if (p == nullptr) return DQMC_EDEVICE;
    // a context on the stack whose scratch pointers lie in this device's
    // static scratch: default pass plan, no top-digit split, no profiling
    dqmc_ctx c{};
    c.device = dev;
    c.ncu = 256;
    c.tiles_cap = kNoAllocTiles;
    c.offs = p;
    c.sums = p + kNoAllocTiles;
    c.counts = (uint32_t *)(p + kNoAllocTiles + kNoAllocSums);
    c.chunkmap = c.counts + kNoAllocTiles;
    for (int i = 0; i <= DQMC_MAX_N; ++i) {
        c.plan_len[i] = 0;
        c.split[i] = 0;
    }
    if (check_common(&c, n) != DQMC_OK) return DQMC_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    if (n <= kLowDigits) {
        LowArgs a = low_args(&c, n);
        a.tt = d_tt;
        a.state = d_state;
        a.list = d_list;
        a.cap = d_list ? list_cap : 0;
        a.count = d_count;
        return launch_low(kLowPrimesTT, a, 1, s) == hipSuccess ? DQMC_OK : DQMC_EDEVICE;
    }
    int rc = enqueue_reduce_high(&c, n, d_tt, 0u, d_state, s);
    if (rc == DQMC_OK) rc = enqueue_extract_tiles(&c, n, kLowReduceCount, d_state, d_list, list_cap, d_count, s);
    return rc;
}

int dqmc_set_split(dqmc_ctx *ctx, int n, int mode)
{
    if (ctx == nullptr) return DQMC_EINVAL;
    ctx->err[0] = 0;
    if (n <= kLowDigits || n > DQMC_MAX_N || mode < -1 || mode > 1)
        return fail(ctx, DQMC_EINVAL, "%s", "the split needs 12 < n <= 25 and mode -1, 0 or 1");
    ctx->split[n] = mode;
    return DQMC_OK;
}

int dqmc_get_split(const dqmc_ctx *ctx, int n)
{
    if (ctx == nullptr) return DQMC_EINVAL;
    return use_split(ctx, n) ? 1 : 0;
}

int dqmc_primes_sliced(dqmc_ctx *ctx, int n, int t, const uint32_t *d_tt, uint32_t flags, uint32_t *d_o,
                       uint32_t *d_m, uint64_t *d_list, uint64_t list_cap, uint64_t *d_count, void *stream)
{
    return dqmc_primes_sliced_multi(ctx, n, t, d_tt, flags, d_o, &d_m, 1, d_list, list_cap, d_count, stream);
}

int dqmc_primes_sliced_multi(dqmc_ctx *ctx, int n, int t, const uint32_t *d_tt, uint32_t flags, uint32_t *d_o,
                             uint32_t *const *d_ms, int nm, uint64_t *d_list, uint64_t list_cap, uint64_t *d_count,
                             void *stream)
{
    if (ctx == nullptr) return DQMC_EINVAL;
    ctx->err[0] = 0;
    if (n < 1 || n > DQMC_SLICED_MAX_N || t < 1 || t > DQMC_SLICED_MAX_T || t > n || n - t > DQMC_MAX_N) {
        char buf[64];
        snprintf(buf, sizeof(buf), "n = %d, t = %d", n, t);
        return fail(ctx, DQMC_EINVAL, "%s: need 1 <= t <= 8, t <= n <= 30 and n - t <= 25", buf);
    }
    const int m = n - t;
    int rc = check_common(ctx, m);
    if (rc != DQMC_OK) return rc;
    if ((flags & ~(uint32_t)DQMC_NEGATE) != 0u) return fail(ctx, DQMC_EINVAL, "%s", "unknown flag bits");
    const uint32_t flip = (flags & DQMC_NEGATE) ? ~0u : 0u;
    if (d_ms == nullptr || nm < 1 || nm > DQMC_SLICED_MAX_STATES)
        return fail(ctx, DQMC_EINVAL, "%s", "need 1 to DQMC_SLICED_MAX_STATES implicant states");
    if (d_tt == nullptr || d_o == nullptr || d_count == nullptr)
        return fail(ctx, DQMC_EINVAL, "%s", "NULL truth table, slice state or count");
    if (!aligned(d_tt, 4) || !aligned(d_o, kStateAlign) || !aligned(d_count, 8) || !aligned(d_list, 8))
        return fail(ctx, DQMC_EINVAL, "%s", "misaligned buffer");
    const uint64_t sw = dqmc_state_words(m);
    std::vector<uint32_t *> states(1, d_o);
    for (int i = 0; i < nm; ++i) {
        if (d_ms[i] == nullptr || !aligned(d_ms[i], kStateAlign))
            return fail(ctx, DQMC_EINVAL, "%s", "NULL or misaligned implicant state");
        for (uint32_t *q : states)
            if (d_ms[i] < q + sw && q < d_ms[i] + sw) return fail(ctx, DQMC_EINVAL, "%s", "the slice states overlap");
        states.push_back(d_ms[i]);
    }
    hipStream_t s = (hipStream_t)stream;
    const uint64_t nslices = pow3(t), slice_cubes = pow3(m);
    // The slices that need each star neighbour's implicant bitmap, in order,
    // for choosing which bitmap to drop when the states are full (the one
    // needed again last).
    std::map<uint64_t, std::vector<uint64_t>> uses;
    for (uint64_t idx = 0; idx < nslices; ++idx)
        for (const SliceKey &k : star_neighbours(idx, t)) uses[k.code()].push_back(idx);
    auto next_use = [&](const SliceKey &k, uint64_t after) -> uint64_t {
        const std::vector<uint64_t> &u = uses[k.code()];
        const auto it = std::upper_bound(u.begin(), u.end(), after);
        return it == u.end() ? ~0ull : *it;
    };
    std::vector<SliceKey> held(nm);  // the function whose implicants state i holds
    std::vector<bool> valid(nm, false);
    for (uint64_t idx = 0; idx < nslices; ++idx) {
        const SliceKey a_key = slice_key(idx, t);
        // primes of f_a into d_o, with the tile summaries
        rc = enqueue_slice_tt(ctx, m, d_tt, a_key.fixed, a_key.stars, flip, ctx->slice_tt, s);
        if (rc == DQMC_OK) rc = enqueue_slice_primes(ctx, m, ctx->slice_tt, d_o, 0, s);
        if (rc != DQMC_OK) return rc;
        // Reduce along each binary top digit j: drop s where s.a[j <- *] is
        // an implicant, i.e. where M of the star neighbour's function is set.
        // The bitmaps already held are applied first; the missing ones are
        // computed with the one needed again soonest last, each into the state
        // whose bitmap is needed again last.
        std::vector<SliceKey> hits, misses;
        for (const SliceKey &k : star_neighbours(idx, t)) {
            bool held_now = false;
            for (int i = 0; i < nm; ++i) held_now = held_now || (valid[i] && held[i] == k);
            (held_now ? hits : misses).push_back(k);
        }
        std::stable_sort(misses.begin(), misses.end(), [&](const SliceKey &x, const SliceKey &y) {
            return next_use(x, idx) > next_use(y, idx);
        });
        for (const SliceKey &k : hits) {
            for (int i = 0; i < nm; ++i) {
                if (valid[i] && held[i] == k) {
                    rc = enqueue_slice_filter(ctx, m, d_o, d_ms[i], 0, s);
                    if (rc != DQMC_OK) return rc;
                    break;
                }
            }
        }
        for (const SliceKey &k : misses) {
            int v = -1;
            for (int i = 0; i < nm && v < 0; ++i)
                if (!valid[i]) v = i;
            if (v < 0) {
                uint64_t far = 0;
                for (int i = 0; i < nm; ++i) {
                    const uint64_t nu = next_use(held[i], idx);
                    if (v < 0 || nu > far) {
                        v = i;
                        far = nu;
                    }
                }
            }
            rc = enqueue_slice_tt(ctx, m, d_tt, k.fixed, k.stars, flip, ctx->slice_tt, s);
            if (rc == DQMC_OK) rc = enqueue_slice_implicants(ctx, m, ctx->slice_tt, d_ms[v], s);
            if (rc == DQMC_OK) rc = enqueue_slice_filter(ctx, m, d_o, d_ms[v], 0, s);
            if (rc != DQMC_OK) return rc;
            held[v] = k;
            valid[v] = true;
        }
        // append the slice's primes: offsets continue from the previous
        // slices' total (two running counters, used alternately)
        uint64_t *total = idx + 1 == nslices ? d_count : ctx->run + (idx & 1);
        const uint64_t *base = idx == 0 ? nullptr : ctx->run + ((idx - 1) & 1);
        rc = enqueue_scan_list(ctx, m, d_o, d_list, d_list ? list_cap : 0, total, base, idx * slice_cubes, s);
        if (rc != DQMC_OK) return rc;
    }
    return DQMC_OK;
}

int dqmc_extract(dqmc_ctx *ctx, int n, const uint32_t *d_state, uint64_t *d_list, uint64_t list_cap,
                 uint64_t *d_count, void *stream)
{
    int rc = check_common(ctx, n);
    if (rc != DQMC_OK) return rc;
    if (d_state == nullptr || d_count == nullptr) return fail(ctx, DQMC_EINVAL, "%s", "NULL state or count");
    if (!aligned(d_state, kStateAlign) || !aligned(d_count, 8) || !aligned(d_list, 8))
        return fail(ctx, DQMC_EINVAL, "%s", "misaligned buffer");
    return enqueue_extract_tiles(ctx, n, kLowCount, const_cast<uint32_t *>(d_state), d_list, list_cap, d_count,
                                 (hipStream_t)stream);
}

int dqmc_bitmap_to_dense(dqmc_ctx *ctx, int n, const uint32_t *d_state, uint64_t *d_dense, void *stream)
{
    int rc = check_common(ctx, n);
    if (rc != DQMC_OK) return rc;
    if (d_state == nullptr || d_dense == nullptr) return fail(ctx, DQMC_EINVAL, "%s", "NULL state or output");
    if (!aligned(d_state, kStateAlign) || !aligned(d_dense, 8))
        return fail(ctx, DQMC_EINVAL, "%s", "misaligned buffer");
    hipStream_t s = (hipStream_t)stream;
    return run_pass(ctx, s, "to_dense", n, state_bytes(n) + 8.0 * (double)dqmc_dense_words(n), 0,
                    [&] { return launch_to_dense(n, d_state, d_dense, s); });
}

}  // extern "C"


extern "C" {

void dqmc_batch_destroy(dqmc_batch *b)
{
    if (b == nullptr) return;
    (void)hipSetDevice(b->ctx->device);
    if (b->mem) (void)hipFree(b->mem);
    delete b;
}

int dqmc_batch_create(dqmc_ctx *ctx, dqmc_job *d_jobs, int32_t njobs, dqmc_batch **out)
{
    if (out != nullptr) *out = nullptr;
    if (ctx == nullptr || out == nullptr) return DQMC_EINVAL;
    ctx->err[0] = 0;
    if (njobs < 0 || (uint32_t)njobs > kBatchMaxJobs || (d_jobs == nullptr && njobs > 0) || !aligned(d_jobs, 8))
        return fail(ctx, DQMC_EINVAL, "%s", "need 0 <= njobs <= 2^20 and an 8-byte aligned device job array");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DQMC_EDEVICE, "%s", "hipSetDevice failed");
    dqmc_batch *b = new dqmc_batch();
    b->ctx = ctx;
    b->d_jobs = d_jobs;
    b->njobs = njobs;
    b->mem = nullptr;
    b->col_cap = 0;
    b->order_mode = 0;
    const uint32_t cap = njobs > 0 ? (uint32_t)njobs : 1u;
    if (hipMalloc(&b->mem, batch_scratch_bytes(cap)) != hipSuccess) {
        dqmc_batch_destroy(b);
        return fail(ctx, DQMC_ENOMEM, "%s", "batch plan allocation failed");
    }
    b->bs = batch_scratch_at(b->mem, cap);
    b->ex = BatchExpect{};
    if (njobs > 0) {
        // the jobs' sizes, by the planner itself: the runs get exact grids
        std::vector<uint32_t> hdr(batch_header_words());
        if (launch_batch_plan(d_jobs, (uint32_t)njobs, b->bs, nullptr) != hipSuccess ||
            hipMemcpy(hdr.data(), b->bs.hdr, hdr.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) {
            dqmc_batch_destroy(b);
            return fail(ctx, DQMC_EDEVICE, "%s", "planning the batch failed");
        }
        batch_expect_from_header(hdr.data(), &b->ex);
    }
    *out = b;
    return DQMC_OK;
}

int dqmc_batch_config(dqmc_batch *b, int32_t col_cap, int32_t order)
{
    if (b == nullptr) return DQMC_EINVAL;
    if (col_cap < 0 || col_cap > kBatchMaxColCap || order < 0 || order >= kBatchModes)
        return fail(b->ctx, DQMC_EINVAL, "%s", "need 0 <= col_cap <= 4 and order 0 or 1");
    b->col_cap = col_cap;
    b->order_mode = order;
    return DQMC_OK;
}

int dqmc_batch_run(dqmc_batch *b, void *stream)
{
    if (b == nullptr) return DQMC_EINVAL;
    dqmc_ctx *ctx = b->ctx;
    ctx->err[0] = 0;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DQMC_EDEVICE, "%s", "hipSetDevice failed");
    if (b->njobs == 0) return DQMC_OK;
    hipStream_t s = (hipStream_t)stream;
    // the job sizes live on the device: no byte model for the profile record
    return run_pass(ctx, s, "batch", -1, 0.0, 8, [&] {
        return launch_batch(b->d_jobs, (uint32_t)b->njobs, b->bs, b->col_cap, b->order_mode, s, &b->ex);
    });
}

int dqmc_primes_batch(dqmc_ctx *ctx, dqmc_job *d_jobs, int32_t njobs, void *stream)
{
    if (ctx == nullptr) return DQMC_EINVAL;
    ctx->err[0] = 0;
    if (njobs < 0 || (uint32_t)njobs > kBatchMaxJobs || (d_jobs == nullptr && njobs > 0) || !aligned(d_jobs, 8))
        return fail(ctx, DQMC_EINVAL, "%s", "need 0 <= njobs <= 2^20 and an 8-byte aligned device job array");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DQMC_EDEVICE, "%s", "hipSetDevice failed");
    if (njobs == 0) return DQMC_OK;
    if ((uint32_t)njobs > ctx->batch_cap) {
        // grow the context's batch scratch (the only allocation of this call;
        // a call that does not grow it only enqueues)
        if (ctx->batch_mem != nullptr) {
            if (hipDeviceSynchronize() != hipSuccess) return fail(ctx, DQMC_EDEVICE, "%s", "synchronize failed");
            (void)hipFree(ctx->batch_mem);
            ctx->batch_mem = nullptr;
            ctx->batch_cap = 0;
        }
        if (hipMalloc(&ctx->batch_mem, batch_scratch_bytes((uint32_t)njobs)) != hipSuccess)
            return fail(ctx, DQMC_ENOMEM, "%s", "batch scratch allocation failed");
        ctx->batch_cap = (uint32_t)njobs;
    }
    const BatchScratch bs = batch_scratch_at(ctx->batch_mem, ctx->batch_cap);
    hipStream_t s = (hipStream_t)stream;
    return run_pass(ctx, s, "batch", -1, 0.0, 8, [&] {
        return launch_batch(d_jobs, (uint32_t)njobs, bs, 0, 0, s);
    });
}

int dqmc_hash_words(dqmc_ctx *ctx, const uint32_t *d_words, uint64_t nwords, uint64_t *d_out, void *stream)
{
    if (ctx == nullptr || d_out == nullptr || (d_words == nullptr && nwords > 0)) return DQMC_EINVAL;
    ctx->err[0] = 0;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DQMC_EDEVICE, "%s", "hipSetDevice failed");
    DQMC_HIP(ctx, launch_hash(d_words, nwords, d_out, (hipStream_t)stream));
    return DQMC_OK;
}

int dqmc_set_plan(dqmc_ctx *ctx, int n, const int32_t *sizes, int ngroups)
{
    if (ctx == nullptr) return DQMC_EINVAL;
    ctx->err[0] = 0;
    if (n <= kLowDigits || n > DQMC_MAX_N || ngroups < 0 || ngroups > DQMC_MAX_N ||
        (ngroups > 0 && sizes == nullptr))
        return fail(ctx, DQMC_EINVAL, "%s", "plan needs 12 < n <= 25 and 0 <= ngroups");
    int sum = 0;
    for (int i = 0; i < ngroups; ++i) {
        if (sizes[i] < 1 || sizes[i] > kMaxGroup) return fail(ctx, DQMC_EINVAL, "%s", "group size outside 1..6");
        sum += sizes[i];
    }
    if (ngroups > 0 && sum != n - kLowDigits) return fail(ctx, DQMC_EINVAL, "%s", "group sizes must sum to n - 12");
    if (ngroups > 0 && n - sizes[ngroups - 1] + 1 > kMaxGroupStart)
        return fail(ctx, DQMC_EINVAL, "%s", "a group may not start above digit 24 (32-bit row offsets)");
    for (int i = 0; i < ngroups; ++i) ctx->plan[n][i] = sizes[i];
    ctx->plan_len[n] = ngroups;
    return DQMC_OK;
}

int dqmc_get_plan(const dqmc_ctx *ctx, int n, int32_t *sizes, int cap)
{
    if (ctx == nullptr || n < 0 || n > DQMC_MAX_N || cap < 0 || (sizes == nullptr && cap > 0)) return DQMC_EINVAL;
    const std::vector<int> v = plan_sizes(ctx, n);
    for (int i = 0; i < (int)v.size() && i < cap; ++i) sizes[i] = v[i];
    return (int)v.size();
}

int dqmc_profile(dqmc_ctx *ctx, int enable)
{
    if (ctx == nullptr) return DQMC_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DQMC_EDEVICE, "%s", "hipSetDevice failed");
    if (enable && !ctx->events_made) {
        for (int i = 0; i < 2 * DQMC_MAX_RECORDS; ++i) DQMC_HIP(ctx, hipEventCreate(&ctx->ev[i]));
        ctx->events_made = true;
    }
    ctx->prof = enable != 0;
    ctx->nrec = 0;
    return DQMC_OK;
}

int dqmc_profile_read(dqmc_ctx *ctx, dqmc_pass_record *out, int cap)
{
    if (ctx == nullptr || (out == nullptr && cap > 0) || cap < 0) return DQMC_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DQMC_EDEVICE, "%s", "hipSetDevice failed");
    const int k = ctx->nrec < cap ? ctx->nrec : cap;
    for (int i = 0; i < k; ++i) {
        DQMC_HIP(ctx, hipEventSynchronize(ctx->ev[2 * i + 1]));
        float ms = 0.f;
        DQMC_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]));
        ctx->rec[i].ms = ms;
        out[i] = ctx->rec[i];
    }
    ctx->nrec = 0;
    return k;
}

int dqmc_flag_units(dqmc_ctx *ctx, uint64_t *h_units)
{
    if (ctx == nullptr || h_units == nullptr) return DQMC_EINVAL;
    for (int i = 0; i < 4; ++i) h_units[i] = 0;
    if (!ctx->flags_used) return DQMC_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DQMC_EDEVICE, "%s", "hipSetDevice failed");
    // three counters in the scan scratch (free between calls)
    unsigned long long *d = (unsigned long long *)ctx->sums;
    DQMC_HIP(ctx, hipMemsetAsync(d, 0, 3 * sizeof(unsigned long long), nullptr));
    DQMC_HIP(ctx, launch_flag_units(ctx->flags_low, ctx->flags_tile, d, nullptr));
    unsigned long long hu[3];
    DQMC_HIP(ctx, hipMemcpy(hu, d, sizeof(hu), hipMemcpyDeviceToHost));
    for (int i = 0; i < 3; ++i) h_units[i] = hu[i];
    h_units[3] = 1;
    return DQMC_OK;
}

}  // extern "C"
