// Internal launchers shared by the kernel files and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dqmc {

// Low tile: the cubes whose digits 13..n are fixed, i.e. 3^min(n-5, 7)
// consecutive blocks (8 * 3^min(n-5, 7) state words, 3^min(n,12) cubes),
// held in LDS.
enum LowMode : int {
    kLowMergeTT = 0,        // truth table -> merged tile (digits 1..12) -> state
    kLowPrimesTT = 1,       // n <= 12: truth table -> M -> O -> state + list
    kLowReduceCount = 2,    // state -> reduce digits 1..12 -> state + tile info
    kLowCount = 3,          // state -> tile info only (no transform, no write)
};

constexpr uint32_t kTileBlocks = 2187;            // 3^7 blocks: digits 6..12
constexpr uint32_t kTileWords = 8 * kTileBlocks;  // 17496 words (69,984 bytes)
// Memory slot of a tile in a state of n >= 13 variables: the tile's words
// and 8 padding words that are always 0, so that the slot (70,016 bytes) is a
// multiple of 128 bytes and every row of a column pass (rows lie a multiple
// of the slot apart) starts on a 128-byte line.
constexpr uint32_t kTileStride = kTileWords + 8;  // 17504 words

// Per-tile summary written by kLowReduceCount / kLowCount: the number of set
// bits, and a bitmap of the 64-word chunks that hold any set bit.
constexpr int kChunkWords = 64;
constexpr int kTileChunks = (kTileWords + kChunkWords - 1) / kChunkWords;  // 274
constexpr int kMapWords = (kTileChunks + 31) / 32;                         // 9

struct LowArgs {
    const uint32_t *tt;
    uint32_t *state;
    uint64_t *list;
    uint64_t cap;
    uint64_t *count;
    uint32_t *counts;   // per tile: number of set bits (count modes)
    uint32_t *chunkmap; // per tile: kMapWords words, bit k = chunk k non-zero
    uint64_t ntiles;
    uint32_t tw;        // words per tile
    uint32_t ts;        // words per tile slot in the state (kTileStride, or tw for one tile)
    int n;
    int lw;             // block digits inside a tile (tw = 8 * 3^lw)
    uint32_t flip;      // XOR applied to the truth-table words (~0u: complement)
    // final reduce (n > 12): per tile, kMapWords words marking the 64-word
    // chunks that may hold a set bit (the others are zero in the state), or
    // nullptr
    const uint32_t *tile_flags;
    // final reduce with chunk flags: tiles left to the full-tile kernel, count
    // at [0] and tile indices from [1] (written by the compact kernel, read by
    // the full-tile kernel; nullptr otherwise)
    uint32_t *deferred;
};

constexpr int kLowThreads = 256;

hipError_t low_setup();

// Exclusive scan of the tile counts into offs (uint64, one per tile) and the
// total into *count.  With base != nullptr every offset and the total start
// at *base (a list continued from an earlier call; base != count).
hipError_t launch_scan_counts(const uint32_t *counts, uint64_t ntiles, uint64_t *offs, uint64_t *count,
                              uint64_t *sums, hipStream_t s, const uint64_t *base = nullptr);
uint64_t scan_scratch_words(uint64_t ntiles);  // size of `sums`
// List of the set bits of the tiles in increasing cube index, using the tile
// summaries and offsets (only chunks marked non-zero are read).
// rho0 is added to every listed cube index (a slice's place in a larger
// function).
hipError_t launch_list(int n, const uint32_t *state, uint32_t tw, uint32_t ts, uint64_t ntiles, const uint32_t *counts,
                       const uint32_t *chunkmap, const uint64_t *offs, uint64_t *list, uint64_t cap, hipStream_t s,
                       uint64_t rho0 = 0);
hipError_t launch_low(int mode, const LowArgs &a, uint64_t nblocks, hipStream_t s);
// Final reduce of full tiles with chunk flags (a.tile_flags and a.deferred
// set): the compact kernel on every tile, then the full-tile kernel on the
// tiles it deferred (more non-zero blocks than its LDS holds).
hipError_t launch_low_compact(const LowArgs &a, hipStream_t s);

// High-digit groups: one pass applies Merge and/or Reduce for a group of
// consecutive digits g0 .. g0+GR+GW-1 (g0 >= 13) with GR digits held in
// registers and GW digits spread over 3^GW wavefronts of one workgroup.
enum ColMode : int {
    kColMerge = 0,        // merge the group; outer digits binary; write * combos
    kColMergeReduce = 1,  // merge then reduce the group; write everything
    kColReduce = 2,       // reduce the group
};

// Highest first digit of a group: a group starting at digit g0 has rows
// L = kTileStride * 3^(g0-13) words apart, and lanes address a row with 32-bit
// offsets (L < 2^32 up to g0 = 24: 3.1e9 words).
constexpr int kMaxGroupStart = 24;

struct ColArgs {
    uint32_t *state;
    uint64_t L;          // words spanned by digits 1..g0-1 (kTileStride * 3^(g0-13))
    uint64_t nlb;        // l-blocks
    uint64_t nouter;     // outer (above the group) combinations launched
    uint64_t nblocks;    // nlb * nouter
    int outer_binary;    // 1: outer index enumerates binary digit combos
    // Column blocks cut per tile slot (col_kernel<4, 2> only): 0, or the
    // blocks per slot (kFlagLowBlocks): block lb covers words 64 (lb mod
    // slot_blocks) .. of slot lb / slot_blocks of the rows, the last one of a
    // slot half full.
    uint32_t slot_blocks;
    // Row flags (col_kernel<4, 2> only; nullptr: none).  The merge+reduce
    // mode writes, per column block, a bit per row of its 729 (set: the row's
    // words of the block hold a set bit after the pass), kFlagWords words per
    // block; it runs with slot_blocks set, so that its blocks are those of
    // the reduce pass.
    // The reduce mode reads kFlagWords words per block in its own row order
    // (launch_flag_transpose) and loads and stores only the flagged rows.
    uint32_t *flags;
};

// Row flags from the top group's merge+reduce (digits 19..24) to the reduce
// of digits 13..18 at n = 24 (plan [6, 6]): both passes have 729 rows per
// column block.  The top pass's block (c, lb) (slot-aligned: words 64 lb ..
// 64 lb + 63 of slot c, in each of its rows 729 kTileStride words apart) is
// the reduce pass's block (lb, o) in its row c for every o.
constexpr uint32_t kFlagWords = 23;                                   // 729 bits
constexpr uint64_t kFlagLowBlocks = (kTileStride + 63) / 64;          // 274 per slot
constexpr uint64_t kFlagTopBlocks = 729ull * kFlagLowBlocks;          // 199746
// Bit o of word c / 32 of block (o, lb) of the reduce pass = bit o of the
// top pass's block (c, lb).
hipError_t launch_flag_transpose(const uint32_t *top, uint32_t *low, hipStream_t s);
// The reduce pass's row flags (rows that may hold a bit as it loads them, a
// superset of what it leaves) as chunk flags of the n = 24 tiles: bit k of
// word k / 32 of tile c + 729 o = bit c of the reduce pass's block (o, k).
hipError_t launch_tile_flags(const uint32_t *low, uint32_t *tiles, uint32_t *deferred, hipStream_t s);
// Bytes the flagged passes move (see dqmc_flag_units) into units[0..2]
// (device, zeroed by the caller).
hipError_t launch_flag_units(const uint32_t *low, const uint32_t *tiles, unsigned long long *units, hipStream_t s);

hipError_t col_setup();    // also runs chunk_setup
hipError_t chunk_setup();  // occupancy caps of the chunked column kernel
hipError_t launch_col(int gr, int gw, int mode, const ColArgs &a, hipStream_t s);
// The chunked form (groups with at most one wave digit; launch_col picks it).
hipError_t launch_col_chunked(int gr, int gw, int mode, const ColArgs &a, hipStream_t s);
int col_lanes_per_block(int gw);  // l values per workgroup

// Batch of many functions (k_batch.hip): jobs with n <= kBatchWholeMaxN run
// whole in one workgroup; jobs with kBatchWholeMaxN < n <= kBatchMaxN run
// tile-parallel, one launch per pass.
constexpr int kBatchWholeMaxN = 12;
constexpr int kBatchMaxN = 16;
constexpr uint32_t kBatchMaxJobs = 1u << 20;
constexpr int kBatchThreads = 768;
constexpr int kBatchModes = 2;       // item orders of the first launch
constexpr int kBatchMaxColCap = 4;   // column-launch workgroups per CU, as a cap (0: none)
constexpr uint32_t kLdsPerCu = 160 * 1024;

// Header of a batch's work items (uint32 words, written by the planner).
constexpr int kBatchHdrWords = 256;

// Device scratch of a batch of up to `cap` jobs, in one allocation.
struct BatchScratch {
    uint32_t *hdr;       // kBatchHdrWords words: ticket, segment sizes, bin bases
    uint32_t *order;     // cap: job indices sorted by n, largest first (stable)
    uint32_t *counts;    // 81 * cap: per tile, set bits of the prime bitmap
    uint32_t *chunkmap;  // 81 * kMapWords * cap: per tile, non-zero chunks
    uint64_t *offs;      // 81 * cap: per tile, list offset within its function
    uint32_t cap;
};

uint64_t batch_scratch_bytes(uint32_t cap);
// Lay out a scratch of batch_scratch_bytes(cap) bytes at `base` (256-byte
// aligned).
BatchScratch batch_scratch_at(void *base, uint32_t cap);

// The valid jobs per n that a batch's launches are sized for (exact = 1), or
// nothing known (exact = 0: the launches are sized by bounds).
struct BatchExpect {
    uint32_t hist[kBatchMaxN + 1];
    uint32_t exact;
};

hipError_t batch_setup();
// Enqueue the planner and the five pass launches for the device-resident job
// array `jobs` (njobs <= s.cap); col_cap = at most this many column-pass
// workgroups per CU (0: no cap), mode 0: whole-function items before the
// truth-table tiles, 1: after them.  With ex->exact the launches get exact
// grids, and a
// run whose jobs' sizes differ from ex->hist does nothing but set every
// status to DQMC_EINVAL.
hipError_t launch_batch(void *jobs, uint32_t njobs, const BatchScratch &s, int col_cap, int mode, hipStream_t st,
                        const BatchExpect *ex = nullptr);
// The planner alone (checks the jobs, writes their statuses and the header).
hipError_t launch_batch_plan(void *jobs, uint32_t njobs, const BatchScratch &s, hipStream_t st);
// The histogram a planner run left in the header (copied to the host).
void batch_expect_from_header(const uint32_t *hdr_host, BatchExpect *ex);
uint32_t batch_header_words();

// Sliced path (k_slice.hip): the truth table of the restriction of f to the
// cube of its top variables given by fixed (bits equal to 1) and stars (bits
// that are *), on its lower m variables; and o &= ~mask on the chunks of each
// tile that the tile summary marks, with a new summary.
hipError_t launch_slice_tt(const uint32_t *tt, int m, uint32_t fixed, uint32_t stars, uint32_t flip, uint32_t *out,
                           hipStream_t s);
hipError_t launch_andnot_map(uint32_t *o, const uint32_t *mask, uint32_t *counts, uint32_t *chunkmap, uint64_t ntiles,
                             uint32_t tw, uint32_t ts, hipStream_t s);

hipError_t launch_fill_u64(uint64_t *p, uint64_t count, uint64_t value, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t s);
hipError_t launch_to_dense(int n, const uint32_t *state, uint64_t *dense, hipStream_t s);
hipError_t launch_hash(const uint32_t *w, uint64_t n, uint64_t *out, hipStream_t s);

}  // namespace dqmc
