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
    int n;
    int lw;             // block digits inside a tile (tw = 8 * 3^lw)
    uint32_t flip;      // XOR applied to the truth-table words (~0u: complement)
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
hipError_t launch_list(int n, const uint32_t *state, uint32_t tw, uint64_t ntiles, const uint32_t *counts,
                       const uint32_t *chunkmap, const uint64_t *offs, uint64_t *list, uint64_t cap, hipStream_t s,
                       uint64_t rho0 = 0);
hipError_t launch_low(int mode, const LowArgs &a, uint64_t nblocks, hipStream_t s);

// High-digit groups: one pass applies Merge and/or Reduce for a group of
// consecutive digits g0 .. g0+GR+GW-1 (g0 >= 13) with GR digits held in
// registers and GW digits spread over 3^GW wavefronts of one workgroup.
enum ColMode : int {
    kColMerge = 0,        // merge the group; outer digits binary; write * combos
    kColMergeReduce = 1,  // merge then reduce the group; write everything
    kColReduce = 2,       // reduce the group
};

// Highest first digit of a group: a group starting at digit g0 has rows
// L = 8 * 3^(g0-6) words apart, and lanes address a row with 32-bit offsets
// (L < 2^32 up to g0 = 24).
constexpr int kMaxGroupStart = 24;

struct ColArgs {
    uint32_t *state;
    uint64_t L;          // 8 * 3^(g0-6): words spanned by digits 1..g0-1
    uint64_t nlb;        // l-blocks
    uint64_t nouter;     // outer (above the group) combinations launched
    uint64_t nblocks;    // nlb * nouter
    int outer_binary;    // 1: outer index enumerates binary digit combos
};

hipError_t col_setup();    // also runs chunk_setup
hipError_t chunk_setup();  // occupancy caps of the chunked column kernel
hipError_t launch_col(int gr, int gw, int mode, const ColArgs &a, hipStream_t s);
// The chunked form (groups with at most one wave digit; launch_col picks it).
hipError_t launch_col_chunked(int gr, int gw, int mode, const ColArgs &a, hipStream_t s);
int col_lanes_per_block(int gw);  // l values per workgroup

// One function of a batch as the batch kernel sees it (device memory).
struct BatchJob {
    const uint32_t *tt;
    uint32_t *state;
    uint64_t *list;
    uint64_t cap;
    uint64_t *count;
    int32_t n;
    int32_t pad;
};

constexpr int kBatchWholeMaxN = 12;  // one workgroup runs the whole function
constexpr int kBatchTileMaxN = 16;   // tile-parallel; larger: the single-function path

hipError_t batch_setup();
// Persistent launch over njobs jobs (n <= kBatchWholeMaxN) in the given
// order (ticket zeroed first).
hipError_t launch_batch(const BatchJob *jobs, const uint32_t *order, uint32_t njobs, uint32_t *ticket,
                        uint32_t grid, hipStream_t s);

// A function with 13 <= n <= kBatchTileMaxN of a batch, run tile-parallel.
// Its 2^(n-12) tiles with binary digits 13..n are work items first_bin..,
// its 3^(n-12) tiles are first_tile.. in the batch's per-tile arrays.
struct TileJob {
    const uint32_t *tt;
    uint32_t *state;
    uint64_t *list;
    uint64_t cap;
    uint64_t *count;
    int32_t n;
    uint32_t first_bin;
    uint32_t first_tile;
    uint32_t pad;
};

struct TileBatch {
    const TileJob *jobs;
    const uint32_t *bin_job;   // per binary-tile work item: its function
    const uint32_t *tile_job;  // per tile: its function
    uint32_t *counts;          // per tile: set bits of the prime bitmap
    uint32_t *chunkmap;        // per tile: kMapWords words of non-zero chunks
    uint64_t *offs;            // per tile: list offset within its function
    uint32_t njobs;
    uint32_t nbin;
    uint32_t ntiles;
};

// The five launches of the tile-parallel batch path.
hipError_t launch_tile_batch(const TileBatch &b, hipStream_t s);

// Host: the work items of m functions with 13 <= n <= kBatchTileMaxN: fills
// tj[0..m), bin_job (2^(n-12) entries per function) and tile_job (3^(n-12)
// per function) and sets b.njobs, b.nbin, b.ntiles.
inline void tile_layout(const BatchJob *jobs, uint32_t m, TileJob *tj, uint32_t *bin_job, uint32_t *tile_job,
                        TileBatch &b)
{
    uint32_t nbin = 0, ntiles = 0;
    for (uint32_t i = 0; i < m; ++i) {
        const BatchJob &j = jobs[i];
        const int h = j.n - 12;
        tj[i] = TileJob{j.tt, j.state, j.list, j.cap, j.count, j.n, nbin, ntiles, 0};
        for (uint32_t k = 0; k < (1u << h); ++k) bin_job[nbin++] = i;
        uint32_t nt = 1;
        for (int q = 0; q < h; ++q) nt *= 3;
        for (uint32_t k = 0; k < nt; ++k) tile_job[ntiles++] = i;
    }
    b.njobs = m;
    b.nbin = nbin;
    b.ntiles = ntiles;
}

// Sliced path (k_slice.hip): the truth table of the restriction of f to the
// cube of its top variables given by fixed (bits equal to 1) and stars (bits
// that are *), on its lower m variables; and o &= ~mask on the chunks of each
// tile that the tile summary marks, with a new summary.
hipError_t launch_slice_tt(const uint32_t *tt, int m, uint32_t fixed, uint32_t stars, uint32_t flip, uint32_t *out,
                           hipStream_t s);
hipError_t launch_andnot_map(uint32_t *o, const uint32_t *mask, uint32_t *counts, uint32_t *chunkmap, uint64_t ntiles,
                             uint32_t tw, hipStream_t s);

hipError_t launch_fill_u64(uint64_t *p, uint64_t count, uint64_t value, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t s);
hipError_t launch_to_dense(int n, const uint32_t *state, uint64_t *dense, hipStream_t s);
hipError_t launch_hash(const uint32_t *w, uint64_t n, uint64_t *out, hipStream_t s);

}  // namespace dqmc
