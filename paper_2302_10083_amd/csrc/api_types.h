// Host-side state behind the opaque handles of the C ABI (dqmc_ctx,
// dqmc_batch); shared by the entry points and the autotuner.
#pragma once

#include "dqmc.h"
#include "launch.h"

struct dqmc_ctx {
    int device;
    int ncu;  // compute units of the device
    // per low tile: count of set bits, non-zero chunk map, list offset
    uint64_t tiles_cap;
    uint32_t *counts;
    uint32_t *chunkmap;
    uint64_t *offs;
    uint64_t *sums;  // per-block sums of the count scan
    uint32_t *slice_tt;  // sliced path: truth table of one slice (2^20 words)
    uint32_t *split_tt;  // top-digit split: truth table of one third (2^19 words)
    uint64_t *run;       // sliced path: running prime counts (2)
    // row flags of the n = 24 passes (plan [6, 6]): the top group's pass
    // writes flags_top, a transpose turns them into flags_low for the reduce
    // of digits 13..18 (kFlagTopBlocks and 729 kFlagLowBlocks blocks of
    // kFlagWords words)
    uint32_t *flags_top;
    uint32_t *flags_low;
    uint32_t *flags_tile;  // the same as chunk flags of the final reduce (3^12 tiles of kMapWords words)
    uint32_t *deferred;    // final reduce: count and list of the tiles the compact kernel left (3^12 + 1 words)
    bool flags_used;       // the last n = 24 computation wrote them
    void *batch_mem;     // dqmc_primes_batch: scratch for up to batch_cap jobs (grown on demand)
    uint32_t batch_cap;
    char err[512];
    // per-pass timing (diagnostics)
    bool prof;
    bool events_made;
    int nrec;
    hipEvent_t ev[2 * DQMC_MAX_RECORDS];
    dqmc_pass_record rec[DQMC_MAX_RECORDS];
    // pass plan overrides: group sizes of digits 13..n (0 groups = default)
    int plan_len[DQMC_MAX_N + 1];
    // top-digit split of dqmc_primes per n: -1 default, 0 off, 1 on
    int split[DQMC_MAX_N + 1];
    int plan[DQMC_MAX_N + 1][DQMC_MAX_N];
};

struct dqmc_batch {
    dqmc_ctx *ctx;
    dqmc_job *d_jobs;  // the caller's device-resident job array
    int32_t njobs;
    void *mem;               // the plan's scratch (one allocation)
    dqmc::BatchScratch bs;   // laid out in mem
    dqmc::BatchExpect ex;    // the jobs' sizes at creation: the launches' exact grids
    int32_t col_cap;         // column-pass workgroups per CU (0: no cap)
    int32_t order_mode;      // order of the first launch's items
};
