/*
 * dqmc.h - C ABI of libdqmc: all prime implicants of a Boolean function from
 * its full truth table, on an AMD Instinct MI355X (gfx950).
 *
 * Method: the dense bit-slice Quine-McCluskey algorithm of Udovenko,
 * "DenseQMC: an efficient bit-slice implementation of the Quine-McCluskey
 * algorithm" (arXiv 2302.10083): the implicant indicator M over all 3^n
 * ternary cubes (MergeAll), the prime indicator O (ReduceAll), then the list
 * of primes (Sec. 4, Alg. 3 and Alg. 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  n         number of variables, 0 <= n <= DQMC_MAX_N.
 *  cube      a string s in {0,1,*}^n (Sec. 2); its index is
 *            rho(s) = sum_{i=1..n} 3^(i-1) rho(s_i), rho(0)=0, rho(1)=1,
 *            rho(*)=2 (Sec. 4.2).  Digit i of a cube carries the literal on
 *            variable x_i.
 *  truth     little-endian uint32 words, dqmc_tt_words(n) of them; bit x
 *  table     (word x/32, bit x%32) is f(x), where variable x_i is bit i-1 of
 *            x.  Bits at x >= 2^n (only when n < 5) are ignored.
 *  state     the 3^n-bit cube bitmap in the "H5" block layout (the bottom
 *            layer of Sec. 4.2 with h = 5): dqmc_state_words(n) uint32 words,
 *            grouped in 256-bit blocks of 8 words; cube rho lives in block
 *            rho/243 at bit p = rho%243, i.e. bit p%32 of the logical word
 *            W = 8*(rho/243) + p/32.  For n <= 12 W is the state word.  For
 *            n > 12 the state is 3^(n-12) slots of 17504 words: a tile of
 *            17496 words (the 2187 blocks of one value of digits 13..n)
 *            followed by 8 words that are always 0, so W lies at word
 *            (W/17496)*17504 + W%17496 (every slot starts on a 128-byte
 *            line).  For n < 5 there is one block and cube rho is bit rho
 *            of it.  Bits 243..255 of every block (bits >= 3^n for n < 5)
 *            are always 0.  The order of the words is increasing rho.
 *            States must be 16-byte aligned (DQMC_EINVAL otherwise).
 *  list      uint64 cube indices rho, strictly increasing.
 *  stream    a hipStream_t passed as void* (NULL = the null stream).
 *
 *  Ownership: the caller owns and allocates every buffer argument (device
 *  memory unless stated otherwise).  The context owns small scratch memory
 *  allocated when it is created, a batch plan owns its job table allocated
 *  by dqmc_batch_create, a server owns the arena it reserves in
 *  dqmc_server_create; no other entry point allocates device memory (the
 *  autotuning calls create and destroy two HIP events).
 *  Asynchrony: compute entry points only enqueue work on `stream` and return;
 *  results are valid after the stream is synchronised.  Argument errors are
 *  found on the host before anything is enqueued and return DQMC_EINVAL;
 *  dqmc_last_error() then describes the problem.
 *  Concurrency: a context's scratch serves one call at a time; calls that use
 *  one context must be ordered (same stream, or synchronised in between).
 *  Use one context per concurrently used stream.
 */
#ifndef DQMC_H
#define DQMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DQMC_MAX_N 25

typedef enum {
    DQMC_OK = 0,
    DQMC_EINVAL = -1,  /* bad argument (n out of range, NULL, bad size) */
    DQMC_ENOMEM = -2,  /* device allocation failed (context creation only) */
    DQMC_EDEVICE = -3, /* a HIP runtime call failed */
    DQMC_ESCRATCH = -4, /* beyond the fixed scratch of dqmc_primes_noalloc */
    DQMC_EIO = -5       /* a tuning file could not be opened, read or written */
} dqmc_status;

typedef struct dqmc_ctx dqmc_ctx;

/* Create a context on HIP device `device` and allocate its scratch (under
 * 100 MB: per-tile summaries and offsets for n = DQMC_MAX_N, and the slice
 * truth tables of the sliced path and of the top-digit split).  Returns DQMC_ENOMEM / DQMC_EDEVICE on failure, with
 * *out set to NULL. */
int dqmc_create(int device, dqmc_ctx **out);

/* Free the context and its scratch.  NULL is ignored.  No call may be in
 * flight on the context. */
void dqmc_destroy(dqmc_ctx *ctx);

/* Message for the last failed call on this context (static storage owned by
 * the context; "" if none).  Thread-compatible, not thread-safe. */
const char *dqmc_last_error(const dqmc_ctx *ctx);

/* Sizes (pure functions; 0 when n is out of range). */
uint64_t dqmc_num_cubes(int n);    /* 3^n (Sec. 4.1: the state has one bit per cube) */
uint64_t dqmc_tt_words(int n);     /* max(1, 2^(n-5)) uint32 words */
uint64_t dqmc_state_words(int n);  /* 8 * 3^max(n-5, 0) uint32 words up to n = 12, 17504 * 3^(n-12) above */
uint64_t dqmc_dense_words(int n);  /* ceil(3^n / 64) uint64 words */

/* Implicant bitmap M (Sec. 4.1, Lemma on MergeAll/ReduceAll; computed by the
 * per-dimension Merge transforms of Alg. 3 / Alg. 4): bit rho of d_state is
 * set iff cube rho is an implicant of f, i.e. f(x) = 1 for every x the cube
 * covers (Sec. 2, Def. of implicant).
 *   d_tt     device, dqmc_tt_words(n) words, read only.
 *   d_state  device, dqmc_state_words(n) words, fully overwritten.
 * Errors: DQMC_EINVAL for n out of range or NULL pointers. */
int dqmc_implicants(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint32_t *d_state, void *stream);

/* Prime implicants (Sec. 2, Def. of prime implicant; Sec. 4.1 ReduceAll and
 * Alg. 4 including its output step): d_state receives the prime bitmap O
 * (bit rho set iff cube rho is a prime implicant), and the primes' indices
 * are written to d_list in increasing order.
 *   d_tt      device, dqmc_tt_words(n) words, read only.
 *   d_state   device, dqmc_state_words(n) words, fully overwritten with O.
 *   d_list    device, room for list_cap uint64; may be NULL (count only).
 *   d_count   device, one uint64: the total number of primes.
 * Capacity: if the total exceeds list_cap, only the list_cap smallest
 * indices are written (this is not an error); O stays in d_state and
 * dqmc_extract can be called again with a larger list. */
int dqmc_primes(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint32_t *d_state, uint64_t *d_list,
                uint64_t list_cap, uint64_t *d_count, void *stream);

/* Complement mode (Sec. 1, "New method": the primes of a function give its
 * DNF, the primes of its complement give its CNF; the dense method suits the
 * CNF of a sparse function).  With flags = DQMC_NEGATE the truth table is
 * complemented as it is loaded: the results are those of dqmc_implicants /
 * dqmc_primes for NOT f, without a complemented copy of the table.  Each
 * prime implicant s of NOT f is the prime clause of f that ORs, for every
 * digit s_i != *, the literal x_i if s_i = 0 and NOT x_i if s_i = 1.
 * flags = 0 is the plain call.  Other bits: DQMC_EINVAL.  Arguments and
 * errors otherwise as dqmc_implicants / dqmc_primes. */
#define DQMC_NEGATE 1u
int dqmc_implicants_ex(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint32_t flags, uint32_t *d_state, void *stream);
int dqmc_primes_ex(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint32_t flags, uint32_t *d_state, uint64_t *d_list,
                   uint64_t list_cap, uint64_t *d_count, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * results as dqmc_primes (prime bitmap O in d_state, sorted list, count), with
 * no context.  Its kernels keep their per-tile summaries, list offsets and
 * scan sums in a fixed device array of the library (27.6 MB: the summaries of
 * the 3^12 tiles of n = 24; held on each device that runs the library until
 * the process ends), so the call allocates nothing.  It runs on the current HIP
 * device with the default pass plan and no top-digit split.
 *   n         0 <= n <= 24.  n = 25 returns DQMC_ESCRATCH (its tile summaries
 *             do not fit the fixed scratch); n outside [0, 25]: DQMC_EINVAL.
 *   d_tt, d_state, d_list, list_cap, d_count: as for dqmc_primes.
 * Calls on one device share that device's scratch: calls that overlap on one
 * device (different streams, or different host threads without ordering)
 * race and give wrong results; order them.  Nothing in the scratch needs to
 * start at zero (every call overwrites what it reads).  The first call on a
 * device looks up the scratch's device address and sets kernel attributes.
 * Errors: DQMC_EINVAL (n, NULL, alignment), DQMC_ESCRATCH, DQMC_EDEVICE; there
 * is no context, so no dqmc_last_error text. */
int dqmc_primes_noalloc(int n, const uint32_t *d_tt, uint32_t *d_state, uint64_t *d_list, uint64_t list_cap,
                        uint64_t *d_count, void *stream);

/* Sparse path (Sec. 5): the classic level-by-level Quine-McCluskey method
 * (Alg. 1) with hash-based neighbour search, for functions of low density,
 * where the number of implicants is far below 3^n.  Cubes are 2n-bit keys
 * (Sec. 5, bit-based representation); each implicant is generated once, at
 * its first star (Sec. 5, avoiding repeated generation); every level is a
 * linear-probing hash set whose redundant entries are marked, never removed
 * (Sec. 5, two-stage custom hash set).  The output is the same as
 * dqmc_primes's list and count (no bitmap), for 0 <= n <= DQMC_SPARSE_MAX_N.
 *   d_tt      device, dqmc_tt_words(n) words (2^(n-5) for n > 25 too).
 *   d_list    device, room for list_cap uint64; may be NULL (count only).
 *   d_count   device, one uint64.
 *   d_work    device workspace of work_bytes (256-byte aligned), owned by the
 *             caller: two levels (list + set), the prime keys and their
 *             sorted copy, and the sort's scratch.
 *   h_need    host uint64[2] or NULL: receives the largest level and the
 *             number of primes seen, also when the workspace was too small;
 *             dqmc_sparse_workspace_bytes(n, h_need[0], h_need[1]) is then
 *             enough for a second call.
 * The call is synchronous: it waits for the stream after every level (the
 * level sizes decide the next launches).  Errors: DQMC_EINVAL (n, NULL,
 * alignment), DQMC_ENOMEM (workspace too small; nothing is written to
 * d_list/d_count), DQMC_EDEVICE. */
#define DQMC_SPARSE_MAX_N 31
uint64_t dqmc_sparse_workspace_bytes(int n, uint64_t max_level, uint64_t max_primes);
int dqmc_sparse_primes(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint64_t *d_list, uint64_t list_cap,
                       uint64_t *d_count, void *d_work, uint64_t work_bytes, uint64_t *h_need, void *stream);

/* Sliced path: functions with more variables than one state can hold
 * (n up to DQMC_SLICED_MAX_N), cut along their top t variables into 3^t
 * slices of m = n - t variables, m <= DQMC_MAX_N.
 * For a cube a over x_{m+1..n} (digit j of a is the literal on x_{m+1+j}),
 * f_a is the function of x_1..x_m that ANDs f over the minterms of a.  The
 * cube s.a (digits 1..m from s, m+1..n from a) is an implicant of f iff s is
 * an implicant of f_a, so MergeAll (Sec. 4.1) of slice a is MergeAll of f_a.
 * The one-step form of ReduceAll (Sec. 4.1, Lemma) splits into the low
 * digits, which give the primes of f_a, and the top digits:
 *     s.a is prime  <=>  s is a prime of f_a and, for every binary digit j
 *                        of a, s is not an implicant of f_{a[j <- *]}.
 * Per slice, in increasing order of a (as a base-3 number, * = 2): the primes
 * of f_a into d_o; for every binary digit j the implicants of f_{a[j <- *]}
 * into d_m (kept from the previous slice when it is the same function; see
 * dqmc_primes_sliced_multi for more states) and d_o &= ~d_m; then the
 * slice's primes are appended to the list.
 *   d_tt      device, the n-variable truth table: 2^(n-5) words (1 for n < 5).
 *   flags     0 or DQMC_NEGATE (the primes of NOT f).
 *   d_o, d_m  device, dqmc_state_words(n - t) words each: slice states, used
 *             as scratch; their contents afterwards are unspecified.  They
 *             must not overlap.
 *   d_list    device, room for list_cap uint64 (may be NULL: count only).
 *   d_count   device, one uint64: the number of primes of f.
 * The list and capacity rules are those of dqmc_primes: the list_cap smallest
 * indices rho over all n digits, in increasing order.  Unlike dqmc_primes
 * there is no n-variable bitmap, so a list that was too small needs a second
 * call.  Errors: DQMC_EINVAL (n, t, NULL, alignment, flags), DQMC_EDEVICE. */
#define DQMC_SLICED_MAX_N 30
#define DQMC_SLICED_MAX_T 8
int dqmc_primes_sliced(dqmc_ctx *ctx, int n, int t, const uint32_t *d_tt, uint32_t flags, uint32_t *d_o,
                       uint32_t *d_m, uint64_t *d_list, uint64_t list_cap, uint64_t *d_count, void *stream);

/* dqmc_primes_sliced with nm implicant states instead of one: d_ms is a
 * host array of nm device pointers (1 <= nm <= DQMC_SLICED_MAX_STATES), each
 * to dqmc_state_words(n - t) words, disjoint from each other and from d_o.
 * The states keep the star neighbours' implicant bitmaps between slices; a
 * missing one goes to the state whose bitmap is needed again last, so more
 * states mean fewer recomputed bitmaps (n = 27, t = 3: 44 with one state, 28
 * with four).  Same results and errors as dqmc_primes_sliced, which is this
 * call with nm = 1. */
#define DQMC_SLICED_MAX_STATES 16
int dqmc_primes_sliced_multi(dqmc_ctx *ctx, int n, int t, const uint32_t *d_tt, uint32_t flags, uint32_t *d_o,
                             uint32_t *const *d_ms, int nm, uint64_t *d_list, uint64_t list_cap, uint64_t *d_count,
                             void *stream);

/* Extraction alone (Alg. 4, output step): every set bit of a state bitmap,
 * as increasing cube indices.  Same list/capacity/count rules as
 * dqmc_primes; d_state is read only. */
int dqmc_extract(dqmc_ctx *ctx, int n, const uint32_t *d_state, uint64_t *d_list, uint64_t list_cap,
                 uint64_t *d_count, void *stream);

/* Repack a block state into the exact 3^n-bit bitmap: bit rho of the
 * little-endian uint64 array d_dense (dqmc_dense_words(n) words, fully
 * overwritten; bits >= 3^n are 0).  Interoperability and tests; not part of
 * the prime computation. */
int dqmc_bitmap_to_dense(dqmc_ctx *ctx, int n, const uint32_t *d_state, uint64_t *d_dense, void *stream);

/* One function of a batch.  The array of jobs lives in HOST memory; the
 * buffers it points to are device memory with the sizes and meaning of
 * dqmc_primes (list may be NULL).  `status` is written by the library:
 * DQMC_OK, or DQMC_EINVAL for a malformed job, which is skipped while the
 * other jobs still run. */
typedef struct {
    int32_t n;
    int32_t status;
    const uint32_t *tt;
    uint32_t *state;
    uint64_t *list;
    uint64_t list_cap;
    uint64_t *count;
} dqmc_job;

/* Prime implicants of many independent functions (the batch bit-slicing of
 * independent executions, Sec. 4.2), from a DEVICE-RESIDENT job array.
 *
 * Every call only enqueues kernels on `stream` and returns.  A planner (one
 * workgroup) checks each job and writes jobs[i].status on the device
 * (DQMC_OK, or DQMC_EINVAL for n outside 0..16, a NULL tt/state/count, or a
 * misaligned buffer: tt 4, state 16, count and list 8 bytes), sorts the valid
 * jobs by n and lays out the work items of every pass; five launches then
 * work through them: the whole-function items (n <= 12: the whole pipeline in
 * one workgroup, largest first) with the truth-table tiles of the jobs with
 * 13 <= n <= 16, then that group's column pass, tile reduces with summaries,
 * count scans and lists.
 * Results are valid after the stream is synchronised; each job's result is
 * exactly what dqmc_primes gives for it alone (list: the min(count,
 * list_cap) smallest primes; list may be NULL).  Functions with n > 16 are
 * not batched: use dqmc_primes.
 *   d_jobs   device array of njobs dqmc_job (8-byte aligned), read by the
 *            kernels, status fields written; the buffers it points to must
 *            stay valid until the work completes.  0 <= njobs <= 2^20.
 *
 * dqmc_primes_batch: uses the context's batch scratch (the job order and the
 * per-tile summaries, about 3.9 KB per job), which the call allocates when
 * njobs exceeds every earlier call's (then it also synchronises the device
 * before freeing the smaller one); other calls allocate nothing.  Calls on one
 * context must be ordered.
 * Plans own their scratch, so that a run allocates nothing and can be
 * captured in a HIP graph and replayed:
 *   dqmc_batch_create: allocates the plan's scratch for njobs jobs and runs
 *     the planner once (synchronously) to learn how many valid jobs of each
 *     n the array holds; the plan's launches are then sized exactly
 *     (dqmc_primes_batch, which knows nothing of the jobs, launches by
 *     bounds: up to 81 tiles per job, the idle workgroups exiting at once).
 *     Between runs the jobs' buffers may change; their sizes may not: a run
 *     that finds different numbers of valid jobs per n does nothing and sets
 *     every status to DQMC_EINVAL.  DQMC_EINVAL (NULL, njobs out of range,
 *     misaligned array), DQMC_ENOMEM, DQMC_EDEVICE.
 *   dqmc_batch_config: col_cap = at most this many workgroups per compute
 *     unit in the column pass (0, the default: as many as its registers
 *     allow, four; 1..4 otherwise), order 0 (default): the whole-function
 *     items (largest first) before the truth-table tiles in the first
 *     launch, 1: after them.  DQMC_EINVAL outside those ranges.
 *   dqmc_batch_run: enqueue the planner and the five launches.
 *   dqmc_batch_destroy: free the plan (no run may be in flight). */
typedef struct dqmc_batch dqmc_batch;
int dqmc_batch_create(dqmc_ctx *ctx, dqmc_job *d_jobs, int32_t njobs, dqmc_batch **out);
int dqmc_batch_config(dqmc_batch *plan, int32_t col_cap, int32_t order);
int dqmc_batch_run(dqmc_batch *plan, void *stream);
void dqmc_batch_destroy(dqmc_batch *plan);
int dqmc_primes_batch(dqmc_ctx *ctx, dqmc_job *d_jobs, int32_t njobs, void *stream);

/* ---------------------------------------------------------------------------
 * Serving: a request loop over one device.
 *
 * Jobs (one truth table each, copied from host memory at submission) are
 * admitted while the device-memory budget and the execution slots allow it:
 * the server reserves its whole budget as one device arena when it is
 * created, and a job takes one block of its footprint - its state
 * (dqmc_state_words(n) words), a list reserve of min(3^n, max(2^18,
 * 3^(n-3)/16)) entries, its truth table and its count, each rounded up to
 * 256 bytes.  Jobs with n <= 16 that are admitted together run as one batch
 * (the planned persistent launch of dqmc_primes_batch); larger jobs run on
 * their own stream and
 * context.  Jobs that arrive
 * while others run are admitted as memory and slots free up (continuous
 * batching), and their work overlaps on the device.  Results stay on the
 * device until released; the result of a job is exactly what dqmc_primes
 * gives for it alone (the list holds min(count, reserve) smallest primes).
 *
 *   dqmc_server_create: budget in bytes of device memory for resident jobs
 *     (0 = 90% of the device memory free at creation; allocated here),
 *     slots = number of concurrent large jobs (streams; 0 = 4).  Starts the
 *     scheduler thread.
 *   dqmc_server_submit: copies the table; *id receives the job id.
 *     DQMC_EINVAL for bad n / NULL, DQMC_ENOMEM if the footprint exceeds the
 *     whole budget.  Never waits for the device.
 *   dqmc_server_poll: 1 if the job finished (*out filled), 0 if not yet,
 *     negative on error (unknown id).  dqmc_server_wait blocks until done;
 *     it returns DQMC_ENOMEM instead if the job cannot be admitted while
 *     nothing runs (the budget is held by results not yet released).
 *   dqmc_server_release: frees a finished job's device memory.
 *   dqmc_server_read: copies a finished job's list (up to cap entries) into
 *     host memory and returns the number copied (negative on error).  The
 *     copy runs without the server's lock (scheduling goes on meanwhile); a
 *     read and a release of the same job must not overlap.
 *   dqmc_server_destroy: waits for running jobs, drops jobs that are
 *     still queued, frees everything; no other call on the server may be
 *     in progress.
 * Times are seconds on one monotonic host clock. */
typedef struct dqmc_server dqmc_server;

typedef struct {
    int32_t n;
    int32_t status;           /* DQMC_OK, or the error of the job's launch */
    uint64_t count;           /* number of primes */
    uint64_t listed;          /* entries in list: min(count, reserve) */
    const uint32_t *state;    /* device: prime bitmap (block layout) */
    const uint64_t *list;     /* device: the smallest `listed` primes, increasing */
    double t_submit, t_admit, t_done;
} dqmc_result;

int dqmc_server_create(int device, uint64_t budget_bytes, int32_t slots, dqmc_server **out);
int dqmc_server_submit(dqmc_server *srv, int32_t n, const uint32_t *h_tt, uint64_t *id);
int dqmc_server_poll(dqmc_server *srv, uint64_t id, dqmc_result *out);
int dqmc_server_wait(dqmc_server *srv, uint64_t id, dqmc_result *out);
int dqmc_server_release(dqmc_server *srv, uint64_t id);
int64_t dqmc_server_read(dqmc_server *srv, uint64_t id, uint64_t *h_list, uint64_t cap);
void dqmc_server_destroy(dqmc_server *srv);

/* Order-dependent 64-bit hash of nwords uint32 device words (diagnostics:
 * comparing device-resident bitmaps without copying them), written to
 * *d_out (device). */
int dqmc_hash_words(dqmc_ctx *ctx, const uint32_t *d_words, uint64_t nwords, uint64_t *d_out, void *stream);

/* ---------------------------------------------------------------------------
 * Tuning: the pass plan.
 *
 * For n > 12 the digits 13..n are processed by column passes over groups of
 * consecutive digits (Alg. 4's top-layer dimensions, several per memory
 * sweep).  dqmc_set_plan chooses the group sizes used by this context for
 * functions with n variables: sizes[0..ngroups) are the group sizes from
 * digit 13 upwards, each in 1..6, summing to n - 12.  ngroups == 0 restores
 * the default plan.  Every plan gives identical results; only speed differs.
 * dqmc_get_plan writes the plan in use (at most cap sizes) and returns the
 * number of groups.  Errors: DQMC_EINVAL for a bad n or bad sizes.
 */
int dqmc_set_plan(dqmc_ctx *ctx, int n, const int32_t *sizes, int ngroups);
int dqmc_get_plan(const dqmc_ctx *ctx, int n, int32_t *sizes, int cap);

/* Top-digit split of dqmc_primes / dqmc_primes_ex (12 < n <= 25): the
 * n-variable state is computed as its three consecutive thirds, the slices
 * of digit n = 0, 1, * (each an (n-1)-variable state of the same block layout),
 * by the identity of dqmc_primes_sliced with t = 1: slice a holds the primes
 * of f_a, and slices 0 and 1 lose the cubes that are implicants of
 * f_* = f_0 AND f_1 (the Lemma of Sec. 4.1, one-step form, on digit n).
 * While slices 0 and 1 are filtered, the * third holds those implicants.  The
 * bitmap, list and count are the same as without the split; only the passes
 * differ (those of n - 1 variables).  mode 1: split, 0: whole-state passes,
 * -1: the default, which splits n = 25 only.  The thirds themselves are
 * never split again.  dqmc_primes_sliced applies the same setting to its
 * (n - t)-variable slices.  dqmc_get_split returns 1 if the split is in use
 * for n, else 0.  Errors: DQMC_EINVAL for a bad n or mode. */
int dqmc_set_split(dqmc_ctx *ctx, int n, int mode);
int dqmc_get_split(const dqmc_ctx *ctx, int n);

/* ---------------------------------------------------------------------------
 * Autotuning: measure the launch choices that leave results unchanged (the
 * batch bit-slicing launch of Sec. 4.2, the grouping of Alg. 4's top-layer
 * dimensions into passes) and keep the fastest.
 *
 * Both calls run the computation several times on the caller's buffers (the
 * outputs end up exactly as after one normal call), time each run with HIP
 * events on `stream`, and wait for the stream before returning.  They return
 * DQMC_EINVAL while `stream` is being captured into a graph, and on bad
 * arguments; a failing run's status is returned as is.  trials (host memory,
 * may be NULL when cap == 0) receives up to cap trials; *ntrials (may be
 * NULL) the number timed.  A trial's ms is its fastest of `reps` timed runs
 * (reps >= 1), each after one untimed run.
 *
 * dqmc_batch_autotune: candidates are the column-pass caps 0, 1, 2 and 3,
 * each with item order 0 and 1 (eight trials); the fastest is set on the plan
 * with dqmc_batch_config.
 *
 * dqmc_plan_autotune (12 < n <= 25): candidates are the plans with the
 * fewest groups up to that number plus extra_groups (0..2): every ordered
 * split of digits 13..n into groups of 1..6 digits, at most
 * DQMC_MAX_PLAN_TRIALS of them, by group count, then lexicographically by
 * sizes; then the top-digit split (dqmc_set_split), reported as a trial with
 * ngroups == 0.  Each is timed on dqmc_primes without a list (the count goes
 * to d_count); the fastest group plan is set with dqmc_set_plan, and the
 * split is switched on (1) if it beat that plan, off (0) otherwise.  d_state
 * holds the last call's result afterwards.  If a run fails, the plan and
 * split mode in force before the call are restored.  cap should leave room
 * for the split trial: DQMC_MAX_PLAN_TRIALS + 1.
 */
typedef struct {
    int32_t col_cap;
    int32_t order;
    float ms;
} dqmc_batch_trial;
int dqmc_batch_autotune(dqmc_batch *plan, int32_t reps, void *stream, dqmc_batch_trial *trials, int32_t cap_trials,
                        int32_t *ntrials);

#define DQMC_MAX_PLAN_TRIALS 64
typedef struct {
    int32_t ngroups;
    int32_t sizes[DQMC_MAX_N];
    float ms;
} dqmc_plan_trial;
int dqmc_plan_autotune(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint32_t *d_state, uint64_t *d_count,
                       int32_t extra_groups, int32_t reps, void *stream, dqmc_plan_trial *trials, int32_t cap,
                       int32_t *ntrials);

/* Tuning cache: a context's per-n settings (group plan and top-digit split)
 * as a JSON file, so that what dqmc_plan_autotune chose on one machine is
 * reused by later processes instead of timed again.  Entries are keyed by
 * the device architecture (hipDeviceProp_t::gcnArchName), n and the setting:
 *
 *   {"format": "dqmc-tune-1", "arch": "gfx950:sramecc+:xnack-",
 *    "plans": [{"n": 24, "groups": [6, 6], "split": -1}, ...]}
 *
 * groups = [] is the default plan, split is the dqmc_set_split mode.
 * dqmc_tune_save writes every n (13..25) whose plan or split is not the
 * default.  dqmc_tune_load applies every entry of a file written for the
 * context's architecture, as dqmc_set_plan and dqmc_set_split would, and
 * stores the number applied in *napplied (may be NULL); a file for another
 * architecture applies nothing and returns DQMC_OK.  Whitespace and the
 * order of keys are free; unknown keys are an error.  Errors: DQMC_EINVAL for
 * NULL arguments, malformed JSON or an entry that dqmc_set_plan /
 * dqmc_set_split would reject (nothing is applied then); DQMC_EIO when the
 * file cannot be opened, read or written; DQMC_EDEVICE when the device's
 * properties cannot be read. */
int dqmc_tune_save(const dqmc_ctx *ctx, const char *path);
int dqmc_tune_load(dqmc_ctx *ctx, const char *path, int32_t *napplied);

/* ---------------------------------------------------------------------------
 * Diagnostics: per-pass device timing.
 *
 * With profiling enabled, every compute call on the context records a HIP
 * event right before and right after each kernel pass it enqueues, on the
 * caller's stream (at most DQMC_MAX_RECORDS passes are kept; later ones are
 * not recorded).  model_bytes is the pass's algorithmic HBM traffic: the
 * state words it must read and write under the pass plan, plus the truth
 * table it reads; for passes that write the prime list, add 8 bytes per
 * listed prime (list_bytes_per_prime = 8).
 */
#define DQMC_MAX_RECORDS 64

typedef struct {
    char pass[40];              /* e.g. "low_merge_tt", "col_reduce_g13_6" */
    int32_t n;
    int32_t list_bytes_per_prime;
    float ms;                   /* elapsed device time of the pass */
    double model_bytes;
} dqmc_pass_record;

/* enable != 0 starts recording (clearing older records); 0 stops. */
int dqmc_profile(dqmc_ctx *ctx, int enable);

/* Waits for the recorded events, copies up to cap records into out (host
 * memory), clears them and returns how many were copied (negative dqmc_status
 * on error). */
int dqmc_profile_read(dqmc_ctx *ctx, dqmc_pass_record *out, int cap);

/* Data-dependent work of the last n = 24 computation on the context that
 * used row and chunk flags (the default plan [6, 6]): the reduce of digits
 * 13..18 loads and stores only the row segments flagged by the top group's
 * pass, and the final reduce loads only the runs of three blocks that touch a
 * flagged 64-word chunk, and stores only the chunks it found non-zero as
 * loaded (a subset of the flagged ones).
 * h_units (host, 4 entries): [0] bytes of the rows the reduce of digits 13..18
 * loads (it stores the same rows), [1] bytes of the runs the final reduce
 * loads, [2] bytes of the flagged chunks (a bound on the final reduce's
 * stores), [3] 1 if the last n = 24
 * computation used the flags (else all 0).  Waits for the context's default
 * stream work it enqueues; call after the computation has finished.  Errors:
 * DQMC_EINVAL (NULL), DQMC_EDEVICE. */
int dqmc_flag_units(dqmc_ctx *ctx, uint64_t *h_units);

#ifdef __cplusplus
}
#endif

#endif /* DQMC_H */
