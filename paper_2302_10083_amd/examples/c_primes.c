/*
 * c_primes - the C ABI of libdqmc used from plain C, without Python or torch:
 * device buffers from hipMalloc, one dqmc_primes call to size the list, a
 * second one to fill it, and dqmc_extract on the bitmap it leaves.  For
 * n <= 16 it also runs dqmc_primes_batch on a device-resident job array of
 * three jobs (the same function with a list, the same function count-only,
 * and a job with n = 17 that the batch rejects), checks the statuses, counts
 * and list against the single call, and prints "batch ok".
 *
 *   c_primes <n> <truth-table file> <output file>
 *
 * The truth-table file holds dqmc_tt_words(n) little-endian uint32 words.
 * The output file receives the count as one uint64, then the count sorted
 * cube indices (uint64) from dqmc_primes, then the same list again from
 * dqmc_extract.  Exit status 0 on success.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "dqmc.h"

#define CHECK_HIP(x)                                                          \
    do {                                                                      \
        hipError_t e_ = (x);                                                  \
        if (e_ != hipSuccess) {                                               \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
            return 2;                                                         \
        }                                                                     \
    } while (0)

#define CHECK_DQMC(ctx, x)                                                    \
    do {                                                                      \
        int rc_ = (x);                                                        \
        if (rc_ != DQMC_OK) {                                                 \
            fprintf(stderr, "%s: %d (%s)\n", #x, rc_, dqmc_last_error(ctx));  \
            return 3;                                                         \
        }                                                                     \
    } while (0)

int main(int argc, char **argv)
{
    if (argc != 4) {
        fprintf(stderr, "usage: %s <n> <truth-table file> <output file>\n", argv[0]);
        return 1;
    }
    const int n = atoi(argv[1]);
    const uint64_t ttw = dqmc_tt_words(n), sw = dqmc_state_words(n);
    if (ttw == 0 || sw == 0) {
        fprintf(stderr, "n = %d is out of range\n", n);
        return 1;
    }
    uint32_t *tt = (uint32_t *)malloc(ttw * 4);
    FILE *f = fopen(argv[2], "rb");
    if (tt == NULL || f == NULL || fread(tt, 4, ttw, f) != ttw) {
        fprintf(stderr, "cannot read %llu words from %s\n", (unsigned long long)ttw, argv[2]);
        return 1;
    }
    fclose(f);

    dqmc_ctx *ctx = NULL;
    if (dqmc_create(0, &ctx) != DQMC_OK) {
        fprintf(stderr, "dqmc_create failed\n");
        return 3;
    }
    uint32_t *d_tt, *d_state;
    uint64_t *d_count, *d_list;
    hipStream_t s;
    CHECK_HIP(hipStreamCreate(&s));
    CHECK_HIP(hipMalloc((void **)&d_tt, ttw * 4));
    CHECK_HIP(hipMalloc((void **)&d_state, sw * 4));
    CHECK_HIP(hipMalloc((void **)&d_count, 8));
    CHECK_HIP(hipMemcpy(d_tt, tt, ttw * 4, hipMemcpyHostToDevice));

    uint64_t count = 0;
    CHECK_DQMC(ctx, dqmc_primes(ctx, n, d_tt, d_state, NULL, 0, d_count, s));
    CHECK_HIP(hipStreamSynchronize(s));
    CHECK_HIP(hipMemcpy(&count, d_count, 8, hipMemcpyDeviceToHost));
    const uint64_t cap = count > 0 ? count : 1;
    CHECK_HIP(hipMalloc((void **)&d_list, cap * 8));
    uint64_t *list = (uint64_t *)malloc(cap * 8);
    uint64_t *list2 = (uint64_t *)malloc(cap * 8);
    if (list == NULL || list2 == NULL) return 1;

    CHECK_DQMC(ctx, dqmc_primes(ctx, n, d_tt, d_state, d_list, count, d_count, s));
    CHECK_HIP(hipStreamSynchronize(s));
    CHECK_HIP(hipMemcpy(list, d_list, count * 8, hipMemcpyDeviceToHost));
    uint64_t count2 = 0;
    CHECK_HIP(hipMemcpy(&count2, d_count, 8, hipMemcpyDeviceToHost));
    if (count2 != count) {
        fprintf(stderr, "count changed between calls: %llu vs %llu\n", (unsigned long long)count,
                (unsigned long long)count2);
        return 4;
    }
    /* the bitmap stays in d_state: list it again */
    CHECK_DQMC(ctx, dqmc_extract(ctx, n, d_state, d_list, count, d_count, s));
    CHECK_HIP(hipStreamSynchronize(s));
    CHECK_HIP(hipMemcpy(list2, d_list, count * 8, hipMemcpyDeviceToHost));

    if (n <= 16) {
        /* the batch call: a device-resident job array, enqueue only */
        uint32_t *d_state2;
        uint64_t *d_list2, *d_count2;
        dqmc_job h_jobs[3], *d_jobs;
        CHECK_HIP(hipMalloc((void **)&d_state2, sw * 4));
        CHECK_HIP(hipMalloc((void **)&d_list2, cap * 8));
        CHECK_HIP(hipMalloc((void **)&d_count2, 16));
        CHECK_HIP(hipMalloc((void **)&d_jobs, sizeof(h_jobs)));
        dqmc_job a = {n, -9, d_tt, d_state2, d_list2, count, d_count2};
        dqmc_job b = {n, -9, d_tt, d_state, NULL, 0, d_count2 + 1};
        dqmc_job c = {17, -9, d_tt, d_state, NULL, 0, d_count};
        h_jobs[0] = a;
        h_jobs[1] = b;
        h_jobs[2] = c;
        CHECK_HIP(hipMemcpy(d_jobs, h_jobs, sizeof(h_jobs), hipMemcpyHostToDevice));
        CHECK_DQMC(ctx, dqmc_primes_batch(ctx, d_jobs, 3, s));
        CHECK_HIP(hipStreamSynchronize(s));
        uint64_t bc[2];
        CHECK_HIP(hipMemcpy(h_jobs, d_jobs, sizeof(h_jobs), hipMemcpyDeviceToHost));
        CHECK_HIP(hipMemcpy(bc, d_count2, 16, hipMemcpyDeviceToHost));
        CHECK_HIP(hipMemcpy(list2, d_list2, count * 8, hipMemcpyDeviceToHost));
        if (h_jobs[0].status != DQMC_OK || h_jobs[1].status != DQMC_OK || h_jobs[2].status != DQMC_EINVAL ||
            bc[0] != count || bc[1] != count) {
            fprintf(stderr, "batch: statuses %d %d %d, counts %llu %llu (want %llu)\n", h_jobs[0].status,
                    h_jobs[1].status, h_jobs[2].status, (unsigned long long)bc[0], (unsigned long long)bc[1],
                    (unsigned long long)count);
            return 5;
        }
        for (uint64_t i = 0; i < count; ++i)
            if (list2[i] != list[i]) {
                fprintf(stderr, "batch list differs at %llu\n", (unsigned long long)i);
                return 5;
            }
        printf("batch ok\n");
        CHECK_HIP(hipFree(d_jobs));
        CHECK_HIP(hipFree(d_count2));
        CHECK_HIP(hipFree(d_list2));
        CHECK_HIP(hipFree(d_state2));
        /* list2 is rewritten by dqmc_extract below */
        CHECK_DQMC(ctx, dqmc_extract(ctx, n, d_state, d_list, count, d_count, s));
        CHECK_HIP(hipStreamSynchronize(s));
        CHECK_HIP(hipMemcpy(list2, d_list, count * 8, hipMemcpyDeviceToHost));
    }

    f = fopen(argv[3], "wb");
    if (f == NULL || fwrite(&count, 8, 1, f) != 1 || fwrite(list, 8, count, f) != count ||
        fwrite(list2, 8, count, f) != count) {
        fprintf(stderr, "cannot write %s\n", argv[3]);
        return 1;
    }
    fclose(f);
    printf("n=%d primes=%llu\n", n, (unsigned long long)count);

    CHECK_HIP(hipFree(d_list));
    CHECK_HIP(hipFree(d_count));
    CHECK_HIP(hipFree(d_state));
    CHECK_HIP(hipFree(d_tt));
    CHECK_HIP(hipStreamDestroy(s));
    dqmc_destroy(ctx);
    free(tt);
    free(list);
    free(list2);
    return 0;
}
