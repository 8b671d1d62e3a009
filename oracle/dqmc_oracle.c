/*
 * CPU oracle for the prime implicants of a Boolean function given by its
 * truth table ("DenseQMC: an efficient bit-slice implementation of the
 * Quine-McCluskey algorithm", Udovenko, arXiv 2302.10083).
 *
 * TEST INFRASTRUCTURE.  This is the plain, slow, definitional computation
 * that the GPU library is checked against.  Only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark load it.  It shares no code,
 * header, table or layout with the GPU library and is never called by it.
 *
 * Conventions (all functions):
 *  - A cube is a string s in {0,1,*}^n (Sec. 2, Def. of minterm) and is
 *    indexed by rho(s) = sum_{i=1..n} 3^(i-1) rho(s_i) with rho(0) = 0,
 *    rho(1) = 1, rho(*) = 2 (Sec. 4.2, notation rho).  Digit i of rho is
 *    floor(rho / 3^(i-1)) mod 3.
 *  - The truth table is a little-endian uint32 array: bit x is f(x), and
 *    variable x_i is bit i-1 of x.  The paper does not fix this map; digit i
 *    of a cube is read as the literal on x_i.
 *  - Cube bitmaps are little-endian uint64 arrays with bit rho = membership.
 *  - M is the set of implicants and O the set of prime implicants.
 *
 * Every function here is pinned by the test suite against facts the paper or
 * the mathematics fixes (printed examples, closed forms, invariants, a
 * set-based brute force on tiny inputs); none is "parity unpinned".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <unistd.h>

#define MAXN 32

uint64_t orc_pow3(int k)
{
    uint64_t p = 1;
    for (int i = 0; i < k; ++i) p *= 3;
    return p;
}

static int tt_bit(const uint32_t *tt, uint64_t x) { return (int)((tt[x >> 5] >> (x & 31)) & 1u); }

static int bm_get(const uint64_t *bm, uint64_t r)
{
    return (int)((__atomic_load_n(&bm[r >> 6], __ATOMIC_RELAXED) >> (r & 63)) & 1u);
}

static void bm_set_atomic(uint64_t *bm, uint64_t r)
{
    __atomic_fetch_or(&bm[r >> 6], 1ULL << (r & 63), __ATOMIC_RELAXED);
}

static void digits_of(int n, uint64_t rho, int *d)
{
    for (int i = 0; i < n; ++i) { d[i] = (int)(rho % 3); rho /= 3; }
}

static int resolve_threads(int nthreads)
{
    if (nthreads > 0) return nthreads;
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

/* ------------------------------------------------------------------------
 * Per-cube definitions (brute force, "O1").
 * ------------------------------------------------------------------------ */

/* Sec. 2, Def. of implicant: the product is an implicant of f iff every
 * input x on which the product evaluates to 1 has f(x) = 1.  The product with
 * string s is 1 exactly on the x that agree with s on every non-* digit. */
int orc_is_implicant(int n, const uint32_t *tt, uint64_t rho)
{
    int d[MAXN];
    digits_of(n, rho, d);
    uint64_t base = 0, freem = 0;
    for (int i = 0; i < n; ++i) {
        if (d[i] == 1) base |= 1ULL << i;
        else if (d[i] == 2) freem |= 1ULL << i;
    }
    uint64_t sub = 0;
    do {
        if (!tt_bit(tt, base | sub)) return 0;
        sub = (sub - freem) & freem;
    } while (sub != 0);
    return 1;
}

/* Sec. 2, Def. of prime implicant: no proper divisor of the product is an
 * implicant.  A proper divisor drops a nonempty set of literals, i.e. turns a
 * nonempty set of non-* digits into *.  Checked here over ALL such sets
 * (exponential in the number of literals; used for small n). */
int orc_is_prime_all_divisors(int n, const uint32_t *tt, uint64_t rho)
{
    if (!orc_is_implicant(n, tt, rho)) return 0;
    int d[MAXN], pos[MAXN], k = 0;
    digits_of(n, rho, d);
    for (int i = 0; i < n; ++i)
        if (d[i] != 2) pos[k++] = i;
    for (uint64_t m = 1; m < (1ULL << k); ++m) {
        uint64_t r = rho;
        for (int j = 0; j < k; ++j)
            if ((m >> j) & 1) r += (uint64_t)(2 - d[pos[j]]) * orc_pow3(pos[j]);
        if (orc_is_implicant(n, tt, r)) return 0;
    }
    return 1;
}

/* Same definition, checking only the divisors that drop one literal.  This
 * is equivalent: if some proper divisor is an implicant, so is every
 * product between it and s, in particular one that drops a single literal
 * (a sub-cube of an implicant is an implicant). */
int orc_is_prime(int n, const uint32_t *tt, uint64_t rho)
{
    if (!orc_is_implicant(n, tt, rho)) return 0;
    uint64_t r = rho, p = 1;
    for (int i = 0; i < n; ++i, p *= 3, r /= 3) {
        uint64_t di = r % 3;
        if (di != 2 && orc_is_implicant(n, tt, rho + (2 - di) * p)) return 0;
    }
    return 1;
}

typedef struct {
    int n, all_divisors;
    const uint32_t *tt;
    uint64_t *M, *O;
    uint64_t nwords;
    uint64_t next;
} brute_job;

static void *brute_worker(void *arg)
{
    brute_job *J = (brute_job *)arg;
    uint64_t N = orc_pow3(J->n);
    for (;;) {
        uint64_t w = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
        if (w >= J->nwords) break;
        uint64_t mw = 0, ow = 0;
        for (uint64_t b = 0; b < 64; ++b) {
            uint64_t r = w * 64 + b;
            if (r >= N) break;
            if (J->M && orc_is_implicant(J->n, J->tt, r)) mw |= 1ULL << b;
            if (J->O) {
                int pr = J->all_divisors ? orc_is_prime_all_divisors(J->n, J->tt, r)
                                         : orc_is_prime(J->n, J->tt, r);
                if (pr) ow |= 1ULL << b;
            }
        }
        if (J->M) J->M[w] = mw;
        if (J->O) J->O[w] = ow;
    }
    return NULL;
}

/* Brute force over all 3^n cubes with the per-cube definitions above.
 * M and O (either may be NULL) receive ceil(3^n/64) words each. */
void orc_bruteforce(int n, const uint32_t *tt, uint64_t *M, uint64_t *O, int all_divisors, int nthreads)
{
    brute_job J = {n, all_divisors, tt, M, O, (orc_pow3(n) + 63) / 64, 0};
    int T = resolve_threads(nthreads);
    pthread_t th[256];
    if (T > 256) T = 256;
    for (int t = 0; t < T; ++t) pthread_create(&th[t], NULL, brute_worker, &J);
    for (int t = 0; t < T; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------
 * Definitional enumerator ("O2"): the Lemma of Sec. 4.1 (MergeAll then
 * ReduceAll), evaluated cube by cube in increasing rho.
 * ------------------------------------------------------------------------ */

/* Implicant bitmap by the Lemma's recursion for M (Sec. 4.1):
 *   M(u) = I(u) = f(u)                    if u has no *,
 *   M(u) = OR over the pairs s + t = u of M(s) AND M(t) otherwise,
 * where s + t = u means s, t agree with u except at one * position i of u,
 * with s_i = 0 and t_i = 1 (Sec. 3, Observation on combining minterms).
 * Both halves have a smaller rho than u, so an increasing-rho sweep sees
 * them finished.  For threading, the sweep is split on the top `t` digits:
 * a block (fixed top digits) only depends on itself and on blocks with one
 * fewer * among the top digits, so blocks are processed level by level
 * (number of * among the top digits), each block sequentially. */
typedef struct {
    int n, t;
    const uint32_t *tt;
    uint64_t *M;
    uint64_t bsize;
    const uint64_t *blocks;
    uint64_t nblocks;
    uint64_t next;
} msweep_job;

static void msweep_block(const msweep_job *J, uint64_t B)
{
    int n = J->n, d[MAXN];
    uint64_t p3[MAXN];
    for (int i = 0; i < n; ++i) p3[i] = orc_pow3(i);
    uint64_t r0 = B * J->bsize, r1 = r0 + J->bsize;
    digits_of(n, r0, d);
    for (uint64_t r = r0; r < r1; ++r) {
        int m = 0, any_star = 0;
        for (int i = 0; i < n && !m; ++i) {
            if (d[i] != 2) continue;
            any_star = 1;
            /* s = u with digit i set to 0, t = u with digit i set to 1 */
            if (bm_get(J->M, r - 2 * p3[i]) && bm_get(J->M, r - p3[i])) m = 1;
        }
        if (!any_star) {
            uint64_t x = 0;
            for (int i = 0; i < n; ++i)
                if (d[i] == 1) x |= 1ULL << i;
            m = tt_bit(J->tt, x);
        }
        if (m) bm_set_atomic(J->M, r);
        for (int i = 0; i < n; ++i) { /* odometer: next rho */
            if (++d[i] < 3) break;
            d[i] = 0;
        }
    }
}

static void *msweep_worker(void *arg)
{
    msweep_job *J = (msweep_job *)arg;
    for (;;) {
        uint64_t k = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
        if (k >= J->nblocks) break;
        msweep_block(J, J->blocks[k]);
    }
    return NULL;
}

void orc_enum_M(int n, const uint32_t *tt, uint64_t *M, int nthreads)
{
    uint64_t N = orc_pow3(n), nw = (N + 63) / 64;
    memset(M, 0, nw * 8);
    int T = resolve_threads(nthreads);
    if (T > 256) T = 256;
    int t = n < 6 ? n : 6;
    uint64_t nb = orc_pow3(t);
    uint64_t *blocks = (uint64_t *)malloc(nb * sizeof(uint64_t));
    for (int lev = 0; lev <= t; ++lev) {
        uint64_t k = 0;
        for (uint64_t B = 0; B < nb; ++B) {
            int stars = 0;
            uint64_t b = B;
            for (int i = 0; i < t; ++i, b /= 3) stars += (b % 3 == 2);
            if (stars == lev) blocks[k++] = B;
        }
        msweep_job J = {n, t, tt, M, orc_pow3(n - t), blocks, k, 0};
        pthread_t th[256];
        int TT = T < (int)k ? T : (int)k;
        for (int i = 0; i < TT; ++i) pthread_create(&th[i], NULL, msweep_worker, &J);
        for (int i = 0; i < TT; ++i) pthread_join(th[i], NULL);
    }
    free(blocks);
}

/* Prime bitmap by the Lemma's formula for O (Sec. 4.1), read with OR: the
 * printed formula uses a big AND, but s is redundant as soon as ONE merge
 * s + t = u has M(u) = 1 (Alg. 1 marks both merged implicants redundant):
 *   O(s) = M(s) AND NOT OR_{i : s_i != *} M(s with digit i set to *).
 * Each cube only reads M, so any range of rho can be evaluated on its own:
 * the range [r0, r0 + nbits) goes to a bitmap whose bit k is cube r0 + k
 * (a "streaming" sweep that never holds the whole O bitmap). */
typedef struct {
    int n;
    const uint64_t *M;
    uint64_t *O;
    uint64_t r0, nbits, nwords;
    uint64_t next;
} osweep_job;

#define OCHUNK 4096 /* words per work item */

static void *osweep_worker(void *arg)
{
    osweep_job *J = (osweep_job *)arg;
    int n = J->n, d[MAXN];
    uint64_t p3[MAXN];
    for (int i = 0; i < n; ++i) p3[i] = orc_pow3(i);
    for (;;) {
        uint64_t c = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
        uint64_t w0 = c * OCHUNK;
        if (w0 >= J->nwords) break;
        uint64_t w1 = w0 + OCHUNK < J->nwords ? w0 + OCHUNK : J->nwords;
        digits_of(n, J->r0 + w0 * 64, d);
        for (uint64_t w = w0; w < w1; ++w) {
            uint64_t ow = 0;
            for (uint64_t b = 0; b < 64; ++b) {
                uint64_t k = w * 64 + b;
                if (k >= J->nbits) break;
                uint64_t r = J->r0 + k;
                if (bm_get(J->M, r)) {
                    int red = 0;
                    for (int i = 0; i < n && !red; ++i)
                        if (d[i] != 2 && bm_get(J->M, r + (uint64_t)(2 - d[i]) * p3[i])) red = 1;
                    if (!red) ow |= 1ULL << b;
                }
                for (int i = 0; i < n; ++i) {
                    if (++d[i] < 3) break;
                    d[i] = 0;
                }
            }
            J->O[w] = ow;
        }
    }
    return NULL;
}

/* O restricted to the cubes r0 <= rho < r1 (r1 <= 3^n), from the whole M:
 * out receives ceil((r1 - r0) / 64) words, bit k = O(r0 + k). */
void orc_enum_O_range(int n, const uint64_t *M, uint64_t r0, uint64_t r1, uint64_t *out, int nthreads)
{
    uint64_t nbits = r1 > r0 ? r1 - r0 : 0;
    osweep_job J = {n, M, out, r0, nbits, (nbits + 63) / 64, 0};
    int T = resolve_threads(nthreads);
    if (T > 256) T = 256;
    pthread_t th[256];
    for (int i = 0; i < T; ++i) pthread_create(&th[i], NULL, osweep_worker, &J);
    for (int i = 0; i < T; ++i) pthread_join(th[i], NULL);
}

void orc_enum_O(int n, const uint64_t *M, uint64_t *O, int nthreads)
{
    orc_enum_O_range(n, M, 0, orc_pow3(n), O, nthreads);
}

/* Set bits of a bitmap of nbits bits whose bit k stands for cube base + k,
 * in increasing order.  Writes the first min(count, cap) entries; returns the
 * count. */
uint64_t orc_extract_bits(uint64_t nbits, const uint64_t *O, uint64_t *list, uint64_t cap, uint64_t base)
{
    uint64_t nw = (nbits + 63) / 64, cnt = 0;
    for (uint64_t w = 0; w < nw; ++w) {
        uint64_t v = O[w];
        while (v) {
            uint64_t k = w * 64 + (uint64_t)__builtin_ctzll(v);
            v &= v - 1;
            if (k >= nbits) break;
            if (list && cnt < cap) list[cnt] = base + k;
            ++cnt;
        }
    }
    return cnt;
}

/* Extraction (Alg. 4, last step): every rho whose bit is set, in increasing
 * rho.  Writes the first min(count, cap) entries; returns the count. */
uint64_t orc_extract(int n, const uint64_t *O, uint64_t *list, uint64_t cap)
{
    return orc_extract_bits(orc_pow3(n), O, list, cap, 0);
}

/* ------------------------------------------------------------------------
 * Per-cube definitions over a sample of cubes (for sizes where the whole
 * bitmap is too large): out[k] = orc_is_prime / orc_is_implicant of rhos[k].
 * ------------------------------------------------------------------------ */
typedef struct {
    int n, what;
    const uint32_t *tt;
    const uint64_t *rhos;
    uint8_t *out;
    uint64_t k;
    uint64_t next;
} sample_job;

static void *sample_worker(void *arg)
{
    sample_job *J = (sample_job *)arg;
    for (;;) {
        uint64_t i0 = __atomic_fetch_add(&J->next, 256, __ATOMIC_RELAXED);
        if (i0 >= J->k) break;
        uint64_t i1 = i0 + 256 < J->k ? i0 + 256 : J->k;
        for (uint64_t i = i0; i < i1; ++i)
            J->out[i] = (uint8_t)(J->what ? orc_is_prime(J->n, J->tt, J->rhos[i])
                                          : orc_is_implicant(J->n, J->tt, J->rhos[i]));
    }
    return NULL;
}

/* what = 1: prime test, 0: implicant test.  Returns the threads used. */
int orc_sample(int n, const uint32_t *tt, const uint64_t *rhos, uint64_t k, uint8_t *out, int what, int nthreads)
{
    sample_job J = {n, what, tt, rhos, out, k, 0};
    int T = resolve_threads(nthreads);
    if (T > 256) T = 256;
    pthread_t th[256];
    for (int i = 0; i < T; ++i) pthread_create(&th[i], NULL, sample_worker, &J);
    for (int i = 0; i < T; ++i) pthread_join(th[i], NULL);
    return T;
}
