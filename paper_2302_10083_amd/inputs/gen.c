/*
 * Seeded synthetic truth-table generators.
 *
 * This file holds no part of the prime-implicant method: it only produces the
 * inputs that the GPU library and the CPU oracle are both run on.
 *
 * Random numbers: counter-based SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014).  Value i of the
 * stream with key k is the SplitMix64 output finaliser applied to
 * k + (i + 1) * GAMMA, where GAMMA is the 64-bit golden-ratio increment; the
 * key of a seed is the finaliser applied to the seed itself.  A uniform
 * double is (v >> 11) * 2^-53.
 *
 * Truth tables: bit x of a little-endian array of uint32 words is f(x), and
 * variable x_i (i = 1..n) is bit i-1 of x.
 */
#include <stdint.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t fin64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t gen_key(uint64_t seed) { return fin64(seed); }

uint64_t gen_u64(uint64_t seed, uint64_t i) { return fin64(fin64(seed) + (i + 1) * GAMMA); }

double gen_uniform(uint64_t seed, uint64_t i) { return (double)(gen_u64(seed, i) >> 11) * 0x1.0p-53; }

void gen_u64_array(uint64_t seed, uint64_t start, uint64_t count, uint64_t *out)
{
    uint64_t k = fin64(seed);
    for (uint64_t j = 0; j < count; ++j) out[j] = fin64(k + (start + j + 1) * GAMMA);
}

static uint64_t tt_words(int n) { return n <= 5 ? 1 : (1ULL << (n - 5)); }

/* f(x) = [u(seed, x) < p] for every x < 2^n.  With or_into != 0 the bits are
 * OR-ed into tt, otherwise tt is overwritten. */
void gen_bernoulli(int n, double p, uint64_t seed, int or_into, uint32_t *tt)
{
    uint64_t k = fin64(seed), N = 1ULL << n, nw = tt_words(n);
    if (!or_into) memset(tt, 0, nw * 4);
    for (uint64_t x = 0; x < N; ++x) {
        double u = (double)(fin64(k + (x + 1) * GAMMA) >> 11) * 0x1.0p-53;
        if (u < p) tt[x >> 5] |= 1u << (x & 31);
    }
}

/* Sequential stream used by the DNF generator. */
typedef struct { uint64_t key, ctr; } stream_t;
static inline uint64_t next_u64(stream_t *s) { return fin64(s->key + (++s->ctr) * GAMMA); }
static inline uint64_t next_below(stream_t *s, uint64_t m) { return next_u64(s) % m; }

/* OR of T random product terms.  Each term: width w uniform in [wlo, whi]
 * (clamped to [0, n]); w distinct variables by a partial Fisher-Yates shuffle;
 * the polarity of each literal is one fair bit.  Every minterm of the term is
 * set in tt.  With or_into == 0 tt is cleared first. */
void gen_dnf(int n, uint32_t T, int wlo, int whi, uint64_t seed, int or_into, uint32_t *tt)
{
    stream_t s = {fin64(seed), 0};
    uint64_t nw = tt_words(n);
    if (!or_into) memset(tt, 0, nw * 4);
    if (wlo > whi) { int t = wlo; wlo = whi; whi = t; }
    uint64_t full = (n >= 64) ? ~0ULL : ((1ULL << n) - 1);
    int perm[64];
    for (uint32_t t = 0; t < T; ++t) {
        int w = wlo + (int)next_below(&s, (uint64_t)(whi - wlo + 1));
        if (w > n) w = n;
        if (w < 0) w = 0;
        for (int j = 0; j < n; ++j) perm[j] = j;
        for (int j = 0; j < w; ++j) {
            int k = j + (int)next_below(&s, (uint64_t)(n - j));
            int tmp = perm[j]; perm[j] = perm[k]; perm[k] = tmp;
        }
        uint64_t care = 0, val = 0;
        for (int j = 0; j < w; ++j) {
            care |= 1ULL << perm[j];
            if (next_u64(&s) & 1) val |= 1ULL << perm[j];
        }
        uint64_t freem = full & ~care, sub = 0;
        do {
            uint64_t x = val | sub;
            tt[x >> 5] |= 1u << (x & 31);
            sub = (sub - freem) & freem;
        } while (sub != 0);
    }
}

/* OR of explicitly given product terms: term j has care mask care[j] and
 * value bits val[j] (val within care). */
void gen_terms(int n, uint32_t T, const uint64_t *care, const uint64_t *val, int or_into, uint32_t *tt)
{
    uint64_t nw = tt_words(n);
    if (!or_into) memset(tt, 0, nw * 4);
    uint64_t full = (n >= 64) ? ~0ULL : ((1ULL << n) - 1);
    for (uint32_t t = 0; t < T; ++t) {
        uint64_t freem = full & ~care[t], v = val[t] & care[t], sub = 0;
        do {
            uint64_t x = v | sub;
            tt[x >> 5] |= 1u << (x & 31);
            sub = (sub - freem) & freem;
        } while (sub != 0);
    }
}
