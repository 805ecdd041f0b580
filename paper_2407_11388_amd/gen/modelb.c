/*
 * Seeded synthetic inputs: model-B random binary CSPs and initial domain states.
 *
 * This file produces inputs only. It holds none of the arc-consistency
 * arithmetic; both the GPU library and the CPU oracle are fed from it.
 *
 * The paper evaluates on randomly generated binary CSPs in which each variable
 * pair is constrained with a given density (Section 5.2, "Benchmark"); domain
 * size and tightness are not stated there. We use the standard "model B"
 * reading of that family: exactly m = floor(p1 * n(n-1)/2 + 1/2) distinct
 * unordered variable pairs carry a constraint, and every relation forbids
 * exactly F = floor(p2 * d^2 + 1/2) distinct value pairs, all drawn uniformly.
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), written from its published
 * definition. Bounded integers use Lemire's multiply-shift method with
 * rejection ("Fast random integer generation in an interval", ACM TOMACS
 * 2019), so draws are exactly uniform. Distinct subsets use Floyd's sampling
 * algorithm (Bentley & Floyd, "A sample of brilliance", CACM 1987), which
 * yields every M-subset of {0..N-1} with equal probability.
 *
 * Layouts produced:
 *   edges[m][2]  int32, x < y, sorted lexicographically;
 *   rel[m][d]    uint64 rows: bit b of rel[e][a] is 1 iff (x_e=a, y_e=b) is
 *                allowed (the relation of the constraint on edge e);
 *   dom[n]       uint64: bit a is 1 iff a is in dom(x).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define MB_API __attribute__((visibility("default")))

static uint64_t sm64_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform integer in [0, bound), bound >= 1 */
static uint64_t rand_below(uint64_t *s, uint64_t bound) {
    uint64_t x = sm64_next(s);
    __uint128_t m = (__uint128_t)x * bound;
    uint64_t l = (uint64_t)m;
    if (l < bound) {
        uint64_t t = (0 - bound) % bound;
        while (l < t) {
            x = sm64_next(s);
            m = (__uint128_t)x * bound;
            l = (uint64_t)m;
        }
    }
    return (uint64_t)(m >> 64);
}

/* uniform double in [0, 1) with 53 random bits */
static double rand_unit(uint64_t *s) {
    return (double)(sm64_next(s) >> 11) * (1.0 / 9007199254740992.0);
}

MB_API uint64_t mb_splitmix64(uint64_t *state) { return sm64_next(state); }

MB_API uint64_t mb_rand_below(uint64_t *state, uint64_t bound) {
    return rand_below(state, bound);
}

/* Seed of independent sub-stream `idx` of a stream seeded with `seed`. */
MB_API uint64_t mb_substream(uint64_t seed, uint64_t idx) {
    uint64_t s = seed + (idx + 1) * 0xD1B54A32D192ED03ull;
    return sm64_next(&s);
}

MB_API int64_t mb_num_edges(int32_t n, double p1) {
    double pairs = (double)n * (double)(n - 1) / 2.0;
    int64_t m = (int64_t)floor(p1 * pairs + 0.5);
    if (m < 0) m = 0;
    if ((double)m > pairs) m = (int64_t)pairs;
    return m;
}

MB_API int32_t mb_num_forbidden(int32_t d, double p2) {
    int32_t f = (int32_t)floor(p2 * (double)d * (double)d + 0.5);
    if (f < 0) f = 0;
    if (f > d * d) f = d * d;
    return f;
}

/*
 * Floyd's algorithm: mark exactly `take` distinct indices of [0, total) in
 * the bitmap `bits` (which must be zero on entry, total bits long).
 */
static void floyd_sample(uint64_t *s, uint64_t total, uint64_t take, uint64_t *bits) {
    for (uint64_t j = total - take; j < total; ++j) {
        uint64_t t = rand_below(s, j + 1);
        if (bits[t >> 6] & (1ull << (t & 63)))
            t = j;
        bits[t >> 6] |= 1ull << (t & 63);
    }
}

/*
 * Model-B instance. Returns 0, or -1 on bad arguments / allocation failure.
 * edges must hold mb_num_edges(n,p1) pairs, rel mb_num_edges(n,p1)*d rows.
 */
MB_API int mb_generate(uint64_t seed, int32_t n, int32_t d, double p1, double p2,
                       int32_t *edges, uint64_t *rel) {
    if (n < 1 || d < 1 || d > 64) return -1;
    uint64_t s = seed;
    int64_t m = mb_num_edges(n, p1);
    uint64_t pairs = (uint64_t)n * (uint64_t)(n - 1) / 2;
    uint64_t *pbits = (uint64_t *)calloc(pairs / 64 + 1, sizeof(uint64_t));
    if (!pbits) return -1;
    floyd_sample(&s, pairs, (uint64_t)m, pbits);
    /* walk the pair index space in order: index = rank of (x,y), x<y, row-major */
    int64_t e = 0;
    uint64_t idx = 0;
    for (int32_t x = 0; x < n - 1; ++x) {
        for (int32_t y = x + 1; y < n; ++y, ++idx) {
            if (pbits[idx >> 6] & (1ull << (idx & 63))) {
                edges[2 * e] = x;
                edges[2 * e + 1] = y;
                ++e;
            }
        }
    }
    free(pbits);
    if (e != m) return -1;

    int32_t f = mb_num_forbidden(d, p2);
    uint64_t cells = (uint64_t)d * (uint64_t)d;
    uint64_t full = (d == 64) ? ~0ull : ((1ull << d) - 1);
    /* Sampling the smaller of the forbidden set and its complement draws the
     * same distribution (a uniform F-subset) with fewer random numbers. */
    int complement = (uint64_t)f * 2 > cells;
    uint64_t take = complement ? cells - (uint64_t)f : (uint64_t)f;
    /* Relation k is drawn from its own sub-stream, so relations are generated
     * in parallel with a result that does not depend on the thread count. */
    uint64_t rel_seed = sm64_next(&s);
    #pragma omp parallel for schedule(static, 4096)
    for (int64_t k = 0; k < m; ++k) {
        uint64_t cbits[64];
        uint64_t ks = mb_substream(rel_seed, (uint64_t)k);
        memset(cbits, 0, sizeof(cbits));
        floyd_sample(&ks, cells, take, cbits);
        uint64_t *rows = rel + (size_t)k * (size_t)d;
        uint64_t init = complement ? 0 : full;
        for (int32_t a = 0; a < d; ++a) rows[a] = init;
        for (uint64_t w = 0; w < (cells + 63) / 64; ++w) {
            uint64_t bw = cbits[w];
            while (bw) {
                int t = __builtin_ctzll(bw);
                bw &= bw - 1;
                uint64_t c = w * 64 + (uint64_t)t;
                uint64_t bit = 1ull << (c % (uint64_t)d);
                if (complement) rows[c / (uint64_t)d] |= bit;   /* allowed cell */
                else rows[c / (uint64_t)d] &= ~bit;             /* forbidden cell */
            }
        }
    }
    return 0;
}

MB_API void mb_full_domains(int32_t n, int32_t d, uint64_t *dom) {
    uint64_t full = (d == 64) ? ~0ull : ((1ull << d) - 1);
    for (int32_t x = 0; x < n; ++x) dom[x] = full;
}

/* Full domains minus exactly `count` distinct (x,a) pairs drawn uniformly. */
MB_API int mb_preremove(uint64_t seed, int32_t n, int32_t d, int64_t count, uint64_t *dom) {
    uint64_t total = (uint64_t)n * (uint64_t)d;
    if (count < 0 || (uint64_t)count > total) return -1;
    uint64_t s = seed;
    uint64_t *bits = (uint64_t *)calloc(total / 64 + 1, sizeof(uint64_t));
    if (!bits) return -1;
    floyd_sample(&s, total, (uint64_t)count, bits);
    mb_full_domains(n, d, dom);
    for (uint64_t i = 0; i < total; ++i)
        if (bits[i >> 6] & (1ull << (i & 63)))
            dom[i / (uint64_t)d] &= ~(1ull << (i % (uint64_t)d));
    free(bits);
    return 0;
}

/*
 * B domain states of one network, each from a random partial assignment:
 * k_s ~ U{0..max_assign}, k_s distinct variables chosen uniformly, each set to
 * a singleton {v}, v ~ U{0..d-1} (drawn in increasing variable order); every
 * other variable keeps its full domain. dom is [B][n]; n_assigned is [B].
 */
MB_API int mb_partial_assign_states(uint64_t seed, int32_t n, int32_t d, int32_t B,
                                    int32_t max_assign, uint64_t *dom, int32_t *n_assigned) {
    if (max_assign > n) max_assign = n;
    uint64_t s = seed;
    uint64_t *bits = (uint64_t *)malloc(((size_t)n / 64 + 1) * sizeof(uint64_t));
    if (!bits) return -1;
    for (int32_t b = 0; b < B; ++b) {
        uint64_t *db = dom + (size_t)b * (size_t)n;
        mb_full_domains(n, d, db);
        int32_t k = (int32_t)rand_below(&s, (uint64_t)max_assign + 1);
        memset(bits, 0, ((size_t)n / 64 + 1) * sizeof(uint64_t));
        floyd_sample(&s, (uint64_t)n, (uint64_t)k, bits);
        for (int32_t x = 0; x < n; ++x)
            if (bits[x >> 6] & (1ull << (x & 63)))
                db[x] = 1ull << rand_below(&s, (uint64_t)d);
        if (n_assigned) n_assigned[b] = k;
    }
    free(bits);
    return 0;
}

/*
 * Parameters of k independent instances of uneven size: per instance, in this
 * order, n ~ U{nmin..nmax}, d ~ U{dmin..dmax}, p1 ~ U[p1lo,p1hi),
 * p2 ~ U[p2lo,p2hi). Instance i is then generated from mb_substream(seed, i).
 */
MB_API void mb_uneven_params(uint64_t seed, int32_t k, int32_t nmin, int32_t nmax,
                             int32_t dmin, int32_t dmax, double p1lo, double p1hi,
                             double p2lo, double p2hi, int32_t *n_out, int32_t *d_out,
                             double *p1_out, double *p2_out) {
    uint64_t s = seed;
    for (int32_t i = 0; i < k; ++i) {
        n_out[i] = nmin + (int32_t)rand_below(&s, (uint64_t)(nmax - nmin + 1));
        d_out[i] = dmin + (int32_t)rand_below(&s, (uint64_t)(dmax - dmin + 1));
        p1_out[i] = p1lo + (p1hi - p1lo) * rand_unit(&s);
        p2_out[i] = p2lo + (p2hi - p2lo) * rand_unit(&s);
    }
}
