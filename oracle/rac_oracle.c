/*
 * CPU oracle for arc-consistency enforcement. TEST INFRASTRUCTURE ONLY:
 * used by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark; the GPU library never links, loads or calls it, and the two
 * share no code.
 *
 * Plain, slow, obviously correct C on 0/1 byte arrays. No bit tricks.
 *
 * Inputs (all host memory, caller-owned):
 *   n, d         number of variables, common domain size (values 0..d-1)
 *   m, edges     m constraints; edge e joins x=edges[2e] and y=edges[2e+1]
 *   rel          [m][d][d] bytes, rel[e][a][b] = 1 iff (x=a, y=b) is allowed
 *                (the relation rel(c_xy) of Section 2's notation)
 *   dom          [n][d] bytes, dom[x][a] = 1 iff (x,a) is in D (in/out)
 *
 * Two functions, two different algorithms for the same closure:
 *
 *   oracle_ac3        the queue-and-revise paradigm the paper contrasts with
 *                     (Section 1): a FIFO of arcs, revise, re-enqueue the arcs
 *                     into a variable whose domain shrank. Runs until the queue
 *                     is empty (it does not stop at a wipe-out), so its result
 *                     is the arc-consistency closure D_ac of Section 3.
 *
 *   oracle_rac_sync   the recurrence of Eq. (1) in the loop of Algorithm 1
 *                     (tensorAC / tensorRevise): synchronous steps over the
 *                     removed set D~; optionally restricted to the variables
 *                     whose domain changed in the previous step (@changed, as
 *                     justified by Proposition 2); stops when a step removes
 *                     nothing (Proposition 1), or at the first wipe-out in the
 *                     paper's throw-on-inconsistency mode.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_API __attribute__((visibility("default")))

/* --------------------------------------------------------------------- */
/* Shared-nothing helpers local to this file                             */
/* --------------------------------------------------------------------- */

/* one directed arc x->y over constraint e; `flip` = 1 when x is edges[2e+1] */
typedef struct {
    int32_t x, y;
    int64_t e;
    int flip;
} arc_t;

/* allowed(x=a, y=b) along an arc */
static int arc_allows(const uint8_t *rel, int32_t d, const arc_t *r, int32_t a, int32_t b) {
    const uint8_t *R = rel + (size_t)r->e * (size_t)d * (size_t)d;
    return r->flip ? R[(size_t)b * d + a] : R[(size_t)a * d + b];
}

static int cmp_i64(const void *p, const void *q) {
    const int64_t a = *(const int64_t *)p, b = *(const int64_t *)q;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Builds both arcs of every constraint: arc 2e is x->y and arc 2e+1 is y->x,
 * so the reverse of arc i is arc i^1. Returns NULL on bad input: a variable
 * out of range, a self-loop, or two constraints on one unordered pair (the
 * CSP of Section 2 has at most one constraint c_xy per pair, and Alg. 2's
 * Cons tensor holds one relation block per ordered pair). */
static arc_t *build_arcs(int32_t n, int64_t m, const int32_t *edges) {
    arc_t *arcs = (arc_t *)malloc(sizeof(arc_t) * (size_t)(2 * m + 1));
    int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    if (!arcs || !keys) { free(arcs); free(keys); return NULL; }
    for (int64_t e = 0; e < m; ++e) {
        int32_t x = edges[2 * e], y = edges[2 * e + 1];
        if (x < 0 || y < 0 || x >= n || y >= n || x == y) { free(arcs); free(keys); return NULL; }
        arcs[2 * e] = (arc_t){x, y, e, 0};
        arcs[2 * e + 1] = (arc_t){y, x, e, 1};
        keys[e] = (int64_t)(x < y ? x : y) * n + (x < y ? y : x);
    }
    qsort(keys, (size_t)m, sizeof(int64_t), cmp_i64);
    for (int64_t e = 1; e < m; ++e)
        if (keys[e] == keys[e - 1]) { free(arcs); free(keys); return NULL; }
    free(keys);
    return arcs;
}

static int any_empty(int32_t n, int32_t d, const uint8_t *dom) {
    for (int32_t x = 0; x < n; ++x) {
        int cnt = 0;
        for (int32_t a = 0; a < d; ++a) cnt += dom[(size_t)x * d + a];
        if (cnt == 0) return 1;
    }
    return 0;
}

/* --------------------------------------------------------------------- */
/* O1: AC-3 (queue of arcs + revise)                                     */
/* --------------------------------------------------------------------- */

/*
 * Returns -1 on bad input, else the status: 0 = every domain non-empty,
 * 1 = some domain empty (wipe-out). stats (optional): [0] = revisions
 * (arcs popped and revised, the #Revision of Table 1), [1] = relation
 * look-ups performed.
 */
OR_API int oracle_ac3(int32_t n, int32_t d, int64_t m, const int32_t *edges,
                      const uint8_t *rel, uint8_t *dom, int64_t *stats) {
    if (n < 1 || d < 1 || m < 0) return -1;
    arc_t *arcs = build_arcs(n, m, edges);
    if (!arcs) return -1;
    int64_t na = 2 * m;

    /* in_arcs of variable v: arcs z->v (to re-enqueue when dom(v) shrinks) */
    int64_t *in_start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *in_list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(na + 1));
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(na + 1));
    uint8_t *queued = (uint8_t *)calloc((size_t)na + 1, 1);
    if (!in_start || !in_list || !fill || !queue || !queued) {
        free(arcs); free(in_start); free(in_list); free(fill); free(queue); free(queued);
        return -1;
    }
    for (int64_t i = 0; i < na; ++i) in_start[arcs[i].y + 1]++;
    for (int32_t v = 0; v < n; ++v) in_start[v + 1] += in_start[v];
    for (int64_t i = 0; i < na; ++i) {
        int32_t v = arcs[i].y;
        in_list[in_start[v] + fill[v]++] = i;
    }

    /* FIFO ring holding each arc at most once */
    int64_t head = 0, count = 0;
    for (int64_t i = 0; i < na; ++i) { queue[i] = i; queued[i] = 1; }
    count = na;

    int64_t revisions = 0, lookups = 0;
    while (count > 0) {
        int64_t ai = queue[head];
        head = (head + 1) % (na ? na : 1);
        count--;
        queued[ai] = 0;
        const arc_t *r = &arcs[ai];
        revisions++;
        int removed = 0;
        for (int32_t a = 0; a < d; ++a) {
            if (!dom[(size_t)r->x * d + a]) continue;
            int supported = 0;
            for (int32_t b = 0; b < d && !supported; ++b) {
                if (!dom[(size_t)r->y * d + b]) continue;
                lookups++;
                if (arc_allows(rel, d, r, a, b)) supported = 1;
            }
            if (!supported) {
                dom[(size_t)r->x * d + a] = 0;
                removed = 1;
            }
        }
        if (removed) {
            /* every arc z->x may have lost a support; the reverse arc y->x of
             * this same constraint (arc ai^1) cannot: a value b of y
             * supported only by a removed value a would need rel(a,b)=1 with
             * b in dom(y), contradicting a's removal */
            for (int64_t k = in_start[r->x]; k < in_start[r->x + 1]; ++k) {
                int64_t zi = in_list[k];
                if (zi == (ai ^ 1) || queued[zi]) continue;
                queue[(head + count) % na] = zi;
                queued[zi] = 1;
                count++;
            }
        }
    }
    if (stats) { stats[0] = revisions; stats[1] = lookups; }
    int status = any_empty(n, d, dom);
    free(arcs); free(in_start); free(in_list); free(fill); free(queue); free(queued);
    return status;
}

/* --------------------------------------------------------------------- */
/* O2: Eq. (1) recurrence, stepped as in Algorithm 1                      */
/* --------------------------------------------------------------------- */

/*
 * dom       [n][d] in/out: D on entry, D \ D~^(iters) on exit.
 * changed0  [n] bytes or NULL: the @changed argument of tensorAC; NULL means
 *           every variable (the first call of the search, Algorithm 2).
 * mode      0: run to the fixpoint even after a wipe-out (the closure D_ac);
 *           1: stop after the first step that leaves a domain empty (the
 *              paper's throw / return-None on inconsistency).
 * incremental  0: every step checks every constraint (Eq. (1) as written);
 *              1: a step after the first checks only constraints c_xy whose
 *                 y changed in the previous step (@changed, Proposition 2).
 * max_steps >= 1. If the last permitted step still removed values the
 *           function returns 2 (not converged) with the state after it.
 * trace     [max_steps][n][d] bytes or NULL: D after each executed step.
 * iters     number of steps executed (K+1 of Proposition 1: the final step
 *           removes nothing; 1 when D is already arc consistent).
 * status    0 consistent / 1 some domain empty at the end.
 * checks    if non-NULL: relation cells in the revised constraints, summed
 *           over steps: for every step and every checked arc x->y, d*d.
 * Returns 0, 2 (max_steps reached while still changing) or -1 (bad input).
 */
OR_API int oracle_rac_sync(int32_t n, int32_t d, int64_t m, const int32_t *edges,
                           const uint8_t *rel, uint8_t *dom, const uint8_t *changed0,
                           int32_t mode, int32_t incremental, int32_t max_steps,
                           uint8_t *trace, int32_t *iters, int32_t *status,
                           int64_t *checks) {
    if (n < 1 || d < 1 || m < 0 || max_steps < 1) return -1;
    arc_t *arcs = build_arcs(n, m, edges);
    if (!arcs) return -1;
    int64_t na = 2 * m;
    size_t nd = (size_t)n * (size_t)d;

    /* D~ (removed values), with D~^(0) = empty; D is read as dom0 \ D~ */
    uint8_t *dom0 = (uint8_t *)malloc(nd);
    uint8_t *tilde = (uint8_t *)calloc(nd, 1);
    uint8_t *next = (uint8_t *)malloc(nd);
    uint8_t *changed = (uint8_t *)malloc((size_t)n);
    uint8_t *changed_next = (uint8_t *)malloc((size_t)n);
    if (!dom0 || !tilde || !next || !changed || !changed_next) {
        free(arcs); free(dom0); free(tilde); free(next); free(changed); free(changed_next);
        return -1;
    }
    memcpy(dom0, dom, nd);
    for (int32_t x = 0; x < n; ++x) changed[x] = changed0 ? (changed0[x] != 0) : 1;

    int64_t ncheck = 0;
    int32_t k = 0;
    int rc = 0;
    for (;;) {
        ++k;
        /* D~^(k) = D~^(k-1) U {(x,a) | exists y: c_xy|(x,a) subset of D~^(k-1)} */
        memcpy(next, tilde, nd);
        for (int64_t i = 0; i < na; ++i) {
            const arc_t *r = &arcs[i];
            if (incremental || k == 1) {
                if (!changed[r->y]) continue;
            }
            ncheck += (int64_t)d * d;
            for (int32_t a = 0; a < d; ++a) {
                size_t xa = (size_t)r->x * d + a;
                if (!dom0[xa] || tilde[xa]) continue;      /* only values still in D */
                /* is every support (y,b) of (x,a) on c_xy already removed? */
                int all_removed = 1;
                for (int32_t b = 0; b < d; ++b) {
                    size_t yb = (size_t)r->y * d + b;
                    if (!dom0[yb]) continue;               /* supports are values of D */
                    if (arc_allows(rel, d, r, a, b) && !tilde[yb]) { all_removed = 0; break; }
                }
                if (all_removed) next[xa] = 1;
            }
        }
        /* the @changed of the next step: variables whose domain shrank */
        int any_change = 0;
        for (int32_t x = 0; x < n; ++x) {
            changed_next[x] = 0;
            for (int32_t a = 0; a < d; ++a)
                if (next[(size_t)x * d + a] != tilde[(size_t)x * d + a]) changed_next[x] = 1;
            any_change |= changed_next[x];
        }
        memcpy(tilde, next, nd);
        memcpy(changed, changed_next, (size_t)n);
        for (size_t i = 0; i < nd; ++i) dom[i] = dom0[i] && !tilde[i];
        if (trace) memcpy(trace + (size_t)(k - 1) * nd, dom, nd);

        if (mode == 1 && any_empty(n, d, dom)) break;   /* throw inconsistency */
        if (!any_change) break;                         /* D~^(K) = D~^(K+1) */
        if (k >= max_steps) { rc = 2; break; }
    }
    if (iters) *iters = k;
    if (status) *status = any_empty(n, d, dom);
    if (checks) *checks = ncheck;
    free(arcs); free(dom0); free(tilde); free(next); free(changed); free(changed_next);
    return rc;
}

/* Is D arc consistent (Section 3's definition)? 1 yes, 0 no, -1 bad input. */
OR_API int oracle_is_ac(int32_t n, int32_t d, int64_t m, const int32_t *edges,
                        const uint8_t *rel, const uint8_t *dom) {
    if (n < 1 || d < 1 || m < 0) return -1;
    arc_t *arcs = build_arcs(n, m, edges);
    if (!arcs) return -1;
    int ok = 1;
    for (int64_t i = 0; i < 2 * m && ok; ++i) {
        const arc_t *r = &arcs[i];
        for (int32_t a = 0; a < d && ok; ++a) {
            if (!dom[(size_t)r->x * d + a]) continue;
            int sup = 0;
            for (int32_t b = 0; b < d && !sup; ++b)
                if (dom[(size_t)r->y * d + b] && arc_allows(rel, d, r, a, b)) sup = 1;
            if (!sup) ok = 0;
        }
    }
    free(arcs);
    return ok;
}
