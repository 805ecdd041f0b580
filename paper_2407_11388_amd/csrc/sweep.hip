// gfx950 kernels of the single-state fixpoint (bit-row and int8-row paths).
//
// One step of the recurrence (Eq. (1); tensorRevise of Algorithm 1): for every
// variable x and value a still in dom(x), a is removed when, on some arc
// x->y whose y is in the previous step's @changed set, no value b of the
// current dom(y) is allowed with a. Step k reads D^(k-1) from dom[(k-1)&1]
// and writes D^(k) to dom[k&1], so steps are synchronous as Eq. (1) requires.
//
// Scheduling: every step is three kernels. The plan kernel lists the problems
// (one problem = one domain state of one network) still running at step k
// and the prefix sums of their work items (whole variables, or a piece of one
// high-degree variable). The revise kernel hands each workgroup one
// contiguous range of those items; it ORs the values that lose their support
// into a per-variable accumulator. The update kernel applies the accumulator
// to D^(k-1), writes D^(k) and the @changed flags of step k, and records per
// problem whether the step removed anything or emptied a domain. The host
// enqueues the steps in rounds (captured HIP graphs of 4, 8, 16, ... steps)
// and reads one counter per round: the number of problems still running. No
// workgroup ever waits on another, and no counter is shared by work items.
#include "rac_internal.h"
#include "rac.h"

namespace rac {

#define DEV __device__ __forceinline__

// Pointers into device memory that arrive through descriptors are generic;
// casting them to the global address space lets the compiler emit global
// loads, which (unlike flat loads) do not count against the LDS wait counter.
#define GLOBAL __attribute__((address_space(1)))
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
template <typename T> DEV const GLOBAL T *as_global(const T *p) {
    return (const GLOBAL T *)p;
}

DEV uint64_t wave_or64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, kWave);
    return v;
}

DEV uint64_t dmask_of(int d) { return d >= 64 ? ~0ull : ((1ull << d) - 1ull); }

// 4 bits -> 4 bytes holding 0/1 (bit i of v becomes byte i). The factor places
// copies of v 7 bits apart, so no two copies overlap and no carry occurs.
DEV uint32_t spread4(uint32_t v) { return (v * 0x00204081u) & 0x01010101u; }

// ---------------------------------------------------------------------------
// Memory protocol. Within a kernel, D^(k-1), the @changed flags of step k-1
// and the control words are read-only (they were written by earlier kernels
// of the stream). The only data written by several workgroups of one kernel
// are the failure accumulators (agent-scope atomic OR, read by the next
// kernel) and a few per-problem words that every writer sets to the same
// value (last step with a change, first step with a wipe-out) or adds to with
// one atomic per workgroup.
// ---------------------------------------------------------------------------

// Where a step reads D^(k-1) and the previous step's @changed set from.
enum ViewKind { VIEW_PLAIN = 0, VIEW_LDS = 1 };

template <int VK>
struct DomView {
    const uint64_t *dom;   // [n] (LDS or global)
    const uint32_t *chg;   // LDS: bit mask; global: flags [n]
    DEV uint64_t get(int32_t y) const { return dom[y]; }
    DEV bool changed(int32_t y) const {
        if (VK == VIEW_LDS) return (chg[y >> 5] >> (y & 31)) & 1u;
        return chg[y] != 0;
    }
};

// ---------------------------------------------------------------------------
// Revision of the units [u0, u1) of one variable x by one wave. Returns the
// values a of x that some re-examined arc leaves without support (bit a set),
// identical in every lane. ALL: every arc is re-examined (the first step
// with @changed = all variables).
// ---------------------------------------------------------------------------

// Per-wave LDS scratch of the bit-row revision.
struct Scratch {
    unsigned long long *failx;   // [kItemVars] values of variable xbase + i found failing
    uint16_t *cmp;               // [kSparseGroups * 64] active arcs of a sparse batch:
                                 // (group within the batch << 6) | arc within the group
};

DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Position of this lane among the set lanes of m below it.
DEV int lane_rank(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Records that the values f of the item's variable slot `own` lost their
// support on some arc. Failures are rare, so the LDS atomic is seldom taken.
DEV void note_fail(const Scratch &S, int32_t own, uint64_t f) {
    if (f)
        (void)__hip_atomic_fetch_or(S.failx + own, (unsigned long long)f, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Bit rows in 64-arc groups (lane = arc). A lane tests each row a of its arc
// against dom(y) and records the rows without support under the variable
// owning the group. Rows of one 16-byte quad without support in dom(y), as
// bits 0..3 (uint32 rows) or 0..1 (uint64 rows).
template <bool WIDE>
DEV uint32_t quad_fail(const u32x4 v, uint64_t dy) {
    if (WIDE) {
        const uint64_t r0 = (uint64_t)v.x | ((uint64_t)v.y << 32);
        const uint64_t r1 = (uint64_t)v.z | ((uint64_t)v.w << 32);
        return ((r0 & dy) == 0 ? 1u : 0u) | ((r1 & dy) == 0 ? 2u : 0u);
    }
    const uint32_t d32 = (uint32_t)dy;
    return ((v.x & d32) == 0 ? 1u : 0u) | ((v.y & d32) == 0 ? 2u : 0u) |
           ((v.z & d32) == 0 ? 4u : 0u) | ((v.w & d32) == 0 ? 8u : 0u);
}

// Every arc re-examined (the first step with @changed = all variables): the
// groups g0 .. g1-1 are cut into units of one group and C row quads (C
// divides qpa); DEPTH units are kept in flight: unit t+DEPTH is issued right
// after unit t is tested. Every row is loaded (padding rows are zero), so no
// load waits for a neighbour index and no load is predicated.
template <int C>
struct GroupUnit {
    u32x4 v[C];
    int32_t y;
    int32_t q0;
    int32_t own;
    bool live;
};

// Cursor over the units of a range of groups: group g, quad chunk c.
struct UnitCursor {
    int64_t g, g1;
    int32_t c, nch;
    DEV void next() {
        if (++c == nch) {
            c = 0;
            ++g;
        }
    }
};

template <int C>
DEV void load_unit(GroupUnit<C> &u, UnitCursor &cur, const GLOBAL u32x4 *__restrict__ rows,
                   const GLOBAL int32_t *__restrict__ nbrp, const GLOBAL int32_t *__restrict__ gown,
                   int32_t xbase, int32_t qpa, int lane) {
    u.live = cur.g < cur.g1;     // wave-uniform
    if (!u.live) return;
    u.y = nbrp[cur.g * kGroup + lane];
    u.own = gown[cur.g] - xbase;
    u.q0 = cur.c * C;
    const GLOBAL u32x4 *base = rows + (cur.g * qpa + u.q0) * kGroup + lane;
#pragma unroll
    for (int q = 0; q < C; ++q) u.v[q] = base[q * kGroup];
    cur.next();
}

template <bool WIDE, int C, class DV>
DEV void test_unit(const GroupUnit<C> &u, const DV &D, const Scratch &S) {
    constexpr int RPQ = WIDE ? 2 : 4;
    static_assert(C * RPQ <= 32, "a unit covers at most 32 rows");
    if (!u.live) return;
    const bool valid = u.y >= 0;
    const uint64_t dy = D.get(valid ? u.y : 0);
    uint32_t f = 0;
#pragma unroll
    for (int q = 0; q < C; ++q) f |= quad_fail<WIDE>(u.v[q], dy) << (q * RPQ);
    if (valid) note_fail(S, u.own, (uint64_t)f << (u.q0 * RPQ));
}

template <bool WIDE, int C, int DEPTH, class DV>
DEV void revise_all(const GLOBAL u32x4 *__restrict__ rows, const GLOBAL int32_t *__restrict__ nbrp,
                    const GLOBAL int32_t *__restrict__ gown, const DV &D, int64_t g0, int64_t g1,
                    int32_t qpa, int32_t xbase, const Scratch &S) {
    const int lane = threadIdx.x & (kWave - 1);
    UnitCursor cur{g0, g1, 0, qpa / C};
    GroupUnit<C> u[DEPTH];
#pragma unroll
    for (int i = 0; i < DEPTH; ++i) load_unit<C>(u[i], cur, rows, nbrp, gown, xbase, qpa, lane);
    while (u[0].live) {
#pragma unroll
        for (int i = 0; i < DEPTH; ++i) {
            test_unit<WIDE, C>(u[i], D, S);
            load_unit<C>(u[i], cur, rows, nbrp, gown, xbase, qpa, lane);
        }
    }
}

// Only the arcs x->y with y in @changed re-examined (steps after the first,
// Proposition 2). The groups are taken kSparseGroups at a time: one load per
// lane per group fetches the neighbours, a ballot per group marks the arcs
// into changed variables, and their positions are compacted in LDS. The
// active arcs are then processed 64 at a time (lane = active arc), in units of
// C row quads, two units in flight. Loads past the last unit repeat the last
// active arc and are never tested, so every load is issued unconditionally.
template <bool WIDE, int C, class DV>
DEV void revise_sparse(const GLOBAL u32x4 *__restrict__ rows, const GLOBAL int32_t *__restrict__ nbrp,
                       const GLOBAL int32_t *__restrict__ gown, const DV &D, int64_t g0,
                       int64_t g1, int32_t qpa, int32_t xbase, const Scratch &S) {
    constexpr int RPQ = WIDE ? 2 : 4;
    const int lane = threadIdx.x & (kWave - 1);
    const int nch = qpa / C;
    struct Unit {
        u32x4 v[C];
        int32_t y, own, q0;
        bool ok;
    };
    for (int64_t gb = g0; gb < g1; gb += kSparseGroups) {
        const int nb = (int)(g1 - gb < kSparseGroups ? g1 - gb : kSparseGroups);
        int32_t y[kSparseGroups];
#pragma unroll
        for (int i = 0; i < kSparseGroups; ++i)
            y[i] = nbrp[(gb + (i < nb ? i : nb - 1)) * kGroup + lane];
        int total = 0;
#pragma unroll
        for (int i = 0; i < kSparseGroups; ++i) {
            const bool act = i < nb && y[i] >= 0 && D.changed(y[i] < 0 ? 0 : y[i]);
            const uint64_t m = __ballot(act);
            if (act) S.cmp[total + lane_rank(m)] = (uint16_t)(i * kGroup + lane);
            total += __popcll(m);
        }
        if (total == 0) continue;
        wave_sync();
        const int nunits = ((total + kWave - 1) / kWave) * nch;
        auto load = [&](int u, Unit &s) {
            const int uc = u < nunits ? u : nunits - 1;
            const int a = uc / nch;
            const int c = uc - a * nch;
            const int p = a * kWave + lane;
            s.ok = u < nunits && p < total;
            const int code = S.cmp[p < total ? p : total - 1];
            const int64_t g = gb + (code >> 6);
            const int l = code & (kGroup - 1);
            s.y = nbrp[g * kGroup + l];
            s.own = gown[g] - xbase;
            s.q0 = c * C;
            const GLOBAL u32x4 *base = rows + (g * qpa + s.q0) * kGroup + l;
#pragma unroll
            for (int q = 0; q < C; ++q) s.v[q] = base[q * kGroup];
        };
        auto test = [&](const Unit &s) {
            const uint64_t dy = D.get(s.y);
            uint32_t f = 0;
#pragma unroll
            for (int q = 0; q < C; ++q) f |= quad_fail<WIDE>(s.v[q], dy) << (q * RPQ);
            if (s.ok) note_fail(S, s.own, (uint64_t)f << (s.q0 * RPQ));
        };
        Unit s0, s1;
        load(0, s0);
        load(1, s1);
        for (int u = 0; u < nunits; u += 2) {
            test(s0);
            load(u + 2, s0);
            test(s1);
            load(u + 3, s1);
        }
        wave_sync();   // every lane has read S.cmp before the next batch rewrites it
    }
}

// The groups g0 .. g1-1 of a bit-row network; failures go to S.failx[own].
template <bool ALL, class DV>
DEV void revise_bits(const NetDesc &N, const DV &D, int64_t g0, int64_t g1, int32_t xbase,
                     const Scratch &S) {
    const GLOBAL u32x4 *rows = as_global((const u32x4 *)N.rows);
    const GLOBAL int32_t *nbrp = as_global(N.nbrp);
    const GLOBAL int32_t *gown = as_global(N.gown);
    if (N.kind == ROW64) {   // qpa is a multiple of 4
        if (ALL) revise_all<true, 4, 2>(rows, nbrp, gown, D, g0, g1, N.qpa, xbase, S);
        else revise_sparse<true, 4>(rows, nbrp, gown, D, g0, g1, N.qpa, xbase, S);
        return;
    }
#define RAC_ROW32(Q, DEP)                                                                   \
    case Q:                                                                                 \
        if (ALL) revise_all<false, Q, DEP>(rows, nbrp, gown, D, g0, g1, Q, xbase, S);       \
        else revise_sparse<false, Q>(rows, nbrp, gown, D, g0, g1, Q, xbase, S);             \
        return;
    switch (N.qpa) {         // ROW32: qpa = 1..8, one chunk per group
        RAC_ROW32(1, 8)
        RAC_ROW32(2, 4)
        RAC_ROW32(3, 3)
        RAC_ROW32(4, 2)
        RAC_ROW32(5, 2)
        RAC_ROW32(6, 2)
        RAC_ROW32(7, 2)
    default:
        if (ALL) revise_all<false, 8, 2>(rows, nbrp, gown, D, g0, g1, 8, xbase, S);
        else revise_sparse<false, 8>(rows, nbrp, gown, D, g0, g1, 8, xbase, S);
        return;
    }
#undef RAC_ROW32
}

// int8 rows (d <= 32, dp = 16 or 32 bytes per row): a lane reads 16 bytes of
// one row a and forms the int32 support count sum_b R[a][b] * dom_y[b] with
// int8 dot products; with 32-byte rows the two halves' counts are summed
// across the lane pair. A row fails when its count is zero. A unit is one
// step of A arcs; kI8Depth units are kept in flight. Addresses past the end
// are clamped to the last arc, whose repeated result is masked off.
constexpr int kI8Depth = 6;

template <bool ALL, class DV>
DEV uint64_t revise_i8(const GLOBAL int8_t *__restrict__ rows, const GLOBAL int32_t *__restrict__ nbr,
                       const DV &D, int64_t j0, int64_t j1, int32_t d, int32_t dp) {
    const int lane = threadIdx.x & (kWave - 1);
    const int lpr = dp >> 4;              // lanes per row: 1 or 2
    const int lpa = d * lpr;              // lanes per arc, <= 64
    const int A = kWave / lpa;
    const int s = lane / lpa;
    const int u0 = lane - s * lpa;        // 16-byte unit within the arc
    const int a = u0 / lpr;
    const int part = u0 - a * lpr;
    const bool active = s < A;
    const int64_t arc_bytes = (int64_t)d * dp;
    bool ok = true;
    i32x4 v[kI8Depth];
    int32_t y[kI8Depth];
    bool in[kI8Depth];
    int64_t jn = j0;                      // first arc of the next unit to load
    auto load = [&](int i) {
        const int64_t j = jn + s;
        in[i] = active && j < j1;
        const int64_t jc = j < j1 ? j : j1 - 1;
        y[i] = nbr[jc];
        bool want = true;
        if (!ALL) want = in[i] && D.changed(y[i]);
        if (want) v[i] = *reinterpret_cast<const GLOBAL i32x4 *>(rows + jc * arc_bytes + u0 * 16);
        if (!ALL) in[i] = want;
        jn += A;
    };
    auto test = [&](int i) {
        const uint32_t dy = (uint32_t)(D.get(y[i]) >> (part * 16)) & 0xFFFFu;
        int cnt = 0;
        cnt = __builtin_amdgcn_sdot4(v[i].x, (int)spread4(dy & 0xFu), cnt, false);
        cnt = __builtin_amdgcn_sdot4(v[i].y, (int)spread4((dy >> 4) & 0xFu), cnt, false);
        cnt = __builtin_amdgcn_sdot4(v[i].z, (int)spread4((dy >> 8) & 0xFu), cnt, false);
        cnt = __builtin_amdgcn_sdot4(v[i].w, (int)spread4((dy >> 12) & 0xFu), cnt, false);
        if (lpr == 2) cnt += __shfl_xor(cnt, 1, kWave);  // every lane executes it
        if (in[i] && cnt == 0) ok = false;
    };
    if (j0 < j1) {
#pragma unroll
        for (int i = 0; i < kI8Depth; ++i) load(i);
        for (int64_t jt = j0; jt < j1; jt += (int64_t)A * kI8Depth) {
#pragma unroll
            for (int i = 0; i < kI8Depth; ++i) {
                test(i);
                load(i);
            }
        }
    }
    const uint64_t fail = (active && part == 0 && !ok) ? (1ull << a) : 0ull;
    return wave_or64(fail);
}

// ---------------------------------------------------------------------------
// Work items
// ---------------------------------------------------------------------------

DEV unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

DEV void or_fail(const Launch &L, int64_t v, uint64_t f) {
    (void)__hip_atomic_fetch_or(L.ws.failacc + v, (unsigned long long)f, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
}

// One work item of a bit-row network: every group of the item's variables
// (or of one piece of a split variable) is revised in one pipeline; the
// failing values of each variable go to its accumulator.
template <bool ALL, class DV>
DEV void process_bits_item(const Launch &L, const NetDesc &N, const DV &D, const int4 it,
                           int64_t off, const Scratch &S) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t nx = it.y - it.x;   // <= kItemVars = kWave (work items are built so)
    S.failx[lane] = 0;
    wave_sync();
    revise_bits<ALL>(N, D, it.z, it.w, it.x, S);
    wave_sync();
    const uint64_t f = lane < nx ? S.failx[lane] : 0ull;
    if (f) or_fail(L, off + it.x + lane, f);
}

// One work item of an int8-row network: variable by variable.
template <bool ALL, class DV>
DEV void process_i8_item(const Launch &L, const NetDesc &N, const DV &D, const int4 it,
                         int32_t pieces, int64_t off) {
    const int lane = threadIdx.x & (kWave - 1);
    const GLOBAL int8_t *rows = as_global((const int8_t *)N.rows);
    const GLOBAL int32_t *nbr = as_global(N.nbr);
    for (int32_t x = it.x; x < it.y; ++x) {
        const int64_t j0 = pieces ? it.z : N.row_ptr[x];
        const int64_t j1 = pieces ? it.w : N.row_ptr[x + 1];
        const uint64_t fail = revise_i8<ALL>(rows, nbr, D, j0, j1, N.d, N.dp);
        if (lane == 0 && fail) or_fail(L, off + x, fail);
    }
}

// One piece of a changed variable y of a bit-row problem, in a step that
// re-examines few arcs (Proposition 2: only arcs x -> y into variables that
// changed in the previous step). The arcs into y are found through y's own
// arcs y -> x, whose reverse arc x -> y sits at rpos in the group layout;
// piece c covers y's arcs 64c .. 64c+63, one per lane. A lane ORs the values
// of x that have no support in D^(k-1)(y) into the accumulator of x.
template <bool WIDE>
DEV void process_push_item(const Launch &L, const NetDesc &N, int k, int64_t off, int32_t y,
                           int32_t c) {
    constexpr int RPQ = WIDE ? 2 : 4;
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t j = N.row_ptr[y] + c * kWave + lane;
    if (j >= N.row_ptr[y + 1]) return;
    const GLOBAL u32x4 *rows = as_global((const u32x4 *)N.rows);
    const uint64_t dy = L.ws.dom[(k - 1) & 1][off + y];
    const int32_t pos = N.rpos[j];
    const int32_t x = N.nbr[j];
    const GLOBAL u32x4 *base = rows + (int64_t)(pos >> 6) * N.qpa * kGroup + (pos & (kGroup - 1));
    uint64_t f = 0;
    if (WIDE) {
        for (int32_t q = 0; q < N.qpa; ++q)
            f |= (uint64_t)quad_fail<true>(base[(int64_t)q * kGroup], dy) << (q * RPQ);
    } else {
        // qpa <= 8 for uint32 rows
        u32x4 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < N.qpa) v[q] = base[q * kGroup];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < N.qpa) f |= (uint64_t)quad_fail<false>(v[q], dy) << (q * RPQ);
    }
    if (f) or_fail(L, off + x, f);
}

// ---------------------------------------------------------------------------
// Step control
// ---------------------------------------------------------------------------

DEV int32_t max_steps(const Launch &L, const NetDesc &N) {
    return L.max_sweeps > 0 ? L.max_sweeps : N.n * N.d + 1;
}

// Does problem p execute step k? Step 1 always; step k > 1 if step k-1
// removed a value (Algorithm 1's loop test), unless the step cap is reached
// or, when stopping on a wipe-out, an earlier step emptied a domain. Only
// words written by earlier kernels decide it (last_change >= k-1 also holds
// while the update kernel of step k raises it to k).
DEV bool active(const Launch &L, const NetDesc &N, const Ctrl &C, int k) {
    if (k > max_steps(L, N)) return false;
    if (k > 1 && C.last_change < k - 1) return false;
    if (L.mode == RAC_STOP_ON_WIPEOUT && C.wipe_step != 0 && C.wipe_step < k) return false;
    return true;
}

// Does step k list its changed variables? Only when step k itself
// re-examined few arcs (at most 4x the push bound): the change sets of later
// steps are usually smaller, and dense steps skip the cost of the list.
DEV bool listed_after(const Launch &L, const NetDesc &N, const Ctrl &C, int k) {
    return L.push_ratio > 0 && N.rpos && C.arcs[(k + 2) % 3] * L.push_ratio <= 4 * N.arcs;
}

// Network of problem p: with uniform_n set, every problem is an instance of
// nets[0] (no table load).
DEV const NetDesc &net_of(const Launch &L, int32_t p) {
    return L.uniform_n > 0 ? L.nets[0] : L.nets[L.prob_net[p]];
}

// Number of problems of a launch (Launch::nprob_dev, else nprob).
DEV int32_t problem_count(const Launch &L) { return L.nprob_dev ? *L.nprob_dev : L.nprob; }

DEV int prob_of_var(const Launch &L, int32_t nprob, int64_t v) {
    if (L.uniform_n > 0)   // 32-bit division whenever the index fits (the 64-bit one is long)
        return v <= 0x7FFFFFFF ? (int)((uint32_t)v / (uint32_t)L.uniform_n)
                               : (int)(v / L.uniform_n);
    int lo = 0, hi = nprob - 1;   // largest p with prob_off[p] <= v
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.prob_off[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The problems that execute step k, with the prefix sums of their item
// counts. One workgroup of 1024 threads; a pass gives thread t up to
// kPlanPer problems t, t + 1024, ... (a wave's loads read consecutive
// problems), whose loads are all issued before any is used (clamped
// indices), so that a pass costs about one memory latency. A thread's
// active problems are listed together, so the list is not in problem order;
// the revise kernel finds items only through the prefix sums.
constexpr int kPlanPer = 4;

// Plan of problems pt + i * 1024, i < per <= R, of one thread: item counts,
// and bit i of on_m / push_m for problem pt + i * 1024.
template <int R>
DEV void plan_problems(const Launch &L, int k, int32_t nprob, int32_t pt, int32_t per,
                       int64_t *items, uint32_t &on_m, uint32_t &push_m, int64_t &tot) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int32_t p = pt + i * 1024;
        const bool valid = i < per && p < nprob;
        const int32_t pc = valid ? p : nprob - 1;
        const NetDesc &N = net_of(L, pc);
        const Ctrl &C = L.ws.ctrl[pc];
        const bool on = valid && active(L, N, C, k);
        // few arcs to re-examine: the changed variables' pieces instead of a
        // scan of every group (step 1 of an incremental start: the pieces of
        // the listed @changed variables bound the arcs). Step k-1 listed its
        // changed variables only if it was itself sparse.
        bool push = false;
        if (L.push_ratio > 0 && N.rpos) {
            if (k > 1)
                push = listed_after(L, N, C, k - 1) && C.arcs[(k - 1) % 3] * L.push_ratio <= N.arcs;
            else if (L.changed0)
                push = (int64_t)C.nchg[0] * N.pchunks * kWave * L.push_ratio <= N.arcs;
        }
        push = push && on;
        const bool all = k == 1 && L.changed0 == nullptr;   // every arc re-examined
        items[i] = !on ? 0 : push ? (int64_t)C.nchg[(k - 1) & 1] * N.pchunks
                                  : all ? N.nitems : N.nitems_inc;
        on_m |= (uint32_t)on << i;
        push_m |= (uint32_t)push << i;
        tot += items[i];
    }
}

__global__ __launch_bounds__(1024) void plan_kernel(Launch L, int k) {
    const int32_t nprob = problem_count(L);
    __shared__ int64_t s_wave[16];
    __shared__ int64_t s_base_items;
    __shared__ int32_t s_wave_n[16];
    __shared__ int32_t s_base_n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        s_base_items = 0;
        s_base_n = 0;
    }
    __syncthreads();
    for (int32_t p0 = 0; p0 < nprob; p0 += 1024 * kPlanPer) {
        const int32_t left = nprob - p0;
        const int32_t per = left >= 1024 * kPlanPer ? kPlanPer : (left + 1023) / 1024;
        const int32_t pt = p0 + (int32_t)threadIdx.x;   // this thread's first problem
        int64_t items[kPlanPer] = {};
        uint32_t on_m = 0, push_m = 0;
        int64_t tot = 0;
        if (pt < nprob) {   // waves past the last problem issue no loads
            if (per == 1)
                plan_problems<1>(L, k, nprob, pt, per, items, on_m, push_m, tot);
            else if (per == 2)
                plan_problems<2>(L, k, nprob, pt, per, items, on_m, push_m, tot);
            else
                plan_problems<kPlanPer>(L, k, nprob, pt, per, items, on_m, push_m, tot);
        }
        const int32_t cnt = __popc(on_m);
        // inclusive scans of the thread totals within the wave, then across waves
        int64_t inc = tot;
        int32_t incn = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t t = __shfl_up(inc, o, 64);
            const int32_t tn = __shfl_up(incn, o, 64);
            if (lane >= o) {
                inc += t;
                incn += tn;
            }
        }
        if (lane == 63) {
            s_wave[wave] = inc;
            s_wave_n[wave] = incn;
        }
        __syncthreads();
        int64_t before = s_base_items + inc - tot;
        int32_t nbefore = s_base_n + incn - cnt;
        for (int w = 0; w < wave; ++w) {
            before += s_wave[w];
            nbefore += s_wave_n[w];
        }
#pragma unroll
        for (int i = 0; i < kPlanPer; ++i)
            if ((on_m >> i) & 1u) {
                L.ws.act[nbefore] = pt + i * 1024;
                L.ws.act_off[nbefore] = before;
                L.ws.act_push[nbefore] = (int32_t)((push_m >> i) & 1u);
                before += items[i];
                ++nbefore;
            }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 0; w < 16; ++w) {
                s_base_items += s_wave[w];
                s_base_n += s_wave_n[w];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        L.ws.act_off[s_base_n] = s_base_items;
        L.ws.plan->nact = s_base_n;
        L.ws.plan->items = s_base_items;
    }
}

// Stage D^(k-1) (and, when only changed arcs are re-examined, the @changed
// flags of step k-1 as a bit mask) of a problem in LDS.
DEV void stage(uint64_t *s_dom, uint32_t *s_chg, const uint64_t *gdom, const uint32_t *gchg,
               int32_t n, bool flags) {
    const int lane = threadIdx.x & (kWave - 1);
    constexpr int kBatch = 8;
    for (int32_t base = 0; base < n; base += kBatch * kWave) {
        uint64_t t[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int32_t v = base + i * kWave + lane;
            t[i] = v < n ? gdom[v] : 0ull;
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int32_t v = base + i * kWave + lane;
            if (v < n) s_dom[v] = t[i];
        }
    }
    if (flags) {
        for (int32_t base = 0; base < n; base += kBatch * kWave) {
            uint32_t t[kBatch];
#pragma unroll
            for (int i = 0; i < kBatch; ++i) {
                const int32_t v = base + i * kWave + lane;
                t[i] = v < n ? gchg[v] : 0u;
            }
#pragma unroll
            for (int i = 0; i < kBatch; ++i) {
                const int32_t b = base + i * kWave;
                const uint64_t m = __ballot(t[i] != 0);
                if (lane == 0 && b < n) {
                    s_chg[b >> 5] = (uint32_t)m;
                    s_chg[(b >> 5) + 1] = (uint32_t)(m >> 32);
                }
            }
        }
    }
    wave_sync();
}

// Step k, revision: workgroup w (one wave) takes items [w*T/G, (w+1)*T/G) of
// the T items the plan listed, stages each problem's D^(k-1) once, and ORs
// the failing values into the accumulators.
__global__ __launch_bounds__(kWave) void revise_kernel(Launch L, int k) {
    extern __shared__ uint64_t s_lds[];
    const Scratch S{reinterpret_cast<unsigned long long *>(s_lds),
                    reinterpret_cast<uint16_t *>(s_lds + kItemVars)};
    uint64_t *s_dom = s_lds + kScratchWords;
    uint32_t *s_chg = reinterpret_cast<uint32_t *>(s_dom + L.stage_vars);
    const int32_t nact = L.ws.plan->nact;
    const int64_t T = L.ws.plan->items;
    const int64_t G = gridDim.x;
    const int64_t c0 = T * blockIdx.x / G, c1 = T * (blockIdx.x + 1) / G;
    if (c0 >= c1) return;
    const bool all = (k == 1) && (L.changed0 == nullptr);
    // the listed problem holding item c0
    int a = 0;
    {
        int hi = nact - 1;
        while (a < hi) {
            const int mid = (a + hi + 1) >> 1;
            if (L.ws.act_off[mid] <= c0) a = mid; else hi = mid - 1;
        }
    }
    int staged = -1;
    for (int64_t c = c0; c < c1; ++c) {
        while (L.ws.act_off[a + 1] <= c) ++a;
        const int32_t p = L.ws.act[a];
        const NetDesc &N = net_of(L, p);
        const int64_t off = L.prob_off[p];
        const int32_t ci = (int32_t)(c - L.ws.act_off[a]);
        if (L.ws.act_push[a]) {
            const int32_t i = ci / N.pchunks;
            const int32_t y = L.ws.clist[(k - 1) & 1][off + i];
            if (N.kind == ROW64) process_push_item<true>(L, N, k, off, y, ci - i * N.pchunks);
            else process_push_item<false>(L, N, k, off, y, ci - i * N.pchunks);
            continue;
        }
        const int4 it = all ? N.items[ci] : N.items_inc[ci];
        const int32_t pieces = all ? N.pieces[ci] : N.pieces_inc[ci];
        const uint64_t *gdom = L.ws.dom[(k - 1) & 1] + off;
        const uint32_t *gchg = L.ws.chg[(k - 1) & 1] + off;
        if (N.n <= L.stage_vars) {
            if (p != staged) {
                stage(s_dom, s_chg, gdom, gchg, N.n, !all);
                staged = p;
            }
            const DomView<VIEW_LDS> D{s_dom, s_chg};
            if (N.kind == ROWI8) {
                if (all) process_i8_item<true>(L, N, D, it, pieces, off);
                else process_i8_item<false>(L, N, D, it, pieces, off);
            } else {
                if (all) process_bits_item<true>(L, N, D, it, off, S);
                else process_bits_item<false>(L, N, D, it, off, S);
            }
        } else {
            const DomView<VIEW_PLAIN> D{gdom, gchg};
            if (N.kind == ROWI8) {
                if (all) process_i8_item<true>(L, N, D, it, pieces, off);
                else process_i8_item<false>(L, N, D, it, pieces, off);
            } else {
                if (all) process_bits_item<true>(L, N, D, it, off, S);
                else process_bits_item<false>(L, N, D, it, off, S);
            }
        }
    }
}

// Block-wide reductions of the update kernel (256 threads = 4 waves).
struct UpdRed {
    unsigned long long deg[4];
    int32_t changed[4], wiped[4];
};

// Step k, update: D^(k)(v) = D^(k-1)(v) minus its accumulated failures, the
// @changed flag of step k (also as a list per problem), and per problem the
// last step with a change, the first step with a wipe-out, the arcs the next
// step re-examines (arcs into changed variables) and the support checks of
// step k (d*d per arc it re-examined).
__global__ __launch_bounds__(256) void update_kernel(Launch L, int k) {
    const int32_t nprob = problem_count(L);
    __shared__ UpdRed s_red;
    const int s_now = k % 3, s_prev = (k + 2) % 3, s_next = (k + 1) % 3;
    const int64_t nv = L.prob_off[nprob];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (blockIdx.x == 0)
        for (int32_t p = threadIdx.x; p < nprob; p += blockDim.x) {
            L.ws.ctrl[p].arcs[s_next] = 0;
            L.ws.ctrl[p].nchg[(k + 1) & 1] = 0;   // the list step k+1 appends to
        }
    int32_t *clist = L.ws.clist[k & 1];
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nv;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = base + threadIdx.x;
        const int64_t vlast = base + blockDim.x - 1 < nv ? base + blockDim.x - 1 : nv - 1;
        const int pb0 = prob_of_var(L, nprob, base), pb1 = prob_of_var(L, nprob, vlast);
        bool ch = false, wp = false, lst = false;
        unsigned long long dg = 0;
        int p = -1;
        int32_t x = 0;
        if (v < nv) {
            p = pb0 == pb1 ? pb0 : prob_of_var(L, nprob, v);
            const NetDesc &N = net_of(L, p);
            Ctrl &C = L.ws.ctrl[p];
            if (active(L, N, C, k)) {
                const uint64_t dx = L.ws.dom[(k - 1) & 1][v];
                const uint64_t f = L.ws.failacc[v];
                if (f) L.ws.failacc[v] = 0;
                const uint64_t nd = dx & ~f & dmask_of(N.d);
                ch = nd != dx;
                wp = nd == 0;
                L.ws.dom[k & 1][v] = nd;
                L.ws.chg[k & 1][v] = ch ? 1u : 0u;
                x = (int32_t)(v - L.prob_off[p]);
                if (ch) dg = (unsigned long long)N.deg[x];
                lst = ch && listed_after(L, N, C, k);
                if (x == 0) C.checks += C.arcs[s_prev] * (long long)N.d * N.d;
            }
        }
        if (pb0 == pb1) {   // the whole block is one problem: one atomic per block
            const uint64_t mc = __ballot(ch), mw = __ballot(wp);
            const unsigned long long ws = wave_sum64(dg);
            const uint64_t ml = __ballot(lst);
            if (ml) {   // the wave's changed variables join the problem's list
                const int leader = __ffsll((unsigned long long)ml) - 1;
                int32_t at = 0;
                if (lane == leader)
                    at = __hip_atomic_fetch_add(&L.ws.ctrl[pb0].nchg[k & 1], __popcll(ml),
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                at = __shfl(at, leader, 64);
                if (lst) clist[L.prob_off[pb0] + at + lane_rank(ml)] = x;
            }
            if (lane == 0) {
                s_red.deg[wave] = ws;
                s_red.changed[wave] = mc != 0;
                s_red.wiped[wave] = mw != 0;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                unsigned long long tdeg = 0;
                int tch = 0, twp = 0;
                for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                    tdeg += s_red.deg[w];
                    tch |= s_red.changed[w];
                    twp |= s_red.wiped[w];
                }
                Ctrl &C = L.ws.ctrl[pb0];
                if (tch) {
                    (void)__hip_atomic_fetch_add(&C.arcs[s_now], (long long)tdeg, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                    C.last_change = k;
                }
                if (twp && C.wipe_step == 0) C.wipe_step = k;
            }
            __syncthreads();
        } else if (p >= 0) {
            Ctrl &C = L.ws.ctrl[p];
            if (ch) {
                (void)__hip_atomic_fetch_add(&C.arcs[s_now], (long long)dg, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
                C.last_change = k;
                if (lst) {
                    const int32_t r = __hip_atomic_fetch_add(&C.nchg[k & 1], 1, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                    clist[L.prob_off[p] + r] = x;
                }
            }
            if (wp && C.wipe_step == 0) C.wipe_step = k;
        }
    }
}

// Step k for many states of one network at once (Launch::shared_rows; uint32
// bit rows, d <= 32): task t covers the 64-arc group g = t mod G of the
// network and the chunk t div G of kSharedStates listed states. Each lane
// loads its arc's rows once and tests them against the neighbour's domain in
// every state of the chunk in which that neighbour changed in step k-1
// (Prop. 2), so a step reads the rows once per chunk of states instead of
// once per state. The next state's change flag and domain are loaded while
// the current one is tested. Failing values go to the accumulators with one
// atomic per (group, state) that has any.
__global__ __launch_bounds__(kWave) void revise_shared_kernel(Launch L, int k) {
    const int32_t nact = L.ws.plan->nact;
    if (nact == 0) return;
    const NetDesc &N = L.nets[0];
    const int64_t G = N.gptr[N.n];
    const int64_t tasks = G * ((nact + kSharedStates - 1) / kSharedStates);
    const int lane = threadIdx.x & (kWave - 1);
    const GLOBAL u32x4 *rows = as_global(reinterpret_cast<const u32x4 *>(N.rows));
    const GLOBAL uint64_t *dom = as_global(L.ws.dom[(k - 1) & 1]);
    const GLOBAL uint32_t *chg = as_global(L.ws.chg[(k - 1) & 1]);
    const GLOBAL int32_t *act = as_global(L.ws.act);
    const int64_t n = L.uniform_n;
    const int qpa = N.qpa;   // <= 8 for uint32 rows
    const uint32_t dmask = (uint32_t)dmask_of(N.d);
    for (int64_t t = blockIdx.x; t < tasks; t += gridDim.x) {
        const int64_t g = t % G;
        const int32_t i0 = (int32_t)(t / G) * kSharedStates;
        const int32_t i1 = nact < i0 + kSharedStates ? nact : i0 + kSharedStates;
        const int32_t x = N.gown[g];
        const int32_t y = N.nbrp[g * kGroup + lane];
        const int32_t yc = y >= 0 ? y : 0;   // padding arcs read variable 0, unused
        u32x4 v[8];
        const GLOBAL u32x4 *q = rows + g * qpa * kGroup + lane;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (i < qpa) v[i] = q[(int64_t)i * kGroup];
        int64_t off_n = (int64_t)act[i0] * n;
        uint32_t cy_n = chg[off_n + yc];
        uint64_t dy_n = dom[off_n + yc];
        for (int32_t i = i0; i < i1; ++i) {
            const int64_t off = off_n;
            const uint32_t cy = cy_n;
            const uint64_t dy = dy_n;
            if (i + 1 < i1) {
                off_n = (int64_t)act[i + 1] * n;
                cy_n = chg[off_n + yc];
                dy_n = dom[off_n + yc];
            }
            const bool on = y >= 0 && cy != 0;
            if (!__ballot(on)) continue;
            uint32_t f = 0;
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c < qpa) f |= quad_fail<false>(v[c], dy) << (4 * c);
            if (!on) f = 0;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) f |= (uint32_t)__shfl_xor((int)f, o, kWave);
            f &= (uint32_t)dom[off + x] & dmask;
            if (lane == 0 && f) or_fail(L, off + x, f);
        }
    }
}

// Small problems in one launch: one workgroup per problem runs every step of
// Eq. (1) with the problem's domains in LDS (double-buffered), so a step
// costs two workgroup barriers instead of three dependent kernel launches.
// Bit rows only (ROW32 / ROW64), n <= kSmallMaxN. Outputs as the finish
// kernel writes them: domains, step count, status, support checks, and
// rc_out = 1 when a problem stopped at the step cap unconverged.
//
// A step re-examines the arcs x -> y into the variables y changed in the
// previous step (Prop. 2) in one of two ways, chosen per step by their number:
// * scan: wave w takes the 64-arc groups w, w + waves, ... (lane = arc; a
//   group's arcs all leave one variable x), tests the rows of each arc into a
//   changed variable against that variable's domain and ORs the failures of x
//   into its LDS word. The next group's neighbour indices are loaded while
//   the current one is tested, a group's row quads up to 8 at a time.
// * walk: the changed variables' own arcs y -> x, numbered consecutively
//   over the step's list of changed variables, 64 per wave at a time; a lane
//   finds its variable y by a binary search over the list's arc offsets,
//   reads the rows of the reverse arc x -> y (through NetDesc::rpos) and ORs
//   the values of x without support in dom(y) into x's LDS word.
// The update phase removes the failures, and lists the changed variables
// with their arc offsets (one 64-bit LDS atomic per variable: list length in
// the high word, arcs in the low word, so offsets grow with the list index).
template <bool WIDE>
DEV void small_scan(const NetDesc &N, const uint64_t *__restrict__ dom, const uint8_t *__restrict__ chg,
                    unsigned long long *failx, int wave, int nwaves, int lane) {
    constexpr int RPQ = WIDE ? 2 : 4;   // rows per quad
    const GLOBAL u32x4 *rows = as_global(reinterpret_cast<const u32x4 *>(N.rows));
    const GLOBAL int32_t *nbrp = as_global(N.nbrp);
    const GLOBAL int32_t *gown = as_global(N.gown);
    const int64_t ngroups = N.gptr[N.n];
    const int qpa = N.qpa;
    const uint64_t dmask = dmask_of(N.d);
    int64_t g = wave;
    int32_t y_next = -1, x_next = 0;
    if (g < ngroups) {
        y_next = nbrp[g * kGroup + lane];
        x_next = gown[g];
    }
    for (; g < ngroups; g += nwaves) {
        const int32_t y = y_next, x = x_next;
        const int64_t gn = g + nwaves;
        if (gn < ngroups) {
            y_next = nbrp[gn * kGroup + lane];
            x_next = gown[gn];
        }
        const int32_t yc = y >= 0 ? y : 0;   // padding arcs read variable 0, unused
        const bool on = y >= 0 && chg[yc];
        if (!__ballot(on)) continue;
        const uint64_t dy = on ? dom[yc] : ~0ull;   // lanes off: every row has support
        const GLOBAL u32x4 *q = rows + g * qpa * kGroup + lane;
        uint64_t f = 0;
        for (int c0 = 0; c0 < qpa; c0 += 8) {
            u32x4 v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (c0 + i < qpa) v[i] = q[(int64_t)(c0 + i) * kGroup];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (c0 + i < qpa) f |= (uint64_t)quad_fail<WIDE>(v[i], dy) << ((c0 + i) * RPQ);
        }
        if (!on) f = 0;
        f = wave_or64(f) & dom[x] & dmask;
        if (lane == 0 && f)
            (void)__hip_atomic_fetch_or(failx + x, (unsigned long long)f, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

template <bool WIDE>
DEV void small_walk(const NetDesc &N, const uint64_t *__restrict__ dom, const uint16_t *__restrict__ clist,
                    const uint32_t *__restrict__ cstart, int32_t ncl, int64_t arcs,
                    unsigned long long *failx, int wave, int nwaves, int lane) {
    constexpr int RPQ = WIDE ? 2 : 4;
    const GLOBAL u32x4 *rows = as_global(reinterpret_cast<const u32x4 *>(N.rows));
    const GLOBAL int32_t *row_ptr = as_global(N.row_ptr);
    const GLOBAL int32_t *nbr = as_global(N.nbr);
    const GLOBAL int32_t *rpos = as_global(N.rpos);
    const int qpa = N.qpa;
    const uint64_t dmask = dmask_of(N.d);
    for (int64_t t0 = (int64_t)wave * kWave; t0 < arcs; t0 += (int64_t)nwaves * kWave) {
        const int64_t t = t0 + lane;
        if (t >= arcs) continue;
        // the list entry i with cstart[i] <= t < cstart[i + 1]
        int32_t lo = 0, hi = ncl - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if ((int64_t)cstart[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int32_t y = clist[lo];
        const int32_t j = row_ptr[y] + (int32_t)(t - cstart[lo]);
        const int32_t x = nbr[j];
        const int32_t pos = rpos[j];
        const GLOBAL u32x4 *q = rows + (int64_t)(pos >> 6) * qpa * kGroup + (pos & (kGroup - 1));
        const uint64_t dy = dom[y];
        uint64_t f = 0;
        for (int c0 = 0; c0 < qpa; c0 += 8) {
            u32x4 v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (c0 + i < qpa) v[i] = q[(int64_t)(c0 + i) * kGroup];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (c0 + i < qpa) f |= (uint64_t)quad_fail<WIDE>(v[i], dy) << ((c0 + i) * RPQ);
        }
        f &= dom[x] & dmask;
        if (f)
            (void)__hip_atomic_fetch_or(failx + x, (unsigned long long)f, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

__global__ __launch_bounds__(kSmallMaxThreads) void small_fixpoint_kernel(Launch L) {
    // dom[2][n] and fail[n] (8 bytes), cstart[2][n] (4), clist[2][n] (2), chg[2][n] (1)
    extern __shared__ uint64_t s_lds[];
    __shared__ int32_t s_any[2], s_wipe;
    __shared__ unsigned long long s_list[2];   // (list length << 32) + arcs of the listed variables
    const int32_t nprob = problem_count(L);
    // one problem at a time per workgroup (the grid may be smaller than the
    // problem count: the search launches one grid for every round)
    for (int32_t p = blockIdx.x; p < nprob; p += gridDim.x) {
        const NetDesc &N = net_of(L, p);
        const int32_t n = N.n;
        const int64_t off = L.uniform_n > 0 ? (int64_t)p * L.uniform_n : L.prob_off[p];
        uint64_t *dom0 = s_lds, *dom1 = s_lds + n;
        unsigned long long *failx = reinterpret_cast<unsigned long long *>(s_lds + 2 * n);
        uint32_t *cst0 = reinterpret_cast<uint32_t *>(s_lds + 3 * n), *cst1 = cst0 + n;
        uint16_t *cl0 = reinterpret_cast<uint16_t *>(cst1 + n), *cl1 = cl0 + n;
        uint8_t *chg0 = reinterpret_cast<uint8_t *>(cl1 + n), *chg1 = chg0 + n;
        const GLOBAL int32_t *deg = as_global(N.deg);
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
        if (tid == 0) {
            s_list[0] = 0;
            s_wipe = 0;
        }
        __syncthreads();
        for (int32_t x = tid; x < n; x += blockDim.x) {
            dom0[x] = L.din[off + x];
            const bool c = L.changed0 ? L.changed0[off + x] != 0 : true;
            chg0[x] = c ? 1 : 0;
            failx[x] = 0;
            if (c && L.changed0) {   // the initial list (all variables: scanned, not listed)
                const unsigned long long at = __hip_atomic_fetch_add(
                    &s_list[0], (1ull << 32) + (unsigned long long)deg[x], __ATOMIC_RELAXED,
                    __HIP_MEMORY_SCOPE_WORKGROUP);
                cl0[at >> 32] = (uint16_t)x;
                cst0[at >> 32] = (uint32_t)at;
            }
        }
        __syncthreads();
        int32_t ncl = (int32_t)(s_list[0] >> 32);
        int64_t arcs_cur = L.changed0 ? (int64_t)(s_list[0] & 0xFFFFFFFFull) : N.arcs;
        const int32_t maxs = max_steps(L, N);
        long long arcs_total = 0;   // re-examined arcs over all steps
        int32_t k = 0, last_change = 0, wipe_step = 0;
        uint64_t *cur = dom0, *nxt = dom1;
        uint8_t *cin = chg0, *cout = chg1;
        while (k < maxs) {
            ++k;
            const int li = (k - 1) & 1, lo = k & 1;   // lists: read (step k-1's), written (step k's)
            // revise: walk the changed variables' arcs when they are listed (every
            // step but a first one that starts from all variables) and at most a
            // quarter of the network's arcs; else scan the groups
            const bool listed = k > 1 || L.changed0 != nullptr;
            if (N.rpos && listed && arcs_cur * kSmallWalkRatio <= N.arcs) {
                const uint16_t *cl = li ? cl1 : cl0;
                const uint32_t *cs = li ? cst1 : cst0;
                if (N.kind == ROW64)
                    small_walk<true>(N, cur, cl, cs, ncl, arcs_cur, failx, wave, nwaves, lane);
                else
                    small_walk<false>(N, cur, cl, cs, ncl, arcs_cur, failx, wave, nwaves, lane);
            } else {
                if (N.kind == ROW64)
                    small_scan<true>(N, cur, cin, failx, wave, nwaves, lane);
                else
                    small_scan<false>(N, cur, cin, failx, wave, nwaves, lane);
            }
            arcs_total += arcs_cur;
            if (tid == 0) {
                s_any[lo] = 0;
                s_list[lo] = 0;
            }
            __syncthreads();   // every failure of step k recorded
            uint16_t *clo = lo ? cl1 : cl0;
            uint32_t *cso = lo ? cst1 : cst0;
            int any = 0, wiped = 0;
            for (int32_t x = tid; x < n; x += blockDim.x) {
                const uint64_t o = cur[x], nd = o & ~failx[x] & dmask_of(N.d);
                nxt[x] = nd;
                const bool c = nd != o;
                cout[x] = c ? 1 : 0;
                failx[x] = 0;
                any |= c;
                wiped |= nd == 0;
                if (c) {
                    const unsigned long long at = __hip_atomic_fetch_add(
                        &s_list[lo], (1ull << 32) + (unsigned long long)deg[x], __ATOMIC_RELAXED,
                        __HIP_MEMORY_SCOPE_WORKGROUP);
                    clo[at >> 32] = (uint16_t)x;
                    cso[at >> 32] = (uint32_t)at;
                }
            }
            if (__ballot(any) && lane == 0) atomicOr(&s_any[lo], 1);
            if (__ballot(wiped) && lane == 0) atomicOr(&s_wipe, 1);
            __syncthreads();   // the step's change and wipe-out words and its list
            const bool changed = s_any[lo] != 0;
            ncl = (int32_t)(s_list[lo] >> 32);
            arcs_cur = (int64_t)(s_list[lo] & 0xFFFFFFFFull);
            if (changed) last_change = k;
            if (s_wipe && wipe_step == 0) wipe_step = k;
            uint64_t *t64 = cur;
            cur = nxt;
            nxt = t64;
            uint8_t *t8 = cin;
            cin = cout;
            cout = t8;
            if (!changed) break;
            if (L.mode == RAC_STOP_ON_WIPEOUT && wipe_step != 0) break;
        }
        int32_t iters, rc = 0;
        if (L.mode == RAC_STOP_ON_WIPEOUT && wipe_step != 0) {
            iters = wipe_step;
        } else if (last_change < maxs) {
            iters = last_change + 1;
        } else {
            iters = maxs;
            rc = 1;
        }
        for (int32_t x = tid; x < n; x += blockDim.x) L.dout[off + x] = cur[x];
        if (tid == 0) {
            if (L.iters_out) L.iters_out[p] = iters;
            if (L.status_out) L.status_out[p] = wipe_step != 0 ? RAC_WIPEOUT : RAC_CONSISTENT;
            if (L.checks_out) L.checks_out[p] = arcs_total * N.d * N.d;
            if (rc && L.rc_out) atomicOr(L.rc_out, 1);
        }
        __syncthreads();   // the LDS is free for the next problem
    }
}

// Clears one word (the non-convergence flag before a fused launch).
__global__ void clear_word_kernel(int32_t *w) {
    if (threadIdx.x == 0) *w = 0;
}

__global__ void init_kernel(Launch L) {
    const int32_t nprob = problem_count(L);
    const int64_t nv = L.prob_off[nprob];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < nv; v += nthreads) {
        L.ws.dom[0][v] = L.din[v];
        const bool c = L.changed0 ? L.changed0[v] != 0 : true;
        L.ws.chg[0][v] = c ? 1u : 0u;
        L.ws.failacc[v] = 0;
    }
    for (int64_t p = tid; p < nprob; p += nthreads) {
        const NetDesc &N = net_of(L, p);
        Ctrl &C = L.ws.ctrl[p];
        // arcs step 1 re-examines (arcs1 < 0: summed by list_changed0_kernel)
        C.arcs[0] = L.changed0 ? (L.arcs1 < 0 ? 0 : L.arcs1) : N.arcs;
        C.arcs[1] = 0;
        C.arcs[2] = 0;
        C.checks = 0;
        C.last_change = 0;
        C.wipe_step = 0;
        C.nchg[0] = 0;
        C.nchg[1] = 0;
    }
    if (tid == 0 && L.rc_out) *L.rc_out = 0;
}

// With an initial @changed set: list its variables per problem (the
// changed-variable list of "step 0"), after init_kernel has zeroed the counts;
// with arcs1 < 0 also each problem's arcs into them (sum of deg).
__global__ void list_changed0_kernel(Launch L) {
    const int32_t nprob = problem_count(L);
    const int64_t nv = L.prob_off[nprob];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    for (int64_t base = tid - lane; base < nv; base += nthreads) {
        const int64_t v = base + lane;
        const bool c = v < nv && L.changed0[v];
        const int64_t vl = base + 63 < nv ? base + 63 : nv - 1;
        const int p0 = prob_of_var(L, nprob, base), p1 = prob_of_var(L, nprob, vl);
        const uint64_t m = __ballot(c);
        if (!m) continue;
        if (p0 == p1) {   // one problem: one atomic for the wave
            const int leader = __ffsll((unsigned long long)m) - 1;
            int32_t at = 0;
            if (lane == leader)
                at = __hip_atomic_fetch_add(&L.ws.ctrl[p0].nchg[0], __popcll(m), __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
            at = __shfl(at, leader, 64);
            if (c) L.ws.clist[0][L.prob_off[p0] + at + lane_rank(m)] = (int32_t)(v - L.prob_off[p0]);
            if (L.arcs1 < 0) {
                const NetDesc &N = net_of(L, p0);
                const unsigned long long dg =
                    wave_sum64(c ? (unsigned long long)N.deg[v - L.prob_off[p0]] : 0ull);
                if (lane == leader)
                    (void)__hip_atomic_fetch_add(&L.ws.ctrl[p0].arcs[0], (long long)dg,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else if (c) {
            const int p = prob_of_var(L, nprob, v);
            const int32_t r = __hip_atomic_fetch_add(&L.ws.ctrl[p].nchg[0], 1, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
            L.ws.clist[0][L.prob_off[p] + r] = (int32_t)(v - L.prob_off[p]);
            if (L.arcs1 < 0)
                (void)__hip_atomic_fetch_add(&L.ws.ctrl[p].arcs[0],
                                             (long long)net_of(L, p).deg[v - L.prob_off[p]],
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ void finish_kernel(Launch L) {
    const int32_t nprob = problem_count(L);
    const int64_t nv = L.prob_off[nprob];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    auto iters_of = [&](int p, int32_t *rc) {
        const NetDesc &N = net_of(L, p);
        const Ctrl &C = L.ws.ctrl[p];
        const int32_t maxs = max_steps(L, N);
        if (L.mode == RAC_STOP_ON_WIPEOUT && C.wipe_step != 0) {
            *rc = 0;
            return C.wipe_step;
        }
        if (C.last_change < maxs) {
            *rc = 0;
            return C.last_change + 1;
        }
        *rc = 1;
        return maxs;
    };
    for (int64_t v = tid; v < nv; v += nthreads) {
        const int p = prob_of_var(L, nprob, v);
        int32_t rc;
        const int32_t it = iters_of(p, &rc);
        L.dout[v] = L.ws.dom[it & 1][v];
    }
    for (int64_t p = tid; p < nprob; p += nthreads) {
        const Ctrl &C = L.ws.ctrl[p];
        int32_t rc;
        const int32_t it = iters_of((int)p, &rc);
        if (L.iters_out) L.iters_out[p] = it;
        if (L.status_out) L.status_out[p] = C.wipe_step != 0 ? RAC_WIPEOUT : RAC_CONSISTENT;
        if (L.checks_out) L.checks_out[p] = C.checks;
        if (rc && L.rc_out) atomicOr(L.rc_out, 1);
    }
}

// Relation row a of an arc from the per-constraint rows rel[e][a] (bit b =
// (a,b) allowed). src = 2e + flip; flip = 1 for the arc y->x, whose row b is
// column b of the constraint's matrix. Rows a >= d are empty.
DEV uint64_t arc_row(const uint64_t *rel, int32_t src, int32_t d, int32_t a) {
    if (src < 0 || a >= d) return 0;
    const uint64_t *R = rel + (int64_t)(src >> 1) * d;
    if ((src & 1) == 0) return R[a];
    uint64_t row = 0;
    for (int b = 0; b < d; ++b) row |= ((R[b] >> a) & 1ull) << b;
    return row;
}

// Bit rows in the 64-arc group layout: thread (g, q, l) writes quad q of arc
// l of group g. src_p[g*64+l] is the arc's source code, -1 for padding.
__global__ void pack_bits_kernel(const uint64_t *rel, const int32_t *src_p, int64_t groups,
                                 int32_t d, int32_t qpa, int32_t kind, uint4 *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= groups * qpa * kGroup) return;
    const int32_t l = (int32_t)(i % kGroup);
    const int64_t gq = i / kGroup;
    const int32_t q = (int32_t)(gq % qpa);
    const int64_t g = gq / qpa;
    const int32_t src = src_p[g * kGroup + l];
    uint4 v;
    if (kind == ROW32) {
        v.x = (uint32_t)arc_row(rel, src, d, 4 * q);
        v.y = (uint32_t)arc_row(rel, src, d, 4 * q + 1);
        v.z = (uint32_t)arc_row(rel, src, d, 4 * q + 2);
        v.w = (uint32_t)arc_row(rel, src, d, 4 * q + 3);
    } else {
        const uint64_t r0 = arc_row(rel, src, d, 2 * q);
        const uint64_t r1 = arc_row(rel, src, d, 2 * q + 1);
        v.x = (uint32_t)r0;
        v.y = (uint32_t)(r0 >> 32);
        v.z = (uint32_t)r1;
        v.w = (uint32_t)(r1 >> 32);
    }
    out[i] = v;
}

// 0/1 int8 rows: out[j][a][b], rows_per_arc rows of dp bytes, zero beyond d.
__global__ void pack_i8_kernel(const uint64_t *rel, const int32_t *arc_src, int64_t arcs,
                               int32_t d, int32_t rows_per_arc, int32_t dp, int8_t *out) {
    const int64_t words_per_row = dp / 4;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= arcs * rows_per_arc * words_per_row) return;
    const int64_t q = i % words_per_row;
    const int64_t r = i / words_per_row;
    const int32_t a = (int32_t)(r % rows_per_arc);
    const int64_t j = r / rows_per_arc;
    const uint64_t row = arc_row(rel, arc_src[j], d, a);
    uint32_t w = 0;
    for (int t = 0; t < 4; ++t) {
        const int b = (int)(q * 4) + t;
        if (b < d && ((row >> b) & 1ull)) w |= 1u << (8 * t);
    }
    reinterpret_cast<uint32_t *>(out)[i] = w;
}

}  // namespace rac
