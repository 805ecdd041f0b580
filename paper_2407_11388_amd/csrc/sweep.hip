// gfx950 kernels of the single-state fixpoint (bit-row and int8-row paths).
//
// One step of the recurrence (Eq. (1); tensorRevise of Algorithm 1): for every
// variable x and value a still in dom(x), a is removed when, on some arc
// x->y whose y is in the previous step's @changed set, no value b of the
// current dom(y) is allowed with a. Step k reads D^(k-1) from dom[(k-1)&1]
// and writes D^(k) to dom[k&1], so steps are synchronous as Eq. (1) requires.
//
// Scheduling: one persistent launch runs every step of every problem (one
// problem = one domain state of one network). A problem's step is cut into
// work items (whole variables, or a piece of one high-degree variable). A
// workgroup claims an item with one atomic on the problem's ticket word
// (step << 32 | item). The workgroup that completes the last item of a step
// finalises it: it reads the step's change / wipe-out flags and either
// publishes the next step's ticket (release) or retires the problem. Item
// claims are ordered after the previous step's completion by that ticket, so
// no workgroup ever waits on another: idle workgroups only poll for new
// tickets, with a bounded number of polls.
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

template <typename T> DEV T ld_rlx(T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> DEV T ld_acq(T *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> DEV void st_rlx(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> DEV void st_rel(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> DEV T add_ar(T *p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> DEV T or_ar(T *p, T v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> DEV T max_ar(T *p, T v) {
    return __hip_atomic_fetch_max(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> DEV T xchg_ar(T *p, T v) {
    return __hip_atomic_exchange(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
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

constexpr int kUnroll = 4;

// ---------------------------------------------------------------------------
// Memory protocol. Data another workgroup wrote in this launch (domains of
// steps >= 1, change flags, control words) is only ever read with agent-scope
// relaxed atomics, which the hardware keeps coherent across the XCDs' L2
// caches without cache-wide write-back or invalidation, and written the same
// way. Before a wave signals that an item is complete it waits until its own
// stores and atomics have been performed (vmcnt(0)). A claimer reads nothing
// of a step before its claim atomic has returned that step's ticket. Step 1
// reads D^(0), written by the previous kernel, with ordinary loads. Relation
// rows, arc lists and work items are read-only during the launch.
// ---------------------------------------------------------------------------

DEV void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Where a step reads D^(k-1) and the previous step's @changed set from.
enum ViewKind { VIEW_PLAIN = 0, VIEW_LDS = 1, VIEW_COHERENT = 2 };

template <int VK>
struct DomView {
    const uint64_t *dom;   // [n] (LDS or global)
    const uint32_t *chg;   // LDS: bit mask; global: flags [n]
    DEV uint64_t get(int32_t y) const {
        if (VK == VIEW_COHERENT) return ld_rlx(const_cast<uint64_t *>(dom + y));
        return dom[y];
    }
    DEV bool changed(int32_t y) const {
        if (VK == VIEW_LDS) return (chg[y >> 5] >> (y & 31)) & 1u;
        if (VK == VIEW_COHERENT) return ld_rlx(const_cast<uint32_t *>(chg + y)) != 0;
        return chg[y] != 0;
    }
};

// ---------------------------------------------------------------------------
// Revision of the units [u0, u1) of one variable x by one wave. Returns the
// values a of x that some re-examined arc leaves without support (bit a set),
// identical in every lane. ALL: every arc is re-examined (the first step
// with @changed = all variables).
// ---------------------------------------------------------------------------

// Bit rows in 64-arc groups (lane = arc). A lane tests each row a of its arc
// against dom(y) and records the rows without support; OR-ing those masks
// over the lanes and groups gives the values that lose all support on some
// arc. Work is cut into units of one group and C row quads (C divides qpa);
// DEPTH units are kept in flight: unit t+DEPTH is issued right after unit t
// is tested. In the first step every row is loaded (padding rows are zero),
// so no load waits for a neighbour index and no load is predicated.
// Rows of one 16-byte quad without support in dom(y), as bits 0..3 (uint32
// rows) or 0..1 (uint64 rows).
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

template <int C>
struct GroupUnit {
    u32x4 v[C];
    int32_t y;
    int32_t q0;
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

template <bool ALL, int C, class DV>
DEV void load_unit(GroupUnit<C> &u, UnitCursor &cur, const GLOBAL u32x4 *__restrict__ rows,
                   const GLOBAL int32_t *__restrict__ nbrp, const DV &D, int32_t qpa, int lane) {
    u.live = cur.g < cur.g1;     // wave-uniform
    if (!u.live) return;
    u.y = nbrp[cur.g * kGroup + lane];
    u.q0 = cur.c * C;
    const GLOBAL u32x4 *base = rows + (cur.g * qpa + u.q0) * kGroup + lane;
    if (ALL) {
#pragma unroll
        for (int q = 0; q < C; ++q) u.v[q] = base[q * kGroup];
    } else {
        if (u.y >= 0 && D.changed(u.y)) {
#pragma unroll
            for (int q = 0; q < C; ++q) u.v[q] = base[q * kGroup];
        }
    }
    cur.next();
}

template <bool ALL, bool WIDE, int C, class DV>
DEV uint64_t test_unit(const GroupUnit<C> &u, const DV &D) {
    constexpr int RPQ = WIDE ? 2 : 4;
    static_assert(C * RPQ <= 32, "a unit covers at most 32 rows");
    if (!u.live) return 0;
    const bool valid = u.y >= 0 && (ALL || D.changed(u.y < 0 ? 0 : u.y));
    const uint64_t dy = D.get(valid ? u.y : 0);
    uint32_t f = 0;
#pragma unroll
    for (int q = 0; q < C; ++q) f |= quad_fail<WIDE>(u.v[q], dy) << (q * RPQ);
    if (!valid) f = 0;
    return (uint64_t)f << (u.q0 * RPQ);
}

template <bool ALL, bool WIDE, int C, int DEPTH, class DV>
DEV uint64_t revise_groups(const GLOBAL u32x4 *__restrict__ rows,
                           const GLOBAL int32_t *__restrict__ nbrp, const DV &D, int64_t g0,
                           int64_t g1, int32_t qpa) {
    const int lane = threadIdx.x & (kWave - 1);
    UnitCursor cur{g0, g1, 0, qpa / C};
    GroupUnit<C> u[DEPTH];
#pragma unroll
    for (int i = 0; i < DEPTH; ++i) load_unit<ALL, C>(u[i], cur, rows, nbrp, D, qpa, lane);
    uint64_t fail = 0;
    while (u[0].live) {
#pragma unroll
        for (int i = 0; i < DEPTH; ++i) {
            fail |= test_unit<ALL, WIDE, C>(u[i], D);
            load_unit<ALL, C>(u[i], cur, rows, nbrp, D, qpa, lane);
        }
    }
    return wave_or64(fail);
}

template <bool ALL, class DV>
DEV uint64_t revise_bits(const NetDesc &N, const DV &D, int64_t g0, int64_t g1) {
    const GLOBAL u32x4 *rows = as_global((const u32x4 *)N.rows);
    const GLOBAL int32_t *nbrp = as_global(N.nbrp);
    if (N.kind == ROW64)   // qpa is a multiple of 4
        return revise_groups<ALL, true, 4, 2>(rows, nbrp, D, g0, g1, N.qpa);
    switch (N.qpa) {       // ROW32: qpa = 1..8, one chunk per group
    case 1: return revise_groups<ALL, false, 1, 8>(rows, nbrp, D, g0, g1, 1);
    case 2: return revise_groups<ALL, false, 2, 4>(rows, nbrp, D, g0, g1, 2);
    case 3: return revise_groups<ALL, false, 3, 3>(rows, nbrp, D, g0, g1, 3);
    case 4: return revise_groups<ALL, false, 4, 2>(rows, nbrp, D, g0, g1, 4);
    case 5: return revise_groups<ALL, false, 5, 2>(rows, nbrp, D, g0, g1, 5);
    case 6: return revise_groups<ALL, false, 6, 2>(rows, nbrp, D, g0, g1, 6);
    case 7: return revise_groups<ALL, false, 7, 2>(rows, nbrp, D, g0, g1, 7);
    default: return revise_groups<ALL, false, 8, 2>(rows, nbrp, D, g0, g1, 8);
    }
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

template <bool ALL, class DV>
DEV uint64_t revise(const NetDesc &N, const DV &D, int64_t u0, int64_t u1) {
    if (N.kind != ROWI8) return revise_bits<ALL>(N, D, u0, u1);
    return revise_i8<ALL>(as_global((const int8_t *)N.rows), as_global(N.nbr), D, u0, u1, N.d,
                          N.dp);
}

// ---------------------------------------------------------------------------
// Per-problem bookkeeping
// ---------------------------------------------------------------------------

struct ItemFlags {
    int changed;
    int wiped;
    unsigned long long degsum;
};

// New domain of x after step k: D^(k)(x) = D^(k-1)(x) minus the failing values.
DEV void update_var(const NetDesc &N, uint64_t *dnext, uint32_t *chg_next, int32_t x,
                    uint64_t dx, uint64_t fail, ItemFlags &f) {
    const uint64_t nx = dx & ~fail & dmask_of(N.d);
    const bool changed = nx != dx;
    st_rlx(dnext + x, nx);
    st_rlx(chg_next + x, changed ? 1u : 0u);
    if (changed) {
        f.changed = 1;
        f.degsum += (unsigned long long)N.deg[x];
    }
    if (nx == 0) f.wiped = 1;
}

template <bool ALL, class DV>
DEV void process_item(const Launch &L, const NetDesc &N, const DV &D, int k, const int4 it,
                      int32_t pieces, int64_t off, ItemFlags &f) {
    uint64_t *dnext = L.ws.dom[k & 1] + off;
    uint32_t *chg_next = L.ws.chg[k & 1] + off;
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t *up = N.kind == ROWI8 ? N.row_ptr : N.gptr;
    if (pieces == 0) {
        // whole variables, one after the other
        for (int32_t x = it.x; x < it.y; ++x) {
            const uint64_t dx = D.get(x);
            uint64_t fail = 0;
            if (dx != 0) fail = revise<ALL>(N, D, up[x], up[x + 1]);
            if (lane == 0) update_var(N, dnext, chg_next, x, dx, fail, f);
        }
        return;
    }
    // one piece of a split variable: the last piece to finish (over all
    // workgroups) writes the variable
    const int32_t x = it.x;
    const uint64_t dx = D.get(x);
    const uint64_t fail = dx != 0 ? revise<ALL>(N, D, it.z, it.w) : 0ull;
    if (lane == 0) {
        uint64_t *acc = L.ws.failacc + off + x;
        int32_t *cnt = L.ws.xcnt + off + x;
        if (fail) (void)__hip_atomic_fetch_or(acc, fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_stores();
        const int32_t arrived = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == pieces - 1) {
            const uint64_t ftot = __hip_atomic_exchange(acc, (uint64_t)0, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            st_rlx(cnt, 0);
            update_var(N, dnext, chg_next, x, dx, ftot, f);
        }
    }
}

// Lane 0, after the wave finished an item of lane `lane` of step k and its
// stores were performed.
DEV void complete_item(const Launch &L, const NetDesc &N, int p, int k, int lane,
                       const ItemFlags &f) {
    Ctrl *C = L.ws.ctrl + p;
    Lane *lanes = L.ws.lanes + (int64_t)p * L.lanes_per_prob;
    if (f.changed) {
        (void)__hip_atomic_fetch_max(&C->last_change, (int32_t)k, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        (void)__hip_atomic_fetch_add(&C->degsum[k & 1], f.degsum, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    }
    if (f.wiped)
        (void)__hip_atomic_fetch_or(&C->wiped, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wait_stores();
    const int32_t lane_done = __hip_atomic_fetch_add(&lanes[lane].finish, 1, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
    if (lane_done != lanes[lane].count - 1) return;
    const int32_t nl = C->nlanes;
    const int32_t all_done = __hip_atomic_fetch_add(&C->lanes_done, 1, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    if (all_done != nl - 1) return;

    // last item of step k: finalise the step (Algorithm 1's loop test)
    const bool changed = ld_rlx(&C->last_change) == k;
    const bool wiped = ld_rlx(&C->wiped) != 0;
    const int32_t maxs = L.max_sweeps > 0 ? L.max_sweeps : N.n * N.d + 1;
    const bool stop_on_wipe = (L.mode == RAC_STOP_ON_WIPEOUT) && wiped;
    if (changed && !stop_on_wipe && k < maxs) {
        const unsigned long long ds = __hip_atomic_exchange(
            &C->degsum[k & 1], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st_rlx(&C->checks, ld_rlx(&C->checks) + (long long)ds * N.d * N.d);
        for (int32_t l = 0; l < nl; ++l) st_rlx(&lanes[l].finish, 0);
        st_rlx(&C->lanes_done, 0);
        wait_stores();
        for (int32_t l = 0; l < nl; ++l) st_rlx(&lanes[l].ticket, (unsigned long long)(k + 1) << 32);
    } else {
        st_rlx(&C->iters, (int32_t)k);
        st_rlx(&C->status, wiped ? (int32_t)RAC_WIPEOUT : (int32_t)RAC_CONSISTENT);
        st_rlx(&C->rc, (changed && !stop_on_wipe) ? (int32_t)RAC_ENOTCONVERGED : 0);
        wait_stores();
        st_rlx(&C->done, 1);
        (void)__hip_atomic_fetch_add(&L.ws.global->active, -1, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Claim an item (whole wave). 1 = claimed, 0 = nothing claimable now,
// -1 = leave. Every (problem, lane) pair is a slot. The wave first tries its
// cursor slot alone, then probes 64 slots at once and claims from the first
// slot with items left. The result is the same in every lane.
DEV int probe_slots(const Launch &L, int64_t first, int32_t width, int64_t nslots,
                    int64_t &cursor, int &p_out, int &k_out, int &c_out, int &lane_out) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t lpp = L.lanes_per_prob;
    int64_t slot = first + lane;
    while (slot >= nslots) slot -= nslots;
    bool cand = false;
    int32_t cnt = 0, start = 0;
    if (lane < width) {
        const int32_t p = (int32_t)(slot / lpp);
        const int32_t l = (int32_t)(slot - (int64_t)p * lpp);
        if (l < L.ws.ctrl[p].nlanes) {
            Lane *ln = L.ws.lanes + slot;
            cnt = ln->count;
            start = ln->start;
            cand = (int32_t)(ld_rlx(&ln->ticket) & 0xFFFFFFFFull) < cnt;
        }
    }
    uint64_t m = __ballot(cand);
    while (m) {
        const int src = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        unsigned long long tk = 0;
        if (lane == src)
            tk = __hip_atomic_fetch_add(&L.ws.lanes[slot].ticket, 1ull, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        tk = __shfl(tk, src, kWave);
        const int32_t c = (int32_t)(tk & 0xFFFFFFFFull);
        if (c < __shfl(cnt, src, kWave)) {
            const int64_t sslot = __shfl(slot, src, kWave);
            cursor = sslot;
            p_out = (int32_t)(sslot / lpp);
            lane_out = (int32_t)(sslot - (int64_t)p_out * lpp);
            k_out = (int32_t)(tk >> 32);
            c_out = __shfl(start, src, kWave) + c;
            return 1;
        }
    }
    return 0;
}

DEV int try_claim(const Launch &L, int64_t &cursor, int &p_out, int &k_out, int &c_out,
                  int &lane_out, int spins) {
    Global *G = L.ws.global;
    if (ld_rlx(&G->error) != 0) return -1;
    if (ld_rlx(&G->active) <= 0) return -1;
    const int64_t nslots = (int64_t)L.nprob * L.lanes_per_prob;
    if (probe_slots(L, cursor, 1, nslots, cursor, p_out, k_out, c_out, lane_out)) return 1;
    // While its own problem is still running, an idle wave mostly re-probes
    // its own lane (the next step's tickets appear on every lane at once) and
    // scans the other slots only every fourth poll, which keeps the polling
    // traffic on the ticket lines low.
    const int32_t cp = (int32_t)(cursor / L.lanes_per_prob);
    if (spins > 0 && (spins & 3) != 3 && ld_rlx(&L.ws.ctrl[cp].done) == 0) return 0;
    for (int64_t base = 1; base <= nslots; base += kWave) {
        const int32_t width = (int32_t)((nslots - base + 1) < kWave ? (nslots - base + 1) : kWave);
        int64_t first = cursor + base;
        while (first >= nslots) first -= nslots;
        if (probe_slots(L, first, width, nslots, cursor, p_out, k_out, c_out, lane_out)) return 1;
    }
    return 0;
}

// Stage D^(k-1) (and, after step 1, the previous step's change flags) of a
// problem in LDS. Step 1 reads what the init kernel wrote: ordinary loads.
DEV void stage(uint64_t *s_dom, uint32_t *s_chg, const uint64_t *gdom, const uint32_t *gchg,
               int32_t n, bool coherent, bool flags) {
    const int lane = threadIdx.x & (kWave - 1);
    constexpr int kBatch = 8;
    for (int32_t base = 0; base < n; base += kBatch * kWave) {
        uint64_t t[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int32_t v = base + i * kWave + lane;
            t[i] = v < n ? (coherent ? ld_rlx(const_cast<uint64_t *>(gdom + v)) : gdom[v]) : 0ull;
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
                t[i] = v < n ? (coherent ? ld_rlx(const_cast<uint32_t *>(gchg + v)) : gchg[v]) : 0u;
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
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The persistent fixpoint kernel: one wave per workgroup, each an independent
// worker that claims items through the tickets. No workgroup ever waits for
// another, so the kernel is correct whether or not all of its workgroups are
// resident at once.
__global__ __launch_bounds__(kWave) void sweep_kernel(Launch L) {
    extern __shared__ uint64_t s_stage[];
    uint64_t *s_dom = s_stage;
    uint32_t *s_chg = reinterpret_cast<uint32_t *>(s_stage + L.stage_vars);
    const int lane = threadIdx.x & (kWave - 1);
    int64_t cursor = (int64_t)(blockIdx.x % (unsigned)((int64_t)L.nprob * L.lanes_per_prob));
    int spins = 0;
    int staged_p = -1, staged_k = -1;
    for (;;) {
        int p = 0, k = 0, c = 0, ln = 0;
        const int r = try_claim(L, cursor, p, k, c, ln, spins);
        if (r < 0) return;
        if (r == 0) {
            if (++spins > L.spin_limit) {
                if (lane == 0)
                    (void)__hip_atomic_fetch_or(&L.ws.global->error, 1, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            __builtin_amdgcn_s_sleep(32);
            continue;
        }
        spins = 0;
        const NetDesc &N = L.nets[L.prob_net[p]];
        const int64_t off = L.prob_off[p];
        const int4 it = N.items[c];
        const int32_t pieces = N.pieces[c];
        const bool all = (k == 1) && (L.changed0 == nullptr);
        const uint64_t *gdom = L.ws.dom[(k - 1) & 1] + off;
        const uint32_t *gchg = L.ws.chg[(k - 1) & 1] + off;
        ItemFlags fl{0, 0, 0ull};
        if (N.n <= L.stage_vars) {
            if (p != staged_p || k != staged_k) {
                stage(s_dom, s_chg, gdom, gchg, N.n, k > 1, !all);
                staged_p = p;
                staged_k = k;
            }
            const DomView<VIEW_LDS> D{s_dom, s_chg};
            if (all) process_item<true>(L, N, D, k, it, pieces, off, fl);
            else process_item<false>(L, N, D, k, it, pieces, off, fl);
        } else if (k == 1) {
            const DomView<VIEW_PLAIN> D{gdom, gchg};
            if (all) process_item<true>(L, N, D, k, it, pieces, off, fl);
            else process_item<false>(L, N, D, k, it, pieces, off, fl);
        } else {
            const DomView<VIEW_COHERENT> D{gdom, gchg};
            process_item<false>(L, N, D, k, it, pieces, off, fl);
        }
        wait_stores();
        if (lane == 0) complete_item(L, N, p, k, ln, fl);
    }
}

// ---------------------------------------------------------------------------
// Set-up and result kernels
// ---------------------------------------------------------------------------

DEV int prob_of_var(const Launch &L, int64_t v) {
    int lo = 0, hi = L.nprob - 1;   // largest p with prob_off[p] <= v
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.prob_off[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void init_kernel(Launch L) {
    const int64_t nv = L.prob_off[L.nprob];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < nv; v += nthreads) {
        L.ws.dom[0][v] = L.din[v];
        L.ws.chg[0][v] = L.changed0 ? (uint32_t)(L.changed0[v] != 0) : 1u;
        L.ws.chg[1][v] = 0;
        L.ws.failacc[v] = 0;
        L.ws.xcnt[v] = 0;
    }
    for (int64_t p = tid; p < L.nprob; p += nthreads) {
        const NetDesc &N = L.nets[L.prob_net[p]];
        Ctrl *C = L.ws.ctrl + p;
        const int32_t nl = N.nitems < L.lanes_per_prob ? N.nitems : L.lanes_per_prob;
        C->degsum[0] = 0;
        C->degsum[1] = 0;
        C->checks = (L.changed0 && L.checks1 >= 0) ? L.checks1 : (long long)N.arcs * N.d * N.d;
        C->lanes_done = 0;
        C->nlanes = nl;
        C->last_change = 0;
        C->wiped = 0;
        C->done = 0;
        C->iters = 0;
        C->status = 0;
        C->rc = 0;
        Lane *lanes = L.ws.lanes + p * L.lanes_per_prob;
        for (int32_t l = 0; l < L.lanes_per_prob; ++l) {
            const int32_t st = l < nl ? (int32_t)((int64_t)N.nitems * l / nl) : 0;
            const int32_t en = l < nl ? (int32_t)((int64_t)N.nitems * (l + 1) / nl) : 0;
            lanes[l].ticket = 1ull << 32;
            lanes[l].finish = 0;
            lanes[l].start = st;
            lanes[l].count = en - st;
        }
    }
    if (tid == 0) {
        L.ws.global->active = L.nprob;
        L.ws.global->error = 0;
        if (L.rc_out) *L.rc_out = 0;
    }
}

__global__ void finish_kernel(Launch L) {
    const int64_t nv = L.prob_off[L.nprob];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < nv; v += nthreads) {
        const int p = prob_of_var(L, v);
        const int32_t k = L.ws.ctrl[p].iters;
        L.dout[v] = L.ws.dom[k & 1][v];
    }
    for (int64_t p = tid; p < L.nprob; p += nthreads) {
        const Ctrl &C = L.ws.ctrl[p];
        if (L.iters_out) L.iters_out[p] = C.iters;
        if (L.status_out) L.status_out[p] = C.status;
        if (L.checks_out) L.checks_out[p] = C.checks;
        if (C.rc != 0 && L.rc_out) atomicOr(L.rc_out, 1);
        if (!C.done && L.rc_out) atomicOr(L.rc_out, 2);
    }
    if (tid == 0 && L.ws.global->error != 0 && L.rc_out) atomicOr(L.rc_out, 2);
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
