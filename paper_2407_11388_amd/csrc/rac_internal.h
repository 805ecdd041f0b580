// Internal types shared by the host code and the gfx950 kernels of librac.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rac {

constexpr int kWave = 64;                  // CDNA wavefront width
constexpr int kStageMax = 2048;            // networks up to this many variables are staged in LDS

// How the relation rows of a network are stored for one path.
//
// Bit rows (ROW32 / ROW64): the arcs of each variable are padded to a
// multiple of 64 and stored in groups of 64 arcs. Within a group, the rows of
// one arc are cut into 16-byte quads (4 uint32 rows or 2 uint64 rows), and
// quad q of the 64 arcs is stored contiguously: quad q of arc l of group g is
// at byte g*qpa*1024 + q*1024 + l*16. A wave reads one group with lane = arc,
// each of its loads covering 1 KiB of consecutive memory.
//
// int8 rows (ROWI8): arcs unpadded, arc j holds d rows of dp bytes (0/1).
enum RowKind : int32_t {
    ROW32 = 0,  // uint32 rows (d <= 32); dp = d rounded up to 4 rows; qpa = dp/4
    ROW64 = 1,  // uint64 rows (d <= 64); dp = d rounded up to 8 rows; qpa = dp/2
    ROWI8 = 2   // 0/1 int8 rows (d <= 32); dp = bytes per row = d rounded up to 16
};

constexpr int kGroup = 64;        // arcs per group of the bit-row layout

// Bit-row work items hold at most kItemVars whole variables (one per lane when
// the item's variables are updated). Steps that re-examine only the arcs into
// changed variables look at kSparseGroups groups at a time.
constexpr int kItemVars = 64;
constexpr int kSparseGroups = 16;
// Per-wave LDS scratch in front of the staged domains, in 8-byte words: the
// failing values of the item's variables (kItemVars words) and the compacted
// active arcs of a sparse batch (kSparseGroups * 64 16-bit codes).
constexpr int kScratchWords = kItemVars + kSparseGroups * kGroup / 4;
// States per task of revise_shared_kernel (each task reads one group's rows once).
constexpr int kSharedStates = 16;

// Small problems in one launch (small_fixpoint_kernel): at most kSmallMaxN
// variables, one workgroup of up to kSmallMaxThreads per problem; LDS of
// 3 * 8 + 2 * 4 + 2 * 2 + 2 bytes per variable.
constexpr int kSmallMaxN = 2048;
constexpr int kSmallMaxThreads = 1024;
constexpr int kSmallWalkRatio = 4;   // walk the changed variables' arcs when at most 1/4 of all
inline size_t small_lds_bytes(int32_t n) { return (size_t)n * 38 + 16; }
// Threads of the workgroup for networks of at most `groups` 64-arc groups:
// about 4 groups per wave and step, 1 to max_waves (<= 16) waves.
inline int small_threads(int64_t groups, int max_waves) {
    int w = 1;
    while (w < max_waves && w < 16 && (int64_t)w * 4 < groups) w <<= 1;
    return w * 64;
}

// One network as seen by the sweep kernel (device memory, read-only).
// Arcs leaving x: row_ptr[x] .. row_ptr[x+1]-1 (to nbr[j]); in the padded
// group layout, groups gptr[x] .. gptr[x+1]-1 with nbrp[g*64 + l] the
// neighbour of arc l of group g, or -1 for padding.
struct NetDesc {
    const int32_t *row_ptr;   // [n+1]
    const int32_t *nbr;       // [arcs]
    const int32_t *gptr;      // [n+1] group offsets (bit rows)
    const int32_t *nbrp;      // [groups*64] (bit rows)
    const int32_t *gown;      // [groups] the variable group g belongs to (bit rows)
    const int32_t *rpos;      // [arcs] for arc j (y -> x in CSR order): the position g*64 + l
                              // of the reverse arc x -> y in the group layout (bit rows),
                              // or null (int8 rows)
    const int32_t *deg;       // [n]
    const void *rows;
    const int4 *items;        // [nitems] {x_begin, x_end, unit_begin, unit_end}; units are
                              // groups for bit rows, arcs for int8 rows
    const int32_t *pieces;    // [nitems] 0: whole variables; k >= 1: one piece of x split in k
    const int4 *items_inc;    // [nitems_inc] the items of steps that re-examine only the arcs
    const int32_t *pieces_inc;// into changed variables (may be finer; else the same table)
    int32_t nitems_inc;
    int32_t n, d, dp, kind;
    int32_t nitems, qpa;
    int32_t pchunks;          // pieces of 64 arcs of the largest degree (bit rows)
    int64_t arcs;
};

// Control words of one problem (one domain state of one network).
struct Ctrl {
    long long arcs[3];      // arcs[k % 3]: arcs into variables step k changed = arcs that
                            // step k+1 re-examines (arcs[0]: those of step 1)
    long long checks;       // support checks so far (d*d per re-examined arc)
    int32_t last_change;    // last step that removed a value (0 = none)
    int32_t wipe_step;      // first step after which some domain was empty (0 = none)
    int32_t nchg[2];        // nchg[k & 1]: variables step k changed (listed in Workspace::clist)
    int32_t pad[6];         // 64 bytes
};

// The problems that execute the next step and the prefix sums of their item
// counts (written by the plan kernel).
struct Plan {
    int32_t nact;
    int32_t pad;
    int64_t items;
};

// Device workspace of a set of problems; variable v of problem p lives at off[p] + v.
struct Workspace {
    uint64_t *dom[2];     // double buffer: step k reads dom[(k-1)&1], writes dom[k&1]
    uint32_t *chg[2];     // chg[k&1][v] = 1 iff step k shrank dom(v); chg[0] starts as @changed
    uint64_t *failacc;    // values found failing in the current step (OR), cleared by the update
    Ctrl *ctrl;           // [nprob]
    Plan *plan;           // [1]
    int32_t *act;         // [nprob] problems of the next step
    int64_t *act_off;     // [nprob + 1] their item prefix sums
    int32_t *act_push;    // [nprob] 1: the listed problem's items are its changed variables
    int32_t *clist[2];    // clist[k & 1][off + i]: the i-th variable step k changed
};

// Everything one enforcement needs (passed by value to every kernel).
struct Launch {
    const NetDesc *nets;      // [nnet]
    const int32_t *prob_net;  // [nprob]
    const int64_t *prob_off;  // [nprob + 1]
    int32_t nprob;
    int32_t mode;             // RAC_RUN_TO_FIXPOINT / RAC_STOP_ON_WIPEOUT
    int32_t max_sweeps;       // 0: per network n*d + 1
    int32_t stage_vars;       // LDS staging capacity in variables (0: none)
    Workspace ws;
    const uint64_t *din;      // [prob_off[nprob]] initial domains
    uint64_t *dout;           // [prob_off[nprob]] results
    int32_t *iters_out;       // [nprob] or null
    int32_t *status_out;      // [nprob] or null
    const uint8_t *changed0;  // [prob_off[nprob]] initial @changed flags, or null (= all)
    long long *checks_out;    // [nprob] or null
    long long arcs1;          // with changed0: arcs step 1 re-examines, per problem
                              // (< 0: each problem's sum of deg over its @changed set)
    int32_t *rc_out;          // [1]: 1 if some problem reached max_sweeps unconverged
    int32_t push_ratio;       // steps k >= 2 of a bit-row problem that re-examine at most
                              // arcs / push_ratio arcs go variable by variable (0: never)
    int32_t uniform_n;        // > 0: every problem is an instance of nets[0] with uniform_n
                              // variables, prob_off[p] = p * uniform_n (else 0)
    const int32_t *nprob_dev; // non-null: the number of problems is *nprob_dev (<= nprob),
                              // read on the device when each kernel starts, so that one
                              // captured graph serves calls with different counts
    int32_t shared_rows;      // 1: every problem a state of nets[0] (uint32 rows) and the
                              // steps revise with revise_shared_kernel
    int32_t pad_;
};

// Records a message for rac_last_error() and returns `code` (rac_host.hip).
int set_error(int code, const char *fmt, ...);

// Kernel entry points (defined in sweep.hip), launched by rac_host.hip.
__global__ void init_kernel(Launch L);
__global__ void list_changed0_kernel(Launch L);
__global__ void plan_kernel(Launch L, int k);
__global__ void revise_kernel(Launch L, int k);
__global__ void revise_shared_kernel(Launch L, int k);
__global__ void update_kernel(Launch L, int k);
__global__ void finish_kernel(Launch L);
__global__ void small_fixpoint_kernel(Launch L);
__global__ void clear_word_kernel(int32_t *w);
__global__ void pack_bits_kernel(const uint64_t *rel, const int32_t *src_p, int64_t groups,
                                 int32_t d, int32_t qpa, int32_t kind, uint4 *out);
__global__ void pack_i8_kernel(const uint64_t *rel, const int32_t *arc_src, int64_t arcs,
                               int32_t d, int32_t rows_per_arc, int32_t dp, int8_t *out);

// Batched MAC search (search.hip). The control block of a search on the
// device: the stack size and the current round's nodes, and the counts so far.
struct SearchCtl {
    long long ssize;      // nodes on the stack
    long long base;       // stack index of the round's first node (ssize - P)
    long long nodes, solutions, failures, sweeps, rounds;
    int32_t P;            // nodes of the current round (0: none)
    int32_t done;         // 1: the search has ended (stack empty, limit reached, or rc)
    int32_t complete;     // 1: the stack emptied (the whole tree was explored)
    int32_t rc;           // OR of the enforcements' return flags (1: step cap reached)
};
__global__ void search_begin_kernel(SearchCtl *ctl, int32_t batch, long long max_solutions,
                                    long long max_nodes);
__global__ void search_end_kernel(SearchCtl *ctl, const long long *stats);
__global__ void search_branch_kernel(const uint64_t *stack, const SearchCtl *ctl, int32_t n,
                                     int32_t *bvar, int32_t *nchild);
__global__ void search_offsets_kernel(const int32_t *nchild, const SearchCtl *ctl, int32_t *coff,
                                      int32_t *total, int32_t *rc);
__global__ void search_expand_kernel(const uint64_t *stack, const SearchCtl *ctl, int32_t n,
                                     const int32_t *bvar, const int32_t *coff, uint64_t *cdom,
                                     uint8_t *cchg);
__global__ void search_classify_kernel(const uint64_t *cres, const int32_t *status, int32_t n,
                                       const int32_t *count, int32_t *is_sol, int32_t *is_open);
__global__ void search_lists_kernel(const int32_t *is_sol, const int32_t *is_open,
                                    const int32_t *iters, const int32_t *count, const int32_t *rc,
                                    int32_t *sol_off, int32_t *open_off, long long *stats);
__global__ void search_push_kernel(const uint64_t *cres, int32_t n, const int32_t *count,
                                   const int32_t *is_sol, const int32_t *is_open,
                                   const int32_t *sol_off, const int32_t *open_off, uint64_t *stack,
                                   const SearchCtl *ctl, int32_t *sol_list);
__global__ void search_best_kernel(const uint64_t *cres, int32_t n, const int32_t *sol_list,
                                   const int32_t *sol_off, const int32_t *count, uint64_t *best,
                                   int32_t *has_best);

}  // namespace rac
