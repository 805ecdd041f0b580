/*
 * rac.h — Recurrent Arc Consistency (RAC) enforcement on AMD Instinct MI355X
 * (gfx950). C ABI.
 *
 * The operation (Section 3 of the paper): given a binary CSP — variables
 * x = 0..n-1 with values 0..d-1, current domains D = {(x,a)}, and binary
 * constraints c_xy with allowed-pair relations rel(c_xy) (Section 2) —
 * compute the arc-consistency closure D_ac, the union of all arc-consistent
 * subsets of D. It is computed by the recurrence of Eq. (1): in every step,
 * every value (x,a) that has, on some constraint c_xy, no allowed partner b
 * left in the current dom(y) is removed, all at once; steps repeat until one
 * removes nothing (Proposition 1). After the first step only constraints into
 * variables whose domain changed in the previous step are re-examined
 * (Proposition 2; Algorithm 1's @changed). On a GPU each step is one pass over
 * the relation rows; per-problem change and wipe-out words stay on the
 * device, and the host enqueues steps in rounds of 4, 8, 16, ... (captured
 * HIP graphs), reading one counter per round instead of one per step.
 *
 * Conventions shared by every entry point
 *   Domains    uint64 per variable: bit a is set iff a is in dom(x). Bits >= d
 *              must be zero (RAC_EINVAL). 1 <= d <= 64.
 *   Edges      int32 [m][2]; edge e constrains x = edges[2e] and
 *              y = edges[2e+1]; x != y; at most one constraint per unordered
 *              pair (a duplicate, including (y,x) after (x,y), is RAC_EINVAL).
 *              Edge (x,y) with relation R yields the arc x->y with R and the
 *              arc y->x with R transposed.
 *   Result     dom is replaced by the closure; iters is the number of steps
 *              executed, the last of which removed nothing (1 if D was
 *              already arc consistent); status is RAC_WIPEOUT iff some domain
 *              is empty at the end. A wipe-out is a result, not an error: the
 *              paper's enforcer throws / returns None there (Algorithm 1).
 *   Modes      RAC_RUN_TO_FIXPOINT (default) keeps stepping after a wipe-out,
 *              so dom is always the closure D_ac; RAC_STOP_ON_WIPEOUT stops
 *              after the first step that leaves a domain empty, as Algorithm 1
 *              does, and returns the state after that step.
 *   Ownership  create copies every input; the caller keeps its arrays. A net
 *              owns its device memory until rac_destroy. Host-pointer entry
 *              points are synchronous. Device-pointer entry points enqueue on
 *              the given HIP stream and return; their buffers must stay valid
 *              until the stream reaches the end of the call. Calls on one net
 *              (or group) must not overlap in time.
 *   Errors     negative return codes; on error, outputs are unspecified.
 *              rac_strerror() names a code; rac_last_error() gives a message
 *              for the calling thread's last failure.
 */
#ifndef RAC_H
#define RAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rac_net rac_net;
typedef struct rac_group rac_group;

enum {
    RAC_OK = 0,
    RAC_EINVAL = -1,          /* bad argument, layout or value */
    RAC_ENOMEM = -2,          /* host or device allocation failed */
    RAC_EHIP = -3,            /* a HIP runtime call failed */
    RAC_EUNSUPPORTED = -4,    /* valid input outside what a path supports */
    RAC_ENOTCONVERGED = -5,   /* max_sweeps reached while values were still being removed */
    RAC_ENODEV = -6,          /* no usable gfx950 device */
    RAC_ETIMEOUT = -7         /* the batched matrix-core path ended with a state that had
                                 neither stopped nor been handed to the bit-row path (an
                                 internal failure: no valid input produces it) */
};

enum { RAC_CONSISTENT = 0, RAC_WIPEOUT = 1 };
enum { RAC_RUN_TO_FIXPOINT = 0, RAC_STOP_ON_WIPEOUT = 1 };

/* Which kernels compute the support tests. */
enum {
    RAC_PATH_AUTO = 0,   /* the autotuner chooses per call */
    RAC_PATH_BITS = 1,   /* relation rows as bit masks; support = (row & dom(y)) != 0 */
    RAC_PATH_INT8 = 2,   /* relation as 0/1 int8 blocks; support count = int32 dot product */
    RAC_PATH_MFMA = 3,   /* batched states: int8 x int8 -> int32 matrix-core products */
    RAC_PATH_FUSED = 4   /* bit rows; one workgroup per state runs every step in one launch,
                            domains in LDS (n <= 2048; else RAC_EUNSUPPORTED at the call) */
};

typedef struct rac_options {
    int32_t mode;         /* RAC_RUN_TO_FIXPOINT or RAC_STOP_ON_WIPEOUT */
    int32_t max_sweeps;   /* 0: n*d + 1, the bound of Proposition 1 */
    int32_t path;         /* RAC_PATH_* */
    int32_t use_graph;    /* 1 (default): replay captured HIP graphs; 0: direct launches */
    int32_t item_bytes;   /* 0: autotuned; else target relation bytes per work item */
    int32_t profile;      /* 1: time every launch of the dominant kernel with HIP events
                             (rac_stats.kernel_ms / kernel_launches); 0 (default): off */
    int32_t tune;         /* with path RAC_PATH_AUTO and item_bytes 0, how the path and work-item
                             size are chosen: 0 (default) the autotuner's table for the call's
                             shape, measured on the call's own inputs the first time a shape is
                             seen (the environment variable RAC_TUNE=rules or =measure overrides
                             this default); 1: fixed rules, no measurement; 2: measure again.
                             A call with max_sweeps > 0 is never measured: it uses the table
                             entry when there is one, else the fixed rules */
    int32_t reserved;     /* must be zero */
} rac_options;

/* Per-call counters of the last enforcement on a net or group. */
typedef struct rac_stats {
    int64_t support_checks;  /* sum over steps and states of d*d per re-examined arc
                                (arcs x->y with y changed in the previous step) */
    int64_t sweeps;          /* sum over states of the steps executed */
    int64_t relation_bytes;  /* relation bytes the kernels were asked to stream */
    double device_ms;        /* device time of the enforcement kernels (HIP events) */
    double kernel_ms;        /* with options.profile: summed duration of the dominant
                                kernel's launches that had work (the revise kernel of each
                                executed step, or the matrix-core step kernel) */
    int64_t kernel_launches; /* with options.profile: number of those launches */
    int64_t algo_ops;        /* algorithmic int8 operations of the matrix-core step kernel:
                                2*d*d per (arc, active state, step); 0 on other paths */
    int32_t path;            /* RAC_PATH_* actually used */
    int32_t item_bytes;      /* work-item size used by the bit / int8 path */
    float first_kernel_ms;   /* with options.profile: duration of the dominant kernel's
                                launch of step 1 (every arc of every state re-examined) */
    int32_t tune_source;     /* where the call's path and item size came from: 0 fixed rules
                                or the caller's options, 1 the table shipped with the library,
                                2 the user's table file, 3 measured by this call */
} rac_stats;

/* Fills *opt with the defaults. */
void rac_default_options(rac_options *opt);

/*
 * Creates a network from 0/1 bytes: rel is [m][d][d], rel[e][a][b] = 1 iff
 * (x_e = a, y_e = b) is allowed (any nonzero byte counts as 1). The relation
 * tensor of the paper (Algorithm 2, init) restricted to its constrained pairs.
 * opt may be NULL (defaults). On success *out receives the net.
 */
int rac_create(int32_t n, int32_t d, int64_t m, const int32_t *edges, const uint8_t *rel,
               const rac_options *opt, rac_net **out);

/*
 * Same, with each relation row packed: rel_rows is [m][d] uint64, bit b of
 * rel_rows[e][a] = 1 iff (x_e = a, y_e = b) is allowed. Bits >= d must be 0.
 */
int rac_create_bits(int32_t n, int32_t d, int64_t m, const int32_t *edges,
                    const uint64_t *rel_rows, const rac_options *opt, rac_net **out);

/*
 * Same, from the dense relation tensor R[x][a][y][b] (uint8, n*d*n*d bytes,
 * the Cons tensor of Algorithm 2 in [x,a,y,b] order) plus the edge list that
 * says which pairs are constrained. Blocks of unconstrained pairs are never
 * read. The block R[y,.,x,.] must equal the transpose of R[x,.,y,.] for every
 * edge (RAC_EINVAL otherwise).
 */
int rac_create_dense(int32_t n, int32_t d, const uint8_t *R, int64_t m, const int32_t *edges,
                     const rac_options *opt, rac_net **out);

void rac_destroy(rac_net *net);

/*
 * Enforces arc consistency on one domain state (tensorAC of Algorithm 1).
 * dom: [n] host uint64, in/out. changed: NULL = every variable changed (the
 * first call); else n_changed variable indices forming the initial @changed
 * set, with the precondition that D without those variables' reductions was
 * already arc consistent (Proposition 2) — the caller's promise, not checked.
 * iters, status: host int32, may be NULL.
 */
int rac_enforce(rac_net *net, uint64_t *dom, const int32_t *changed, int32_t n_changed,
                int32_t *iters, int32_t *status);

/*
 * Enforces arc consistency on B independent domain states of one network
 * (e.g. search nodes under different partial assignments). dom: [B][n] host
 * uint64, in/out; iters, status: [B] host int32 (may be NULL). Every state
 * starts with @changed = all variables.
 */
int rac_enforce_batch(rac_net *net, int32_t B, uint64_t *dom, int32_t *iters, int32_t *status);

/*
 * Device-pointer form of rac_enforce_batch: d_dom_in [B][n] and d_dom_out
 * [B][n] uint64 (may be the same buffer), d_iters and d_status [B] int32, all
 * in device memory of the net's device; enqueued on `stream` (a hipStream_t,
 * NULL = the null stream). The host may wait on the stream while the call
 * runs (between rounds of steps, to read how many states are still running);
 * the call returns once the last kernels are enqueued. Errors detected on the
 * device (max_sweeps reached) are reported by rac_sync_status(), or by the
 * next call on the net: every other entry point on the net first waits for a
 * device-pointer call still in flight, since it shares the net's workspace.
 */
int rac_enforce_batch_device(rac_net *net, int32_t B, const uint64_t *d_dom_in,
                             uint64_t *d_dom_out, int32_t *d_iters, int32_t *d_status,
                             void *stream);

/* Waits for the net's last device-pointer call (the end of its work on the
 * caller's stream, not the whole device) and returns its error code. */
int rac_sync_status(rac_net *net);

/*
 * For callers that cannot allocate device memory during the call (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid it):
 * rac_enforce_batch_device on the bit-row path with every workspace buffer in
 * one fixed 64 MiB device array of the library instead of memory allocated
 * for the net. Arguments as for rac_enforce_batch_device (device pointers of
 * the net's device; d_dom_in may equal d_dom_out; d_iters, d_status may be
 * NULL); results are equal to that entry point's. Always the bit-row path,
 * whatever options.path says. It waits on `stream` between rounds of steps
 * and at the end, so the results are complete when it returns, and it
 * returns the call's own error code (RAC_ENOTCONVERGED at max_sweeps); it
 * does not wait for, or report, an earlier device-pointer call on the net.
 * B * n is limited by the array: about 64 MiB / (40 * n + 100) states; larger
 * calls return RAC_EINVAL and do nothing. The array is per process and per
 * device and keeps the last call's contents; each call sets every part it
 * reads first. Calls from several host threads are serialised by the
 * library; work that another process or library places on the same buffers
 * would race, and none does.
 */
int rac_enforce_batch_noalloc(rac_net *net, int32_t B, const uint64_t *d_dom_in,
                              uint64_t *d_dom_out, int32_t *d_iters, int32_t *d_status,
                              void *stream);

/*
 * Many independent networks of uneven n, d and density, one domain state
 * each, enforced together: every step of every network runs in the same
 * kernels (one captured graph per round of steps). dom[i] is [n_i] host
 * uint64 for nets[i], in/out; iters, status: [k] host int32 (may be NULL).
 * Equivalent to k calls of rac_enforce, each with @changed = all.
 */
int rac_enforce_multi(int32_t k, rac_net *const *nets, uint64_t *const *dom, int32_t *iters,
                      int32_t *status);

/*
 * A group fixes a list of nets once (device descriptor tables, its own work
 * items, the autotuned choice per net and a captured graph), so repeated
 * calls avoid that set-up. rac_group_enforce has the semantics of
 * rac_enforce_multi. With opt's path automatic, item_bytes 0 and tuning not
 * set to fixed rules, the first rac_group_enforce call measures the group's
 * work-item size (the one from the group's total work and smaller ones) on
 * its own inputs and keeps the fastest; rac_group_enforce_device calls use
 * the size in effect. The nets must outlive the group; calls on the member
 * nets themselves stay valid and do not affect the group.
 */
int rac_group_create(int32_t k, rac_net *const *nets, const rac_options *opt, rac_group **out);
int rac_group_enforce(rac_group *g, uint64_t *const *dom, int32_t *iters, int32_t *status);
/* Device-pointer form: d_dom is [sum_i n_i] uint64 in device memory, the
 * states of nets[0..k-1] back to back, in/out; d_iters, d_status [k]. */
int rac_group_enforce_device(rac_group *g, uint64_t *d_dom, int32_t *d_iters,
                             int32_t *d_status, void *stream);
int rac_group_sync_status(rac_group *g);
void rac_group_destroy(rac_group *g);

/*
 * Batched MAC search (Algorithm 2: depth-first search that enforces arc
 * consistency after every assignment). The root domains `dom` ([n] host
 * uint64) are enforced first. Every open node then branches on the variable
 * with the smallest domain of size > 1 (lowest index on ties) into one child
 * per value (ascending); each child is enforced with @changed = {that
 * variable} (Proposition 2: its parent was arc consistent). A child whose
 * enforcement empties a domain is a failure; one whose domains are all
 * singletons is a solution (an arc-consistent state of singletons satisfies
 * every constraint); the others stay open. Up to `batch` open nodes (0: 256)
 * are taken from the top of a LIFO stack per round and all their children
 * are enforced together on the device.
 *   max_solutions, max_nodes: stop once that many solutions were found or
 *     nodes enforced (0: no limit); the round in progress completes.
 *   solution: [n] host uint64 or NULL; receives the lexicographically
 *     smallest solution found (value of variable 0 first), if any.
 * With no limit hit (out->complete = 1) the explored tree, the counts and the
 * returned solution do not depend on `batch`. Domains and relations as for
 * rac_enforce. The children are enforced on the fused path (RAC_PATH_FUSED,
 * or RAC_PATH_AUTO when a state's bit rows take at most 2 MiB), where the
 * rounds run from the device and the host reads their counts once per batch
 * of up to 8 rounds; else on the net's bit-row path (int8 if that is the
 * net's path), one host read per round. Limits are checked before each round
 * either way.
 */
typedef struct rac_search_result {
    int64_t solutions;   /* solutions found */
    int64_t nodes;       /* nodes enforced: the root and every child */
    int64_t failures;    /* enforced nodes that wiped out */
    int64_t rounds;      /* batched rounds (device enforcement calls after the root) */
    int64_t sweeps;      /* recurrence steps of all enforced nodes (Table 1's #Recurrence
                            summed; each child stops at its first wipe-out) */
    int32_t complete;    /* 1: the whole tree was explored */
    int32_t reserved;
    double search_ms;    /* wall-clock time of the call */
} rac_search_result;

int rac_search(rac_net *net, const uint64_t *dom, int64_t max_solutions, int64_t max_nodes,
               int32_t batch, uint64_t *solution, rac_search_result *out);

/* Counters of the last call on a net / group (host-pointer calls, or after a
 * rac_sync_status / rac_group_sync_status). */
int rac_net_stats(const rac_net *net, rac_stats *out);
int rac_group_stats(const rac_group *g, rac_stats *out);

/* Sizes of a net (any pointer may be NULL). */
int rac_net_info(const rac_net *net, int32_t *n, int32_t *d, int64_t *m, int64_t *arcs);

const char *rac_strerror(int code);
const char *rac_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RAC_H */
