// Kernels of the batched MAC search (Algorithm 2: depth-first search that
// enforces arc consistency after every assignment). A round takes the top P
// nodes of the device stack, branches each on one variable, enforces all
// children together (@changed = the assigned variable, Proposition 2), and
// sorts the children into failures, solutions and nodes pushed back onto the
// stack. The round's sizes live in a device control block (SearchCtl): the
// begin kernel sets P and the base of the popped nodes from the stack size,
// the end kernel adds the round's counts and sets the new stack size, so that
// rounds can follow each other with no host read in between.
#include "rac.h"
#include "rac_internal.h"

namespace rac {

namespace {

__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// Exclusive prefix sums of cnt[0..N) into off[0..N], off[N] = total, by one
// workgroup of 1024 threads (16 waves), in chunks of 1024.
__device__ void block_scan(const int32_t *cnt, int32_t N, int32_t *off) {
    __shared__ int32_t s_wave[16];
    __shared__ int32_t s_base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (int32_t c0 = 0; c0 < N; c0 += 1024) {
        const int32_t i = c0 + (int32_t)threadIdx.x;
        const int32_t v = i < N ? cnt[i] : 0;
        int32_t inc = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (lane == 63) s_wave[wave] = inc;
        __syncthreads();
        int32_t before = s_base;
        for (int w = 0; w < wave; ++w) before += s_wave[w];
        if (i < N) off[i] = before + inc - v;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < 16; ++w) s_base += s_wave[w];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[N] = s_base;
}

}  // namespace

// Start of a round: the search ends when the stack is empty (complete) or a
// limit is reached (checked before each round, as the round in progress
// completes); else the round takes the top min(stack, batch) nodes.
__global__ void search_begin_kernel(SearchCtl *ctl, int32_t batch, long long max_solutions,
                                    long long max_nodes) {
    if (threadIdx.x != 0) return;
    SearchCtl &c = *ctl;
    c.P = 0;
    if (c.done) return;
    if (c.ssize == 0) {
        c.done = 1;
        c.complete = 1;
        return;
    }
    if ((max_solutions > 0 && c.solutions >= max_solutions) || (max_nodes > 0 && c.nodes >= max_nodes)) {
        c.done = 1;
        return;
    }
    c.P = (int32_t)(c.ssize < batch ? c.ssize : batch);
    c.base = c.ssize - c.P;
}

// End of a round: the counts of its C children (stats from
// search_lists_kernel) and the new stack size; an enforcement that reports
// the step cap ends the search.
__global__ void search_end_kernel(SearchCtl *ctl, const long long *stats) {
    if (threadIdx.x != 0) return;
    SearchCtl &c = *ctl;
    if (c.P == 0) return;
    const long long C = stats[4];
    c.nodes += C;
    c.sweeps += stats[0];
    c.solutions += stats[1];
    c.failures += C - stats[1] - stats[2];
    c.ssize = c.base + stats[2];
    c.rounds += 1;
    c.rc |= (int32_t)stats[3];
    if (c.rc) c.done = 1;
}

// Branching choice of node i (one wave per node): the variable with the
// smallest domain of size > 1 (lowest index on ties), and its domain size
// (the node's number of children). Nodes on the stack are arc consistent,
// not wiped out and not yet solutions, so such a variable exists.
__global__ __launch_bounds__(64) void search_branch_kernel(const uint64_t *stack,
                                                           const SearchCtl *ctl, int32_t n,
                                                           int32_t *bvar, int32_t *nchild) {
    const int32_t P = ctl->P;
    const int lane = threadIdx.x;
    for (int32_t i = blockIdx.x; i < P; i += gridDim.x) {
        const uint64_t *dom = stack + (ctl->base + i) * n;
        int best = 0x7FFFFFFF;   // (size << 20) | variable, sizes <= 64, n < 2^20
        for (int32_t x = lane; x < n; x += 64) {
            const int s = __popcll(dom[x]);
            if (s > 1) best = min(best, (s << 20) | x);
        }
        best = wave_min_int(best);
        if (lane == 0) {
            bvar[i] = best & 0xFFFFF;
            nchild[i] = best >> 20;
        }
    }
}

// Child offsets: coff[i] = children of nodes 0..i-1, coff[P] = all children,
// also stored in *total (the problem count of the round's enforcement); the
// enforcement's step-cap flag starts clear.
__global__ __launch_bounds__(1024) void search_offsets_kernel(const int32_t *nchild,
                                                              const SearchCtl *ctl, int32_t *coff,
                                                              int32_t *total, int32_t *rc) {
    const int32_t P = ctl->P;
    if (threadIdx.x == 0) *rc = 0;   // the round's enforcement ORs its step-cap flag here
    block_scan(nchild, P, coff);
    // thread 0 wrote coff[P] itself
    if (threadIdx.x == 0) *total = coff[P];
}

// Children of node i (one workgroup per node): child j takes the j-th value
// of the branching variable (ascending); its @changed set is that variable.
__global__ __launch_bounds__(256) void search_expand_kernel(const uint64_t *stack,
                                                            const SearchCtl *ctl, int32_t n,
                                                            const int32_t *bvar,
                                                            const int32_t *coff, uint64_t *cdom,
                                                            uint8_t *cchg) {
    const int32_t P = ctl->P;
    for (int32_t i = blockIdx.x; i < P; i += gridDim.x) {
        const int32_t xb = bvar[i];
        const uint64_t *dom = stack + (ctl->base + i) * n;
        const int32_t c0 = coff[i], c1 = coff[i + 1];
        uint64_t rest = dom[xb];
        for (int32_t c = c0; c < c1; ++c) {
            const uint64_t v = rest & (~rest + 1ull);   // lowest remaining value
            rest &= rest - 1ull;
            uint64_t *out = cdom + (int64_t)c * n;
            uint8_t *chg = cchg + (int64_t)c * n;
            for (int32_t x = threadIdx.x; x < n; x += blockDim.x) {
                out[x] = x == xb ? v : dom[x];
                chg[x] = x == xb ? 1 : 0;
            }
        }
    }
}

// Kind of each enforced child, as 0/1 flags for the list scans that follow:
// a solution (not wiped out, every domain a singleton) or open (not wiped
// out, some domain larger); neither means a failure. One wave per child,
// *count children (the workgroups stride over them).
__global__ __launch_bounds__(64) void search_classify_kernel(const uint64_t *cres,
                                                             const int32_t *status, int32_t n,
                                                             const int32_t *count,
                                                             int32_t *is_sol, int32_t *is_open) {
    const int32_t C = *count;
    const int lane = threadIdx.x;
    for (int32_t c = blockIdx.x; c < C; c += gridDim.x) {
        const uint64_t *dom = cres + (int64_t)c * n;
        int multi = 0;
        for (int32_t x = lane; x < n; x += 64) multi |= __popcll(dom[x]) > 1;
        multi = __any(multi) ? 1 : 0;
        if (lane == 0) {
            const bool wiped = status[c] == RAC_WIPEOUT;
            is_sol[c] = (!wiped && !multi) ? 1 : 0;
            is_open[c] = (!wiped && multi) ? 1 : 0;
        }
    }
}

// Offsets of the solution and open lists (two scans in one workgroup), and
// the round's summary for the host in one block: stats[0] = recurrence steps
// of all C = *count children, stats[1] = solutions, stats[2] = open children,
// stats[3] = the step kernels' return flags (*rc), stats[4] = C.
__global__ __launch_bounds__(1024) void search_lists_kernel(const int32_t *is_sol,
                                                            const int32_t *is_open,
                                                            const int32_t *iters,
                                                            const int32_t *count,
                                                            const int32_t *rc, int32_t *sol_off,
                                                            int32_t *open_off, long long *stats) {
    __shared__ long long s_steps;
    const int32_t C = *count;
    block_scan(is_sol, C, sol_off);
    // thread 0 wrote sol_off[C] itself
    if (threadIdx.x == 0) stats[1] = sol_off[C];
    __syncthreads();
    block_scan(is_open, C, open_off);
    if (threadIdx.x == 0) {
        stats[2] = open_off[C];
        stats[3] = *rc;
        stats[4] = C;
        s_steps = 0;
    }
    __syncthreads();
    long long t = 0;
    for (int32_t c = threadIdx.x; c < C; c += blockDim.x) t += iters[c];
    for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long *)&s_steps, (unsigned long long)t);
    __syncthreads();
    if (threadIdx.x == 0) stats[0] = s_steps;
}

// Open children go onto the stack above the round's base, the last child
// lowest, so that the first child (the smallest value of the first node)
// ends on top; solutions are listed in child order. One workgroup per child,
// C = *count children (the workgroups stride over them).
__global__ __launch_bounds__(256) void search_push_kernel(const uint64_t *cres, int32_t n,
                                                          const int32_t *count,
                                                          const int32_t *is_sol,
                                                          const int32_t *is_open,
                                                          const int32_t *sol_off,
                                                          const int32_t *open_off, uint64_t *stack,
                                                          const SearchCtl *ctl, int32_t *sol_list) {
    const int32_t C = *count;
    if (ctl->P == 0) return;
    const long long base = ctl->base;
    for (int32_t c = blockIdx.x; c < C; c += gridDim.x) {
        if (is_sol[c] && threadIdx.x == 0) sol_list[sol_off[c]] = c;
        if (!is_open[c]) continue;
        const int32_t nopen = open_off[C];
        const int64_t at = base + (nopen - 1 - open_off[c]);
        const uint64_t *src = cres + (int64_t)c * n;
        uint64_t *dst = stack + at * n;
        for (int32_t x = threadIdx.x; x < n; x += blockDim.x) dst[x] = src[x];
    }
}

namespace {

// Whether assignment a is lexicographically smaller than b (n singleton
// domains each; the first variable where they differ decides, and there the
// lower bit is the smaller value). Whole wave, uniform result.
__device__ __forceinline__ bool wave_lex_less(const uint64_t *a, const uint64_t *b, int32_t n) {
    const int lane = threadIdx.x & 63;
    for (int32_t x0 = 0; x0 < n; x0 += 64) {
        const int32_t x = x0 + lane;
        const uint64_t va = x < n ? a[x] : 0ull, vb = x < n ? b[x] : 0ull;
        const uint64_t diff = __ballot(va != vb);
        if (diff) {
            const int f = __ffsll((unsigned long long)diff) - 1;
            return __shfl((int)(va < vb), f, 64) != 0;
        }
    }
    return false;
}

}  // namespace

// The lexicographically smallest solution (value of variable 0 first, then
// 1, ...) among `best` (if has_best) and the listed solutions of the *count
// children. One workgroup
// of 16 waves: each wave keeps the smallest of every 16th listed solution,
// then wave 0 merges the wave results with `best`.
__global__ __launch_bounds__(1024) void search_best_kernel(const uint64_t *cres, int32_t n,
                                                           const int32_t *sol_list,
                                                           const int32_t *sol_off,
                                                           const int32_t *count, uint64_t *best,
                                                           int32_t *has_best) {
    __shared__ int32_t s_win[16];
    const int32_t ns = sol_off[*count];
    if (ns == 0) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int32_t win = -1;   // index into sol_list
    for (int32_t k = wave; k < ns; k += 16) {
        if (win < 0 || wave_lex_less(cres + (int64_t)sol_list[k] * n,
                                     cres + (int64_t)sol_list[win] * n, n))
            win = k;
    }
    if (lane == 0) s_win[wave] = win;
    __syncthreads();
    if (wave != 0) return;
    const bool had = *has_best != 0;
    const uint64_t *cur = had ? best : nullptr;
    for (int w = 0; w < 16; ++w) {
        const int32_t k = s_win[w];
        if (k < 0) continue;
        const uint64_t *cand = cres + (int64_t)sol_list[k] * n;
        if (!cur || wave_lex_less(cand, cur, n)) cur = cand;
    }
    if (cur && cur != best) {
        for (int32_t x = lane; x < n; x += 64) best[x] = cur[x];
        if (lane == 0) *has_best = 1;
    }
}

}  // namespace rac
