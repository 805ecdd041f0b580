// Batched-state path: support counts of many domain states of one network as
// int8 x int8 -> int32 matrix-core products (gfx950 MFMA).
#pragma once

#include <vector>

#include "rac.h"
#include "rac_internal.h"

namespace rac {

struct MfmaData {
    bool ready = false;
    int32_t n = 0, d = 0;
    int64_t arcs = 0;
    void *impl = nullptr;   // device buffers and events (mfma.hip)
};

// Whether the autotuner sends B states of a network with domain size d to the
// matrix-core path rather than the bit-row path.
bool mfma_auto_choice(int32_t d, int32_t n, int64_t arcs, int32_t B);

int mfma_ensure(MfmaData &md, int32_t n, int32_t d, int64_t arcs, const int32_t *row_ptr,
                const int32_t *nbr, const int32_t *deg, const uint64_t *rel,
                const int32_t *arc_src, const std::vector<int32_t> &h_row_ptr,
                hipStream_t stream);
// Enqueues the init kernel and matrix-core steps for B states (device input
// d_in [B][n]; the final domains of the states that stop go to d_out [B][n]).
// Stops when every state has stopped, at the step cap, or when at most
// `handoff` states remain active (0: never hand off). *k_out is the last step
// run, *p_out the number of states left for the caller to finish with
// mfma_handoff / (another path) / mfma_merge. Waits on the device only to read
// the active-state count between steps.
int mfma_start(MfmaData &md, int32_t B, const uint64_t *d_in, uint64_t *d_out, int32_t mode,
               int32_t max_sweeps, int32_t profile, int32_t handoff, hipStream_t stream,
               int32_t *k_out, int32_t *p_out);
// Writes the P remaining states as bit masks [P][n] and their step-k change
// flags [P][n] (the @changed set to continue from).
int mfma_handoff(MfmaData &md, int32_t k, uint64_t *d_bits, uint8_t *d_changed, hipStream_t stream);
// Takes back their results (the domains go to d_out): domains [P][n], steps
// run after step k, status,
// support checks of those steps, and the other path's return flags.
int mfma_merge(MfmaData &md, int32_t k, const uint64_t *d_bits, const int32_t *d_it,
               const int32_t *d_st, const long long *d_chk, const int32_t *d_rc,
               hipStream_t stream);
// Writes every state's step count and status (the domains are in d_out).
int mfma_finish(MfmaData &md, int32_t *d_iters, int32_t *d_status, hipStream_t stream);
// Waits for the last call and fills the counters; returns its error code.
int mfma_collect(MfmaData &md, rac_stats *stats);
void mfma_release(MfmaData &md);

}  // namespace rac
