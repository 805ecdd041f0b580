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
int mfma_enforce_host(MfmaData &md, int32_t B, uint64_t *dom, int32_t *iters, int32_t *status,
                      int32_t mode, int32_t max_sweeps, int32_t profile, hipStream_t stream,
                      rac_stats *stats);
int mfma_enforce_device(MfmaData &md, int32_t B, const uint64_t *d_in, uint64_t *d_out,
                        int32_t *d_iters, int32_t *d_status, int32_t mode, int32_t max_sweeps,
                        int32_t profile, hipStream_t stream);
int mfma_sync_status(MfmaData &md, rac_stats *stats);
void mfma_release(MfmaData &md);

}  // namespace rac
