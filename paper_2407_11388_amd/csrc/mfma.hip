// Batched-state matrix-core path (gfx950 int8 MFMA).
#include "rac_mfma.h"

namespace rac {

bool mfma_auto_choice(int32_t, int32_t, int64_t, int32_t) { return false; }

int mfma_ensure(MfmaData &, int32_t, int32_t, int64_t, const int32_t *, const int32_t *,
                const int32_t *, const uint64_t *, const int32_t *, const std::vector<int32_t> &,
                hipStream_t) {
    return set_error(RAC_EUNSUPPORTED, "matrix-core path not available");
}
int mfma_enforce_host(MfmaData &, int32_t, uint64_t *, int32_t *, int32_t *, int32_t, int32_t,
                      hipStream_t, rac_stats *) {
    return set_error(RAC_EUNSUPPORTED, "matrix-core path not available");
}
int mfma_enforce_device(MfmaData &, int32_t, const uint64_t *, uint64_t *, int32_t *, int32_t *,
                        int32_t, int32_t, hipStream_t) {
    return set_error(RAC_EUNSUPPORTED, "matrix-core path not available");
}
int mfma_sync_status(MfmaData &, rac_stats *) { return RAC_OK; }
void mfma_release(MfmaData &md) { md.ready = false; }

}  // namespace rac
