// Batched evolution and the adjoint gradient (filled in below).
#include "../../include/z2h.h"

extern "C" {
z2h_status z2h_adjoint(const z2h_plan *, const void *, void *, size_t, const z2h_schedule *,
                       const z2h_couplings *, double *, double *, double *, void *) {
    return Z2H_ERR_UNSUPPORTED;
}
z2h_status z2h_batch_create(int32_t, const int32_t *, const int32_t *, const z2h_schedule *, const z2h_init *,
                            const z2h_couplings *, z2h_dtype, z2h_batch **out, size_t *, size_t *, uint64_t *) {
    if (out) *out = nullptr;
    return Z2H_ERR_UNSUPPORTED;
}
z2h_status z2h_batch_run(z2h_batch *, void *, void *, size_t, double *, void *) { return Z2H_ERR_UNSUPPORTED; }
void z2h_batch_destroy(z2h_batch *) {}
}
