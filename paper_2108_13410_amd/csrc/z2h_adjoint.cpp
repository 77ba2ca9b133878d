// Adjoint gradient of the final energy with respect to the per-step
// schedule values (reverse evolution with the inverse passes).
#include "z2h_runtime.h"

using namespace z2h;
using namespace z2h::rt;

extern "C" {
z2h_status z2h_adjoint(const z2h_plan *, const void *, void *, size_t, const z2h_schedule *,
                       const z2h_couplings *, double *, double *, double *, void *) {
    return fail(Z2H_ERR_UNSUPPORTED, "adjoint not available yet");
}
}
