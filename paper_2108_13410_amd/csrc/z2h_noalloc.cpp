// z2h_evolve without a workspace argument and without any allocation, for
// callers that cannot allocate device memory (code under graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The scratch that z2h_evolve takes from the caller's workspace (the z
// passes' per-tile norm partials and, for per-step schedules, the device
// copies of sZ/sX) lives here in one file-scope device array.  Each device
// holds its own copy of the array for the life of the process; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device, looked up once per device and kept.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "z2h_runtime.h"

using namespace z2h;
using namespace z2h::rt;

namespace {

constexpr size_t kScratchBytes = Z2H_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size is a multiple of 256 bytes");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];

// Device address of this device's scratch array (looked up once per device).
z2h_status scratch_ptr(void **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(Z2H_ERR_UNSUPPORTED, "device index %d", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(Z2H_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return Z2H_OK;
}

// Scratch bytes a call needs: z2h_evolve's workspace figure.
// z2h_evolve's workspace without its phase-table chunk: here every
// workgroup builds its own table (the fixed array stays small).
size_t scratch_need(const Plan &P, const z2h_schedule *sched) {
    size_t need = ws_evolve_size(P) - ws_tables_size(P);
    if (sched->sZ || sched->sX) need += align256(sizeof(double) * 2 * (size_t)std::max<int64_t>(sched->steps, 0)) + 256;
    return need;
}

}  // namespace

extern "C" {

z2h_status z2h_evolve_noalloc(const z2h_plan *plan, void *d_state, const z2h_schedule *sched, double *d_norms,
                              void *stream) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        const Plan &P = plan->P;
        z2h_status st = validate_state_ptr(d_state, "d_state");
        if (st) return st;
        if ((st = validate_schedule(P, sched))) return st;
        const size_t need = scratch_need(P, sched);
        if (need > kScratchBytes)
            return fail(Z2H_ERR_UNSUPPORTED, "scratch of %zu bytes needed, the fixed array holds %zu", need,
                        kScratchBytes);
        const bool arrays = sched->sZ || sched->sX;
        if (arrays) {
            for (int64_t k = 0; k < sched->steps; ++k) {
                if ((sched->sZ && !std::isfinite(sched->sZ[k])) || (sched->sX && !std::isfinite(sched->sX[k])))
                    return fail(Z2H_ERR_INVALID, "schedule value at step %lld not finite", (long long)k);
            }
        }
        if ((st = check_device_(P))) return st;
        void *base = nullptr;
        if ((st = scratch_ptr(&base))) return st;
        hipStream_t s = (hipStream_t)stream;
        // Same carve-up as z2h_evolve's workspace, over the fixed array.
        // Nothing needs clearing: the norm partials are written by a z pass
        // before the next pass reads them, and the schedule copies are
        // written before the first pass.
        Carver c{(char *)base, 0};
        JobSet J;
        memset(&J, 0, sizeof J);
        J.inl = make_job(sched, 0);
        J.inl.norm_part = (double *)c.take(sizeof(double) * norm_parts(P));
        J.inl.norm_trace = d_norms;
        if (arrays) {
            double *dz = (double *)c.take(sizeof(double) * sched->steps);
            double *dx = (double *)c.take(sizeof(double) * sched->steps);
            if (sched->sZ) HIP_TRY(hipMemcpyAsync(dz, sched->sZ, sizeof(double) * sched->steps, hipMemcpyHostToDevice, s));
            if (sched->sX) HIP_TRY(hipMemcpyAsync(dx, sched->sX, sizeof(double) * sched->steps, hipMemcpyHostToDevice, s));
            // the host arrays may be reused as soon as this call returns
            HIP_TRY(hipStreamSynchronize(s));
            J.inl.sZ = sched->sZ ? dz : nullptr;
            J.inl.sX = sched->sX ? dx : nullptr;
        }
        J.h_jobs = &J.inl;
        J.njobs = 1;
        return run_levels(P, d_state, J, s);
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_evolve_noalloc");
    }
}

}  // extern "C"
