// Autotuner: times candidate pass schedules of a lattice on the device and
// keeps the fastest for later plans and batches of that lattice, precision
// and batch size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "z2h_runtime.h"

using namespace z2h;
using namespace z2h::rt;

namespace {

// Device buffers shared by every candidate of one tuning run.
struct TuneBufs {
    void *states = nullptr, *parts = nullptr, *jobs = nullptr, *inits = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneBufs() {
        if (states) (void)hipFree(states);
        if (parts) (void)hipFree(parts);
        if (jobs) (void)hipFree(jobs);
        if (inits) (void)hipFree(inits);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Milliseconds of S Trotter steps of `batch` states with plan P.
z2h_status time_steps(const Plan &P, TuneBufs &B, int batch, int S, hipStream_t s, float &ms) {
    std::vector<JobDev> h(batch);
    const size_t parts_per_job = ((size_t)1 << (P.n - 8)) + ((size_t)1 << (P.n - 18 > 0 ? P.n - 18 : 0));
    z2h_schedule sc;
    memset(&sc, 0, sizeof sc);
    sc.start = {1.0, 1.0, 0.0, 0.0};
    sc.end = {1.0, 1.0, 0.3, 0.3};
    sc.steps = S;
    sc.dt = 0.02;
    sc.k_end = S;
    sc.renorm = P.c128 ? 0 : 1;
    for (int j = 0; j < batch; ++j) {
        h[j] = make_job(&sc, (uint64_t)j << P.n);
        h[j].norm_part = (double *)B.parts + (size_t)j * parts_per_job;
    }
    HIP_TRY(hipMemcpy(B.jobs, h.data(), sizeof(JobDev) * batch, hipMemcpyHostToDevice));
    JobSet J;
    memset(&J, 0, sizeof J);
    J.d_jobs = (const JobDev *)B.jobs;
    J.h_jobs = h.data();
    J.njobs = batch;
    HIP_TRY(hipEventRecord(B.e0, s));
    z2h_status st = run_levels(P, B.states, J, s);
    if (st) return st;
    HIP_TRY(hipEventRecord(B.e1, s));
    HIP_TRY(hipEventSynchronize(B.e1));
    HIP_TRY(hipEventElapsedTime(&ms, B.e0, B.e1));
    return Z2H_OK;
}

}  // namespace

extern "C" {

z2h_status z2h_plan_create_config(int32_t Lx, int32_t Ly, z2h_dtype dtype, const char *schedule, z2h_plan **out) {
    try {
        if (!out || !schedule) return fail(Z2H_ERR_INVALID, "NULL argument");
        *out = nullptr;
        if (dtype != Z2H_C64 && dtype != Z2H_C128) return fail(Z2H_ERR_INVALID, "bad dtype %d", dtype);
        z2h_plan *p = new (std::nothrow) z2h_plan;
        if (!p) return fail(Z2H_ERR_OOM, "out of host memory");
        z2h_status st = plan_with_config(Lx, Ly, dtype == Z2H_C128, schedule, p->P);
        if (st) {
            delete p;
            return st;
        }
        p->P.device = -1;
        int ndev = 0, dev = 0;
        if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0 && hipGetDevice(&dev) == hipSuccess) p->P.device = dev;
        *out = p;
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in plan creation");
    }
}

z2h_status z2h_tune_candidates(int32_t Lx, int32_t Ly, z2h_dtype dtype, char *buf, size_t len) {
    z2h_status st = check_lattice(Lx, Ly);
    if (st) return st;
    if (!buf || !len) return fail(Z2H_ERR_INVALID, "NULL argument");
    std::string all;
    for (const auto &c : tune_candidates(Lx, Ly, dtype == Z2H_C128)) all += c + "\n";
    if (all.size() + 1 > len) return fail(Z2H_ERR_INVALID, "buffer of %zu bytes, %zu needed", len, all.size() + 1);
    memcpy(buf, all.c_str(), all.size() + 1);
    return Z2H_OK;
}

z2h_status z2h_tune_load(const char *cache_path) {
    if (!cache_path) return fail(Z2H_ERR_INVALID, "cache_path is NULL");
    return tune_load(cache_path);
}

z2h_status z2h_autotune(int32_t Lx, int32_t Ly, z2h_dtype dtype, int32_t batch, const char *cache_path,
                        char *best, size_t best_len, double *best_ms_per_step) {
    try {
        z2h_status st = check_lattice(Lx, Ly);
        if (st) return st;
        if (dtype != Z2H_C64 && dtype != Z2H_C128) return fail(Z2H_ERR_INVALID, "bad dtype %d", dtype);
        const int n = 2 * Lx * Ly;
        const bool c128 = dtype == Z2H_C128;
        const size_t esize = c128 ? 16 : 8;
        if (batch < 1 || (uint64_t)batch * (esize << n) > (96ull << 30))
            return fail(Z2H_ERR_INVALID, "batch %d out of range (states above 96 GiB)", batch);
        if (n <= 14) return fail(Z2H_ERR_UNSUPPORTED, "n = %d runs in one workgroup; nothing to tune", n);
        std::vector<std::string> cands = tune_candidates(Lx, Ly, c128);
        if (cands.empty()) return fail(Z2H_ERR_UNSUPPORTED, "no candidate schedules for n = %d", n);
        HIP_TRY(prepare_kernels());
        TuneBufs B;
        const size_t sb = (size_t)batch * (esize << n);
        if (hipMalloc(&B.states, sb) != hipSuccess) return fail(Z2H_ERR_OOM, "trial states of %zu bytes", sb);
        if (hipMalloc(&B.parts, sizeof(double) * (size_t)batch * (((size_t)1 << (n - 8)) + ((size_t)1 << (n - 18 > 0 ? n - 18 : 0)))) != hipSuccess)
            return fail(Z2H_ERR_OOM, "trial partials");
        if (hipMalloc(&B.jobs, sizeof(JobDev) * batch) != hipSuccess) return fail(Z2H_ERR_OOM, "trial jobs");
        if (hipMalloc(&B.inits, sizeof(InitJob) * batch) != hipSuccess) return fail(Z2H_ERR_OOM, "trial inits");
        HIP_TRY(hipEventCreate(&B.e0));
        HIP_TRY(hipEventCreate(&B.e1));
        hipStream_t s = nullptr;
        // |+...+> in every trial state
        {
            Plan P0;
            if ((st = make_plan(Lx, Ly, c128, 0, P0, batch))) return st;
            std::vector<InitJob> ij(batch);
            for (int j = 0; j < batch; ++j) ij[j] = init_job(P0, Z2H_INIT_PLUS, (uint64_t)j << n);
            HIP_TRY(hipMemcpy(B.inits, ij.data(), sizeof(InitJob) * batch, hipMemcpyHostToDevice));
            InitArgs a;
            memset(&a, 0, sizeof a);
            a.states = B.states;
            a.jobs = (const InitJob *)B.inits;
            a.lat = P0.lat;
            hipError_t e = launch_init(c128, a, (unsigned)batch, s);
            if (e != hipSuccess) return fail(Z2H_ERR_HIP, "init failed: %s", hipGetErrorString(e));
        }
        double best_t = 1e300;
        std::string best_cfg;
        for (const auto &cfg : cands) {
            Plan P;
            if (plan_with_config(Lx, Ly, c128, cfg.c_str(), P) != Z2H_OK) continue;
            float alo = 0, ahi = 0, w = 0;
            // warm-up, then the difference of a long and a short ramp removes
            // the first and last transform passes; large states (a warm-up
            // above 50 ms) are timed once over fewer steps
            if ((st = time_steps(P, B, batch, 2, s, w))) return st;
            // a 2-step ramp is about 3 steps of passes: skip candidates whose
            // warm-up is far behind the best so far
            if (best_t < 1e300 && w > 1.5 * 3.0 * best_t) continue;
            const bool big = w > 50.0f;
            const int lo = big ? 1 : 2, hi = big ? 3 : 6, reps = big ? 1 : 2;
            double t = 1e300;
            for (int r = 0; r < reps; ++r) {
                if ((st = time_steps(P, B, batch, lo, s, alo))) return st;
                if ((st = time_steps(P, B, batch, hi, s, ahi))) return st;
                t = std::min(t, (double)(ahi - alo) / (double)(hi - lo));
            }
            if (t < best_t) {
                best_t = t;
                best_cfg = cfg;
            }
        }
        if (best_cfg.empty()) return fail(Z2H_ERR_UNSUPPORTED, "no candidate schedule could be timed");
        tune_store(n, c128, batch, best_cfg);
        if (cache_path) {
            FILE *f = fopen(cache_path, "a");
            if (!f) return fail(Z2H_ERR_INVALID, "cannot append to %s", cache_path);
            fprintf(f, "%d %d %d %s\n", n, c128 ? 1 : 0, tune_batch_class(batch), best_cfg.c_str());
            fclose(f);
        }
        if (best && best_len) snprintf(best, best_len, "%s", best_cfg.c_str());
        if (best_ms_per_step) *best_ms_per_step = best_t;
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_autotune");
    }
}

}  // extern "C"
