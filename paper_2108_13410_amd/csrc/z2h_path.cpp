// Piecewise-linear parameter paths with observable traces (Sec. III, V):
// each leg is a linear ramp run in segments through z2h_evolve, with an
// observation after every segment.
#include <string.h>

#include <algorithm>
#include <cmath>

#include "z2h_runtime.h"

using namespace z2h;
using namespace z2h::rt;

namespace {

// Samples of a path: the initial one, then per leg with steps the segment ends.
int64_t path_samples(const z2h_path &p) {
    int64_t n = 1;
    for (int i = 0; i + 1 < p.nvert; ++i) {
        const int64_t M = p.steps[i];
        if (M <= 0) continue;
        n += p.trace_every > 0 ? (M + p.trace_every - 1) / p.trace_every : 1;
    }
    return n;
}

z2h_status check_path(const z2h_path *p) {
    if (!p) return fail(Z2H_ERR_INVALID, "path is NULL");
    if (p->nvert < 2 || p->nvert > (1 << 16)) return fail(Z2H_ERR_INVALID, "path with %d vertices", p->nvert);
    if (!p->vert || !p->steps) return fail(Z2H_ERR_INVALID, "path vertices or steps NULL");
    if (!std::isfinite(p->dt)) return fail(Z2H_ERR_INVALID, "dt not finite");
    if (p->sampling < 0 || p->sampling > 1 || p->order < 0 || p->order > 1 || p->renorm < 0 || p->renorm > 1)
        return fail(Z2H_ERR_INVALID, "sampling, order and renorm must be 0 or 1");
    if (p->trace_every < 0) return fail(Z2H_ERR_INVALID, "trace_every %d < 0", p->trace_every);
    for (int i = 0; i < p->nvert; ++i) {
        const double *c = &p->vert[i].JA;
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(c[k])) return fail(Z2H_ERR_INVALID, "vertex %d not finite", i);
        if (i + 1 < p->nvert && p->steps[i] < 0) return fail(Z2H_ERR_INVALID, "leg %d: %lld steps", i, (long long)p->steps[i]);
    }
    return Z2H_OK;
}

z2h_couplings lerp(const z2h_couplings &a, const z2h_couplings &b, double s) {
    return {a.JA + s * (b.JA - a.JA), a.JB + s * (b.JB - a.JB), a.hx + s * (b.hx - a.hx), a.hz + s * (b.hz - a.hz)};
}

}  // namespace

extern "C" {

z2h_status z2h_path_evolve(const z2h_plan *plan, void *d_state, void *d_ws, size_t ws_bytes,
                           const z2h_path *path, const uint64_t *zmasks, int32_t nz,
                           const uint64_t *xmasks, int32_t nx, double *d_trace, int64_t trace_cap,
                           int64_t *n_samples, void *stream) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        z2h_status st = check_path(path);
        if (st) return st;
        const int64_t ns = path_samples(*path);
        if (n_samples) *n_samples = ns;
        if (!d_trace) return Z2H_OK;
        if (trace_cap < ns) return fail(Z2H_ERR_WORKSPACE, "trace holds %lld samples, %lld needed",
                                        (long long)trace_cap, (long long)ns);
        const Plan &P = plan->P;
        const size_t need = std::max(ws_evolve_size(P), ws_observe_size(P));
        if (ws_bytes < need) return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
        int64_t idx = 0;
        auto observe = [&](const z2h_couplings &H) {
            return z2h_observe(plan, d_state, d_ws, ws_bytes, &H, zmasks, nz, xmasks, nx, nullptr,
                               d_trace + (size_t)idx++ * Z2H_OBS_DOUBLES, stream);
        };
        if ((st = observe(path->vert[0]))) return st;
        for (int i = 0; i + 1 < path->nvert; ++i) {
            const int64_t M = path->steps[i];
            if (M <= 0) continue;
            z2h_schedule s;
            memset(&s, 0, sizeof s);
            s.start = path->vert[i];
            s.end = path->vert[i + 1];
            s.steps = M;
            s.dt = path->dt;
            s.sampling = path->sampling;
            s.order = path->order;
            s.renorm = path->renorm;
            const int64_t every = path->trace_every > 0 ? path->trace_every : M;
            for (int64_t k0 = 0; k0 < M; k0 += every) {
                s.k_begin = k0;
                s.k_end = std::min(M, k0 + every);
                if ((st = z2h_evolve(plan, d_state, d_ws, ws_bytes, &s, nullptr, stream))) return st;
                if ((st = observe(lerp(path->vert[i], path->vert[i + 1], (double)s.k_end / (double)M)))) return st;
            }
        }
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_path_evolve");
    }
}

}  // extern "C"
