// Piecewise-linear parameter paths with observable traces (Sec. III, V):
// each leg is a linear ramp run in segments through z2h_evolve, with an
// observation after every segment.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

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

// ---- many paths at once

// Segments of leg i when all paths advance together: every `every` steps of
// the longest path's leg (one segment when every = 0).
int64_t leg_segments(const z2h_path *paths, int np, int i) {
    int64_t M = 0;
    for (int j = 0; j < np; ++j) M = std::max<int64_t>(M, paths[j].steps[i]);
    if (M <= 0) return 0;
    const int64_t e = paths[0].trace_every;
    return e > 0 ? (M + e - 1) / e : 1;
}

struct PathsLayout {
    double *norm, *partZ, *partX, *H;
    void *scratch;
    uint64_t *d_off;
    JobDev *d_jobs;
    size_t bytes;
};

PathsLayout paths_layout(const Plan &P, int np, int64_t maxseg, char *base) {
    Carver c{base, 0};
    PathsLayout L;
    L.norm = (double *)c.take(sizeof(double) * np * norm_parts(P));
    L.scratch = P.K > 1 ? c.take((P.esize << P.n) * (size_t)np) : nullptr;
    L.partZ = (double *)c.take(sizeof(double) * np * obs_workers(P.geom[0]) * kObsQ);
    L.partX = (double *)c.take(sizeof(double) * np * obs_workers(P.geom[P.K - 1]) * kObsQ);
    L.d_off = (uint64_t *)c.take(sizeof(uint64_t) * np);
    L.d_jobs = (JobDev *)c.take(sizeof(JobDev) * np * (size_t)maxseg);
    L.H = (double *)c.take(sizeof(double) * 4 * np * (size_t)(maxseg + 1));
    L.bytes = align256(c.off);
    return L;
}

z2h_status check_paths(int np, const z2h_path *paths, int64_t *nsamples, int64_t *maxseg) {
    if (np < 1 || np > (1 << 16)) return fail(Z2H_ERR_INVALID, "npaths = %d", np);
    if (!paths) return fail(Z2H_ERR_INVALID, "paths is NULL");
    z2h_status st;
    for (int j = 0; j < np; ++j) {
        if ((st = check_path(&paths[j]))) return st;
        if (paths[j].nvert != paths[0].nvert) return fail(Z2H_ERR_INVALID, "path %d: %d vertices, path 0 has %d", j,
                                                          paths[j].nvert, paths[0].nvert);
        if (paths[j].trace_every != paths[0].trace_every)
            return fail(Z2H_ERR_INVALID, "path %d: trace interval differs from path 0's", j);
        if (paths[j].order != paths[0].order) return fail(Z2H_ERR_INVALID, "path %d: step order differs from path 0's", j);
        for (int i = 0; i + 1 < paths[j].nvert; ++i)
            if (paths[j].steps[i] > (1 << 30)) return fail(Z2H_ERR_INVALID, "path %d leg %d: too many steps", j, i);
    }
    int64_t ns = 1, mx = 1;
    for (int i = 0; i + 1 < paths[0].nvert; ++i) {
        const int64_t g = leg_segments(paths, np, i);
        ns += g;
        mx = std::max(mx, g);
    }
    *nsamples = ns;
    *maxseg = mx;
    return Z2H_OK;
}

}  // namespace

extern "C" {

z2h_status z2h_paths_sizes(const z2h_plan *plan, int32_t npaths, const z2h_path *paths, int64_t *n_samples,
                           size_t *ws_bytes) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        int64_t ns = 0, mx = 0;
        z2h_status st = check_paths(npaths, paths, &ns, &mx);
        if (st) return st;
        if (n_samples) *n_samples = ns;
        if (ws_bytes) *ws_bytes = paths_layout(plan->P, npaths, mx, nullptr).bytes;
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_paths_sizes");
    }
}

z2h_status z2h_paths_evolve(const z2h_plan *plan, int32_t npaths, void *d_states, void *d_ws, size_t ws_bytes,
                            const z2h_path *paths, const uint64_t *zmasks, int32_t nz, const uint64_t *xmasks,
                            int32_t nx, double *d_trace, void *stream) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        const Plan &P = plan->P;
        int64_t ns = 0, maxseg = 0;
        z2h_status st = check_paths(npaths, paths, &ns, &maxseg);
        if (st) return st;
        if ((st = validate_state_ptr(d_states, "d_states"))) return st;
        if (!d_trace) return fail(Z2H_ERR_INVALID, "d_trace is NULL");
        if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(Z2H_ERR_INVALID, "d_ws NULL or not 256-byte aligned");
        const PathsLayout need = paths_layout(P, npaths, maxseg, nullptr);
        if (ws_bytes < need.bytes) return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need.bytes);
        uint32_t zl[Z2H_MAX_LOOPS], xl[Z2H_MAX_LOOPS];
        if ((st = check_loop_masks(P, zmasks, nz, "zmasks", zl))) return st;
        if ((st = check_loop_masks(P, xmasks, nx, "xmasks", xl))) return st;
        if ((st = check_device_(P))) return st;
        HIP_TRY(prepare_kernels());
        hipStream_t s = (hipStream_t)stream;
        const PathsLayout L = paths_layout(P, npaths, maxseg, (char *)d_ws);
        const int np = npaths;
        const uint64_t elems = 1ull << P.n;
        std::vector<uint64_t> off(np);
        for (int j = 0; j < np; ++j) off[j] = (uint64_t)j * elems;
        HIP_TRY(hipMemcpyAsync(L.d_off, off.data(), sizeof(uint64_t) * np, hipMemcpyHostToDevice, s));

        ObsBuffers B;
        memset(&B, 0, sizeof B);
        B.scratch = L.scratch;
        B.src_off = L.d_off;
        B.dst_off = L.d_off;
        B.partZ = L.partZ;
        B.partX = L.partX;
        int64_t sample = 0;
        std::vector<double> hH((size_t)4 * np * (maxseg + 1));
        // sample 0: every path's initial state at its first vertex
        for (int j = 0; j < np; ++j) memcpy(&hH[4 * j], &paths[j].vert[0].JA, 4 * sizeof(double));
        HIP_TRY(hipMemcpyAsync(L.H, hH.data(), sizeof(double) * 4 * np, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // the host arrays are reused below
        B.H = L.H;
        B.out = d_trace;
        if ((st = run_observe(P, d_states, np, B, zl, nz, xl, nx, s))) return st;
        ++sample;

        const int64_t every = paths[0].trace_every;
        std::vector<JobDev> rec;
        std::vector<int> order(np);
        for (int i = 0; i + 1 < paths[0].nvert; ++i) {
            const int64_t nseg = leg_segments(paths, np, i);
            if (nseg == 0) continue;
            // records of every segment of this leg (each segment's jobs ordered
            // by decreasing step count, as the level sequencer requires), and the
            // couplings each path is observed with after it
            rec.assign((size_t)nseg * np, JobDev{});
            for (int64_t g = 0; g < nseg; ++g) {
                std::vector<JobDev> seg(np);
                for (int j = 0; j < np; ++j) {
                    const z2h_path &pj = paths[j];
                    const int64_t M = pj.steps[i];
                    const int64_t e = every > 0 ? every : std::max<int64_t>(M, 1);
                    z2h_schedule sc;
                    memset(&sc, 0, sizeof sc);
                    sc.start = pj.vert[i];
                    sc.end = pj.vert[i + 1];
                    sc.steps = M;
                    sc.dt = pj.dt;
                    sc.sampling = pj.sampling;
                    sc.order = pj.order;
                    sc.renorm = pj.renorm;
                    sc.k_begin = std::min<int64_t>(g * e, M);
                    sc.k_end = std::min<int64_t>((g + 1) * e, M);
                    seg[j] = make_job(&sc, off[j]);
                    seg[j].norm_part = L.norm + (size_t)j * norm_parts(P);
                    const double f = M > 0 ? (double)sc.k_end / (double)M : 1.0;
                    const z2h_couplings h = lerp(pj.vert[i], pj.vert[i + 1], f);
                    memcpy(&hH[((size_t)g * np + j) * 4], &h.JA, 4 * sizeof(double));
                }
                std::iota(order.begin(), order.end(), 0);
                std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return seg[a].steps > seg[b].steps; });
                for (int r = 0; r < np; ++r) rec[(size_t)g * np + r] = seg[order[r]];
            }
            HIP_TRY(hipMemcpyAsync(L.d_jobs, rec.data(), sizeof(JobDev) * rec.size(), hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(L.H, hH.data(), sizeof(double) * 4 * np * nseg, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
            for (int64_t g = 0; g < nseg; ++g) {
                JobSet J;
                memset(&J, 0, sizeof J);
                J.d_jobs = L.d_jobs + (size_t)g * np;
                J.h_jobs = rec.data() + (size_t)g * np;
                J.njobs = np;
                if ((st = run_levels(P, d_states, J, s))) return st;
                B.H = L.H + (size_t)g * np * 4;
                B.out = d_trace + (size_t)sample * np * kObsQ;
                if ((st = run_observe(P, d_states, np, B, zl, nz, xl, nx, s))) return st;
                ++sample;
            }
            // the records and couplings of the next leg overwrite these
            HIP_TRY(hipStreamSynchronize(s));
        }
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_paths_evolve");
    }
}


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
