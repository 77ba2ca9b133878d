// Batched ramps: many phase-diagram points and lattices of uneven size
// evolved together and recorded once in a HIP graph.
//
// Jobs are grouped by lattice.  Groups whose states need several passes per
// step run level by level on the caller's stream: one launch per level covers
// every tile of every job still running (jobs are sorted by decreasing step
// count so the running jobs are a prefix).  Groups small enough to live in one
// workgroup run on a second stream inside the same graph, concurrently with
// the level launches.  Observables follow on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <vector>

#include "z2h_runtime.h"

using namespace z2h;
using namespace z2h::rt;


namespace {

struct Group {
    Plan P;
    std::vector<int> jobs;        // global job indices, decreasing level count
    std::vector<JobDev> h_jobs;   // host copies of the device records
    std::vector<InitJob> h_init;
    std::vector<JobDev> h_p1p;    // jobs whose initial state needs the transform
    std::vector<uint64_t> h_off;  // element offsets
    std::vector<double> h_H;      // observed couplings, 4 per job
    std::vector<int32_t> h_out;   // output row per job
    uint32_t zl[kMaxLoops], xl[kMaxLoops];
    int nz, nx;
    // device copies (inside the batch's table allocation)
    JobDev *d_jobs, *d_p1p;
    double *parts_norm;           // per-job norm partials of the z passes (batch-owned)
    InitJob *d_init;
    uint64_t *d_off;
    double *d_H;
    int32_t *d_out;
    // workspace pieces (set per workspace): observable partials only
    double *partZ, *partX;
    // packed level sequence (groups of several passes per step whose step
    // counts differ): jobs run one after another in slots
    bool packed;
    PackedLevels pack;
    bool tables;                  // precomputed phase tables allowed (Z2H_TUNE "tables=0" disables)
    void *d_tabs;                 // precomputed phase tables (batch-owned), or null
    uint64_t tab_stride;          // bytes per job record in d_tabs
};

}  // namespace

struct z2h_batch {
    int njobs;
    bool c128;
    size_t esize;
    std::vector<Group> groups;
    std::vector<uint64_t> byte_off;
    size_t states_bytes, ws_bytes;
    void *d_tables;
    size_t tables_bytes;
    hipStream_t side;            // second branch of the graph (one-workgroup lattices)
    hipStream_t cap;             // stream the graph is recorded on
    hipEvent_t fork, join;
    // graph cache
    hipGraphExec_t exec;
    void *g_states, *g_ws;
    double *g_obs;
    int chunk_jobs;                  // jobs evolved together (0: all)
    // traced runs (z2h_batch_run_trace): graph and the inputs it was recorded for
    hipGraphExec_t exec_t;
    void *t_states, *t_ws;
    double *t_obs, *t_trace;
    int t_every;
    // segment records of traced runs: batch-owned, uploaded for one interval
    void *d_trace_tab;
    size_t trace_tab_bytes;
    int t_up_every;                  // interval the uploaded records belong to (0: none)
    std::vector<TimedLaunch> timed;  // event pairs of the last timed run
    int device;
};

static void loops_for(const Plan &P, uint32_t *zl, int &nz, uint32_t *xl, int &nx) {
    uint64_t z[kMaxLoops], x[kMaxLoops];
    int32_t a = 0, c = 0;
    z2h_loop_masks(P.Lx, P.Ly, z, &a, x, &c);
    for (int j = 0; j < a; ++j) zl[j] = (uint32_t)z[j];
    for (int j = 0; j < c; ++j) xl[j] = (uint32_t)x[j];
    nz = a;
    nx = c;
}

static void free_batch(z2h_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->exec_t) (void)hipGraphExecDestroy(b->exec_t);
    for (auto &t : b->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    if (b->d_tables) (void)hipFree(b->d_tables);
    if (b->d_trace_tab) (void)hipFree(b->d_trace_tab);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    delete b;
}

// Phase tables precomputed at creation for a group whose states are
// cache-resident (at most 64 MiB together) and whose phase passes run
// full-window kernels: such launch-latency-bound passes copy a ready table
// instead of building one per workgroup.  Large groups (the scan) build
// them per workgroup, hidden behind their tile loads.  Bytes for every
// level of every job of the group (0: none).
static int group_max_levels(const Group &g) {
    int mx = 0;
    for (const JobDev &h : g.h_jobs) mx = std::max(mx, job_levels(g.P, h));
    return mx;
}

static uint64_t group_tab_stride(const Group &g) {
    return align256((size_t)group_max_levels(g) * (size_t)(g.P.nst + 1) * (g.P.n + 1) * g.P.esize);
}

static size_t group_tables_bytes(const Group &g) {
    const Plan &P = g.P;
    if (!g.tables || P.K < 2 || !P.geom[0].full || !P.geom[P.K - 1].full) return 0;
    if ((P.esize << P.n) * g.jobs.size() > ((size_t)64 << 20)) return 0;
    const size_t bytes = group_tab_stride(g) * g.jobs.size();
    return bytes <= ((size_t)256 << 20) ? bytes : 0;
}

// Workspace layout of a batch: transformed-copy scratch mirroring the state
// buffer, then per group the observable records.  Every piece is written
// before it is read within one run, so the caller may use the workspace for
// anything else between runs.  (Job records and norm partials, which the
// device records point to, are the batch's own.)
static size_t layout_ws(z2h_batch *b, char *base) {
    Carver c{base, 0};
    void *scratch = c.take(b->states_bytes);
    (void)scratch;
    for (auto &g : b->groups) {
        const size_t nj = g.jobs.size();
        g.partZ = (double *)c.take(sizeof(double) * nj * obs_workers(g.P.geom[0]) * kObsQ);
        g.partX = (double *)c.take(sizeof(double) * nj * obs_workers(g.P.geom[g.P.K - 1]) * kObsQ);
    }
    return align256(c.off);
}

// Record (or run) the whole batch on stream s.
static z2h_status enqueue(z2h_batch *b, void *states, void *ws, double *obs, hipStream_t s) {
    void *scratch = ws;  // first piece of the workspace
    // initial states
    for (auto &g : b->groups) {
        InitArgs a;
        memset(&a, 0, sizeof a);
        a.states = states;
        a.jobs = g.d_init;
        a.lat = g.P.lat;
        hipError_t e = launch_init(g.P.c128, a, (unsigned)g.jobs.size(), s);
        if (e != hipSuccess) return fail(Z2H_ERR_HIP, "init launch failed: %s", hipGetErrorString(e));
        if (!g.h_p1p.empty()) {
            JobSet J;
            memset(&J, 0, sizeof J);
            J.d_jobs = g.d_p1p;
            J.h_jobs = g.h_p1p.data();
            J.njobs = (int)g.h_p1p.size();
            z2h_status st = full_transform(g.P, states, J, s);
            if (st) return st;
        }
    }
    // evolution: resident groups on the side stream, level groups on s
    bool forked = false;
    for (auto &g : b->groups) {
        JobSet J;
        memset(&J, 0, sizeof J);
        J.d_jobs = g.d_jobs;
        J.h_jobs = g.h_jobs.data();
        J.njobs = (int)g.jobs.size();
        if (g.P.K == 1) {
            if (!forked) {
                HIP_TRY(hipEventRecord(b->fork, s));
                HIP_TRY(hipStreamWaitEvent(b->side, b->fork, 0));
                forked = true;
            }
            z2h_status st = run_levels(g.P, states, J, b->side);
            if (st) return st;
        }
    }
    for (auto &g : b->groups) {
        if (g.P.K == 1) continue;
        // Jobs run in chunks whose states fit the last-level cache together:
        // every level of a chunk then streams from the 256 MB MALL instead of
        // HBM.  Chunks keep the decreasing-step order, so each chunk's running
        // jobs are still a prefix.
        const int nj = (int)g.jobs.size();
        if (g.packed) {
            JobSet J;
            memset(&J, 0, sizeof J);
            J.d_jobs = g.d_jobs;
            J.h_jobs = g.h_jobs.data();
            J.njobs = nj;
            J.d_btabs = g.d_tabs;
            J.btab_stride = g.tab_stride;
            z2h_status st = run_levels_packed(g.P, states, J, g.pack, s);
            if (st) return st;
            continue;
        }
        const int chunk = b->chunk_jobs > 0 ? b->chunk_jobs : nj;
        for (int c0 = 0; c0 < nj; c0 += chunk) {
            JobSet J;
            memset(&J, 0, sizeof J);
            J.d_jobs = g.d_jobs + c0;
            J.h_jobs = g.h_jobs.data() + c0;
            J.njobs = std::min(chunk, nj - c0);
            J.d_btabs = g.d_tabs ? (const char *)g.d_tabs + (size_t)c0 * g.tab_stride : nullptr;
            J.btab_stride = g.tab_stride;
            z2h_status st = run_levels(g.P, states, J, s);
            if (st) return st;
        }
    }
    if (forked) {
        HIP_TRY(hipEventRecord(b->join, b->side));
        HIP_TRY(hipStreamWaitEvent(s, b->join, 0));
    }
    // observables
    for (auto &g : b->groups) {
        ObsBuffers B;
        memset(&B, 0, sizeof B);
        B.scratch = scratch;
        B.src_off = g.d_off;
        B.dst_off = g.d_off;
        B.partZ = g.partZ;
        B.partX = g.partX;
        B.H = g.d_H;
        B.out = obs;
        B.out_index = g.d_out;
        z2h_status st = run_observe(g.P, states, (int)g.jobs.size(), B, g.zl, g.nz, g.xl, g.nx, s);
        if (st) return st;
    }
    return Z2H_OK;
}

// ---------------------------------------------------------------- traces
//
// A traced run splits every job's ramp into segments of `every` steps
// (steps [s*every, (s+1)*every) of job j, clipped to its M steps) and observes
// all jobs after each segment.  Segments join with unmerged x halves, so the
// sampled states are exactly those of the uninterrupted Trotter product.  The
// per-segment job records and observation couplings live after the batch's
// own workspace.

static int64_t trace_samples(const z2h_batch *b, int every) {
    int64_t maxM = 0;
    for (const auto &g : b->groups)
        for (const auto &J : g.h_jobs) maxM = std::max<int64_t>(maxM, J.steps);
    return maxM <= 0 ? 0 : (maxM + every - 1) / every;
}

// Bytes of the segment records of a traced run (batch-owned table).
static size_t trace_tab_size(const z2h_batch *b, int64_t nseg) {
    Carver c{nullptr, 0};
    for (const auto &g : b->groups) {
        c.take(sizeof(JobDev) * g.h_jobs.size() * (size_t)nseg);
        c.take(sizeof(double) * 4 * g.h_jobs.size() * (size_t)nseg);
    }
    return align256(c.off);
}

struct TracePieces {
    std::vector<JobDev *> d_seg;              // per group: nseg x nj records
    std::vector<double *> d_segH;             // per group: nseg x nj x 4 couplings
    std::vector<std::vector<JobDev>> h_seg;   // host copies (step counts for the launch sequence)
};

static void trace_layout(const z2h_batch *b, int64_t nseg, char *tab, TracePieces &T) {
    Carver c{tab, 0};
    T.d_seg.clear();
    T.d_segH.clear();
    for (const auto &g : b->groups) {
        T.d_seg.push_back((JobDev *)c.take(sizeof(JobDev) * g.h_jobs.size() * (size_t)nseg));
        T.d_segH.push_back((double *)c.take(sizeof(double) * 4 * g.h_jobs.size() * (size_t)nseg));
    }
}

// Host records of every segment (norm partials: the batch's own).
static void trace_records(const z2h_batch *b, int every, int64_t nseg, TracePieces &T,
                          std::vector<std::vector<double>> &H) {
    T.h_seg.assign(b->groups.size(), {});
    H.assign(b->groups.size(), {});
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const Group &g = b->groups[gi];
        const size_t nj = g.h_jobs.size();
        auto &rec = T.h_seg[gi];
        auto &hh = H[gi];
        rec.resize(nj * (size_t)nseg);
        hh.resize(4 * nj * (size_t)nseg);
        for (int64_t sg = 0; sg < nseg; ++sg) {
            for (size_t j = 0; j < nj; ++j) {
                JobDev r = g.h_jobs[j];
                r.lev0 = 0;  // segments run level-synchronously, never packed
                const int64_t M = r.M;
                const int64_t k0 = std::min<int64_t>(sg * every, M), k1 = std::min<int64_t>((sg + 1) * every, M);
                r.k_begin = (int32_t)k0;
                r.steps = (int32_t)(k1 - k0);
                r.norm_trace = nullptr;
                rec[(size_t)sg * nj + j] = r;
                const double f = M > 0 ? (double)k1 / (double)M : 1.0;
                for (int q = 0; q < 4; ++q) hh[((size_t)sg * nj + j) * 4 + q] = r.c0[q] + f * (r.c1[q] - r.c0[q]);
            }
        }
    }
}

static z2h_status enqueue_init(z2h_batch *b, void *states, hipStream_t s) {
    for (auto &g : b->groups) {
        InitArgs a;
        memset(&a, 0, sizeof a);
        a.states = states;
        a.jobs = g.d_init;
        a.lat = g.P.lat;
        hipError_t e = launch_init(g.P.c128, a, (unsigned)g.jobs.size(), s);
        if (e != hipSuccess) return fail(Z2H_ERR_HIP, "init launch failed: %s", hipGetErrorString(e));
        if (!g.h_p1p.empty()) {
            JobSet J;
            memset(&J, 0, sizeof J);
            J.d_jobs = g.d_p1p;
            J.h_jobs = g.h_p1p.data();
            J.njobs = (int)g.h_p1p.size();
            z2h_status st = full_transform(g.P, states, J, s);
            if (st) return st;
        }
    }
    return Z2H_OK;
}

static z2h_status enqueue_observe(z2h_batch *b, void *states, void *scratch, double *out,
                                  const std::vector<const double *> &Hsel, hipStream_t s) {
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        Group &g = b->groups[gi];
        ObsBuffers B;
        memset(&B, 0, sizeof B);
        B.scratch = scratch;
        B.src_off = g.d_off;
        B.dst_off = g.d_off;
        B.partZ = g.partZ;
        B.partX = g.partX;
        B.H = Hsel[gi];
        B.out = out;
        B.out_index = g.d_out;
        z2h_status st = run_observe(g.P, states, (int)g.jobs.size(), B, g.zl, g.nz, g.xl, g.nx, s);
        if (st) return st;
    }
    return Z2H_OK;
}

static z2h_status enqueue_traced(z2h_batch *b, void *states, void *ws, double *obs, double *trace,
                                 int64_t nseg, const TracePieces &T, hipStream_t s) {
    z2h_status st = enqueue_init(b, states, s);
    if (st) return st;
    std::vector<const double *> Hs(b->groups.size());
    for (int64_t sg = 0; sg < nseg; ++sg) {
        for (size_t gi = 0; gi < b->groups.size(); ++gi) {
            const Group &g = b->groups[gi];
            const size_t nj = g.h_jobs.size();
            JobSet J;
            memset(&J, 0, sizeof J);
            J.d_jobs = T.d_seg[gi] + (size_t)sg * nj;
            J.h_jobs = T.h_seg[gi].data() + (size_t)sg * nj;
            J.njobs = (int)nj;
            if ((st = run_levels(g.P, states, J, s))) return st;
            Hs[gi] = T.d_segH[gi] + (size_t)sg * nj * 4;
        }
        if ((st = enqueue_observe(b, states, ws, trace + (size_t)sg * b->njobs * kObsQ, Hs, s))) return st;
    }
    for (size_t gi = 0; gi < b->groups.size(); ++gi) Hs[gi] = b->groups[gi].d_H;
    return enqueue_observe(b, states, ws, obs, Hs, s);
}


// Slot count for a packed level group, or 0 to keep the level-synchronous
// launches: the cheaper sequence under the launch cost model above, over
// slot counts whose launches fill one or two waves of resident workgroups.
static int choose_slots(const Plan &P, const std::vector<JobDev> &h_jobs, int device) {
    const int nj = (int)h_jobs.size();
    const int Pp = 2 * (P.K - 1);
    int cus = 256;
    if (device >= 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && v > 0) cus = v;
    }
    // workgroups per job and pass, and resident workgroups (LDS-limited,
    // at most four per compute unit) of the widest pass
    double waves_per_job = 0.0;
    for (int k = 0; k < P.K; ++k) {
        const GroupGeom &g = P.geom[k];
        const double blocks = (double)(1ull << g.tiles_log2) / (g.pair >= 2 ? 2.0 : 1.0);
        const int per_cu = std::max(1, std::min(4, (int)(kMaxLdsBytes / std::max<size_t>(1, lds_bytes(P, g, g.R)))));
        waves_per_job = std::max(waves_per_job, blocks / ((double)per_cu * cus));
    }
    if (waves_per_job <= 0.0) return 0;
    std::vector<int64_t> nl(nj);
    int64_t mx = 0;
    for (int j = 0; j < nj; ++j) {
        const JobDev &h = h_jobs[j];
        nl[j] = h.steps <= 0 ? 0 : (h.order == 0 ? Pp * (h.steps + 1) + 1 : Pp * h.steps + 1);
        mx = std::max(mx, nl[j]);
    }
    const double t0 = 7.0, t1 = 8.0;  // microseconds per launch and per wave
    auto launch = [&](int active) { return active ? t0 + t1 * std::ceil(active * waves_per_job - 1e-9) : 0.0; };
    // level-synchronous: job j is active at levels [0, nl[j])
    std::vector<int64_t> sorted(nl);
    std::sort(sorted.begin(), sorted.end(), std::greater<int64_t>());
    double best = 0.0;
    {
        int active = nj;
        for (int64_t L = 0; L < mx; ++L) {
            while (active > 0 && sorted[active - 1] <= L) --active;
            best += launch(active);
        }
    }
    int best_slots = 0;
    const int one_wave = std::max(1, (int)std::floor(1.0 / waves_per_job + 1e-9));
    for (int slots : {one_wave, 2 * one_wave}) {
        if (slots >= nj) continue;
        std::vector<JobDev> tmp(h_jobs);
        PackedLevels L;
        pack_levels(P, tmp, slots, L);
        double cost = 0.0;
        for (const auto &a : L.active) cost += launch((int)a.size());
        if (cost < best) {
            best = cost;
            best_slots = slots;
        }
    }
    return best_slots;
}

extern "C" {

z2h_status z2h_loop_masks(int32_t Lx, int32_t Ly, uint64_t *zl, int32_t *nz, uint64_t *xl, int32_t *nx) {
    z2h_status st = check_lattice(Lx, Ly);
    if (st) return st;
    if (!zl || !nz || !xl || !nx) return fail(Z2H_ERR_INVALID, "NULL argument");
    uint64_t stars[kMaxStab], pl[kMaxStab];
    build_masks(Lx, Ly, stars, pl);
    uint64_t strip = 0, W1 = 0, W2 = 0, V1 = 0, V2 = 0;
    for (int x = 0; x < std::min(3, Lx); ++x) strip ^= pl[x];
    const uint64_t ell = pl[0] ^ pl[1] ^ pl[Lx];
    for (int x = 0; x < Lx; ++x) {
        W1 |= 1ull << link_bit(Lx, Ly, x, 0, 0);
        V1 |= 1ull << link_bit(Lx, Ly, x, 0, 1);
    }
    for (int y = 0; y < Ly; ++y) {
        W2 |= 1ull << link_bit(Lx, Ly, 0, y, 1);
        V2 |= 1ull << link_bit(Lx, Ly, 0, y, 0);
    }
    zl[0] = strip;
    zl[1] = ell;
    zl[2] = W1;
    zl[3] = W2;
    *nz = 4;
    xl[0] = V1;
    xl[1] = V2;
    *nx = 2;
    return Z2H_OK;
}

z2h_status z2h_batch_create(int32_t njobs, const int32_t *Lx, const int32_t *Ly, const z2h_schedule *sched,
                            const z2h_init *init, const z2h_couplings *obsH, z2h_dtype dtype, z2h_batch **out,
                            size_t *states_bytes, size_t *ws_bytes, uint64_t *state_offsets) {
    try {
        if (!out) return fail(Z2H_ERR_INVALID, "out is NULL");
        *out = nullptr;
        if (njobs <= 0 || njobs > (1 << 20)) return fail(Z2H_ERR_INVALID, "njobs = %d", njobs);
        if (!Lx || !Ly || !sched || !init || !obsH || !states_bytes || !ws_bytes || !state_offsets)
            return fail(Z2H_ERR_INVALID, "NULL argument");
        if (dtype != Z2H_C64 && dtype != Z2H_C128) return fail(Z2H_ERR_INVALID, "bad dtype %d", dtype);
        const bool c128 = dtype == Z2H_C128;
        z2h_batch *b = new (std::nothrow) z2h_batch();
        if (!b) return fail(Z2H_ERR_OOM, "out of host memory");
        b->njobs = njobs;
        b->c128 = c128;
        b->esize = c128 ? 16 : 8;
        b->device = -1;
        (void)hipGetDevice(&b->device);
        // group by lattice, validate
        std::map<std::pair<int, int>, int> gid;
        for (int j = 0; j < njobs; ++j) {
            z2h_status st = check_lattice(Lx[j], Ly[j]);
            if (st) { free_batch(b); return st; }
            auto key = std::make_pair(Lx[j], Ly[j]);
            if (!gid.count(key)) {
                Group g{};
                int count = 0;
                for (int i = 0; i < njobs; ++i) count += (Lx[i] == Lx[j] && Ly[i] == Ly[j]);
                st = make_plan(Lx[j], Ly[j], c128, 0, g.P, count);
                if (st) { free_batch(b); return st; }
                g.P.device = b->device;
                gid[key] = (int)b->groups.size();
                b->groups.push_back(g);
            }
            if ((st = validate_schedule(b->groups[gid[key]].P, &sched[j]))) { free_batch(b); return st; }
            if (sched[j].sZ || sched[j].sX) { free_batch(b); return fail(Z2H_ERR_INVALID, "job %d: per-step schedule arrays are not supported in batches", j); }
            if (sched[j].k_begin != 0 || sched[j].k_end != sched[j].steps) { free_batch(b); return fail(Z2H_ERR_INVALID, "job %d: batches run whole ramps", j); }
            if (init[j] < Z2H_INIT_PSI1 || init[j] > Z2H_INIT_PLUS) { free_batch(b); return fail(Z2H_ERR_INVALID, "job %d: bad init kind", j); }
            const double *h = &obsH[j].JA;
            for (int k = 0; k < 4; ++k)
                if (!std::isfinite(h[k])) { free_batch(b); return fail(Z2H_ERR_INVALID, "job %d: observed couplings not finite", j); }
            b->groups[gid[key]].jobs.push_back(j);
        }
        // slot count of packed level groups: Z2H_TUNE "slots=N" (0: never
        // pack), else automatic (-1)
        int pack_slots = -1;
        if (const char *tv = getenv("Z2H_TUNE")) {
            int v;
            const char *q = strstr(tv, "slots=");
            if (q && sscanf(q, "slots=%d", &v) == 1 && v >= 0) pack_slots = v;
        }
        // precomputed phase tables: Z2H_TUNE "tables=0" disables them
        bool tables = true;
        if (const char *tv = getenv("Z2H_TUNE")) {
            int v;
            const char *q = strstr(tv, "tables=");
            if (q && sscanf(q, "tables=%d", &v) == 1) tables = v != 0;
        }
        for (auto &g : b->groups) g.tables = tables;
        // per group: order jobs by decreasing level count
        for (auto &g : b->groups) {
            const int Pp = 2 * (g.P.K - 1);
            auto nlev = [&](int j) {
                const z2h_schedule &s = sched[j];
                return s.steps <= 0 ? 0 : (s.order == 0 ? Pp * (s.steps + 1) + 1 : Pp * s.steps + 1);
            };
            std::stable_sort(g.jobs.begin(), g.jobs.end(), [&](int a, int c) {
                return g.P.K == 1 ? sched[a].steps > sched[c].steps : nlev(a) > nlev(c);
            });
        }
        // state offsets: the states of a group are contiguous, in the group's
        // job order, at the stride of one state (a multiple of 256 bytes)
        b->byte_off.resize(njobs);
        size_t off = 0;
        for (auto &g : b->groups) {
            for (int j : g.jobs) {
                off = align256(off);
                b->byte_off[j] = off;
                state_offsets[j] = off;
                off += b->esize << (2 * Lx[j] * Ly[j]);
            }
        }
        b->states_bytes = align256(off);
        // records
        size_t tbytes = 0;
        for (auto &g : b->groups) {
            for (int j : g.jobs) {
                const uint64_t eoff = b->byte_off[j] / b->esize;
                g.h_jobs.push_back(make_job(&sched[j], eoff));
                g.h_init.push_back(init_job(g.P, init[j], eoff));
                if (init[j] == Z2H_INIT_PSI1P) g.h_p1p.push_back(make_job(&sched[j], eoff));
                g.h_off.push_back(eoff);
                g.h_H.insert(g.h_H.end(), {obsH[j].JA, obsH[j].JB, obsH[j].hx, obsH[j].hz});
                g.h_out.push_back(j);
            }
            loops_for(g.P, g.zl, g.nz, g.xl, g.nx);
            const size_t nj = g.jobs.size();
            // Packing (step counts that differ): level-synchronous launches
            // shrink as jobs finish, down to a few jobs per launch; jobs packed
            // into slots and run back to back keep every launch the same size.
            // A launch costs about t0 + t1 per wave of resident workgroups
            // (measured on MI355X: ~7 us + ~8 us per wave), so the host
            // compares the level-synchronous sequence with slot counts whose
            // launches fill one or two waves and keeps the cheapest.
            g.packed = false;
            if (g.P.K > 1 && nj > 1 && (1 << g.P.geom[0].tiles_log2) <= kReduceChunk && pack_slots != 0) {
                const int slots = pack_slots > 0 ? pack_slots : choose_slots(g.P, g.h_jobs, b->device);
                if (slots > 0 && slots < (int)nj) {
                    pack_levels(g.P, g.h_jobs, slots, g.pack);
                    g.packed = true;
                    tbytes += align256(sizeof(int32_t) * std::max<size_t>(1, g.pack.off.back()));
                }
            }
            tbytes += group_tables_bytes(g);
            tbytes += align256(sizeof(JobDev) * nj) + align256(sizeof(double) * nj * norm_parts(g.P)) +
                      align256(sizeof(JobDev) * std::max<size_t>(1, g.h_p1p.size())) +
                      align256(sizeof(InitJob) * nj) + align256(sizeof(uint64_t) * nj) +
                      align256(sizeof(double) * 4 * nj) + align256(sizeof(int32_t) * nj);
        }
        b->ws_bytes = layout_ws(b, nullptr);
        // device tables (the batch's only allocation)
        b->tables_bytes = tbytes;
        if (hipMalloc(&b->d_tables, tbytes) != hipSuccess) {
            free_batch(b);
            return fail(Z2H_ERR_OOM, "device allocation of %zu bytes failed", tbytes);
        }
        Carver c{(char *)b->d_tables, 0};
        for (auto &g : b->groups) {
            const size_t nj = g.jobs.size();
            g.d_jobs = (JobDev *)c.take(sizeof(JobDev) * nj);
            g.parts_norm = (double *)c.take(sizeof(double) * nj * norm_parts(g.P));
            for (size_t j = 0; j < nj; ++j) g.h_jobs[j].norm_part = g.parts_norm + j * norm_parts(g.P);
            g.d_tabs = nullptr;
            g.tab_stride = 0;
            if (const size_t tb = group_tables_bytes(g)) {
                g.d_tabs = c.take(tb);
                g.tab_stride = group_tab_stride(g);
            }
            g.d_p1p = (JobDev *)c.take(sizeof(JobDev) * std::max<size_t>(1, g.h_p1p.size()));
            g.d_init = (InitJob *)c.take(sizeof(InitJob) * nj);
            g.d_off = (uint64_t *)c.take(sizeof(uint64_t) * nj);
            g.d_H = (double *)c.take(sizeof(double) * 4 * nj);
            g.d_out = (int32_t *)c.take(sizeof(int32_t) * nj);
            std::vector<int32_t> flat;
            if (g.packed) {
                g.pack.d_idx = (int32_t *)c.take(sizeof(int32_t) * std::max<size_t>(1, g.pack.off.back()));
                flat.reserve(g.pack.off.back());
                for (const auto &a : g.pack.active) flat.insert(flat.end(), a.begin(), a.end());
            }
            bool ok = hipMemcpy(g.d_jobs, g.h_jobs.data(), sizeof(JobDev) * nj, hipMemcpyHostToDevice) == hipSuccess &&
                      hipMemcpy(g.d_init, g.h_init.data(), sizeof(InitJob) * nj, hipMemcpyHostToDevice) == hipSuccess &&
                      hipMemcpy(g.d_off, g.h_off.data(), sizeof(uint64_t) * nj, hipMemcpyHostToDevice) == hipSuccess &&
                      hipMemcpy(g.d_H, g.h_H.data(), sizeof(double) * 4 * nj, hipMemcpyHostToDevice) == hipSuccess &&
                      hipMemcpy(g.d_out, g.h_out.data(), sizeof(int32_t) * nj, hipMemcpyHostToDevice) == hipSuccess &&
                      (g.h_p1p.empty() || hipMemcpy(g.d_p1p, g.h_p1p.data(), sizeof(JobDev) * g.h_p1p.size(),
                                                    hipMemcpyHostToDevice) == hipSuccess) &&
                      (flat.empty() || hipMemcpy((void *)g.pack.d_idx, flat.data(), sizeof(int32_t) * flat.size(),
                                                 hipMemcpyHostToDevice) == hipSuccess);
            if (!ok) {
                free_batch(b);
                return fail(Z2H_ERR_HIP, "upload of batch tables failed");
            }
        }
        // phase tables of the cache-resident groups: every level of every
        // job, computed once here (the schedules of a batch are fixed)
        for (auto &g : b->groups) {
            if (!g.d_tabs) continue;
            TablesArgs ta;
            memset(&ta, 0, sizeof ta);
            ta.tabs = g.d_tabs;
            ta.jobs = g.d_jobs;
            ta.stride = g.tab_stride;
            ta.lat = g.P.lat;
            ta.lev0 = 0;
            ta.K = g.P.K;
            if (launch_tables(g.P.c128, ta, (unsigned)group_max_levels(g), nullptr, (unsigned)g.jobs.size()) !=
                hipSuccess) {
                free_batch(b);
                return fail(Z2H_ERR_HIP, "table kernel launch failed");
            }
            if (hipDeviceSynchronize() != hipSuccess) {
                free_batch(b);
                return fail(Z2H_ERR_HIP, "table kernels failed");
            }
        }
        if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess) {
            free_batch(b);
            return fail(Z2H_ERR_HIP, "stream/event creation failed");
        }
        // Chunking (jobs evolved together) is off by default: measured on
        // MI355X, cache-sized chunks ran slower than one launch per level
        // over all jobs, whose grids hide latency better.
        b->chunk_jobs = 0;
        {
            if (const char *tv = getenv("Z2H_TUNE")) {
                int v;
                const char *q = strstr(tv, "chunk=");
                if (q && sscanf(q, "chunk=%d", &v) == 1 && v >= 0) b->chunk_jobs = v;
            }
        }
        *states_bytes = b->states_bytes;
        *ws_bytes = b->ws_bytes;
        *out = b;
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_batch_create");
    }
}

z2h_status z2h_batch_run(z2h_batch *b, void *d_states, void *d_ws, size_t ws_bytes, double *d_obs, void *stream) {
    try {
        if (!b) return fail(Z2H_ERR_INVALID, "batch is NULL");
        z2h_status st = validate_state_ptr(d_states, "d_states");
        if (st) return st;
        if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(Z2H_ERR_INVALID, "d_ws NULL or not 256-byte aligned");
        if (!d_obs) return fail(Z2H_ERR_INVALID, "d_obs is NULL");
        if (ws_bytes < b->ws_bytes) return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, b->ws_bytes);
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || (b->device >= 0 && dev != b->device))
            return fail(Z2H_ERR_INVALID, "batch used on another device");
        hipStream_t s = (hipStream_t)stream;
        if (t_timing) {
            // Timed run: the same launch sequence issued directly on the
            // caller's stream with an event pair around every pass kernel
            // (event records inside a graph carry no timestamps).
            HIP_TRY(hipStreamSynchronize(s));
            for (auto &t : b->timed) {
                (void)hipEventDestroy(t.a);
                (void)hipEventDestroy(t.b);
            }
            b->timed.clear();
            HIP_TRY(prepare_kernels());
            layout_ws(b, (char *)d_ws);
            std::vector<TimedLaunch> saved;
            saved.swap(t_launches);
            st = enqueue(b, d_states, d_ws, d_obs, s);
            b->timed.swap(t_launches);
            t_launches.swap(saved);
            return st;
        }
        if (!b->exec || b->g_states != d_states || b->g_ws != d_ws || b->g_obs != d_obs) {
            if (b->exec) {
                HIP_TRY(hipStreamSynchronize(s));
                (void)hipGraphExecDestroy(b->exec);
                b->exec = nullptr;
            }
            HIP_TRY(prepare_kernels());
            layout_ws(b, (char *)d_ws);
            // recorded on the batch's own stream (the caller's may be the
            // legacy default stream, which cannot be captured)
            HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
            st = enqueue(b, d_states, d_ws, d_obs, b->cap);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(b->cap, &graph);
            if (st) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return fail(Z2H_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(Z2H_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
            b->g_states = d_states;
            b->g_ws = d_ws;
            b->g_obs = d_obs;
        }
        HIP_TRY(hipGraphLaunch(b->exec, s));
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_batch_run");
    }
}

z2h_status z2h_batch_timing(z2h_batch *b, int64_t counts[4], double ms[4]) {
    if (!b || !counts || !ms) return fail(Z2H_ERR_INVALID, "NULL argument");
    for (int k = 0; k < 4; ++k) {
        counts[k] = 0;
        ms[k] = 0;
    }
    for (auto &t : b->timed) {
        float x = 0;
        if (hipEventSynchronize(t.b) != hipSuccess || hipEventElapsedTime(&x, t.a, t.b) != hipSuccess)
            return fail(Z2H_ERR_HIP, "event timing failed");
        counts[t.kind] += 1;
        ms[t.kind] += x;
    }
    return Z2H_OK;
}

z2h_status z2h_batch_trace_sizes(const z2h_batch *b, int32_t every, int64_t *samples_per_job, size_t *ws_bytes) {
    if (!b) return fail(Z2H_ERR_INVALID, "batch is NULL");
    if (every < 1) return fail(Z2H_ERR_INVALID, "trace interval %d < 1", every);
    const int64_t ns = trace_samples(b, every);
    if (samples_per_job) *samples_per_job = ns;
    if (ws_bytes) *ws_bytes = b->ws_bytes;
    return Z2H_OK;
}

z2h_status z2h_batch_run_trace(z2h_batch *b, void *d_states, void *d_ws, size_t ws_bytes, double *d_obs,
                               int32_t every, double *d_trace, void *stream) {
    try {
        if (!b) return fail(Z2H_ERR_INVALID, "batch is NULL");
        z2h_status st = validate_state_ptr(d_states, "d_states");
        if (st) return st;
        if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(Z2H_ERR_INVALID, "d_ws NULL or not 256-byte aligned");
        if (!d_obs || !d_trace) return fail(Z2H_ERR_INVALID, "d_obs or d_trace is NULL");
        if (every < 1) return fail(Z2H_ERR_INVALID, "trace interval %d < 1", every);
        for (const auto &g : b->groups)
            for (const auto &J : g.h_jobs)
                if (J.order != g.h_jobs[0].order)
                    return fail(Z2H_ERR_INVALID, "traced batches need one step order per lattice");
        const int64_t nseg = trace_samples(b, every);
        if (ws_bytes < b->ws_bytes) return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, b->ws_bytes);
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || (b->device >= 0 && dev != b->device))
            return fail(Z2H_ERR_INVALID, "batch used on another device");
        hipStream_t s = (hipStream_t)stream;
        HIP_TRY(prepare_kernels());
        layout_ws(b, (char *)d_ws);
        if (b->t_up_every != every) {
            // The interval changed: earlier runs' graph and records are
            // retired before the table is reused or replaced.
            HIP_TRY(hipStreamSynchronize(s));
            HIP_TRY(hipStreamSynchronize(b->cap));
            if (b->exec_t) {
                (void)hipGraphExecDestroy(b->exec_t);
                b->exec_t = nullptr;
            }
            b->t_up_every = 0;
            const size_t need = trace_tab_size(b, nseg);
            if (need > b->trace_tab_bytes) {
                if (b->d_trace_tab) (void)hipFree(b->d_trace_tab);
                b->d_trace_tab = nullptr;
                b->trace_tab_bytes = 0;
                if (hipMalloc(&b->d_trace_tab, need) != hipSuccess)
                    return fail(Z2H_ERR_OOM, "device allocation of %zu bytes for segment records failed", need);
                b->trace_tab_bytes = need;
            }
        }
        TracePieces T;
        std::vector<std::vector<double>> H;
        trace_layout(b, nseg, (char *)b->d_trace_tab, T);
        trace_records(b, every, nseg, T, H);
        if (b->t_up_every != every) {
            for (size_t gi = 0; gi < b->groups.size(); ++gi) {
                HIP_TRY(hipMemcpy(T.d_seg[gi], T.h_seg[gi].data(), sizeof(JobDev) * T.h_seg[gi].size(),
                                  hipMemcpyHostToDevice));
                HIP_TRY(hipMemcpy(T.d_segH[gi], H[gi].data(), sizeof(double) * H[gi].size(), hipMemcpyHostToDevice));
            }
            b->t_up_every = every;
        }
        if (t_timing) {
            HIP_TRY(hipStreamSynchronize(s));
            for (auto &t : b->timed) {
                (void)hipEventDestroy(t.a);
                (void)hipEventDestroy(t.b);
            }
            b->timed.clear();
            std::vector<TimedLaunch> saved;
            saved.swap(t_launches);
            st = enqueue_traced(b, d_states, d_ws, d_obs, d_trace, nseg, T, s);
            b->timed.swap(t_launches);
            t_launches.swap(saved);
            return st;
        }
        if (!b->exec_t || b->t_states != d_states || b->t_ws != d_ws || b->t_obs != d_obs ||
            b->t_trace != d_trace || b->t_every != every) {
            if (b->exec_t) {
                HIP_TRY(hipStreamSynchronize(s));
                (void)hipGraphExecDestroy(b->exec_t);
                b->exec_t = nullptr;
            }
            HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
            st = enqueue_traced(b, d_states, d_ws, d_obs, d_trace, nseg, T, b->cap);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(b->cap, &graph);
            if (st) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return fail(Z2H_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&b->exec_t, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(Z2H_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
            b->t_states = d_states;
            b->t_ws = d_ws;
            b->t_obs = d_obs;
            b->t_trace = d_trace;
            b->t_every = every;
        }
        HIP_TRY(hipGraphLaunch(b->exec_t, s));
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_batch_run_trace");
    }
}

void z2h_batch_destroy(z2h_batch *b) { free_batch(b); }

}  // extern "C"
