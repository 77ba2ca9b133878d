// Host runtime internals of libz2h shared by the single-state, batch and
// adjoint entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/z2h.h"
#include "z2h_internal.h"
#include "z2h_kernels.h"

namespace z2h {

// Pass schedule of one lattice and precision.
struct Plan {
    int Lx, Ly, n, nst;
    bool c128;
    size_t esize;
    int K;                       // groups (1: whole state in one workgroup)
    GroupGeom geom[kMaxGroups];
    LatticeDev lat;
    int device;
    int nt;                      // streaming loads/stores in the pass kernels
    int xcd;                     // bit j: XCD-major block order in the passes over group j
    int tables;                  // phase tables precomputed per evolve call (0: built per workgroup)
};

namespace rt {

extern thread_local std::string g_err;
z2h_status fail(z2h_status code, const char *fmt, ...);

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ::z2h::rt::fail(Z2H_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace carve-up (256-byte aligned pieces); base null = size only.
struct Carver {
    char *base;
    size_t off;
    void *take(size_t bytes) {
        off = align256(off);
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

int link_bit(int Lx, int Ly, int x, int y, int dir);
void build_masks(int Lx, int Ly, uint64_t *st, uint64_t *pl);
z2h_status check_lattice(int Lx, int Ly);
LatticeDev make_latdev(int Lx, int Ly);
z2h_status make_plan(int Lx, int Ly, bool c128, int max_tile_bits, Plan &P, int batch_hint);
z2h_status plan_with_config(int Lx, int Ly, bool c128, const char *cfg, Plan &P);
std::vector<std::string> tune_candidates(int Lx, int Ly, bool c128);
void tune_store(int n, bool c128, int batch, const std::string &cfg);
z2h_status tune_load(const char *path);
int tune_batch_class(int batch);
size_t lds_bytes(const Plan &P, const GroupGeom &g, int R);
// A group with a layout window across the two runs of a split group: the
// component-exchange pass kernels, the observables, the adjoint and the
// Hamiltonian passes load such windows; the other pass kernels do not.
bool geom_straddles(const GroupGeom &g);
size_t obs_lds_bytes(const Plan &P, const GroupGeom &g, int R);
int obs_workers(const GroupGeom &g);
size_t obs_records(const Plan &P);
size_t norm_parts(const Plan &P);
size_t ws_evolve_size(const Plan &P);
size_t ws_observe_size(const Plan &P);
size_t ws_adjoint_size(const Plan &P);

z2h_status validate_state_ptr(const void *p, const char *what);
z2h_status validate_schedule(const Plan &P, const z2h_schedule *s);
JobDev make_job(const z2h_schedule *s, uint64_t offset);
InitJob init_job(const Plan &P, int kind, uint64_t offset);
int pass_kind_of(const LevelOp &op);
z2h_status check_device_(const Plan &P);
z2h_status check_loop_masks(const Plan &P, const uint64_t *m, int32_t cnt, const char *what,
                            uint32_t *out);

// Per-kernel event timing (z2h_timing_enable / z2h_timing_read).
struct TimedLaunch {
    hipEvent_t a, b;
    int kind;
};
extern thread_local bool t_timing;
extern thread_local std::vector<TimedLaunch> t_launches;
hipEvent_t get_event();
void timed_begin(hipStream_t s, hipEvent_t &e0, hipEvent_t &e1);
void timed_end(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int kind);

// The jobs of one launch sequence: a device array (batches) or one inline
// record carried in the kernel argument block (single state).
struct JobSet {
    const JobDev *d_jobs;   // device array or null
    JobDev inl;             // used when d_jobs is null
    const JobDev *h_jobs;   // host copies (step counts, order), same order as d_jobs
    int njobs;
    const int32_t *d_jidx;  // packed launch: block-job b runs d_jobs[d_jidx[b]] (device), or null
    void *d_tabs;           // single inline job: room for the phase tables of kTabChunk levels, or null
    int tab_lev0;           // first level whose table d_tabs holds
    const void *d_btabs;    // batch group: precomputed tables of every level of d_jobs[r] at
    uint64_t btab_stride;   // d_btabs + r * btab_stride (bytes), or null
};

// Levels whose phase tables one table launch precomputes for a single state
// (the evolve workspace holds one chunk).
constexpr int kTabChunk = 1024;
size_t ws_tables_size(const Plan &P);
int job_levels(const Plan &P, const JobDev &h);  // levels of a job's pass sequence

// Packed level sequence of a batch group: jobs run one after another in
// slots, job j's level 0 at launch level lev0[j] (a multiple of the passes
// per step, so every job of a launch visits the same group).  active[L]
// lists the jobs (indices into the group's records) running at launch level
// L; d_idx + off[L] is the same list on the device.
struct PackedLevels {
    std::vector<std::vector<int32_t>> active;
    std::vector<size_t> off;
    const int32_t *d_idx;
};

// Slots by longest-processing-time assignment; fills lev0 of every host
// record and the per-level lists.
void pack_levels(const Plan &P, std::vector<JobDev> &h_jobs, int slots, PackedLevels &L);
z2h_status run_levels_packed(const Plan &P, void *states, const JobSet &J, const PackedLevels &L, hipStream_t s);

z2h_status launch_one_level(const Plan &P, void *states, const JobSet &J, int lev, int group,
                            int rn_parts, bool force_plain, int kind, hipStream_t s,
                            int kind_hint = -1);
z2h_status full_transform(const Plan &P, void *states, const JobSet &J, hipStream_t s);
z2h_status run_levels(const Plan &P, void *states, const JobSet &J, hipStream_t s);

// Observables of njobs states; records and outputs in device memory.
struct ObsBuffers {
    void *scratch;                      // transformed copies (K > 1)
    const uint64_t *src_off, *dst_off;  // device arrays or null (single state at offset 0)
    double *partZ, *partX;              // njobs * workers * kObsQ each
    const double *H;                    // njobs * 4 (device) or null: H_inline
    double H_inline[4];
    double *out;                        // kObsQ doubles per job
    const int32_t *out_index;           // device: output row of each job, or null (identity)
};

z2h_status run_observe(const Plan &P, const void *states, int njobs, const ObsBuffers &B,
                       const uint32_t *zl, int nz, const uint32_t *xl, int nx, hipStream_t s);

}  // namespace rt
}  // namespace z2h

struct z2h_plan {
    z2h::Plan P;
};
