// Kernel argument blocks and launchers of libz2h (host <-> device boundary
// inside the library; not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "z2h_internal.h"

namespace z2h {

constexpr int kDosBins = 33;
constexpr int kMaxLdsBytes = 160 * 1024;

struct LevelArgs {
    void *states;              // base of the state buffer (complex elements)
    const JobDev *jobs;        // device array of jobs in this launch
    GroupGeom geom;            // group visited at this level
    LatticeDev lat;
    int32_t level, K, group;
    int32_t rn_parts;          // partial norms to sum when a pass renormalizes
    int32_t force_plain;       // 1: plain transform of "group" regardless of the level
    int32_t nt;                // 1: nontemporal (streaming) loads and stores of the state
    int32_t kind_hint;         // pass kind shared by every job of the launch, or -1
    int32_t jmode;             // 0: job jb's state starts at jbase + jb * jstride (elements)
                               // 1: at its record's offset
    uint64_t jbase, jstride;
    int32_t njobs;             // jobs of this launch
    int32_t xcd;               // 1: XCD-major block order (consecutive tiles on one XCD)
    const int32_t *jidx;       // job of block-job b is jobs[jidx[b]] (packed batches), or null: jobs[b]
    const void *tabs;          // precomputed phase tables, or null.  Single state: the tables of
                               // levels tab_lev0, tab_lev0 + 1, ..  Batch group (tab_stride > 0):
                               // record r's level l at tabs + r * tab_stride + l * entries
    uint64_t tab_stride;       // bytes per job record (0: single state)
    int32_t tab_lev0;
    int32_t pad3;
    JobDev job_inline;         // used when jobs is null (single state)
};

// Phase tables of a run of levels of one job, precomputed for the pass
// kernels (single-state evolution).
struct TablesArgs {
    void *tabs;                // (nst + 1)(n + 1) complex entries per level, level lev0 first
    JobDev job;                // the job (jobs null)
    const JobDev *jobs;        // or: job blockIdx.y of this device array, its tables at tabs + y * stride
    uint64_t stride;           // bytes per job when jobs is set
    LatticeDev lat;
    int32_t lev0, K;
};

struct ResidentArgs {
    void *states;
    const JobDev *jobs;
    GroupGeom geom;            // whole state as one tile
    LatticeDev lat;
    int32_t job0;              // first job of this launch
    int32_t pad;
    JobDev job_inline;         // used when jobs is null (single state)
};

struct ObsArgs {
    const void *src;           // state buffer read
    void *dst;                 // transformed copy written (or null)
    const uint64_t *src_off;   // per-job element offsets (device), or null: offset 0
    const uint64_t *dst_off;
    GroupGeom geom;
    LatticeDev lat;
    uint32_t zloops[kMaxLoops], xloops[kMaxLoops];
    int32_t nz, nx;
    int32_t redZ, doH, redX;
    int32_t pad;
    double *part_z;            // per-workgroup records of computational-basis sums (or null)
    double *part_x;            // per-workgroup records of Hadamard-basis sums (or null)
};

struct FinalArgs {
    const double *partZ, *partX;
    int32_t nrecZ, nrecX;      // records per job
    int32_t n, pad;
    const double *H;           // couplings per job (4 doubles), or null: H_inline
    double *out;               // kObsQ doubles per job
    const int32_t *out_index;  // output row of each job (or null: the job index)
    double H_inline[4];
};

struct InitJob {
    uint64_t offset;           // element offset of the state
    int32_t kind;              // 0 plaquette-even, 1 star-even (before the transform), 2 zero, 3 plus
    int32_t pad;
    double amp;
};

struct InitArgs {
    void *states;
    const InitJob *jobs;       // device array (gridDim.y jobs) or null: one_job
    InitJob one_job;
    LatticeDev lat;
};

// Reverse-sweep pass of the adjoint: operates on psi (A) and the adjoint
// state lambda (B) with the same transforms, undoing one forward level.
struct AdjArgs {
    void *A, *B;               // A: psi (or the source of mode 2); B: lambda (or the destination of mode 2)
    GroupGeom geom;
    LatticeDev lat;
    JobDev job;                // schedule of the forward ramp (couplings, dt, device sZ/sX)
    LevelOp op;                // forward level being undone
    int32_t mode;              // 0: plain transform of A (and B if set); 1: inverse phase of A and B with
                               // gradient reduction; 2: B = diag * A (real diagonal of the energy)
    int32_t no_transform;      // 1: act in the current basis without transforming the group
    double dJ, dh;             // diagonal (nst - 2k) dJ + (n - 2w) dh: gradient weight (mode 1) or energy (mode 2)
    double dscale;             // extra real factor of the mode-2 diagonal (2^-n in the Hadamard basis)
    double *part;              // per-block partial sums of Im sum conj(B) D A (mode 1)
};

struct AdjFinalArgs {
    const double *part;        // per-block partials of one level
    int32_t np;                // number of partials
    int32_t pad;
    double *out;               // the level's sum
};

struct AdjGradArgs {
    const double *level_sum;
    double *gZ, *gX;
    int32_t S, K, P, n;
    double dt, inv_norm;
};

hipError_t launch_adj(bool c128, const AdjArgs &a, unsigned nblocks, size_t lds, hipStream_t s);
hipError_t launch_adj_final(const AdjFinalArgs &a, hipStream_t s);
hipError_t launch_adj_grad(const AdjGradArgs &a, hipStream_t s);
hipError_t launch_axpy(bool c128, void *y, const void *x, uint64_t n, hipStream_t s);
bool adj_shape_ok(int R, int NL);

hipError_t launch_level(bool c128, int R, const LevelArgs &a, unsigned nblocks, size_t lds,
                        hipStream_t s);
hipError_t launch_resident(bool c128, int R, const ResidentArgs &a, unsigned njobs, size_t lds,
                           hipStream_t s);
hipError_t launch_obs(bool c128, int R, const ObsArgs &a, unsigned workers, unsigned njobs,
                      size_t lds, hipStream_t s);
hipError_t launch_obs_finalize(const FinalArgs &a, unsigned njobs, hipStream_t s);
hipError_t launch_init(bool c128, const InitArgs &a, unsigned njobs, hipStream_t s);
hipError_t launch_tables(bool c128, const TablesArgs &a, unsigned nlevels, hipStream_t s, unsigned njobs = 1);
hipError_t launch_reduce_parts(const JobDev *jobs, const JobDev &inline_job, int njobs, int parts,
                               hipStream_t s);

LevelOp level_op_host(int lev, int K, int S, int k0, int order);

// Register-window shapes (R, NL) with a compiled straight-line kernel.
bool full_level_ok(int R, int NL);
bool pair_level_ok(bool c128, int R, int NL);  // two-tile blocks compiled for this shape
bool cx_level_ok(int R, int NL);               // component-exchange kernels compiled for this shape
bool full_resident_ok(int R, int NL);

// Set the dynamic-LDS limit of every kernel (call before graph capture).
hipError_t prepare_kernels();

}  // namespace z2h
