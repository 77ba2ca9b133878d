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
    JobDev job_inline;         // used when jobs is null (single state)
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

hipError_t launch_level(bool c128, int R, const LevelArgs &a, unsigned nblocks, size_t lds,
                        hipStream_t s);
hipError_t launch_resident(bool c128, int R, const ResidentArgs &a, unsigned njobs, size_t lds,
                           hipStream_t s);
hipError_t launch_obs(bool c128, int R, const ObsArgs &a, unsigned workers, unsigned njobs,
                      size_t lds, hipStream_t s);
hipError_t launch_obs_finalize(const FinalArgs &a, unsigned njobs, hipStream_t s);
hipError_t launch_init(bool c128, const InitArgs &a, unsigned njobs, hipStream_t s);
hipError_t launch_reduce_parts(const JobDev *jobs, const JobDev &inline_job, int njobs, int parts,
                               hipStream_t s);

LevelOp level_op_host(int lev, int K, int S, int k0, int order);

// Register-window shapes (R, NL) with a compiled straight-line kernel.
bool full_level_ok(int R, int NL);
bool full_resident_ok(int R, int NL);

// Set the dynamic-LDS limit of every kernel (call before graph capture).
hipError_t prepare_kernels();

}  // namespace z2h
