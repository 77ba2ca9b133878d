// Internal types shared by the host runtime and the device kernels of libz2h.
#pragma once

#include <stdint.h>

namespace z2h {

constexpr int kMaxN = 32;        // qubits (indices fit in 32 bits)
constexpr int kMaxStab = 16;     // stars or plaquettes (n/2)
constexpr int kMaxLay = 4;       // register layouts per transform
constexpr int kMaxGroups = 4;    // qubit groups of the transform
constexpr int kObsQ = 56;        // doubles per observable record
constexpr int kMaxLoops = 8;
constexpr int kReduceChunk = 1024;  // block partials per first-stage reduction block

// Lattice data the kernels need: stabilizer masks of both kinds, the
// stabilizers containing each link ("syndrome" columns) and loop masks.
struct LatticeDev {
    int32_t n, nst;                     // links, stars (= plaquettes)
    uint32_t zmask[kMaxStab];           // plaquettes (Z strings)
    uint32_t xmask[kMaxStab];           // stars (X strings)
    uint32_t zsyn[kMaxN];               // bit p set if link l is on plaquette p
    uint32_t xsyn[kMaxN];               // bit v set if link l is on star v
};

// One group of the Walsh-Hadamard transform as a tile pass.  A tile holds
// 2^m elements; local index e = u + 2^c * v with u the c carried low bits of
// the global index and v the bits [b0, b0 + m - c) of the global index.  The
// transform acts on local bits [x0, x1).  The tile number supplies the
// remaining global bits.  Each thread keeps 2^R elements in registers; layout
// j puts local bits [p[j], p[j] + R) in registers; in that layout the
// butterflies run over register bits [blo[j], bhi[j]).
struct GroupGeom {
    int32_t m, c, b0, x0, x1;
    int32_t R;                          // log2 amplitudes per thread
    int32_t full;                       // NL when x1 - x0 = NL * R (straight-line kernel), else 0
    int32_t nlay;
    int32_t p[kMaxLay], blo[kMaxLay], bhi[kMaxLay];
    int32_t tiles_log2;                 // tiles per state = 2^(n - m)
    int32_t pair;                       // 2: each block handles tiles 2u, 2u + 1 (else 1 or 0)
    int32_t lds_blk;                    // full-window LDS block per value of the untransformed bits
    int32_t cx;                         // 1: layout changes exchange the real, then the imaginary
                                        // parts (LDS of one component per slot)
    int32_t hi;                         // > 0: the top hi local bits [m - hi, m) sit at global
    int32_t b1;                         // bits [b1, b1 + hi) instead of continuing from b0
    int32_t pad;
};

// Per-job data for the level-synchronous pass kernel.
struct JobDev {
    uint64_t offset;                    // element offset of the state
    int32_t steps;                      // steps applied by this job (k_end - k_begin)
    int32_t k_begin;                    // first step index
    int32_t M;                          // total steps of the ramp (for s_k)
    int32_t sampling, order, renorm;
    double dt;
    double c0[4], c1[4];                // JA, JB, hx, hz at s = 0 and s = 1
    const double *sZ, *sX;              // per-step schedule values or null (device)
    double *norm_part;                  // partial norms of the last z-type pass
    double *norm_trace;                 // per-step norms or null
    int32_t norm_parts;                 // number of partials written there
    int32_t lev0;                       // launch level at which this job's level 0 runs (0 unless packed)
};

// Pass kinds inside a job's level sequence.
enum PassKind : int32_t {
    kIdle = 0,      // job has no pass at this level
    kPlainH = 1,    // transform of the group only
    kPhaseB = 2,    // transform, diagonal phase of the inner basis, transform
    kPhaseA = 3,    // same, outer basis
    kHalfIn = 4,    // phase then transform (z-x-z order, first z half)
    kHalfOut = 5,   // transform then phase (z-x-z order, last z half)
};

// Level descriptor: what a job does at level "lev" of its pass sequence.
struct LevelOp {
    int32_t group;     // which transform group
    int32_t kind;      // PassKind
    int32_t basis;     // 0: phase/reduction in the computational (Z) basis, 1: X basis
    int32_t ka, kb;    // steps whose half/full phases this pass applies (-1: none)
    int32_t full;      // 1: full-step phase of step ka; 0: half-step phases of ka and kb
    int32_t norm;      // 1: measure the norm in the middle of this pass
    int32_t renorm;    // 1: multiply by 1/sqrt(norm of the previous z pass)
};

}  // namespace z2h
