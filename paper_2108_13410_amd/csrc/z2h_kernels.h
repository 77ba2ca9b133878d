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
hipError_t launch_reduce_parts(const JobDev *jobs, const JobDev &inline_job, int njobs, int parts,
                               hipStream_t s);

// ---- exact solvers (Hamiltonian application, Lanczos, Krylov exponential)

// Lanczos coefficients of iteration k (device): v_k = sigma_k u_k with u_k
// the stored vector; beta_k = |u_k| (|u_0| for the start vector).
struct LanczosCoef {
    double alpha, beta, sigma, pad;
};

// One tile pass of y = H x.  The passes visit groups 0, 1, .., K-1, .., 1, 0;
// the top group multiplies by the Hadamard-basis diagonal between its
// forward and backward transform, and the last pass adds the computational-
// basis diagonal times x.
//
// Lanczos form (lz = 1, K > 1): the first pass also reduces sum D_Z |x|^2 and
// the top pass 2^-n sum D_X |W x|^2, so <x, H x> is known when the last pass
// runs; that pass then writes the next Lanczos vector
//   w = sigma_k (H x - alpha_k x) - beta_k sigma_{k-1} p,
//   alpha_k = sigma_k^2 (sum of both partial sets),
// to w instead of H x to dst, with per-workgroup |w|^2 partials.
struct HamArgs {
    const void *src;           // read by this pass
    void *dst;                 // written by this pass (may equal src)
    const void *x;             // final pass: the vector H acts on; else null
    double *part;              // final pass: per-workgroup Re<x, Hx> partials, or null
    double *part_z;            // first pass: per-workgroup sum D_Z |x|^2, or null
    double *part_x;            // top pass: per-workgroup 2^-n sum D_X |W x|^2, or null
    const void *p;             // Lanczos final pass: previous vector (read if use_prev)
    void *w;                   // Lanczos final pass: output (may equal p)
    double *part_w;            // Lanczos final pass: |w|^2 partials
    const double *apart_z, *apart_x;
    const LanczosCoef *coef;
    int32_t napart_z, napart_x;
    int32_t k, use_prev, lz;
    GroupGeom geom;
    LatticeDev lat;
    int32_t top;               // 1: transform, X-basis diagonal, transform back
    int32_t final_pass;        // 1: add D_Z x after the transform
    double JA, JB, hx, hz;
    double xscale;             // 2^-n: the two unnormalised transforms
};

// w = sigma_k (y - alpha_k u) - beta_k sigma_{k-1} p (elementwise; w may equal p)
// with alpha_k = sigma_k^2 sum(apart); per-block |w|^2 partials.  mode 1:
// partials of |u|^2 only (start vector).
struct VecArgs {
    const void *y, *u, *p;
    void *w;
    uint64_t nelem;
    const double *apart;       // Re<u, H u> partials of the final Hamiltonian pass
    int32_t napart;
    int32_t k;                 // iteration
    int32_t use_prev;          // 0 at k = 0 (p not read)
    int32_t mode;              // 0 update, 1 norm of u
    const LanczosCoef *coef;
    double *part;              // per-block |w|^2 (or |u|^2) partials
};

// One block: coef[k].alpha from the Hamiltonian partials (one or two sets) and coef[k+1]
// (beta, sigma) from the |w|^2 partials; mode 1: coef[0] from |u_0|^2.
struct ScalarArgs {
    const double *apart, *apart2, *wpart;   // alpha: sum of apart and apart2 (may be null)
    int32_t napart, napart2, nwpart;
    int32_t k, mode;
    LanczosCoef *coef;
};

constexpr int kKrylovMax = 32;   // Krylov basis vectors of one exponential

// psi = sum_j c_j u_j (complex coefficients from the host; u_0 may be psi).
struct CombineArgs {
    void *psi;
    const void *u[kKrylovMax];
    double cre[kKrylovMax], cim[kKrylovMax];
    int32_t m, pad;
    uint64_t nelem;
};

constexpr int kVecBlocks = 2048;   // blocks of the elementwise Lanczos kernels
constexpr int kHamWorkersMax = 2048;

hipError_t launch_ham(bool c128, int R, const HamArgs &a, unsigned workers, size_t lds, hipStream_t s);
hipError_t launch_vec(bool c128, const VecArgs &a, unsigned blocks, hipStream_t s);
hipError_t launch_scalar(const ScalarArgs &a, hipStream_t s);
hipError_t launch_combine(bool c128, const CombineArgs &a, unsigned blocks, hipStream_t s);

// ---- gate-level circuit emulation

// One gate on device: kind as in the public header; m = the 2x2 matrix of a
// one-qubit gate (row-major, re/im interleaved), computed on the host in FP64.
struct GateDev {
    int32_t kind, q0, q1, pad;
    double m[8];
};

constexpr int kFuseMaxGates = 40;   // gates applied by one fused tile pass
constexpr int kGateBlocksMax = 4096;

// One fused pass: the tile holds the m qubits lq[0..m) (ascending; the
// gates' qubits are local indices into it) and the tile number supplies the
// other qubits cq[0..nq-m) in ascending order.
struct FusedArgs {
    void *state;
    int32_t nq, m, ngates, pad;
    int32_t lq[16];
    int32_t cq[40];
    GateDev gates[kFuseMaxGates];
};

hipError_t launch_gate(bool c128, void *state, int nq, const GateDev &g, hipStream_t s);
hipError_t launch_fused(bool c128, const FusedArgs &a, hipStream_t s);
hipError_t launch_normalize(bool c128, void *state, int nq, double *part, int nparts, hipStream_t s);

LevelOp level_op_host(int lev, int K, int S, int k0, int order);

// Register-window shapes (R, NL) with a compiled straight-line kernel.
bool full_level_ok(int R, int NL);
bool pair_level_ok(bool c128, int R, int NL);  // two-tile blocks compiled for this shape
bool full_resident_ok(int R, int NL);

// Set the dynamic-LDS limit of every kernel (call before graph capture).
hipError_t prepare_kernels();

}  // namespace z2h
