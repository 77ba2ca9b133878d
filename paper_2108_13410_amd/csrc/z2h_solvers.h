// Kernel argument blocks and launchers of the exact solvers and of the
// gate-level circuit emulation (inside the library; not part of the public
// C ABI).  Kept apart from the Trotter-step kernels' declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "z2h_internal.h"
#include "z2h_kernels.h"

namespace z2h {

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
    int32_t xcd;               // 1: XCD-major block order (partials indexed by logical block)
    int32_t pad;
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

// Ritz-vector accumulation: g = (first ? 0 : g) + s * coef[k].sigma * u.
struct AccArgs {
    void *g;
    const void *u;
    const LanczosCoef *coef;
    double s;
    int32_t k, first;
    uint64_t nelem;
};

// Per-block partials of either Re<a, b> and Im<a, b> (mode 0; two doubles
// per block) or |a - theta b|^2 (mode 1).
struct DotArgs {
    const void *a, *b;
    double theta;
    int32_t mode, pad;
    uint64_t nelem;
    double *part;
};

constexpr int kVecBlocks = 2048;   // blocks of the elementwise Lanczos kernels
constexpr int kHamWorkersMax = 2048;

hipError_t launch_ham(bool c128, int R, const HamArgs &a, unsigned workers, size_t lds, hipStream_t s);
hipError_t launch_vec(bool c128, const VecArgs &a, unsigned blocks, hipStream_t s);
hipError_t launch_scalar(const ScalarArgs &a, hipStream_t s);
hipError_t launch_combine(bool c128, const CombineArgs &a, unsigned blocks, hipStream_t s);
hipError_t launch_acc(bool c128, const AccArgs &a, unsigned blocks, hipStream_t s);
hipError_t launch_dot(bool c128, const DotArgs &a, unsigned blocks, hipStream_t s);

// ---- gate-level circuit emulation

// One gate on device: kind as in the public header; m = the 2x2 matrix of a
// one-qubit gate (row-major, re/im interleaved), computed on the host in FP64.
struct GateDev {
    int32_t kind, q0, q1, pad;
    double m[8];
};

constexpr int kFuseMaxGates = 40;   // gates applied by one fused tile pass
constexpr int kGateBlocksMax = 4096;
constexpr int kRegBits = 5;         // qubits held in a thread's registers

// One fused pass over tiles of m qubits lq[0..m) (ascending); the tile
// number supplies the other qubits cq[0..nq-m) in ascending order.  Local
// bit j of the tile index is qubit lq[j].  Each thread holds 2^kRegBits
// amplitudes of a tile, which differ in kRegBits local bits (the layout);
// the 2^(m-kRegBits) threads of a block differ in the other local bits.
// The gates run in phases: phase p has the layout whose local bits are
// packed 4 bits each, ascending, in bits 0..19 of phase[p], and applies the
// gates up to index phase[p] >> 24 (exclusive).  Gate qubits are register
// bit indices into the layout of their phase.  Loads and stores use the
// home layout, the top kRegBits local bits.  In the register kernels a
// CNOT's q0 is the mask of its control bits (the target flips with their
// parity), and a Hadamard is the unscaled butterfly: the amplitudes are
// multiplied by `scale` (2^(-h/2) for h Hadamards) after the last gate.
struct FusedArgs {
    void *state;
    int32_t nq, m, ngates, nphase;
    double scale;
    int32_t lq[16];
    int32_t cq[40];
    uint32_t phase[kFuseMaxGates];
    GateDev gates[kFuseMaxGates];
};
static_assert(sizeof(FusedArgs) <= 4096, "kernel argument block");

// One register-group pass: each thread holds the 2^kRegBits amplitudes that
// differ in the group's qubits rq[] (its register bits); the 2^nt threads of
// a block differ in qubits tq[]; the block's tile number supplies the other
// qubits cq[].  Gate qubits are register-bit indices.
struct RegArgs {
    void *state;
    int32_t nq, nt, ngates, pad;
    double scale;
    int32_t rq[kRegBits], pad2[3];
    int32_t tq[8];
    int32_t cq[40];
    GateDev gates[kFuseMaxGates];
};
static_assert(sizeof(RegArgs) <= 4096, "kernel argument block");

hipError_t launch_gate(bool c128, void *state, int nq, const GateDev &g, hipStream_t s);
hipError_t launch_reg(bool c128, const RegArgs &a, hipStream_t s);
hipError_t launch_fused(bool c128, const FusedArgs &a, hipStream_t s);
hipError_t launch_normalize(bool c128, void *state, int nq, double *part, int nparts, hipStream_t s);

}  // namespace z2h
