// Device kernels of libz2h: the Trotter step of Sec. III as diagonal phase
// passes around an in-place Walsh-Hadamard transform, for gfx950.
//
// A tile of 2^m complex amplitudes is held by 2^(m-R) threads, 2^R amplitudes
// per thread in registers.  Butterflies over the register bits need no
// communication; the other bits of the tile are brought into registers by an
// exchange through LDS ("layout" change).  Global memory is touched once per
// pass: one coalesced load and one coalesced store of the tile.
//
// The diagonal factors of Eq. (decom) are applied as a table lookup: in the
// computational basis the phase of basis state i depends only on the number
// of odd plaquettes k(i) and the Hamming weight w(i); in the Hadamard basis
// the same holds for stars.  The (k, w) table is built in FP64 by every
// workgroup from the couplings of its step and cast to the storage type.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <set>

#include "z2h_internal.h"
#include "z2h_kernels.h"
#include "z2h_tile.h"

namespace z2h {


// Streaming loads of NT tiles, element by element across the tiles: with
// two tiles of a strided group the two 128-byte halves of each 256-byte row
// are requested back to back.
template <typename Real, int R, int NT, bool SW = false>
__device__ __forceinline__ void load_tiles(Cx<Real> (&v)[NT][1 << R], const Cx<Real> *st,
                                           const LayCtx<R> (&L)[NT]) {
#pragma unroll
    for (int q = 0; q < (1 << R); ++q) {
#pragma unroll
        for (int s = 0; s < NT; ++s) v[s][q] = ldc<Real, true>(st + L[s].i0 + reg_off<R, SW>(L[s], q));
    }
}

// FP64 factors of the phase table live at the start of the exchange
// region: every kernel builds its table while no layout change is in flight
// (before the first exchange of a pass, or after the closing barrier of the
// last one), and the region (at least 2^8 elements) outsizes the factors.
__device__ __forceinline__ double2 *table_scratch(unsigned char *smem) {
    return reinterpret_cast<double2 *>(smem);
}

// Build the phase table T[k][w] = scale * exp(i (alpha (nst - 2k) + beta (n - 2w)))
// in LDS (FP64 angles and products, cast to Real).  Contraction into FMAs is
// off in the schedule, angle and table arithmetic, so every kernel that
// builds a table (in LDS or ahead of time in global memory) rounds the same
// way whatever code surrounds it.  Two stages so that a
// pass can compute the factors while its tile loads are in flight and apply
// the scale (which may depend on a norm reduction) afterwards.
__device__ __forceinline__ void table_factors(double2 *fac, int nst, int n, double alpha, double beta) {
#pragma clang fp contract(off)
    const int t = threadIdx.x, nt = blockDim.x;
    for (int j = t; j < nst + 1 + n + 1; j += nt) {
        double ang = j <= nst ? alpha * (double)(nst - 2 * j) : beta * (double)(n - 2 * (j - nst - 1));
        double s, c;
        sincos(ang, &s, &c);
        fac[j] = make_double2(c, s);
    }
}

template <typename Real>
__device__ __forceinline__ void table_products(Cx<Real> *tab, const double2 *fac, int nst, int n,
                                               double scale) {
#pragma clang fp contract(off)
    const int t = threadIdx.x, nt = blockDim.x;
    __syncthreads();
    const int W = n + 1;
    for (int j = t; j < (nst + 1) * W; j += nt) {
        const int k = j / W, w = j - k * W;
        const double2 a = fac[k], b = fac[nst + 1 + w];
        const double re = (a.x * b.x - a.y * b.y) * scale;
        const double im = (a.x * b.y + a.y * b.x) * scale;
        tab[j] = Cx<Real>{(Real)re, (Real)im};
    }
    __syncthreads();
}

template <typename Real>
__device__ void build_table(Cx<Real> *tab, double2 *fac, int nst, int n, double alpha,
                            double beta, double scale) {
    table_factors(fac, nst, n, alpha, beta);
    table_products<Real>(tab, fac, nst, n, scale);
}

// Multiply every register element by T[k][w]: elements are visited in
// Gray-code order so each step updates the syndrome by one uniform column.
template <typename Real, int R, int PHASE_CHUNK = 0>
__device__ __forceinline__ void apply_phase(Cx<Real> (&v)[1 << R], const LayCtx<R> &L, int basis,
                                            int n, const Cx<Real> *tab) {
    uint32_t s = basis ? L.s0x : L.s0z;
    const Cx<Real> *tw = tab + L.w0;
    const int W = n + 1;
#pragma unroll
    for (int idx = 0; idx < (1 << R); ++idx) {
        const int q = idx ^ (idx >> 1);
        if (idx) s ^= basis ? L.lx[__builtin_ctz(idx)] : L.lz[__builtin_ctz(idx)];
        v[q] = cmul(v[q], tw[__umul24((uint32_t)popc(s), (uint32_t)W) + __builtin_popcount(q)]);
        // keep the table reads of at most eight elements in flight (register
        // pressure when a block holds two tiles)
        if (PHASE_CHUNK && (idx & (PHASE_CHUNK - 1)) == PHASE_CHUNK - 1) __builtin_amdgcn_sched_barrier(0);
    }
}

// Sum of |v_q|^2 over a thread's register elements: pairwise in the storage
// precision (complex64 steps accumulate in FP32), returned as FP64 for the
// block and grid reductions.
template <typename Real, int R>
__device__ __forceinline__ double sumsq(const Cx<Real> (&v)[1 << R]) {
    Real a[1 << R];
#pragma unroll
    for (int q = 0; q < (1 << R); ++q) a[q] = v[q].x * v[q].x + v[q].y * v[q].y;
#pragma unroll
    for (int h = (1 << R) >> 1; h > 0; h >>= 1) {
#pragma unroll
        for (int q = 0; q < h; ++q) a[q] += a[q + h];
    }
    return (double)a[0];
}


// Norm partials and traces live in global memory; accessing them through
// global-address-space pointers keeps them off the LDS counter (generic
// "flat" accesses count on both, and would make LDS waits wait for them).
typedef __attribute__((address_space(1))) double *GlobalDoubles;
__device__ __forceinline__ double gld(const double *p, int64_t i) { return ((GlobalDoubles)p)[i]; }
__device__ __forceinline__ void gst(double *p, int64_t i, double v) { ((GlobalDoubles)p)[i] = v; }

// Job records are read-only during a launch: read them through the constant
// address space so that the (block-uniform) record is fetched with scalar
// loads, whose completion does not wait on the block's outstanding tile loads.
typedef const __attribute__((address_space(4))) uint32_t *ConstWords;
static_assert(sizeof(JobDev) % 4 == 0, "job record is copied in 32-bit words");

__device__ __forceinline__ JobDev job_record(const JobDev *jobs, int jb, const JobDev &inl) {
    if (!jobs) return inl;
    JobDev J;
    uint32_t *d = reinterpret_cast<uint32_t *>(&J);
    const ConstWords src = (ConstWords)(jobs + jb);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(JobDev) / 4); ++i) d[i] = src[i];
    return J;
}

// Job of a packed launch's block-job b (index list read through the constant
// address space: a scalar load).
__device__ __forceinline__ int job_index(const int32_t *jidx, int b) {
    typedef const __attribute__((address_space(4))) int32_t *ConstInts;
    return ((ConstInts)jidx)[b];
}

// ---------------------------------------------------------------- schedule

__device__ __forceinline__ double sched_s(const JobDev &J, int k, int zkind) {
#pragma clang fp contract(off)
    typedef const __attribute__((address_space(4))) double *ConstDoubles;
    const double *arr = zkind ? J.sZ : J.sX;
    if (arr) return ((ConstDoubles)arr)[k];  // read-only; scalar load
    return J.sampling ? (double)(k + 1) / (double)J.M : ((double)k + 0.5) / (double)J.M;
}

// (coupling, field) of the given basis at step k: inner (Z) basis uses
// (JB, hz) at sZ, outer (X) basis uses (JA, hx) at sX.
__device__ __forceinline__ void coup(const JobDev &J, int basis, int k, double &Jc, double &h) {
#pragma clang fp contract(off)
    const double s = sched_s(J, k, basis == 0);
    const int ij = basis == 0 ? 1 : 0, ih = basis == 0 ? 3 : 2;
    Jc = (1.0 - s) * J.c0[ij] + s * J.c1[ij];
    h = (1.0 - s) * J.c0[ih] + s * J.c1[ih];
}

// Angles of a phase pass: full step ka (duration dt) or half steps ka, kb.
__device__ __forceinline__ void phase_angles(const JobDev &J, const LevelOp &op, double &alpha,
                                             double &beta) {
#pragma clang fp contract(off)
    double Ja, ha, Jb = 0, hb = 0;
    coup(J, op.basis, op.ka, Ja, ha);
    if (op.full) {
        alpha = J.dt * Ja;
        beta = J.dt * ha;
        return;
    }
    if (op.kb >= 0) coup(J, op.basis, op.kb, Jb, hb);
    alpha = 0.5 * J.dt * (Ja + Jb);
    beta = 0.5 * J.dt * (ha + hb);
}

// Level sequence of one job (see the host planner for the derivation): the
// visited group zig-zags between group 0 (computational basis reached) and
// group K-1 (Hadamard basis reached).
__host__ __device__ inline LevelOp level_op(int lev, int K, int S, int k0, int order) {
    LevelOp op{0, kIdle, 0, -1, -1, 0, 0, 0};
    const int P = 2 * (K - 1);
    const int nlev = order == 0 ? P * (S + 1) + 1 : P * S + 1;
    if (S <= 0 || lev < 0 || lev >= nlev) return op;
    const int r = lev % P;
    op.group = r <= K - 1 ? r : P - r;
    const int j = lev / P;
    if (op.group != 0 && op.group != K - 1) {
        op.kind = kPlainH;
        return op;
    }
    if (op.group == K - 1 && r == K - 1) {
        // outer visit j
        op.basis = 1;
        if (order == 0) {
            op.kind = kPhaseB;
            if (j == 0) {
                op.ka = k0; op.kb = -1; op.full = 0;
            } else if (j == S) {
                op.ka = k0 + S - 1; op.kb = -1; op.full = 0;
            } else {
                op.ka = k0 + j - 1; op.kb = k0 + j; op.full = 0;
            }
            op.renorm = j >= 1 ? 1 : 0;
        } else {
            op.kind = kPhaseB;
            op.ka = k0 + j; op.full = 1;
            op.renorm = 1;
        }
        return op;
    }
    // inner visit j (group 0)
    op.basis = 0;
    if (order == 0) {
        if (j == 0 || j == S + 1) {
            op.kind = kPlainH;
        } else {
            op.kind = kPhaseB;
            op.ka = k0 + j - 1; op.full = 1;
            op.norm = 1;
        }
    } else {
        if (j == 0) {
            op.kind = kHalfIn; op.ka = k0; op.kb = -1; op.full = 0; op.norm = 1;
        } else if (j == S) {
            op.kind = kHalfOut; op.ka = k0 + S - 1; op.kb = -1; op.full = 0;
        } else {
            op.kind = kPhaseB; op.ka = k0 + j - 1; op.kb = k0 + j; op.full = 0; op.norm = 1;
        }
    }
    return op;
}

// ---------------------------------------------------------------- level kernel

template <typename Real, int R, bool NT, bool SP = false>
__global__ void __launch_bounds__(512) level_kernel(LevelArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const GroupGeom &g = a.geom;
    const uint32_t t = threadIdx.x;
    const uint64_t tiles = 1ull << g.tiles_log2;
    const uint64_t bid = blockIdx.x;
    const int jb = (int)(bid >> g.tiles_log2);
    const uint64_t tile = bid & (tiles - 1);
    const JobDev J = job_record(a.jobs, a.jidx ? job_index(a.jidx, jb) : jb, a.job_inline);
    const LevelOp op = a.force_plain ? LevelOp{a.group, kPlainH, 0, -1, -1, 0, 0, 0}
                                     : level_op(a.level - J.lev0, a.K, J.steps, J.k_begin, J.order);
    if (op.kind == kIdle || op.group != a.group) return;  // uniform per block

    Cx<Real> *lds = reinterpret_cast<Cx<Real> *>(smem);
    const uint32_t lds_elems = (1u << g.m) + (1u << (g.m - R));
    Cx<Real> *tab = lds + lds_elems;
    const int W = a.lat.n + 1;
    double2 *fac = table_scratch(smem);
    double *red = align16<double>(tab + (a.lat.nst + 1) * W);

    const bool has_phase = op.kind != kPlainH;
    const bool preH = op.kind != kHalfIn;
    const bool postH = op.kind == kPhaseB || op.kind == kHalfIn;

    // Phase table (FP64 angles), including the renormalization factor.
    if (has_phase) {
        double alpha, beta;
        phase_angles(J, op, alpha, beta);
        double scale = op.basis ? ldexp(1.0, -a.lat.n) : 1.0;
        if (op.renorm && J.norm_part && (J.renorm || J.norm_trace)) {
            double s = 0.0;
            for (int j = (int)t; j < a.rn_parts; j += blockDim.x) s += gld(J.norm_part, j);
            s = block_sum(s, red);
            if (J.renorm) scale *= 1.0 / sqrt(s);
            if (tile == 0 && t == 0 && J.norm_trace) gst(J.norm_trace, op.ka - J.k_begin, s);
        }
        build_table<Real>(tab, fac, a.lat.nst, a.lat.n, alpha, beta, scale);
    }

    Cx<Real> v[1 << R];
    Cx<Real> *st = reinterpret_cast<Cx<Real> *>(a.states) + J.offset;

    LayCtx<R> L0;
    lay_ctx<R, SP>(L0, g, a.lat, tile, g.p[0], t, false);
    load_tile<Real, R, NT, SP>(v, st, L0);

    int cur = 0;
    if (preH) {
        for (int j = 0; j < g.nlay; ++j) {
            if (j > 0) exchange<Real, R>(v, lds, g.p[j - 1], g.p[j], t);
            butterflies<Real, R>(v, g.blo[j], g.bhi[j]);
        }
        cur = g.nlay - 1;
    }
    // norms are measured only where a renormalization or a trace uses them
    const bool need_norm = op.norm && (J.renorm || J.norm_trace);
    if (has_phase || need_norm) {
        LayCtx<R> Lm;
        lay_ctx<R, SP>(Lm, g, a.lat, tile, g.p[cur], t, has_phase, op.basis);
        if (need_norm) {
            double s = block_sum(sumsq<Real, R>(v), red);
            if (t == 0 && J.norm_part) gst(J.norm_part, tile, s);
        }
        if (has_phase) apply_phase<Real, R>(v, Lm, op.basis, a.lat.n, tab);
    }
    if (postH) {
        if (cur == g.nlay - 1) {
            for (int j = g.nlay - 1; j >= 0; --j) {
                if (j != cur) {
                    exchange<Real, R>(v, lds, g.p[cur], g.p[j], t);
                    cur = j;
                }
                butterflies<Real, R>(v, g.blo[j], g.bhi[j]);
            }
        } else {
            for (int j = 0; j < g.nlay; ++j) {
                if (j != cur) {
                    exchange<Real, R>(v, lds, g.p[cur], g.p[j], t);
                    cur = j;
                }
                butterflies<Real, R>(v, g.blo[j], g.bhi[j]);
            }
        }
    }
    if (cur != 0) exchange<Real, R>(v, lds, g.p[cur], g.p[0], t);
    store_tile<Real, R, NT, SP>(v, st, L0);
}

// ---------------------------------------------------------------- full-window kernels
//
// When a group's transformed bits are an exact multiple NL * R of the
// register window, every layout butterflies all R register bits: the
// transform is straight-line code (no runtime-selected stages, so no register
// copies at control-flow joins), layout j sits at local bit x1 - R (j + 1),
// and each pass kind is its own straight-line path from load to store.

template <typename Real, int R>
__device__ __forceinline__ void bfly_all(Cx<Real> (&v)[1 << R]) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
#pragma unroll
        for (int q = 0; q < (1 << R); ++q) {
            if (!(q & (1 << j))) {
                Cx<Real> a = v[q], b = v[q | (1 << j)];
                v[q] = cadd(a, b);
                v[q | (1 << j)] = csub(a, b);
            }
        }
    }
}

// Layout change through LDS.  The register bits and the thread bits of a
// local index are disjoint, so slot(base | q << p) = slot(base) + slot(q << p):
// one per-thread base plus a block-uniform offset per element.
template <typename Real, int R>
__device__ __forceinline__ void xchg(Cx<Real> (&v)[1 << R], Cx<Real> *lds, int pf, int pt, uint32_t t) {
    const uint32_t bf = slot<R>(lay_base<R>(pf, t)), bt = slot<R>(lay_base<R>(pt, t));
#pragma unroll
    for (int q = 0; q < (1 << R); ++q) lds[bf + slot<R>((uint32_t)q << pf)] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (1 << R); ++q) v[q] = lds[bt + slot<R>((uint32_t)q << pt)];
    __syncthreads();
}

// Transform over the group: layouts 0 .. NL-1 (ends in layout NL-1).
template <typename Real, int R, int NL>
__device__ __forceinline__ void fwd_full(Cx<Real> (&v)[1 << R], Cx<Real> *lds, int x1, uint32_t t) {
    bfly_all<Real, R>(v);
#pragma unroll
    for (int j = 1; j < NL; ++j) {
        xchg<Real, R>(v, lds, x1 - R * j, x1 - R * (j + 1), t);
        bfly_all<Real, R>(v);
    }
}

// Transform over the group starting in layout NL-1 (ends in layout 0).
template <typename Real, int R, int NL>
__device__ __forceinline__ void bwd_full(Cx<Real> (&v)[1 << R], Cx<Real> *lds, int x1, uint32_t t) {
    bfly_all<Real, R>(v);
#pragma unroll
    for (int j = NL - 1; j >= 1; --j) {
        xchg<Real, R>(v, lds, x1 - R * (j + 1), x1 - R * j, t);
        bfly_all<Real, R>(v);
    }
}

// Finish the norm of the previous z pass (thread t already holds partial t)
// and fold 1/sqrt(norm) into the phase table when the job renormalizes.
template <typename Real>
__device__ __forceinline__ void renorm_table(const LevelArgs &a, const JobDev &J, const LevelOp &op,
                                             uint64_t tile, uint32_t t, double part, Cx<Real> *tab,
                                             double *red) {
    for (int j = (int)t + (int)blockDim.x; j < a.rn_parts; j += blockDim.x) part += gld(J.norm_part, j);
    const double s = block_sum(part, red);
    if (tile == 0 && t == 0 && J.norm_trace) gst(J.norm_trace, op.ka - J.k_begin, s);
    if (J.renorm) {
        const Real f = (Real)(1.0 / sqrt(s));
        const int entries = (a.lat.nst + 1) * (a.lat.n + 1);
        for (int j = (int)t; j < entries; j += blockDim.x) {
            tab[j].x *= f;
            tab[j].y *= f;
        }
        __syncthreads();
    }
}

// Rest of one pass over NT consecutive tiles of a block, after their loads
// were issued (v[s] in layout 0 for tile tile0 + s).  The phase table is
// built while the loads are in flight: FP64 factors and unscaled products
// first; the renormalization factor (from the previous z pass's block
// partials, whose load was issued after the tiles') is applied to the table
// after the first transform, when those loads have landed.  Layout changes
// go through LDS one tile at a time (the LDS block holds one tile).
// LDS placement of a tile for the layout changes of a full-window pass.
// Local index e splits into its G transformed bits t = e[x0, x1) and the
// untransformed bits u (carried low bits, then any bits above x1); element e
// goes to slot(t) + u * g.lds_blk.  Register window j covers bits
// [R (NL-1-j), R (NL-j)) of t, so an element's offset within a layout is a
// compile-time constant and each thread keeps one base per layout.  The block
// length (at least the padded 2^G + 2^(G-R)) is chosen by the planner so that
// the lanes of a wave spread over the LDS banks in every layout.
template <int R, int NL>
struct LdsMap {
    uint32_t base[NL];
};

template <int R, int NL, typename Real>
__device__ __forceinline__ void lds_map(LdsMap<R, NL> &M, const GroupGeom &g, uint32_t t) {
    constexpr int G = R * NL;
    const int x0 = g.x0, x1 = g.x1;
    const uint32_t blk = (uint32_t)g.lds_blk;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const uint32_t e = lay_base<R>(x1 - R * (j + 1), t);
        const uint32_t tb = (e >> x0) & ((1u << G) - 1u);
        const uint32_t u = (e & ((1u << x0) - 1u)) | ((e >> x1) << x0);
        M.base[j] = slot<R>(tb) + u * blk;
    }
}

// Layout change from window position PF to PT (positions in rot coordinates).
template <typename Real, int R, int PF, int PT>
__device__ __forceinline__ void xchg_rot(Cx<Real> (&v)[1 << R], Cx<Real> *lds, uint32_t bf, uint32_t bt) {
#pragma unroll
    for (int q = 0; q < (1 << R); ++q) lds[bf + slot<R>((uint32_t)q << PF)] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (1 << R); ++q) v[q] = lds[bt + slot<R>((uint32_t)q << PT)];
    __syncthreads();
}

// Layout change with CX = 1: the real parts, then the imaginary parts,
// through an LDS block of one component per slot (half the bytes of a
// tile), so that two workgroups of a large tile fit on one CU.  Same slots
// as the element exchange; CX = 0 is the element exchange.
template <typename Real, int R, int PF, int PT, int CX>
__device__ __forceinline__ void xchg_rot_x(Cx<Real> (&v)[1 << R], Cx<Real> *lds, uint32_t bf, uint32_t bt) {
    if constexpr (CX == 0) {
        xchg_rot<Real, R, PF, PT>(v, lds, bf, bt);
    } else {
        Real *l = reinterpret_cast<Real *>(lds);
#pragma unroll
        for (int q = 0; q < (1 << R); ++q) l[bf + slot<R>((uint32_t)q << PF)] = v[q].x;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < (1 << R); ++q) v[q].x = l[bt + slot<R>((uint32_t)q << PT)];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < (1 << R); ++q) l[bf + slot<R>((uint32_t)q << PF)] = v[q].y;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < (1 << R); ++q) v[q].y = l[bt + slot<R>((uint32_t)q << PT)];
        __syncthreads();
    }
}

template <typename Real, int R, int NL, int J, int CX = 0>
__device__ __forceinline__ void fwd_rot_from(Cx<Real> (&v)[1 << R], Cx<Real> *lds, const LdsMap<R, NL> &M) {
    if constexpr (J < NL) {
        xchg_rot_x<Real, R, R * (NL - J), R * (NL - 1 - J), CX>(v, lds, M.base[J - 1], M.base[J]);
        bfly_all<Real, R>(v);
        fwd_rot_from<Real, R, NL, J + 1, CX>(v, lds, M);
    }
}

// Transform over the group: layouts 0 .. NL-1 (ends in layout NL-1).
template <typename Real, int R, int NL, int CX = 0>
__device__ __forceinline__ void fwd_rot(Cx<Real> (&v)[1 << R], Cx<Real> *lds, const LdsMap<R, NL> &M) {
    bfly_all<Real, R>(v);
    fwd_rot_from<Real, R, NL, 1, CX>(v, lds, M);
}

template <typename Real, int R, int NL, int J, int CX = 0>
__device__ __forceinline__ void bwd_rot_from(Cx<Real> (&v)[1 << R], Cx<Real> *lds, const LdsMap<R, NL> &M) {
    if constexpr (J >= 1) {
        xchg_rot_x<Real, R, R * (NL - 1 - J), R * (NL - J), CX>(v, lds, M.base[J], M.base[J - 1]);
        bfly_all<Real, R>(v);
        bwd_rot_from<Real, R, NL, J - 1, CX>(v, lds, M);
    }
}

// Transform over the group starting in layout NL-1 (ends in layout 0).
template <typename Real, int R, int NL, int CX = 0>
__device__ __forceinline__ void bwd_rot(Cx<Real> (&v)[1 << R], Cx<Real> *lds, const LdsMap<R, NL> &M) {
    bfly_all<Real, R>(v);
    bwd_rot_from<Real, R, NL, NL - 1, CX>(v, lds, M);
}

// TAB: the kernel may copy a precomputed phase table (a.tabs) instead of
// building it.  Only the any-kind kernels carry that branch: launches with
// tables use them for every phase level, and the single-kind phase kernels
// keep the shorter set-up of the per-workgroup build.
template <typename Real, int R, int NL, int KIND, int NT, int CX = 0, bool TAB = false>
__device__ __forceinline__ void pass_multi(const LevelArgs &a, const JobDev &J, const LevelOp &op, int jrec,
                                           uint64_t tile0, uint32_t t, Cx<Real> (&v)[NT][1 << R],
                                           Cx<Real> *st, const LayCtx<R> (&L0)[NT], Cx<Real> *lds,
                                           Cx<Real> *tab, double2 *fac, double *red, int tab_done = 0) {
    const GroupGeom &g = a.geom;
    const int x1 = g.x1;
    const int p0 = x1 - R, pl = x1 - R * NL;
    constexpr bool kPhase = KIND != kPlainH;
    // norms are measured (z passes) and summed (the next pass) only where a
    // renormalization or a norm trace uses them
    const bool use_norms = J.renorm || J.norm_trace;
    const bool want_norm = kPhase && op.renorm && J.norm_part && use_norms;
    const bool meas_norm = op.norm && use_norms;
    const int nst = a.lat.nst, n = a.lat.n;
    double part = 0.0;
    if constexpr (kPhase) {
        if (want_norm && (int)t < a.rn_parts) part = gld(J.norm_part, t);
        if (TAB && a.tabs) {
            // the level's table was built by tables_kernel with the same
            // arithmetic (once per batch for every job's levels, or per chunk
            // of levels of a single state): copy it into LDS
            typedef typename Vec2<Real>::type V;
            typedef const __attribute__((address_space(1))) V *GTab;
            const int entries = (nst + 1) * (n + 1);
            const GTab src =
                a.tab_stride
                    ? (GTab)((const __attribute__((address_space(1))) unsigned char *)a.tabs +
                             (size_t)(a.jidx ? job_index(a.jidx, jrec) : jrec) * a.tab_stride) +
                          (size_t)(a.level - J.lev0) * entries
                    : (GTab)a.tabs + (size_t)(a.level - a.tab_lev0) * entries;
            // (entries below tab_done were prefetched by the block)
            for (int j = tab_done + (int)t; j < entries; j += blockDim.x) {
                const V w = src[j];
                tab[j] = Cx<Real>{w.x, w.y};
            }
            __syncthreads();
        } else {
            double alpha, beta;
            phase_angles(J, op, alpha, beta);
            table_factors(fac, nst, n, alpha, beta);
            table_products<Real>(tab, fac, nst, n, op.basis ? ldexp(1.0, -n) : 1.0);
        }
    }
    if constexpr (KIND == kHalfIn) {
        if (want_norm) renorm_table<Real>(a, J, op, tile0, t, part, tab, red);
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            LayCtx<R> Ls;
            lay_ctx<R, CX != 0>(Ls, g, a.lat, tile0 + s, p0, t, true, op.basis);
            if (meas_norm) {
                const double q = block_sum(sumsq<Real, R>(v[s]), red);
                if (t == 0 && J.norm_part) gst(J.norm_part, tile0 + s, q);
            }
            apply_phase<Real, R, NT == 2 ? 8 : 0>(v[s], Ls, op.basis, n, tab);
        }
    }
    LdsMap<R, NL> M;
    lds_map<R, NL, Real>(M, g, t);
#pragma unroll
    for (int s = 0; s < NT; ++s) fwd_rot<Real, R, NL, CX>(v[s], lds, M);
    if constexpr (kPhase && KIND != kHalfIn) {
        if (want_norm) renorm_table<Real>(a, J, op, tile0, t, part, tab, red);
    }
    if constexpr (KIND == kPhaseB || KIND == kHalfOut) {
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            LayCtx<R> Lm;
            lay_ctx<R, CX != 0>(Lm, g, a.lat, tile0 + s, pl, t, true, op.basis);
            if constexpr (KIND == kPhaseB) {
                if (meas_norm) {
                    const double q = block_sum(sumsq<Real, R>(v[s]), red);
                    if (t == 0 && J.norm_part) gst(J.norm_part, tile0 + s, q);
                }
            }
            apply_phase<Real, R, NT == 2 ? 8 : 0>(v[s], Lm, op.basis, n, tab);
        }
    }
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        if constexpr (KIND == kPhaseB) {
            bwd_rot<Real, R, NL, CX>(v[s], lds, M);
        } else {
            if constexpr (NL > 1) xchg_rot_x<Real, R, 0, R * (NL - 1), CX>(v[s], lds, M.base[NL - 1], M.base[0]);
        }
        if constexpr (NT == 1) {
            // one tile: the store address is recomputed from an opaque copy
            // of the thread index rather than kept live through the pass
            // (two registers, which spill at the component exchange's
            // register limit).  Two-tile blocks keep it: the registers saved
            // there raise the number of resident blocks, which measured
            // slower on the strided rows they stream.
            uint32_t tt = t;
            asm volatile("" : "+v"(tt));
            LayCtx<R> Ls;
            lay_ctx<R, CX != 0>(Ls, g, a.lat, tile0 + s, x1 - R, tt, false);
            store_tile<Real, R, true, CX != 0>(v[s], st, Ls);
        } else {
            store_tile<Real, R, true, CX != 0>(v[s], st, L0[s]);
        }
    }
}

// KS: the pass kind every job of the launch has at this level (kPhaseB or
// kPlainH), or kAnyKind when the kinds differ or are rarer (half passes of
// the z-x-z order) and each block selects its job's kind.  When jobs are laid out at a uniform stride
// (a.jstride, elements; a.jmode 0) the tile loads are issued before the job
// record is read.
constexpr int kAnyKind = -1;

// KS kPhaseTab: every job of the launch has a phase pass (kPhaseB) and the
// level's table was precomputed for a single state (a.tabs, no per-job
// stride).  The block loads its share of the table before its tile loads,
// so the table's arrival does not wait behind the tile's, and writes it to
// LDS once the tile loads are in flight.
constexpr int kPhaseTab = 8;
constexpr int kTabPre = 3;  // table entries prefetched per thread

// NT: consecutive tiles per block (1, or 2 for strided groups whose tiles
// carry 128-byte rows: the two tiles of a block differ only in the lowest
// tile bit, so each block reads and writes 256 contiguous bytes per row).
template <typename Real, int R, int NL, int KS, int NT, int CX>
__device__ __forceinline__ void level_body(const LevelArgs &a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const GroupGeom &g = a.geom;
    const uint32_t t = threadIdx.x;
    constexpr int kNTlog = NT == 2 ? 1 : 0;
    const int blog = g.tiles_log2 - kNTlog;  // blocks per state = 2^blog
    const uint64_t bid = a.xcd ? xcd_major(blockIdx.x, gridDim.x) : blockIdx.x;
    const int jb = (int)(bid >> blog);
    const uint64_t tile0 = (bid & ((1ull << blog) - 1)) << kNTlog;
    Cx<Real> *base = reinterpret_cast<Cx<Real> *>(a.states);

    Cx<Real> v[NT][1 << R];
    LayCtx<R> L0[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) lay_ctx<R, CX != 0>(L0[s], g, a.lat, tile0 + s, g.x1 - R, t, false);
    // The tile loads are issued at one point of the code (two load sites
    // would hold registers for both and spill).  With a uniform job stride
    // (jmode 0) they go out before the job record is read; otherwise the
    // record (scalar loads) gives the state's offset first, and a block whose
    // job has no pass at this level returns before loading.
    Cx<Real> *st = base + a.jbase + (uint64_t)jb * a.jstride;
    // TP: one state's precomputed table; TA (any-kind kernels): a batch's
    // per-job tables, fetched ahead where the job record is read first
    constexpr bool TP = KS == kPhaseTab, TA = KS == kAnyKind;
    typedef typename Vec2<Real>::type TV;
    typedef const __attribute__((address_space(1))) TV *GTab;
    TV pre[TP || TA ? kTabPre : 1];
    bool prefetched = false;
    const int entries = (a.lat.nst + 1) * (a.lat.n + 1);
    if constexpr (TP) {
        const GTab src = (GTab)a.tabs + (size_t)(a.level - a.tab_lev0) * entries;
#pragma unroll
        for (int i = 0; i < kTabPre; ++i) {
            const int j = (int)t + i * (int)blockDim.x;
            if (j < entries) pre[i] = src[j];
        }
        prefetched = true;
    }
    JobDev J;
    LevelOp op;
    const bool early = a.jmode != 0;
    if (early) {
        const int jrec = a.jidx ? job_index(a.jidx, jb) : jb;
        J = job_record(a.jobs, jrec, a.job_inline);
        op = a.force_plain ? LevelOp{a.group, kPlainH, 0, -1, -1, 0, 0, 0}
                           : level_op(a.level - J.lev0, a.K, J.steps, J.k_begin, J.order);
        if (op.kind == kIdle || op.group != a.group) return;  // uniform per block
        st = base + J.offset;
        if constexpr (TA) {
            if (a.tabs && a.tab_stride && op.kind != kPlainH) {
                const GTab src = (GTab)((const __attribute__((address_space(1))) unsigned char *)a.tabs +
                                        (size_t)jrec * a.tab_stride) +
                                 (size_t)(a.level - J.lev0) * entries;
#pragma unroll
                for (int i = 0; i < kTabPre; ++i) {
                    const int j = (int)t + i * (int)blockDim.x;
                    if (j < entries) pre[i] = src[j];
                }
                prefetched = true;
            }
        }
    }
    load_tiles<Real, R, NT, CX != 0>(v, st, L0);
    if (!early) {
        J = job_record(a.jobs, a.jidx ? job_index(a.jidx, jb) : jb, a.job_inline);
        op = a.force_plain ? LevelOp{a.group, kPlainH, 0, -1, -1, 0, 0, 0}
                           : level_op(a.level - J.lev0, a.K, J.steps, J.k_begin, J.order);
        if (op.kind == kIdle || op.group != a.group) return;  // uniform per block
    }

    Cx<Real> *lds = reinterpret_cast<Cx<Real> *>(smem);
    const uint32_t lds_elems = (1u << (g.m - R * NL)) * (uint32_t)g.lds_blk;
    // the exchange region holds one element (CX: one component) per slot
    Cx<Real> *tab = CX ? align16<Cx<Real>>(reinterpret_cast<Real *>(smem) + lds_elems) : lds + lds_elems;
    const int W = a.lat.n + 1;
    double2 *fac = table_scratch(smem);
    double *red = align16<double>(tab + (a.lat.nst + 1) * W);

    int tab_done = 0;  // table entries already in LDS
    if constexpr (TP || TA) {
        if (prefetched) {
#pragma unroll
            for (int i = 0; i < kTabPre; ++i) {
                const int j = (int)t + i * (int)blockDim.x;
                if (j < entries) tab[j] = Cx<Real>{pre[i].x, pre[i].y};
            }
            const int done = kTabPre * (int)blockDim.x;
            tab_done = done < entries ? done : entries;
        }
    }
    if constexpr (TP) {
        pass_multi<Real, R, NL, kPhaseB, NT, CX, true>(a, J, op, jb, tile0, t, v, st, L0, lds, tab, fac, red, tab_done);
    } else if constexpr (KS != kAnyKind) {
        pass_multi<Real, R, NL, KS, NT, CX>(a, J, op, jb, tile0, t, v, st, L0, lds, tab, fac, red);
    } else {
        switch (op.kind) {
            case kPhaseB: pass_multi<Real, R, NL, kPhaseB, NT, CX, true>(a, J, op, jb, tile0, t, v, st, L0, lds, tab, fac, red, tab_done); break;
            case kPlainH: pass_multi<Real, R, NL, kPlainH, NT, CX, true>(a, J, op, jb, tile0, t, v, st, L0, lds, tab, fac, red); break;
            case kHalfIn: pass_multi<Real, R, NL, kHalfIn, NT, CX, true>(a, J, op, jb, tile0, t, v, st, L0, lds, tab, fac, red, tab_done); break;
            default: pass_multi<Real, R, NL, kHalfOut, NT, CX, true>(a, J, op, jb, tile0, t, v, st, L0, lds, tab, fac, red, tab_done); break;
        }
    }
}

template <typename Real, int R, int NL, int KS, int NT>
__global__ void __launch_bounds__(512) level_kernel_full(LevelArgs a) {
    level_body<Real, R, NL, KS, NT, 0>(a);
}

// One tile per workgroup with the component exchange: two workgroups per CU
// (complex64: four waves per SIMD, so at most 128 registers per thread).
template <typename Real, int R, int NL, int KS>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 ? 4 : 2)))
level_kernel_cx(LevelArgs a) {
    level_body<Real, R, NL, KS, 1, 1>(a);
}

// Phase tables of levels lev0 + blockIdx.x of one job, written to global
// memory in the layout of the LDS table (one block per level; plain levels
// leave their slot unwritten).
template <typename Real>
__global__ void __launch_bounds__(256) tables_kernel(TablesArgs a) {
    __shared__ double2 fac[kMaxStab + 1 + kMaxN + 1];
    const JobDev J = a.jobs ? job_record(a.jobs, (int)blockIdx.y, a.job) : a.job;
    const int lev = a.lev0 + (int)blockIdx.x;
    const LevelOp op = level_op(lev, a.K, J.steps, J.k_begin, J.order);
    if (op.kind == kIdle || op.kind == kPlainH) return;  // uniform per block
    const int nst = a.lat.nst, n = a.lat.n;
    double alpha, beta;
    phase_angles(J, op, alpha, beta);
    table_factors(fac, nst, n, alpha, beta);
    unsigned char *base = reinterpret_cast<unsigned char *>(a.tabs) + (size_t)blockIdx.y * a.stride;
    Cx<Real> *tab = reinterpret_cast<Cx<Real> *>(base) + (size_t)blockIdx.x * (nst + 1) * (n + 1);
    table_products<Real>(tab, fac, nst, n, op.basis ? ldexp(1.0, -n) : 1.0);
}

hipError_t launch_tables(bool c128, const TablesArgs &a, unsigned nlevels, hipStream_t s, unsigned njobs) {
    if (nlevels == 0 || njobs == 0) return hipSuccess;
    if (c128)
        hipLaunchKernelGGL(tables_kernel<double>, dim3(nlevels, njobs), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(tables_kernel<float>, dim3(nlevels, njobs), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- resident kernel
//
// Whole ramp of a small lattice inside one workgroup: the state never leaves
// registers between steps.  Same operation order, angles and renormalization
// rule as the level sequence of the pass kernels.  The whole state is one
// group of NL * R = n transformed bits.

template <typename Real, int R, int NL>
__global__ void __launch_bounds__(512) resident_kernel(ResidentArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const GroupGeom &g = a.geom;
    const uint32_t t = threadIdx.x;
    const JobDev J = job_record(a.jobs, a.job0 + blockIdx.x, a.job_inline);
    const int S = J.steps, k0 = J.k_begin;
    if (S <= 0) return;
    const int n = a.lat.n, nst = a.lat.nst, W = n + 1;
    const int x1 = g.x1, p0 = x1 - R, pl = x1 - R * NL;

    Cx<Real> *lds = reinterpret_cast<Cx<Real> *>(smem);
    const uint32_t lds_elems = (1u << g.m) + (1u << (g.m - R));
    Cx<Real> *tab = lds + lds_elems;
    double2 *fac = table_scratch(smem);
    double *red = align16<double>(tab + (nst + 1) * W);

    Cx<Real> v[1 << R];
    Cx<Real> *st = reinterpret_cast<Cx<Real> *>(a.states) + J.offset;
    LayCtx<R> L0, Lt;
    lay_ctx<R>(L0, g, a.lat, 0, p0, t, true);
    lay_ctx<R>(Lt, g, a.lat, 0, pl, t, true);
    load_tile<Real, R>(v, st, L0);

    double last_norm = 1.0;
    const double two_mn = ldexp(1.0, -n);

    // outer (Hadamard-basis) phase: transform, phase, transform back
    auto outer = [&](const LevelOp &op, bool have_norm) {
        double alpha, beta;
        phase_angles(J, op, alpha, beta);
        double scale = two_mn;
        if (op.renorm && have_norm) {
            if (J.renorm) scale *= 1.0 / sqrt(last_norm);
            if (t == 0 && J.norm_trace) gst(J.norm_trace, op.ka - k0, last_norm);
        }
        build_table<Real>(tab, fac, nst, n, alpha, beta, scale);
        fwd_full<Real, R, NL>(v, lds, x1, t);
        apply_phase<Real, R>(v, Lt, 1, n, tab);
        bwd_full<Real, R, NL>(v, lds, x1, t);
    };
    // inner (computational-basis) phase, with the norm measured first
    auto inner = [&](const LevelOp &op) {
        double alpha, beta;
        phase_angles(J, op, alpha, beta);
        if (op.norm) last_norm = block_sum(sumsq<Real, R>(v), red);
        build_table<Real>(tab, fac, nst, n, alpha, beta, 1.0);
        apply_phase<Real, R>(v, L0, 0, n, tab);
    };

    // The level sequence with K = 2 groups, walked in its fixed pattern:
    // order 0: X(0) [Z(j) X(j+1)] ..., order 1: Z(0) [X(j) Z(j+1)] ...
    const int P = 2;
    if (J.order == 0) {
        outer(level_op(1, 2, S, k0, 0), false);
        for (int j = 1; j <= S; ++j) {
            inner(level_op(P * j, 2, S, k0, 0));
            outer(level_op(P * j + 1, 2, S, k0, 0), true);
        }
    } else {
        inner(level_op(0, 2, S, k0, 1));
        for (int j = 0; j < S; ++j) {
            outer(level_op(P * j + 1, 2, S, k0, 1), true);
            inner(level_op(P * (j + 1), 2, S, k0, 1));
        }
    }
    store_tile<Real, R>(v, st, L0);
}

// ---------------------------------------------------------------- adjoint
//
// Reverse evolution for the gradient of <psi_M|H|psi_M> with respect to the
// per-step schedule values.  Every forward level is undone on psi and on the
// adjoint state lambda = H psi_M with the same transforms and the conjugate
// phase (the level's real scale factor is kept, so the scale bookkeeping of
// the unnormalized transforms matches the forward sweep).  At a diagonal
// level the sum Im sum_i conj(lambda_i) D_i psi_i is reduced in FP64, with
// D = dH/ds diagonal in that basis.

template <typename Real, int R>
__device__ __forceinline__ double adj_reduce(const Cx<Real> (&a)[1 << R], const Cx<Real> (&b)[1 << R],
                                             const LayCtx<R> &L, int basis, int nst, int n, double dJ, double dh) {
    uint32_t s = basis ? L.s0x : L.s0z;
    double acc = 0.0;
#pragma unroll
    for (int idx = 0; idx < (1 << R); ++idx) {
        const int q = idx ^ (idx >> 1);
        if (idx) s ^= basis ? L.lx[__builtin_ctz(idx)] : L.lz[__builtin_ctz(idx)];
        const double im = (double)b[q].x * (double)a[q].y - (double)b[q].y * (double)a[q].x;
        const int k = popc(s), w = L.w0 + __builtin_popcount(q);
        acc += (dJ * (double)(nst - 2 * k) + dh * (double)(n - 2 * w)) * im;
    }
    return acc;
}

// Real diagonal table T[k][w] = scale (dJ (nst - 2k) + dh (n - 2w)), FP64 cast.
template <typename Real>
__device__ void build_diag_table(Cx<Real> *tab, int nst, int n, double dJ, double dh, double scale) {
    const int W = n + 1;
    for (int j = threadIdx.x; j < (nst + 1) * W; j += blockDim.x) {
        const int k = j / W, w = j - k * W;
        tab[j] = Cx<Real>{(Real)(scale * (dJ * (double)(nst - 2 * k) + dh * (double)(n - 2 * w))), (Real)0};
    }
    __syncthreads();
}

template <typename Real, int R, int NL>
__global__ void __launch_bounds__(512) adj_kernel(AdjArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const GroupGeom &g = a.geom;
    const uint32_t t = threadIdx.x;
    const uint64_t tile = blockIdx.x;
    const int n = a.lat.n, nst = a.lat.nst, W = n + 1;
    Cx<Real> *lds = reinterpret_cast<Cx<Real> *>(smem);
    const uint32_t lds_elems = (1u << g.m) + (1u << (g.m - R));
    Cx<Real> *tab = lds + lds_elems;
    double2 *fac = table_scratch(smem);
    double *red = align16<double>(tab + (nst + 1) * W);
    const int x1 = g.x1, p0 = x1 - R, pl = x1 - R * NL;
    Cx<Real> *A = reinterpret_cast<Cx<Real> *>(a.A);
    Cx<Real> *B = reinterpret_cast<Cx<Real> *>(a.B);
    LayCtx<R> L0, Lm;
    lay_ctx<R, true>(L0, g, a.lat, tile, p0, t, true);
    lay_ctx<R, true>(Lm, g, a.lat, tile, a.no_transform ? p0 : pl, t, true);
    Cx<Real> va[1 << R], vb[1 << R];

    if (a.mode == 0) {
        load_tile<Real, R, false, true>(va, A, L0);
        fwd_full<Real, R, NL>(va, lds, x1, t);
        if (NL > 1) xchg<Real, R>(va, lds, pl, p0, t);
        store_tile<Real, R, false, true>(va, A, L0);
        if (B) {
            load_tile<Real, R, false, true>(vb, B, L0);
            fwd_full<Real, R, NL>(vb, lds, x1, t);
            if (NL > 1) xchg<Real, R>(vb, lds, pl, p0, t);
            store_tile<Real, R, false, true>(vb, B, L0);
        }
        return;
    }
    if (a.mode == 2) {
        build_diag_table<Real>(tab, nst, n, a.dJ, a.dh, a.dscale);
        load_tile<Real, R, false, true>(va, A, L0);
        if (!a.no_transform) fwd_full<Real, R, NL>(va, lds, x1, t);
        apply_phase<Real, R>(va, Lm, a.op.basis, n, tab);
        if (!a.no_transform) bwd_full<Real, R, NL>(va, lds, x1, t);
        store_tile<Real, R, false, true>(va, B, L0);
        return;
    }
    // mode 1: undo a diagonal level on both states, reducing the gradient
    {
        double alpha, beta;
        phase_angles(a.job, a.op, alpha, beta);
        const double scale = a.op.basis ? ldexp(1.0, -n) : 1.0;
        build_table<Real>(tab, fac, nst, n, -alpha, -beta, scale);
    }
    load_tile<Real, R, false, true>(va, A, L0);
    load_tile<Real, R, false, true>(vb, B, L0);
    if (!a.no_transform) {
        fwd_full<Real, R, NL>(va, lds, x1, t);
        fwd_full<Real, R, NL>(vb, lds, x1, t);
    }
    const double acc = block_sum(adj_reduce<Real, R>(va, vb, Lm, a.op.basis, nst, n, a.dJ, a.dh), red);
    if (t == 0 && a.part) a.part[tile] = acc;
    apply_phase<Real, R>(va, Lm, a.op.basis, n, tab);
    apply_phase<Real, R>(vb, Lm, a.op.basis, n, tab);
    if (!a.no_transform) bwd_full<Real, R, NL>(va, lds, x1, t);
    store_tile<Real, R, false, true>(va, A, L0);
    if (!a.no_transform) bwd_full<Real, R, NL>(vb, lds, x1, t);
    store_tile<Real, R, false, true>(vb, B, L0);
}

// Sum of one level's per-block partials (fixed order).
__global__ void adj_final_kernel(AdjFinalArgs a) {
    __shared__ double red[16];
    double s = 0.0;
    for (int j = threadIdx.x; j < a.np; j += blockDim.x) s += a.part[j];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *a.out = s;
}

// Gradient of each schedule value from the level sums (x-z-x order): the
// z part of step k sits at inner visit k + 1, its two x halves at outer
// visits k and k + 1.
__global__ void adj_grad_kernel(AdjGradArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.S) return;
    const int inner = a.P * (k + 1);
    const int outer0 = (a.K - 1) + a.P * k, outer1 = (a.K - 1) + a.P * (k + 1);
    a.gZ[k] = 2.0 * a.dt * a.level_sum[inner] * a.inv_norm;
    a.gX[k] = a.dt * ldexp(1.0, -a.n) * (a.level_sum[outer0] + a.level_sum[outer1]) * a.inv_norm;
}

template <typename Real>
__global__ void axpy_kernel(Cx<Real> *y, const Cx<Real> *x, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        y[i] = cadd(y[i], x[i]);
}

// ---------------------------------------------------------------- observables

// Per-thread accumulation of one basis' observables for the elements in
// registers: [0] sum |a|^2, [1] sum |a|^2 (nst - 2k), [2] sum |a|^2 (n - 2w),
// [3..10] loop parities, [11..11+n] weight histogram (computational basis).
template <typename Real, int R>
__device__ __forceinline__ void obs_accum(const Cx<Real> (&v)[1 << R], const LayCtx<R> &L,
                                          int basis, const LatticeDev &lat, const uint32_t *loops,
                                          int nloops, bool dos, double *acc) {
    uint32_t s = basis ? L.s0x : L.s0z;
    double dl[R + 1];
#pragma unroll
    for (int j = 0; j <= R; ++j) dl[j] = 0.0;
    uint32_t lp[kMaxLoops];
#pragma unroll
    for (int j = 0; j < kMaxLoops; ++j) lp[j] = j < nloops ? (popc((uint32_t)L.i0 & loops[j]) & 1) : 0;
#pragma unroll
    for (int idx = 0; idx < (1 << R); ++idx) {
        const int q = idx ^ (idx >> 1);
        if (idx) {
            const int r = __builtin_ctz(idx);
            s ^= basis ? L.lx[r] : L.lz[r];
#pragma unroll
            for (int j = 0; j < kMaxLoops; ++j)
                if (j < nloops) lp[j] ^= (loops[j] >> reg_bit(L, r)) & 1u;
        }
        const double p2 = (double)v[q].x * (double)v[q].x + (double)v[q].y * (double)v[q].y;
        const int k = popc(s);
        const int w = L.w0 + __builtin_popcount(q);
        acc[0] += p2;
        acc[1] += p2 * (double)(lat.nst - 2 * k);
        acc[2] += p2 * (double)(lat.n - 2 * w);
#pragma unroll
        for (int j = 0; j < kMaxLoops; ++j)
            if (j < nloops) acc[3 + j] += lp[j] ? -p2 : p2;
        dl[__builtin_popcount(q)] += p2;
    }
    if (dos) {
#pragma unroll
        for (int b = 0; b < kDosBins; ++b) {
            double x = 0.0;
#pragma unroll
            for (int j = 0; j <= R; ++j) x += (L.w0 + j == b) ? dl[j] : 0.0;
            acc[11 + b] += x;
        }
    }
}

template <typename Real, int R>
__global__ void __launch_bounds__(512) obs_kernel(ObsArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const GroupGeom &g = a.geom;
    const uint32_t t = threadIdx.x;
    const int job = blockIdx.y;
    const uint64_t tiles = 1ull << g.tiles_log2;
    Cx<Real> *lds = reinterpret_cast<Cx<Real> *>(smem);
    const uint32_t lds_elems = (1u << g.m) + (1u << (g.m - R));
    double *red = reinterpret_cast<double *>(lds + lds_elems);
    const Cx<Real> *src = reinterpret_cast<const Cx<Real> *>(a.src) + (a.src_off ? a.src_off[job] : 0);
    Cx<Real> *dst = a.dst ? reinterpret_cast<Cx<Real> *>(a.dst) + (a.dst_off ? a.dst_off[job] : 0) : nullptr;

    constexpr int NA = 11 + kDosBins;
    double accz[NA], accx[11];
#pragma unroll
    for (int j = 0; j < NA; ++j) accz[j] = 0.0;
#pragma unroll
    for (int j = 0; j < 11; ++j) accx[j] = 0.0;

    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        Cx<Real> v[1 << R];
        LayCtx<R> L0;
        lay_ctx<R, true>(L0, g, a.lat, tile, g.p[0], t, a.redZ != 0);
        load_tile<Real, R, false, true>(v, src, L0);
        if (a.redZ) obs_accum<Real, R>(v, L0, 0, a.lat, a.zloops, a.nz, true, accz);
        int cur = 0;
        if (a.doH) {
            for (int j = 0; j < g.nlay; ++j) {
                if (j > 0) exchange<Real, R>(v, lds, g.p[j - 1], g.p[j], t);
                butterflies<Real, R>(v, g.blo[j], g.bhi[j]);
                cur = j;
            }
        }
        if (a.redX) {
            LayCtx<R> Lm;
            lay_ctx<R, true>(Lm, g, a.lat, tile, g.p[cur], t, true);
            obs_accum<Real, R>(v, Lm, 1, a.lat, a.xloops, a.nx, false, accx);
        }
        if (dst) {
            if (cur != 0) exchange<Real, R>(v, lds, g.p[cur], g.p[0], t);
            store_tile<Real, R, false, true>(v, dst, L0);
        }
    }
    const size_t rec = ((size_t)job * gridDim.x + blockIdx.x) * kObsQ;
    if (a.redZ && a.part_z) {
        for (int j = 0; j < NA; ++j) {
            const double s = block_sum(accz[j], red);
            if (t == 0) a.part_z[rec + j] = s;
        }
    }
    if (a.redX && a.part_x) {
        for (int j = 0; j < 11; ++j) {
            const double s = block_sum(accx[j], red);
            if (t == 0) a.part_x[rec + j] = s;
        }
    }
}

// Sum the per-workgroup records of every job and form the observables.
__global__ void obs_finalize_kernel(FinalArgs a) {
    const int job = blockIdx.x;
    const int t = threadIdx.x;
    __shared__ double sz[kObsQ], sx[kObsQ];
    if (t < kObsQ) {
        double s = 0.0, x = 0.0;
        const double *pz = a.partZ + (size_t)job * a.nrecZ * kObsQ;
        const double *px = a.partX + (size_t)job * a.nrecX * kObsQ;
        for (int r = 0; r < a.nrecZ; ++r) s += pz[(size_t)r * kObsQ + t];
        for (int r = 0; r < a.nrecX; ++r) x += px[(size_t)r * kObsQ + t];
        sz[t] = s;
        sx[t] = x;
    }
    __syncthreads();
    if (t == 0) {
        const int n = a.n;
        double *o = a.out + (size_t)(a.out_index ? a.out_index[job] : job) * kObsQ;
        const double *c = a.H ? a.H + 4 * job : a.H_inline;
        const double nz = sz[0], nxr = sx[0];
        const double sumB = sz[1] / nz, mz = sz[2] / (n * nz);
        const double sumA = sx[1] / nxr, mx = sx[2] / (n * nxr);
        o[0] = nz;
        o[2] = sumA;
        o[3] = sumB;
        o[4] = mx;
        o[5] = mz;
        o[1] = -c[0] * sumA - c[1] * sumB - c[2] * n * mx - c[3] * n * mz;
        for (int j = 0; j < kMaxLoops; ++j) {
            o[6 + j] = sz[3 + j] / nz;
            o[14 + j] = sx[3 + j] / nxr;
        }
        for (int b = 0; b < kDosBins; ++b) o[22 + b] = sz[11 + b] / nz;
        o[55] = nxr * ldexp(1.0, -n);
    }
}

// ---------------------------------------------------------------- init / misc

template <typename Real>
__global__ void init_kernel(InitArgs a) {
    const InitJob J = a.jobs ? a.jobs[blockIdx.y] : a.one_job;
    Cx<Real> *st = reinterpret_cast<Cx<Real> *>(a.states) + J.offset;
    const uint64_t N = 1ull << a.lat.n;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (J.kind == 0) {
            v = syndrome_direct(a.lat.zmask, a.lat.nst, i) == 0 ? J.amp : 0.0;
        } else if (J.kind == 1) {
            v = syndrome_direct(a.lat.xmask, a.lat.nst, i) == 0 ? J.amp : 0.0;
        } else if (J.kind == 2) {
            v = i == 0 ? 1.0 : 0.0;
        } else {
            v = J.amp;
        }
        st[i] = Cx<Real>{(Real)v, (Real)0};
    }
}

// In-place sum of each job's partial norms into entry 0 (fixed order).
// Norm of a z pass with more block partials than a pass kernel should read:
// stage 1 sums chunks of kReduceChunk partials (block x of job y) into the
// slots after the partials, stage 2 sums the slots into partial 0.  Fixed
// summation order, so results do not depend on scheduling.
__global__ void reduce_parts_stage1(const JobDev *jobs, JobDev inl, int parts) {
    __shared__ double red[16];
    const JobDev J = job_record(jobs, blockIdx.y, inl);
    if (!J.norm_part) return;
    const int lo = blockIdx.x * kReduceChunk;
    const int hi = min(parts, lo + kReduceChunk);
    double s = 0.0;
    for (int j = lo + (int)threadIdx.x; j < hi; j += blockDim.x) s += gld(J.norm_part, j);
    s = block_sum(s, red);
    if (threadIdx.x == 0) gst(J.norm_part, parts + blockIdx.x, s);
}

__global__ void reduce_parts_stage2(const JobDev *jobs, JobDev inl, int parts, int chunks) {
    __shared__ double red[16];
    const JobDev J = job_record(jobs, blockIdx.x, inl);
    if (!J.norm_part) return;
    double s = 0.0;
    for (int j = (int)threadIdx.x; j < chunks; j += blockDim.x) s += gld(J.norm_part, parts + j);
    s = block_sum(s, red);
    if (threadIdx.x == 0) gst(J.norm_part, 0, s);
}

// ---------------------------------------------------------------- launchers

// Raise the dynamic-LDS limit of a kernel once to the largest block any plan
// uses, so that no attribute call happens while a stream is being captured.
static std::mutex g_lds_mu;
static std::set<const void *> g_lds_done;

static hipError_t set_lds(const void *fn, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_lds_mu);
    if (g_lds_done.count(fn)) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e == hipSuccess) g_lds_done.insert(fn);
    return e;
}

template <typename Real, int R, bool NT>
static hipError_t do_level_nt(const LevelArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    if (a.geom.hi) {  // a group in two runs of qubits: the kernel with their address map
        const void *fs = reinterpret_cast<const void *>(&level_kernel<Real, R, NT, true>);
        hipError_t e = set_lds(fs, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((level_kernel<Real, R, NT, true>), grid, dim3(1u << (a.geom.m - R)), lds, s, a);
        return hipGetLastError();
    }
    const void *fn = reinterpret_cast<const void *>(&level_kernel<Real, R, NT>);
    hipError_t e = set_lds(fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((level_kernel<Real, R, NT>), grid, dim3(1u << (a.geom.m - R)), lds, s, a);
    return hipGetLastError();
}

template <typename Real, int R, int NL, int KS, int NT>
static hipError_t do_level_full_ks(const LevelArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    const void *fn = reinterpret_cast<const void *>(&level_kernel_full<Real, R, NL, KS, NT>);
    hipError_t e = set_lds(fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((level_kernel_full<Real, R, NL, KS, NT>), grid, dim3(1u << (a.geom.m - R)), lds, s, a);
    return hipGetLastError();
}

template <typename Real, int R, int NL, int NT>
static hipError_t do_level_full_nt(const LevelArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    // precomputed tables: one state's tables are prefetched by the phase
    // kernels compiled for them; per-job tables are read by the any-kind kernels
    if (a.kind_hint == kPhaseB && !a.tabs) return do_level_full_ks<Real, R, NL, kPhaseB, NT>(a, grid, lds, s);
    if (a.kind_hint == kPhaseB && !a.tab_stride) return do_level_full_ks<Real, R, NL, kPhaseTab, NT>(a, grid, lds, s);
    if (a.kind_hint == kPlainH) return do_level_full_ks<Real, R, NL, kPlainH, NT>(a, grid, lds, s);
    return do_level_full_ks<Real, R, NL, kAnyKind, NT>(a, grid, lds, s);
}

// Shapes with a two-tile variant (complex64 only: two register windows of
// 2^R complex doubles would not fit the register budget).
#define Z2H_PAIR_SHAPES(X) X(5, 2) X(4, 2) X(4, 3) X(3, 2) X(3, 3)

// Shapes with a component-exchange variant (one tile per workgroup).
#define Z2H_CX_SHAPES(X) X(5, 2)

template <typename Real, int R, int NL, int KS>
static hipError_t do_level_cx_ks(const LevelArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    const void *fn = reinterpret_cast<const void *>(&level_kernel_cx<Real, R, NL, KS>);
    hipError_t e = set_lds(fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((level_kernel_cx<Real, R, NL, KS>), grid, dim3(1u << (a.geom.m - R)), lds, s, a);
    return hipGetLastError();
}

template <typename Real, int R, int NL>
static hipError_t do_level_full(const LevelArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    if (a.geom.cx) {
#define Z2H_CX_CALL(r, nl)                                                                               \
        if (R == r && NL == nl) {                                                                        \
            if (a.kind_hint == kPhaseB && (!a.tabs || !a.tab_stride)) return do_level_cx_ks<Real, r, nl, kPhaseB>(a, grid, lds, s); \
            if (a.kind_hint == kPlainH) return do_level_cx_ks<Real, r, nl, kPlainH>(a, grid, lds, s);    \
            return do_level_cx_ks<Real, r, nl, kAnyKind>(a, grid, lds, s);                               \
        }
        Z2H_CX_SHAPES(Z2H_CX_CALL)
#undef Z2H_CX_CALL
        return hipErrorInvalidValue;
    }
    if (a.geom.pair == 2) {
        if constexpr (sizeof(Real) == 4) {
#define Z2H_PAIR_CALL(r, nl) \
            if (R == r && NL == nl) return do_level_full_nt<Real, r, nl, 2>(a, dim3(grid.x / 2), lds, s);
            Z2H_PAIR_SHAPES(Z2H_PAIR_CALL)
#undef Z2H_PAIR_CALL
        }
        return hipErrorInvalidValue;
    }
    return do_level_full_nt<Real, R, NL, 1>(a, grid, lds, s);
}

bool cx_level_ok(int R, int NL) {
#define Z2H_OK_CX(r, nl) if (R == r && NL == nl) return true;
    Z2H_CX_SHAPES(Z2H_OK_CX)
#undef Z2H_OK_CX
    return false;
}

bool pair_level_ok(bool c128, int R, int NL) {
    if (c128) return false;
#define Z2H_OK_PAIR(r, nl) if (R == r && NL == nl) return true;
    Z2H_PAIR_SHAPES(Z2H_OK_PAIR)
#undef Z2H_OK_PAIR
    return false;
}

// (R, NL) shapes compiled as straight-line kernels.
#define Z2H_FULL_LEVEL_SHAPES(X) \
    X(5, 1) X(5, 2) X(5, 3) X(4, 1) X(4, 2) X(4, 3) X(3, 1) X(3, 2) X(3, 3) X(2, 2) X(2, 3) X(2, 4)
#define Z2H_FULL_RESIDENT_SHAPES(X) X(2, 4) X(4, 2) X(4, 3) X(3, 4) X(5, 2)
#define Z2H_ADJ_SHAPES(X) Z2H_FULL_LEVEL_SHAPES(X) X(3, 4)

bool full_level_ok(int R, int NL) {
#define Z2H_OK_SHAPE(r, nl) if (R == r && NL == nl) return true;
    Z2H_FULL_LEVEL_SHAPES(Z2H_OK_SHAPE)
    return false;
}

bool full_resident_ok(int R, int NL) {
    Z2H_FULL_RESIDENT_SHAPES(Z2H_OK_SHAPE)
#undef Z2H_OK_SHAPE
    return false;
}

template <typename Real>
static hipError_t level_full_dispatch(const LevelArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    const int R = a.geom.R, NL = a.geom.full;
#define Z2H_CALL_SHAPE(r, nl) \
    if (R == r && NL == nl) return do_level_full<Real, r, nl>(a, grid, lds, s);
    Z2H_FULL_LEVEL_SHAPES(Z2H_CALL_SHAPE)
#undef Z2H_CALL_SHAPE
    return hipErrorInvalidValue;
}

template <typename Real, int R>
static hipError_t do_level(const LevelArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    if (a.geom.m - R < 6 || a.geom.m - R > 9) return hipErrorInvalidConfiguration;  // launch bounds
    if (a.geom.full) return level_full_dispatch<Real>(a, grid, lds, s);
    return a.nt ? do_level_nt<Real, R, true>(a, grid, lds, s) : do_level_nt<Real, R, false>(a, grid, lds, s);
}

template <typename Real, int R, int NL>
static hipError_t do_resident_shape(const ResidentArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    const void *fn = reinterpret_cast<const void *>(&resident_kernel<Real, R, NL>);
    hipError_t e = set_lds(fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((resident_kernel<Real, R, NL>), grid, dim3(1u << (a.geom.m - R)), lds, s, a);
    return hipGetLastError();
}

template <typename Real, int R>
static hipError_t do_resident(const ResidentArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    if (a.geom.m - R < 6 || a.geom.m - R > 9) return hipErrorInvalidConfiguration;  // launch bounds
    const int NL = a.geom.full;
#define Z2H_CALL_SHAPE(r, nl) \
    if (R == r && NL == nl) return do_resident_shape<Real, r, nl>(a, grid, lds, s);
    Z2H_FULL_RESIDENT_SHAPES(Z2H_CALL_SHAPE)
#undef Z2H_CALL_SHAPE
    return hipErrorInvalidValue;
}

template <typename Real, int R>
static hipError_t do_obs(const ObsArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    if (a.geom.m - R < 6 || a.geom.m - R > 9) return hipErrorInvalidConfiguration;  // launch bounds
    const void *fn = reinterpret_cast<const void *>(&obs_kernel<Real, R>);
    hipError_t e = set_lds(fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((obs_kernel<Real, R>), grid, dim3(1u << (a.geom.m - R)), lds, s, a);
    return hipGetLastError();
}

#define Z2H_DISPATCH(FN, ARGS, GRID, LDS, S)                               \
    do {                                                                   \
        if (c128) {                                                        \
            switch (R) {                                                   \
                case 2: return FN<double, 2>(ARGS, GRID, LDS, S);          \
                case 3: return FN<double, 3>(ARGS, GRID, LDS, S);          \
                case 4: return FN<double, 4>(ARGS, GRID, LDS, S);          \
                case 5: return FN<double, 5>(ARGS, GRID, LDS, S);          \
            }                                                              \
        } else {                                                           \
            switch (R) {                                                   \
                case 2: return FN<float, 2>(ARGS, GRID, LDS, S);           \
                case 3: return FN<float, 3>(ARGS, GRID, LDS, S);           \
                case 4: return FN<float, 4>(ARGS, GRID, LDS, S);           \
                case 5: return FN<float, 5>(ARGS, GRID, LDS, S);           \
            }                                                              \
        }                                                                  \
        return hipErrorInvalidValue;                                       \
    } while (0)

template <typename Real>
static hipError_t prep_real() {
    hipError_t e = hipSuccess;
#define Z2H_PREP_GEN(r)                                                                                   \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel<Real, r, false>), kMaxLdsBytes); \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel<Real, r, true>), kMaxLdsBytes);  \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&obs_kernel<Real, r>), kMaxLdsBytes);
    Z2H_PREP_GEN(2) Z2H_PREP_GEN(3) Z2H_PREP_GEN(4) Z2H_PREP_GEN(5)
#undef Z2H_PREP_GEN
#define Z2H_PREP_FULL(r, nl) \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel_full<Real, r, nl, kAnyKind, 1>), kMaxLdsBytes); \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel_full<Real, r, nl, kPhaseB, 1>), kMaxLdsBytes); \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel_full<Real, r, nl, kPhaseTab, 1>), kMaxLdsBytes); \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel_full<Real, r, nl, kPlainH, 1>), kMaxLdsBytes);
    Z2H_FULL_LEVEL_SHAPES(Z2H_PREP_FULL)
#undef Z2H_PREP_FULL
    if constexpr (sizeof(Real) == 4) {
#define Z2H_PREP_PAIR(r, nl) \
        if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel_full<Real, r, nl, kAnyKind, 2>), kMaxLdsBytes); \
        if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel_full<Real, r, nl, kPhaseB, 2>), kMaxLdsBytes); \
        if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel_full<Real, r, nl, kPhaseTab, 2>), kMaxLdsBytes); \
        if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel_full<Real, r, nl, kPlainH, 2>), kMaxLdsBytes);
        Z2H_PAIR_SHAPES(Z2H_PREP_PAIR)
#undef Z2H_PREP_PAIR
    }
#define Z2H_PREP_CX(r, nl) \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel_cx<Real, r, nl, kAnyKind>), kMaxLdsBytes); \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel_cx<Real, r, nl, kPhaseB>), kMaxLdsBytes); \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&level_kernel_cx<Real, r, nl, kPlainH>), kMaxLdsBytes);
    Z2H_CX_SHAPES(Z2H_PREP_CX)
#undef Z2H_PREP_CX
#define Z2H_PREP_RES(r, nl) \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&resident_kernel<Real, r, nl>), kMaxLdsBytes);
    Z2H_FULL_RESIDENT_SHAPES(Z2H_PREP_RES)
#undef Z2H_PREP_RES
    return e;
}

hipError_t prepare_kernels() {
#define Z2H_PREP_ADJ(r, nl)                                                                               \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&adj_kernel<float, r, nl>), kMaxLdsBytes); \
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void *>(&adj_kernel<double, r, nl>), kMaxLdsBytes);
    hipError_t e = hipSuccess;
    Z2H_ADJ_SHAPES(Z2H_PREP_ADJ)
#undef Z2H_PREP_ADJ
    if (e == hipSuccess) e = prep_real<float>();
    if (e == hipSuccess) e = prep_real<double>();
    return e;
}

hipError_t launch_level(bool c128, int R, const LevelArgs &a, unsigned nblocks, size_t lds,
                        hipStream_t s) {
    Z2H_DISPATCH(do_level, a, dim3(nblocks), lds, s);
}

hipError_t launch_resident(bool c128, int R, const ResidentArgs &a, unsigned njobs, size_t lds,
                           hipStream_t s) {
    Z2H_DISPATCH(do_resident, a, dim3(njobs), lds, s);
}

hipError_t launch_obs(bool c128, int R, const ObsArgs &a, unsigned workers, unsigned njobs,
                      size_t lds, hipStream_t s) {
    Z2H_DISPATCH(do_obs, a, dim3(workers, njobs), lds, s);
}

hipError_t launch_obs_finalize(const FinalArgs &a, unsigned njobs, hipStream_t s) {
    hipLaunchKernelGGL(obs_finalize_kernel, dim3(njobs), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init(bool c128, const InitArgs &a, unsigned njobs, hipStream_t s) {
    const uint64_t N = 1ull << a.lat.n;
    uint64_t blocks = (N + 255) / 256;
    const uint64_t cap = njobs > 64 ? 64 : 4096;
    if (blocks > cap) blocks = cap;
    if (c128)
        hipLaunchKernelGGL(init_kernel<double>, dim3((unsigned)blocks, njobs), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(init_kernel<float>, dim3((unsigned)blocks, njobs), dim3(256), 0, s, a);
    return hipGetLastError();
}

bool adj_shape_ok(int R, int NL) {
#define Z2H_OK_SHAPE(r, nl) if (R == r && NL == nl) return true;
    Z2H_ADJ_SHAPES(Z2H_OK_SHAPE)
#undef Z2H_OK_SHAPE
    return false;
}

template <typename Real, int R, int NL>
static hipError_t do_adj(const AdjArgs &a, unsigned nblocks, size_t lds, hipStream_t s) {
    const void *fn = reinterpret_cast<const void *>(&adj_kernel<Real, R, NL>);
    hipError_t e = set_lds(fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((adj_kernel<Real, R, NL>), dim3(nblocks), dim3(1u << (a.geom.m - R)), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_adj(bool c128, const AdjArgs &a, unsigned nblocks, size_t lds, hipStream_t s) {
    const int R = a.geom.R, NL = a.geom.full;
    if (a.geom.m - R < 6 || a.geom.m - R > 9) return hipErrorInvalidConfiguration;  // launch bounds
#define Z2H_CALL_SHAPE(r, nl)                                                                  \
    if (R == r && NL == nl)                                                                    \
        return c128 ? do_adj<double, r, nl>(a, nblocks, lds, s) : do_adj<float, r, nl>(a, nblocks, lds, s);
    Z2H_ADJ_SHAPES(Z2H_CALL_SHAPE)
#undef Z2H_CALL_SHAPE
    return hipErrorInvalidValue;
}

hipError_t launch_adj_final(const AdjFinalArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(adj_final_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_grad(const AdjGradArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(adj_grad_kernel, dim3((a.S + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_axpy(bool c128, void *y, const void *x, uint64_t n, hipStream_t s) {
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (c128)
        hipLaunchKernelGGL(axpy_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<Cx<double> *>(y), reinterpret_cast<const Cx<double> *>(x), n);
    else
        hipLaunchKernelGGL(axpy_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<Cx<float> *>(y), reinterpret_cast<const Cx<float> *>(x), n);
    return hipGetLastError();
}

LevelOp level_op_host(int lev, int K, int S, int k0, int order) {
    return level_op(lev, K, S, k0, order);
}

hipError_t launch_reduce_parts(const JobDev *jobs, const JobDev &inl, int njobs, int parts,
                               hipStream_t s) {
    const int chunks = (parts + kReduceChunk - 1) / kReduceChunk;  // slots after the partials (norm_parts)
    hipLaunchKernelGGL(reduce_parts_stage1, dim3(chunks, njobs), dim3(256), 0, s, jobs, inl, parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_parts_stage2, dim3(njobs), dim3(256), 0, s, jobs, inl, parts, chunks);
    return hipGetLastError();
}

}  // namespace z2h
