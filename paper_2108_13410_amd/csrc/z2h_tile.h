// Generic tile machinery shared by the device kernels of libz2h.
//
// A tile of 2^m complex amplitudes is held by 2^(m-R) threads, 2^R amplitudes
// per thread in registers.  A "layout" p places local bits [p, p + R) in
// registers; butterflies act on register bits and an exchange through LDS
// moves the tile from one layout to another.  GroupGeom (z2h_internal.h)
// maps local tile bits to global state bits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "z2h_internal.h"
#include "z2h_kernels.h"

namespace z2h {

template <typename Real>
struct __attribute__((aligned(2 * sizeof(Real)))) Cx {
    Real x, y;
};

template <typename Real>
__device__ __forceinline__ Cx<Real> cadd(Cx<Real> a, Cx<Real> b) { return {a.x + b.x, a.y + b.y}; }
template <typename Real>
__device__ __forceinline__ Cx<Real> csub(Cx<Real> a, Cx<Real> b) { return {a.x - b.x, a.y - b.y}; }
template <typename Real>
__device__ __forceinline__ Cx<Real> cmul(Cx<Real> a, Cx<Real> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__device__ __forceinline__ int popc(uint32_t v) { return __builtin_popcount(v); }

// Next 16-byte boundary at or after p (LDS sub-buffers; the host sizes the
// dynamic LDS block with the same rounding).
// The padding is added to the original pointer (not rebuilt from an
// integer) so the compiler still knows the result points into LDS and emits
// ds_* instructions rather than flat ones for it.
template <typename T, typename U>
__device__ __forceinline__ T *align16(U *p) {
    const uintptr_t pad = (16u - (uint32_t)(reinterpret_cast<uintptr_t>(p) & 15u)) & 15u;
    return reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(p) + pad);
}

// Local index of register element q of thread t in layout p.
template <int R>
__device__ __forceinline__ uint32_t lay_base(int p, uint32_t t) {
    return (t & ((1u << p) - 1u)) | ((t >> p) << (p + R));
}

// LDS slot of local index e: one pad element every 2^R elements keeps every
// layout's accesses free of bank conflicts.
template <int R>
__device__ __forceinline__ uint32_t slot(uint32_t e) { return e + (e >> R); }

// Global index (within the state) of local index e of tile "tile".  Local
// bits [0, c) are global [0, c); the transformed bits follow from b0, except
// in a group split in two runs (hi > 0), whose top hi local bits sit at
// [b1, b1 + hi).  The tile index fills the remaining global bits in
// ascending order.  SPLIT: the kernel may be given split groups (the
// planner gives them only to the kernels compiled with it).
template <bool SPLIT = false>
__device__ __forceinline__ uint64_t glob(const GroupGeom &g, uint64_t tile, uint32_t e) {
    const uint32_t cm = (1u << g.c) - 1u;
    const int tlo_bits = g.b0 - g.c;
    const uint64_t tlo = tile & ((1ull << tlo_bits) - 1ull);
    if (!SPLIT || !g.hi)
        return (uint64_t)(e & cm) | (tlo << g.c) | ((uint64_t)(e >> g.c) << g.b0) |
               ((tile >> tlo_bits) << (g.b0 + g.m - g.c));
    const int ga = g.m - g.c - g.hi;            // bits of the run at b0
    const int tmid_bits = g.b1 - (g.b0 + ga);   // tile bits between the runs
    const uint64_t tmid = (tile >> tlo_bits) & ((1ull << tmid_bits) - 1ull);
    const uint64_t thi = tile >> (tlo_bits + tmid_bits);
    const uint32_t et = e >> g.c;
    return (uint64_t)(e & cm) | (tlo << g.c) | ((uint64_t)(et & ((1u << ga) - 1u)) << g.b0) |
           (tmid << (g.b0 + ga)) | ((uint64_t)(et >> ga) << g.b1) | (thi << (g.b1 + g.hi));
}

// Global bit position of local bit x.
template <bool SPLIT = false>
__device__ __forceinline__ int gbit(const GroupGeom &g, int x) {
    if (!SPLIT) return x < g.c ? x : g.b0 + (x - g.c);
    return x < g.c ? x : (g.hi && x >= g.m - g.hi) ? g.b1 + (x - (g.m - g.hi)) : g.b0 + (x - g.c);
}

template <typename Real, int R>
__device__ __forceinline__ void butterflies(Cx<Real> (&v)[1 << R], int blo, int bhi) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (j >= blo && j < bhi) {
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
}

template <typename Real, int R>
__device__ __forceinline__ void exchange(Cx<Real> (&v)[1 << R], Cx<Real> *lds, int pf, int pt,
                                         uint32_t t) {
    const uint32_t bf = lay_base<R>(pf, t), bt = lay_base<R>(pt, t);
#pragma unroll
    for (int q = 0; q < (1 << R); ++q) {
        uint32_t e = bf | ((uint32_t)q << pf);
        lds[slot<R>(e)] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (1 << R); ++q) {
        uint32_t e = bt | ((uint32_t)q << pt);
        v[q] = lds[slot<R>(e)];
    }
    __syncthreads();
}

// Per-thread constants of one layout.  The register bits of a layout are
// global bits [gs, gs + nlo) and, when the window straddles the boundary
// between the two runs of a split group, [gs2, gs2 + R - nlo) (the planner
// never lets a layout straddle the carried/transformed boundary).  Register
// element q sits at global index i0 + reg_off(q): (q << gs) for a window
// inside one run.  s0z/s0x are the plaquette/star syndromes of i0 and lz/lx
// the syndrome columns of the R register bits (uniform across the block).
template <int R>
struct LayCtx {
    uint64_t i0;
    int gs, w0;
    int gs2, nlo;
    uint32_t s0z, s0x;
    uint32_t lz[R], lx[R];
};

// Global offset of register element q.  SW: the layout may straddle two
// runs (only the kernels that take split-window groups pass true; for a
// window inside one run nlo = R and the second term vanishes).
template <int R, bool SW>
__device__ __forceinline__ uint64_t reg_off(const LayCtx<R> &L, int q) {
    if constexpr (SW)
        return ((uint64_t)(q & ((1 << L.nlo) - 1)) << L.gs) | ((uint64_t)(q >> L.nlo) << L.gs2);
    else
        return (uint64_t)q << L.gs;
}

// Global bit of register bit r of a layout.
template <int R>
__device__ __forceinline__ int reg_bit(const LayCtx<R> &L, int r) {
    return r < L.nlo ? L.gs + r : L.gs2 + (r - L.nlo);
}

__device__ __forceinline__ uint32_t syndrome_direct(const uint32_t *masks, int nst, uint64_t i) {
    uint32_t s = 0;
    const uint32_t ii = (uint32_t)i;
    for (int k = 0; k < nst; ++k) s |= (uint32_t)(popc(ii & masks[k]) & 1) << k;
    return s;
}

// want_syn: fill the syndromes; which: 0 plaquettes only, 1 stars only, 2
// both (a phase pass needs only the basis it applies).
template <int R, bool SPLIT = false>
__device__ __forceinline__ void lay_ctx(LayCtx<R> &L, const GroupGeom &g, const LatticeDev &lat,
                                        uint64_t tile, int p, uint32_t t, bool want_syn, int which = 2) {
    L.i0 = glob<SPLIT>(g, tile, lay_base<R>(p, t));
    L.gs = gbit<SPLIT>(g, p);
    if constexpr (SPLIT) {
        const int xb = g.m - g.hi;  // local start of the second run
        L.nlo = (g.hi && p < xb && p + R > xb) ? xb - p : R;
        L.gs2 = g.b1;
    } else {
        L.nlo = R;
        L.gs2 = 0;
    }
    L.w0 = __builtin_popcountll(L.i0);
    if (want_syn) {
        L.s0z = which != 1 ? syndrome_direct(lat.zmask, lat.nst, L.i0) : 0u;
        L.s0x = which != 0 ? syndrome_direct(lat.xmask, lat.nst, L.i0) : 0u;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int b = SPLIT ? reg_bit(L, r) : L.gs + r;
            L.lz[r] = lat.zsyn[b];
            L.lx[r] = lat.xsyn[b];
        }
    }
}

template <typename Real> struct Vec2;
template <> struct Vec2<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct Vec2<double> { typedef double type __attribute__((ext_vector_type(2))); };

// One complex element; NT selects the nontemporal (streaming) cache policy.
template <typename Real, bool NT>
__device__ __forceinline__ Cx<Real> ldc(const Cx<Real> *p) {
    if constexpr (NT) {
        typedef typename Vec2<Real>::type V;
        const V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
        return Cx<Real>{v.x, v.y};
    } else {
        return *p;
    }
}

template <typename Real, bool NT>
__device__ __forceinline__ void stc(Cx<Real> *p, Cx<Real> x) {
    if constexpr (NT) {
        typedef typename Vec2<Real>::type V;
        V v = {x.x, x.y};
        __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
    } else {
        *p = x;
    }
}

template <typename Real, int R, bool NT = false, bool SW = false>
__device__ __forceinline__ void load_tile(Cx<Real> (&v)[1 << R], const Cx<Real> *st,
                                          const LayCtx<R> &L) {
    const Cx<Real> *b = st + L.i0;
#pragma unroll
    for (int q = 0; q < (1 << R); ++q) v[q] = ldc<Real, NT>(b + reg_off<R, SW>(L, q));
}

// The base index is passed through an empty asm statement so that the
// compiler recomputes the 2^R store addresses instead of keeping the load
// addresses alive through the whole pass (2 VGPRs each).
template <typename Real, int R, bool NT = false, bool SW = false>
__device__ __forceinline__ void store_tile(const Cx<Real> (&v)[1 << R], Cx<Real> *st,
                                           const LayCtx<R> &L) {
    uint64_t i0 = L.i0;
    asm volatile("" : "+v"(i0));
    Cx<Real> *b = st + i0;
#pragma unroll
    for (int q = 0; q < (1 << R); ++q) stc<Real, NT>(b + reg_off<R, SW>(L, q), v[q]);
}

// Workgroups of a launch are handed to the eight XCDs in turn (block b to
// XCD b mod 8).  XCD-major order renumbers them so that each XCD walks a
// contiguous range of tiles (of a grid-stride loop's round), so neighbouring
// tiles meet in one L2 and each XCD streams one region of the state.  A
// bijection of [0, nb) when nb is a multiple of 8; other grids keep their
// order.
__device__ __forceinline__ uint32_t xcd_major(uint32_t b, uint32_t nb) {
    return (nb & 7u) ? b : (b & 7u) * (nb >> 3) + (b >> 3);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Deterministic block sum; every thread gets the result.
__device__ double block_sum(double x, double *red) {
    x = wave_sum(x);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = x;
    __syncthreads();
    double s = 0.0;
    for (int j = 0; j < nw; ++j) s += red[j];
    __syncthreads();
    return s;
}

}  // namespace z2h
