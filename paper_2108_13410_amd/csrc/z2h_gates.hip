// Gate kernels for the gate-level emulation of the paper's circuits
// (Sec. III; Eqs. (ini1), (ini2)): one-qubit gates given as 2x2 matrices,
// CNOT, projection on |0>, renormalisation, and two fused passes that keep
// a thread's amplitudes in registers: gate groups on the qubits of an LDS
// tile, applied in register phases, and gate groups on five qubits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <set>

#include "../../include/z2h.h"
#include "z2h_internal.h"
#include "z2h_kernels.h"
#include "z2h_solvers.h"
#include "z2h_tile.h"

namespace z2h {

// Index with a zero bit inserted at position b (the bits from b up move one
// position up).
__device__ __forceinline__ uint64_t insert0(uint64_t i, int b) {
    const uint64_t lo = i & ((1ull << b) - 1ull);
    return ((i >> b) << (b + 1)) | lo;
}

template <typename Real>
__device__ __forceinline__ void apply_2x2(Cx<Real> &a, Cx<Real> &b, const double *m) {
    const Cx<Real> m00{(Real)m[0], (Real)m[1]}, m01{(Real)m[2], (Real)m[3]};
    const Cx<Real> m10{(Real)m[4], (Real)m[5]}, m11{(Real)m[6], (Real)m[7]};
    const Cx<Real> x = a, y = b;
    a = cadd(cmul(m00, x), cmul(m01, y));
    b = cadd(cmul(m10, x), cmul(m11, y));
}

// One gate over the whole state, one pair (or quadruple) per thread step.
template <typename Real>
__global__ void __launch_bounds__(256) gate_kernel(Cx<Real> *st, int nq, GateDev g) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g.kind == Z2H_GATE_CNOT) {
        const int lo = g.q0 < g.q1 ? g.q0 : g.q1, hi = g.q0 < g.q1 ? g.q1 : g.q0;
        const uint64_t n = 1ull << (nq - 2);
        for (uint64_t p = t0; p < n; p += stride) {
            const uint64_t i = insert0(insert0(p, lo), hi) | (1ull << g.q0);
            const uint64_t j = i | (1ull << g.q1);
            const Cx<Real> a = st[i];
            st[i] = st[j];
            st[j] = a;
        }
        return;
    }
    const uint64_t n = 1ull << (nq - 1);
    for (uint64_t p = t0; p < n; p += stride) {
        const uint64_t i = insert0(p, g.q0), j = i | (1ull << g.q0);
        if (g.kind == Z2H_GATE_PROJ0) {
            st[j] = Cx<Real>{(Real)0, (Real)0};
        } else {
            Cx<Real> a = st[i], b = st[j];
            apply_2x2<Real>(a, b, g.m);
            st[i] = a;
            st[j] = b;
        }
    }
}

template <typename Real>
__global__ void __launch_bounds__(256) norm_parts_kernel(const Cx<Real> *st, uint64_t n, double *part) {
    __shared__ double red[8];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const Cx<Real> e = st[i];
        acc += (double)e.x * (double)e.x + (double)e.y * (double)e.y;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Every block sums the partials itself, then scales its share.
template <typename Real>
__global__ void __launch_bounds__(256) scale_kernel(Cx<Real> *st, uint64_t n, const double *part, int nparts) {
    __shared__ double red[8];
    double s = 0.0;
    for (int j = (int)threadIdx.x; j < nparts; j += (int)blockDim.x) s += part[j];
    s = block_sum(s, red);
    const Real f = s > 0.0 ? (Real)(1.0 / sqrt(s)) : (Real)1;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        Cx<Real> e = st[i];
        e.x *= f;
        e.y *= f;
        st[i] = e;
    }
}

// ------------------------------------------------------------ register file

// The 2^kRegBits amplitudes a thread holds, real and imaginary parts
// interleaved in one vector value.  The gates below touch it only through
// compile-time element indices, and a runtime switch picks the
// instantiation for a gate's register bits.  (With an array, merged switch
// cases address the elements through pointer selects, and the array is
// then kept in scratch memory.)
template <typename Real>
struct RegFile {
    typedef Real type __attribute__((ext_vector_type(2 << kRegBits)));
};
template <typename Real>
using Regs = typename RegFile<Real>::type;

// The one-qubit gates in the forms their matrices have (the host builds
// them so): H as the unscaled butterfly [[1, 1], [1, -1]] (the group's
// amplitudes are scaled once at its end); R_x = [[c, i w], [i w, c]]; R_z =
// diag(d0, d1).  Four or eight real operations per amplitude pair instead
// of the sixteen of a general complex 2x2 matrix.
template <typename Real, int B>
__device__ __forceinline__ void reg_h(Regs<Real> &v) {
#pragma unroll
    for (int k = 0; k < (1 << kRegBits); ++k)
        if (!(k & (1 << B))) {
            const int j = k | (1 << B);
            const Real xr = v[2 * k], xi = v[2 * k + 1], yr = v[2 * j], yi = v[2 * j + 1];
            v[2 * k] = xr + yr;
            v[2 * k + 1] = xi + yi;
            v[2 * j] = xr - yr;
            v[2 * j + 1] = xi - yi;
        }
}

template <typename Real, int B>
__device__ __forceinline__ void reg_rx(Regs<Real> &v, const double *m) {
    const Real c = (Real)m[0], w = (Real)m[3];
#pragma unroll
    for (int k = 0; k < (1 << kRegBits); ++k)
        if (!(k & (1 << B))) {
            const int j = k | (1 << B);
            const Real xr = v[2 * k], xi = v[2 * k + 1], yr = v[2 * j], yi = v[2 * j + 1];
            v[2 * k] = c * xr - w * yi;
            v[2 * k + 1] = c * xi + w * yr;
            v[2 * j] = c * yr - w * xi;
            v[2 * j + 1] = c * yi + w * xr;
        }
}

template <typename Real, int B>
__device__ __forceinline__ void reg_rz(Regs<Real> &v, const double *m) {
    const Cx<Real> d0{(Real)m[0], (Real)m[1]}, d1{(Real)m[6], (Real)m[7]};
#pragma unroll
    for (int k = 0; k < (1 << kRegBits); ++k) {
        const Cx<Real> d = (k & (1 << B)) ? d1 : d0;
        const Cx<Real> p = cmul(d, Cx<Real>{v[2 * k], v[2 * k + 1]});
        v[2 * k] = p.x;
        v[2 * k + 1] = p.y;
    }
}

template <typename Real, int B>
__device__ __forceinline__ void reg_proj0(Regs<Real> &v) {
#pragma unroll
    for (int k = 0; k < (1 << kRegBits); ++k)
        if (k & (1 << B)) {
            v[2 * k] = (Real)0;
            v[2 * k + 1] = (Real)0;
        }
}

// CNOT with target bit T and control mask M: the target flips where the
// parity of the control bits is odd (consecutive CNOTs with one target,
// composed).
template <typename Real, int T, int M>
__device__ __forceinline__ void reg_cnot(Regs<Real> &v) {
#pragma unroll
    for (int k = 0; k < (1 << kRegBits); ++k)
        if (!(k & (1 << T)) && (__builtin_popcount(k & M) & 1)) {
            const int j = k | (1 << T);
            const Real x = v[2 * k], y = v[2 * k + 1];
            v[2 * k] = v[2 * j];
            v[2 * k + 1] = v[2 * j + 1];
            v[2 * j] = x;
            v[2 * j + 1] = y;
        }
}

template <typename Real, int T, int M = 1>
__device__ __forceinline__ void reg_cnot_m(Regs<Real> &v, int mask) {
    if constexpr (M < (1 << kRegBits)) {
        if constexpr (!(M & (1 << T))) {
            if (mask == M) {
                reg_cnot<Real, T, M>(v);
                return;
            }
        }
        reg_cnot_m<Real, T, M + 1>(v, mask);
    }
}

template <typename Real>
__device__ __forceinline__ void reg_gate(Regs<Real> &v, const GateDev &g) {
    static_assert(kRegBits == 5, "the switches below cover five register bits");
    if (g.kind == Z2H_GATE_CNOT) {
        switch (g.q1) {
            case 0: reg_cnot_m<Real, 0>(v, g.q0); break;
            case 1: reg_cnot_m<Real, 1>(v, g.q0); break;
            case 2: reg_cnot_m<Real, 2>(v, g.q0); break;
            case 3: reg_cnot_m<Real, 3>(v, g.q0); break;
            default: reg_cnot_m<Real, 4>(v, g.q0); break;
        }
    } else if (g.kind == Z2H_GATE_PROJ0) {
        switch (g.q0) {
            case 0: reg_proj0<Real, 0>(v); break;
            case 1: reg_proj0<Real, 1>(v); break;
            case 2: reg_proj0<Real, 2>(v); break;
            case 3: reg_proj0<Real, 3>(v); break;
            default: reg_proj0<Real, 4>(v); break;
        }
    } else if (g.kind == Z2H_GATE_H) {
        switch (g.q0) {
            case 0: reg_h<Real, 0>(v); break;
            case 1: reg_h<Real, 1>(v); break;
            case 2: reg_h<Real, 2>(v); break;
            case 3: reg_h<Real, 3>(v); break;
            default: reg_h<Real, 4>(v); break;
        }
    } else if (g.kind == Z2H_GATE_RX) {
        switch (g.q0) {
            case 0: reg_rx<Real, 0>(v, g.m); break;
            case 1: reg_rx<Real, 1>(v, g.m); break;
            case 2: reg_rx<Real, 2>(v, g.m); break;
            case 3: reg_rx<Real, 3>(v, g.m); break;
            default: reg_rx<Real, 4>(v, g.m); break;
        }
    } else {
        switch (g.q0) {
            case 0: reg_rz<Real, 0>(v, g.m); break;
            case 1: reg_rz<Real, 1>(v, g.m); break;
            case 2: reg_rz<Real, 2>(v, g.m); break;
            case 3: reg_rz<Real, 3>(v, g.m); break;
            default: reg_rz<Real, 4>(v, g.m); break;
        }
    }
}

template <typename Real>
__device__ __forceinline__ void scale_regs(Regs<Real> &v, Real f) {
#pragma unroll
    for (int k = 0; k < (2 << kRegBits); ++k) v[k] *= f;
}

// Register k of a thread whose base index is `base`: the bits of k select
// the offsets off[0..kRegBits).
template <typename Real>
__device__ __forceinline__ void load_regs(Regs<Real> &v, const Cx<Real> *st, uint64_t base,
                                          const uint64_t (&off)[kRegBits]) {
#pragma unroll
    for (int k = 0; k < (1 << kRegBits); ++k) {
        uint64_t i = base;
#pragma unroll
        for (int b = 0; b < kRegBits; ++b)
            if (k & (1 << b)) i |= off[b];
        const Cx<Real> e = st[i];
        v[2 * k] = e.x;
        v[2 * k + 1] = e.y;
    }
}

template <typename Real>
__device__ __forceinline__ void store_regs(const Regs<Real> &v, Cx<Real> *st, uint64_t base,
                                           const uint64_t (&off)[kRegBits]) {
#pragma unroll
    for (int k = 0; k < (1 << kRegBits); ++k) {
        uint64_t i = base;
#pragma unroll
        for (int b = 0; b < kRegBits; ++b)
            if (k & (1 << b)) i |= off[b];
        st[i] = Cx<Real>{v[2 * k], v[2 * k + 1]};
    }
}

// The bits of x deposited, lowest first, at the qubits q[0..n).
__device__ __forceinline__ uint64_t deposit(uint64_t x, const int32_t *q, int n) {
    uint64_t g = 0;
    for (int j = 0; j < n; ++j) g |= ((x >> j) & 1ull) << q[j];
    return g;
}

// ------------------------------------------------------------- tile phases

// Local index of register 0 of thread t in the layout with register bits
// S[0] < ... < S[kRegBits-1]: t's bits fill the other local bits in order.
__device__ __forceinline__ uint32_t spread(uint32_t t, const int (&S)[kRegBits]) {
    uint32_t x = t;
#pragma unroll
    for (int b = 0; b < kRegBits; ++b) x = ((x >> S[b]) << (S[b] + 1)) | (x & ((1u << S[b]) - 1u));
    return x;
}

// LDS slot of local index i: one pad element after every 256-byte row, so
// threads whose indices differ only in higher bits reach different banks.
// For indices with disjoint bits the slot is additive, slot(a | b) =
// slot(a) + slot(b) (the low parts of a and b add without a carry), so a
// register's slot is the thread's slot plus a block-uniform offset.
template <typename Real>
constexpr int kPadShift = sizeof(Real) == 8 ? 4 : 5;

template <typename Real>
__device__ __forceinline__ uint32_t lds_slot(uint32_t i) {
    return i + (i >> kPadShift<Real>);
}

template <typename Real>
constexpr size_t tile_lds_bytes(int m) {
    return (((size_t)1 << m) + ((size_t)1 << m >> kPadShift<Real>)) * sizeof(Cx<Real>);
}

__device__ __forceinline__ void unpack_layout(uint32_t code, int (&S)[kRegBits]) {
#pragma unroll
    for (int b = 0; b < kRegBits; ++b) S[b] = (int)((code >> (4 * b)) & 15u);
}

// Move the tile from layout `from` to layout `to` through LDS.
template <typename Real>
__device__ __forceinline__ void relayout(Regs<Real> &v, Cx<Real> *lds, uint32_t t, uint32_t from, uint32_t to) {
    int S[kRegBits];
    uint32_t so[kRegBits];
    unpack_layout(from, S);
    uint32_t base = lds_slot<Real>(spread(t, S));
#pragma unroll
    for (int b = 0; b < kRegBits; ++b) so[b] = lds_slot<Real>(1u << S[b]);
    __syncthreads();  // every thread is done with the previous contents
#pragma unroll
    for (int k = 0; k < (1 << kRegBits); ++k) {
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < kRegBits; ++b)
            if (k & (1 << b)) o += so[b];
        lds[base + o] = Cx<Real>{v[2 * k], v[2 * k + 1]};
    }
    __syncthreads();
    unpack_layout(to, S);
    base = lds_slot<Real>(spread(t, S));
#pragma unroll
    for (int b = 0; b < kRegBits; ++b) so[b] = lds_slot<Real>(1u << S[b]);
#pragma unroll
    for (int k = 0; k < (1 << kRegBits); ++k) {
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < kRegBits; ++b)
            if (k & (1 << b)) o += so[b];
        const Cx<Real> e = lds[base + o];
        v[2 * k] = e.x;
        v[2 * k + 1] = e.y;
    }
}

// A group of gates on the qubits of one tile of 2^m amplitudes.  Each
// thread loads its 2^kRegBits amplitudes in the home layout (its own bits
// are the tile's lowest qubits, which keeps the loads coalesced), applies
// the gates phase by phase in registers, changing layout through LDS
// between phases whose register bits differ, and stores in the home layout.
// Two padded complex64 tiles (66 KiB each) fit a CU's LDS; the register
// budget is set for the two waves per SIMD that this allows.
template <typename Real>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 ? 2 : 1)))
fused_kernel(FusedArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    Cx<Real> *lds = reinterpret_cast<Cx<Real> *>(smem);
    Cx<Real> *st = reinterpret_cast<Cx<Real> *>(a.state);
    const uint32_t t = threadIdx.x;
    const int lt = a.m - kRegBits, nc = a.nq - a.m;
    uint32_t home = 0;
#pragma unroll
    for (int b = 0; b < kRegBits; ++b) home |= (uint32_t)(lt + b) << (4 * b);
    uint64_t off[kRegBits];
#pragma unroll
    for (int b = 0; b < kRegBits; ++b) off[b] = 1ull << a.lq[lt + b];
    const uint64_t toff = deposit(t, a.lq, lt);
    // tile numbers deposited at the qubits cq[]: advanced by a masked add
    const uint64_t mask = deposit(~0ull, a.cq, nc), step = deposit(gridDim.x, a.cq, nc);
    uint64_t tb = deposit(blockIdx.x, a.cq, nc);
    const uint64_t tiles = 1ull << nc;
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        Regs<Real> v;
        load_regs<Real>(v, st, tb | toff, off);
        uint32_t cur = home;
        int g = 0;
        for (int p = 0; p < a.nphase; ++p) {
            const uint32_t lay = a.phase[p] & 0xFFFFFu;
            if (lay != cur) {
                relayout<Real>(v, lds, t, cur, lay);
                cur = lay;
            }
            for (const int end = (int)(a.phase[p] >> 24); g < end; ++g) reg_gate<Real>(v, a.gates[g]);
        }
        if (cur != home) relayout<Real>(v, lds, t, cur, home);
        if (a.scale != 1.0) scale_regs<Real>(v, (Real)a.scale);
        uint64_t base = tb | toff;
        // keeps the 32 store addresses from being computed before the gates
        asm volatile("" : "+v"(base));
        store_regs<Real>(v, st, base, off);
        tb = ((tb | ~mask) + step) & mask;
    }
}

// A group of gates on at most five qubits, applied in registers: load the
// thread's 32 amplitudes, apply every gate, store.  No LDS and no barriers.
template <typename Real>
__global__ void __launch_bounds__(256) reg_kernel(RegArgs a) {
    Cx<Real> *st = reinterpret_cast<Cx<Real> *>(a.state);
    const uint64_t tpart = deposit(threadIdx.x, a.tq, a.nt);
    uint64_t off[kRegBits];
#pragma unroll
    for (int i = 0; i < kRegBits; ++i) off[i] = 1ull << a.rq[i];
    const int ncq = a.nq - kRegBits - a.nt;
    const uint64_t mask = deposit(~0ull, a.cq, ncq), step = deposit(gridDim.x, a.cq, ncq);
    uint64_t tb = deposit(blockIdx.x, a.cq, ncq);
    const uint64_t tiles = 1ull << ncq;
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        Regs<Real> v;
        load_regs<Real>(v, st, tb | tpart, off);
        for (int g = 0; g < a.ngates; ++g) reg_gate<Real>(v, a.gates[g]);
        if (a.scale != 1.0) scale_regs<Real>(v, (Real)a.scale);
        uint64_t base = tb | tpart;
        asm volatile("" : "+v"(base));
        store_regs<Real>(v, st, base, off);
        tb = ((tb | ~mask) + step) & mask;
    }
}

// ---------------------------------------------------------------- launchers

// Largest padded tile: 2^13 complex64 or 2^12 complex128 amplitudes.
constexpr size_t kTileLdsMax = 69632;
static_assert(tile_lds_bytes<float>(13) <= kTileLdsMax && tile_lds_bytes<double>(12) <= kTileLdsMax, "tile LDS");

static unsigned blocks_for(uint64_t work) {
    const uint64_t b = (work + 255) / 256;
    return (unsigned)(b < (uint64_t)kGateBlocksMax ? (b ? b : 1) : (uint64_t)kGateBlocksMax);
}

hipError_t launch_gate(bool c128, void *state, int nq, const GateDev &g, hipStream_t s) {
    const unsigned nb = blocks_for(1ull << (nq - 1));
    if (c128)
        hipLaunchKernelGGL(gate_kernel<double>, dim3(nb), dim3(256), 0, s, (Cx<double> *)state, nq, g);
    else
        hipLaunchKernelGGL(gate_kernel<float>, dim3(nb), dim3(256), 0, s, (Cx<float> *)state, nq, g);
    return hipGetLastError();
}

static std::mutex g_lds_mu;
static std::set<const void *> g_lds_done;

// Raise a kernel's dynamic-LDS limit once (tiles above 64 KiB).
static hipError_t allow_lds(const void *fn, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_lds_mu);
    if (g_lds_done.count(fn)) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTileLdsMax);
    if (e == hipSuccess) g_lds_done.insert(fn);
    return e;
}

hipError_t launch_fused(bool c128, const FusedArgs &a, hipStream_t s) {
    if (a.m < kRegBits + 1 || a.m > 13 || a.nq - a.m > 40) return hipErrorInvalidValue;
    const uint64_t tiles = 1ull << (a.nq - a.m);
    const unsigned nb = (unsigned)(tiles < (uint64_t)kGateBlocksMax ? tiles : (uint64_t)kGateBlocksMax);
    const unsigned nt = 1u << (a.m - kRegBits);
    const size_t lds = c128 ? tile_lds_bytes<double>(a.m) : tile_lds_bytes<float>(a.m);
    if (lds > kTileLdsMax || nt > 256) return hipErrorInvalidValue;
    const void *fn = c128 ? reinterpret_cast<const void *>(&fused_kernel<double>)
                          : reinterpret_cast<const void *>(&fused_kernel<float>);
    hipError_t e = allow_lds(fn, lds);
    if (e != hipSuccess) return e;
    if (c128)
        hipLaunchKernelGGL(fused_kernel<double>, dim3(nb), dim3(nt), lds, s, a);
    else
        hipLaunchKernelGGL(fused_kernel<float>, dim3(nb), dim3(nt), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_reg(bool c128, const RegArgs &a, hipStream_t s) {
    const uint64_t tiles = 1ull << (a.nq - kRegBits - a.nt);
    const unsigned nb = (unsigned)(tiles < (uint64_t)kGateBlocksMax ? tiles : (uint64_t)kGateBlocksMax);
    if (c128)
        hipLaunchKernelGGL(reg_kernel<double>, dim3(nb), dim3(1u << a.nt), 0, s, a);
    else
        hipLaunchKernelGGL(reg_kernel<float>, dim3(nb), dim3(1u << a.nt), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_normalize(bool c128, void *state, int nq, double *part, int nparts, hipStream_t s) {
    const uint64_t n = 1ull << nq;
    const unsigned nb = blocks_for(n) < (unsigned)nparts ? blocks_for(n) : (unsigned)nparts;
    if (c128) {
        hipLaunchKernelGGL(norm_parts_kernel<double>, dim3(nb), dim3(256), 0, s, (const Cx<double> *)state, n, part);
        hipLaunchKernelGGL(scale_kernel<double>, dim3(nb), dim3(256), 0, s, (Cx<double> *)state, n, part, (int)nb);
    } else {
        hipLaunchKernelGGL(norm_parts_kernel<float>, dim3(nb), dim3(256), 0, s, (const Cx<float> *)state, n, part);
        hipLaunchKernelGGL(scale_kernel<float>, dim3(nb), dim3(256), 0, s, (Cx<float> *)state, n, part, (int)nb);
    }
    return hipGetLastError();
}

}  // namespace z2h
