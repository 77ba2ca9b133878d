// Gate kernels for the gate-level emulation of the paper's circuits
// (Sec. III; Eqs. (ini1), (ini2)): one-qubit gates given as 2x2 matrices,
// CNOT, projection on |0>, renormalisation, and a fused pass that applies a
// group of gates to tiles held in LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Global index of a tile's element: local bit j sits at qubit lq[j], tile
// bit j at qubit cq[j].
__device__ __forceinline__ uint64_t local_offset(const FusedArgs &a, uint32_t e) {
    uint64_t g = 0;
    for (int j = 0; j < a.m; ++j) g |= (uint64_t)((e >> j) & 1u) << a.lq[j];
    return g;
}

__device__ __forceinline__ uint64_t tile_base(const FusedArgs &a, uint64_t tile) {
    uint64_t g = 0;
    for (int j = 0; j < a.nq - a.m; ++j) g |= ((tile >> j) & 1ull) << a.cq[j];
    return g;
}

// A group of gates on the qubits of one tile: load the 2^m amplitudes of a
// tile (the four lowest qubits are always local, so each row is 16
// contiguous amplitudes), apply the gates one after another in LDS, store.
template <typename Real>
__global__ void __launch_bounds__(256) fused_kernel(FusedArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    Cx<Real> *lds = reinterpret_cast<Cx<Real> *>(smem);
    Cx<Real> *st = reinterpret_cast<Cx<Real> *>(a.state);
    const uint32_t T = 1u << a.m, t = threadIdx.x, nt = blockDim.x;
    const uint64_t tiles = 1ull << (a.nq - a.m);
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint64_t base = tile_base(a, tile);
        for (uint32_t e = t; e < T; e += nt) lds[e] = st[base | local_offset(a, e)];
        __syncthreads();
        for (int k = 0; k < a.ngates; ++k) {
            const GateDev &g = a.gates[k];
            if (g.kind == Z2H_GATE_CNOT) {
                const int lo = g.q0 < g.q1 ? g.q0 : g.q1, hi = g.q0 < g.q1 ? g.q1 : g.q0;
                for (uint32_t p = t; p < (T >> 2); p += nt) {
                    const uint32_t i = (uint32_t)insert0(insert0(p, lo), hi) | (1u << g.q0);
                    const uint32_t j = i | (1u << g.q1);
                    const Cx<Real> x = lds[i];
                    lds[i] = lds[j];
                    lds[j] = x;
                }
            } else {
                for (uint32_t p = t; p < (T >> 1); p += nt) {
                    const uint32_t i = (uint32_t)insert0(p, g.q0), j = i | (1u << g.q0);
                    if (g.kind == Z2H_GATE_PROJ0) {
                        lds[j] = Cx<Real>{(Real)0, (Real)0};
                    } else {
                        Cx<Real> x = lds[i], y = lds[j];
                        apply_2x2<Real>(x, y, g.m);
                        lds[i] = x;
                        lds[j] = y;
                    }
                }
            }
            __syncthreads();
        }
        for (uint32_t e = t; e < T; e += nt) st[base | local_offset(a, e)] = lds[e];
        __syncthreads();
    }
}

// Gates on register bits: every one-qubit gate, CNOT and projection acts
// on pairs of a thread's own registers, with the bit positions fixed at
// compile time (a runtime switch picks the instantiation).
template <typename Real, int B>
__device__ __forceinline__ void reg_1q(Cx<Real> (&v)[1 << kRegBits], const double *m) {
#pragma unroll
    for (int k = 0; k < (1 << kRegBits); ++k)
        if (!(k & (1 << B))) apply_2x2<Real>(v[k], v[k | (1 << B)], m);
}

template <typename Real, int B>
__device__ __forceinline__ void reg_proj0(Cx<Real> (&v)[1 << kRegBits]) {
#pragma unroll
    for (int k = 0; k < (1 << kRegBits); ++k)
        if (k & (1 << B)) v[k] = Cx<Real>{(Real)0, (Real)0};
}

template <typename Real, int C, int T>
__device__ __forceinline__ void reg_cnot(Cx<Real> (&v)[1 << kRegBits]) {
    if constexpr (C != T) {
#pragma unroll
        for (int k = 0; k < (1 << kRegBits); ++k)
            if ((k & (1 << C)) && !(k & (1 << T))) {
                const Cx<Real> x = v[k];
                v[k] = v[k | (1 << T)];
                v[k | (1 << T)] = x;
            }
    }
}

template <typename Real, int C>
__device__ __forceinline__ void reg_cnot_t(Cx<Real> (&v)[1 << kRegBits], int t) {
    switch (t) {
        case 0: reg_cnot<Real, C, 0>(v); break;
        case 1: reg_cnot<Real, C, 1>(v); break;
        case 2: reg_cnot<Real, C, 2>(v); break;
        case 3: reg_cnot<Real, C, 3>(v); break;
        default: reg_cnot<Real, C, 4>(v); break;
    }
}

template <typename Real>
__device__ __forceinline__ void reg_gate(Cx<Real> (&v)[1 << kRegBits], const GateDev &g) {
    static_assert(kRegBits == 5, "the switches below cover five register bits");
    if (g.kind == Z2H_GATE_CNOT) {
        switch (g.q0) {
            case 0: reg_cnot_t<Real, 0>(v, g.q1); break;
            case 1: reg_cnot_t<Real, 1>(v, g.q1); break;
            case 2: reg_cnot_t<Real, 2>(v, g.q1); break;
            case 3: reg_cnot_t<Real, 3>(v, g.q1); break;
            default: reg_cnot_t<Real, 4>(v, g.q1); break;
        }
    } else if (g.kind == Z2H_GATE_PROJ0) {
        switch (g.q0) {
            case 0: reg_proj0<Real, 0>(v); break;
            case 1: reg_proj0<Real, 1>(v); break;
            case 2: reg_proj0<Real, 2>(v); break;
            case 3: reg_proj0<Real, 3>(v); break;
            default: reg_proj0<Real, 4>(v); break;
        }
    } else {
        switch (g.q0) {
            case 0: reg_1q<Real, 0>(v, g.m); break;
            case 1: reg_1q<Real, 1>(v, g.m); break;
            case 2: reg_1q<Real, 2>(v, g.m); break;
            case 3: reg_1q<Real, 3>(v, g.m); break;
            default: reg_1q<Real, 4>(v, g.m); break;
        }
    }
}

// A group of gates on at most five qubits, applied in registers: load the
// thread's 32 amplitudes, apply every gate, store.  No LDS and no barriers.
template <typename Real>
__global__ void __launch_bounds__(256) reg_kernel(RegArgs a) {
    Cx<Real> *st = reinterpret_cast<Cx<Real> *>(a.state);
    const uint32_t t = threadIdx.x;
    uint64_t tpart = 0;
    for (int j = 0; j < a.nt; ++j) tpart |= (uint64_t)((t >> j) & 1u) << a.tq[j];
    uint64_t roff[kRegBits];
#pragma unroll
    for (int i = 0; i < kRegBits; ++i) roff[i] = 1ull << a.rq[i];
    const int ncq = a.nq - kRegBits - a.nt;
    const uint64_t tiles = 1ull << ncq;
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        uint64_t base = tpart;
        for (int j = 0; j < ncq; ++j) base |= ((tile >> j) & 1ull) << a.cq[j];
        Cx<Real> v[1 << kRegBits];
#pragma unroll
        for (int k = 0; k < (1 << kRegBits); ++k) {
            uint64_t i = base;
#pragma unroll
            for (int b = 0; b < kRegBits; ++b)
                if (k & (1 << b)) i |= roff[b];
            v[k] = st[i];
        }
        for (int g = 0; g < a.ngates; ++g) reg_gate<Real>(v, a.gates[g]);
        // recompute the store addresses rather than keep the 32 load
        // addresses alive through the gates (two registers each)
        asm volatile("" : "+v"(base));
#pragma unroll
        for (int k = 0; k < (1 << kRegBits); ++k) {
            uint64_t i = base;
#pragma unroll
            for (int b = 0; b < kRegBits; ++b)
                if (k & (1 << b)) i |= roff[b];
            st[i] = v[k];
        }
    }
}

// ---------------------------------------------------------------- launchers

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

hipError_t launch_fused(bool c128, const FusedArgs &a, hipStream_t s) {
    const uint64_t tiles = 1ull << (a.nq - a.m);
    const unsigned nb = (unsigned)(tiles < (uint64_t)kGateBlocksMax ? tiles : (uint64_t)kGateBlocksMax);
    const size_t lds = (size_t)(c128 ? 16 : 8) << a.m;
    if (lds > 65536) return hipErrorInvalidValue;
    if (c128)
        hipLaunchKernelGGL(fused_kernel<double>, dim3(nb), dim3(256), lds, s, a);
    else
        hipLaunchKernelGGL(fused_kernel<float>, dim3(nb), dim3(256), lds, s, a);
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
