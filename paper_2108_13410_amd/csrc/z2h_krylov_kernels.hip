// Device kernels of the exact solvers of libz2h: the Hamiltonian of the
// mapped model (Sec. II, Eq. effi) applied to a state, and the vector
// operations of the Lanczos recurrence that the ground-energy and Krylov
// time-evolution entry points build on (the exact references of Sec. VII).
//
// H = D_Z + 2^-n W D_X W, with W the unnormalised Walsh-Hadamard transform
// over all links, D_Z(i) = -JB (nst - 2 k_p(i)) - hz (n - 2 w(i)) the
// plaquette and z-field terms in the computational basis and D_X the star and
// x-field terms in the Hadamard basis (same form with k_v and hx).  The
// transform reuses the tile passes of the Trotter step: one pass per group
// up to the top group, which multiplies by D_X between its forward and
// backward transform, and one pass per group back down; the last pass adds
// D_Z x.  Nothing is exponentiated, so the diagonal is computed per element
// from the syndrome and the Hamming weight.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <set>

#include "z2h_internal.h"
#include "z2h_kernels.h"
#include "z2h_solvers.h"
#include "z2h_tile.h"

namespace z2h {

// Value of one basis' diagonal at syndrome s and weight w.
__device__ __forceinline__ double diag_value(int nst, int n, uint32_t s, int w, double J, double h) {
    return -(J * (double)(nst - 2 * popc(s)) + h * (double)(n - 2 * w));
}

// v *= scale * D_X for the register elements of layout L (Hadamard basis);
// accx (if not null) accumulates scale * sum D_X |v|^2 of the values before
// (a pointer: the accumulator then lives in a scratch slot rather than in
// one of the registers the two prefetched tiles need).
template <typename Real, int R>
__device__ __forceinline__ void mul_diag_x(Cx<Real> (&v)[1 << R], const LayCtx<R> &L, const LatticeDev &lat,
                                           double J, double h, double scale, double *accx) {
    uint32_t s = L.s0x;
#pragma unroll
    for (int idx = 0; idx < (1 << R); ++idx) {
        const int q = idx ^ (idx >> 1);
        if (idx) s ^= L.lx[__builtin_ctz(idx)];
        const double dd = scale * diag_value(lat.nst, lat.n, s, L.w0 + __builtin_popcount(q), J, h);
        if (accx) *accx += dd * ((double)v[q].x * (double)v[q].x + (double)v[q].y * (double)v[q].y);
        const Real d = (Real)dd;
        v[q].x *= d;
        v[q].y *= d;
    }
}

// sum D_Z |v|^2 over the register elements of layout L (computational basis).
template <typename Real, int R>
__device__ __forceinline__ double diag_norm_z(const Cx<Real> (&v)[1 << R], const LayCtx<R> &L,
                                              const LatticeDev &lat, double J, double h) {
    uint32_t s = L.s0z;
    double acc = 0.0;
#pragma unroll
    for (int idx = 0; idx < (1 << R); ++idx) {
        const int q = idx ^ (idx >> 1);
        if (idx) s ^= L.lz[__builtin_ctz(idx)];
        acc += diag_value(lat.nst, lat.n, s, L.w0 + __builtin_popcount(q), J, h) *
               ((double)v[q].x * (double)v[q].x + (double)v[q].y * (double)v[q].y);
    }
    return acc;
}

// Elements of x at the register positions of layout L, eight Gray-code steps
// at a time (each chunk covers eight register elements), so that at most
// eight extra elements of each operand are live beside the tile.
template <int R>
struct Chunk {
    static constexpr int C = (1 << R) < 8 ? (1 << R) : 8;
};

// v += D_Z x for the register elements of layout L (computational basis),
// accumulating Re(conj(x) v) of the result.
template <typename Real, int R, bool SP>
__device__ __forceinline__ void add_diag_z(Cx<Real> (&v)[1 << R], const Cx<Real> *x, const LayCtx<R> &L,
                                           const LatticeDev &lat, double J, double h, double &acc) {
    constexpr int C = Chunk<R>::C;
    uint32_t s = L.s0z;
    const Cx<Real> *b = x + L.i0;
#pragma unroll
    for (int c0 = 0; c0 < (1 << R); c0 += C) {
        Cx<Real> xv[C];
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int q = (c0 + i) ^ ((c0 + i) >> 1);
            xv[i] = b[reg_off<R, SP>(L, q)];
        }
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int idx = c0 + i, q = idx ^ (idx >> 1);
            if (idx) s ^= L.lz[__builtin_ctz(idx)];
            const Real d = (Real)diag_value(lat.nst, lat.n, s, L.w0 + __builtin_popcount(q), J, h);
            v[q].x += d * xv[i].x;
            v[q].y += d * xv[i].y;
            acc += (double)xv[i].x * (double)v[q].x + (double)xv[i].y * (double)v[q].y;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Lanczos form of the last pass: with v = (2^-n W D_X W u) at the register
// positions of layout L, write w = sig (v + D_Z u - alpha u) - cp p and
// accumulate |w|^2.
template <typename Real, int R, bool SP>
__device__ __forceinline__ void lanczos_out(const Cx<Real> (&v)[1 << R], const Cx<Real> *u, const Cx<Real> *p,
                                            Cx<Real> *w, const LayCtx<R> &L, const LatticeDev &lat, double J,
                                            double h, double sig, double alpha, double cp, bool use_prev,
                                            double &acc) {
    constexpr int C = Chunk<R>::C;
    uint32_t s = L.s0z;
    const Cx<Real> *bu = u + L.i0;
    const Cx<Real> *bp = p + L.i0;
    Cx<Real> *bw = w + L.i0;
    const Real rs = (Real)sig, rc = (Real)cp;
#pragma unroll
    for (int c0 = 0; c0 < (1 << R); c0 += C) {
        Cx<Real> uv[C], pv[C];
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int q = (c0 + i) ^ ((c0 + i) >> 1);
            uv[i] = bu[reg_off<R, SP>(L, q)];
            pv[i] = use_prev ? bp[reg_off<R, SP>(L, q)] : Cx<Real>{(Real)0, (Real)0};
        }
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int idx = c0 + i, q = idx ^ (idx >> 1);
            if (idx) s ^= L.lz[__builtin_ctz(idx)];
            const Real d = (Real)(diag_value(lat.nst, lat.n, s, L.w0 + __builtin_popcount(q), J, h) - alpha);
            Cx<Real> r{rs * (v[q].x + d * uv[i].x) - rc * pv[i].x, rs * (v[q].y + d * uv[i].y) - rc * pv[i].y};
            bw[reg_off<R, SP>(L, q)] = r;
            acc += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// PF: the next tile's elements are loaded while the current one is
// transformed (two register tiles; used where they fit without spilling).
template <typename Real, int R, bool PF, bool SP>
__global__ void __launch_bounds__(512) ham_kernel(HamArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const GroupGeom &g = a.geom;
    const uint32_t t = threadIdx.x;
    const uint64_t tiles = 1ull << g.tiles_log2;
    Cx<Real> *lds = reinterpret_cast<Cx<Real> *>(smem);
    const uint32_t lds_elems = (1u << g.m) + (1u << (g.m - R));
    double *red = reinterpret_cast<double *>(lds + lds_elems);
    const Cx<Real> *src = reinterpret_cast<const Cx<Real> *>(a.src);
    Cx<Real> *dst = reinterpret_cast<Cx<Real> *>(a.dst);
    const Cx<Real> *x = reinterpret_cast<const Cx<Real> *>(a.x);
    const bool lz = a.lz && a.final_pass;
    double acc = 0.0, accz = 0.0, accx = 0.0;

    // Lanczos coefficients of this iteration (every block sums the partials
    // of the first and the top pass itself)
    double sig = 0.0, alpha = 0.0, cp = 0.0;
    if (lz) {
        const LanczosCoef ck = a.coef[a.k];
        sig = ck.sigma;
        double sm = 0.0;
        for (int j = (int)t; j < a.napart_z; j += (int)blockDim.x) sm += a.apart_z[j];
        for (int j = (int)t; j < a.napart_x; j += (int)blockDim.x) sm += a.apart_x[j];
        alpha = sig * sig * block_sum(sm, red);
        cp = a.use_prev ? ck.beta * a.coef[a.k - 1].sigma : 0.0;
    }

    const bool syn0 = a.final_pass || a.part_z;
    // logical block: first tile of the grid-stride walk and partial slot
    const uint32_t lb = a.xcd ? xcd_major(blockIdx.x, gridDim.x) : blockIdx.x;
    uint64_t tile = lb;
    Cx<Real> vn[PF ? (1 << R) : 1];
    LayCtx<R> Ln;
    if constexpr (PF) {
        if (tile < tiles) {
            lay_ctx<R, SP>(Ln, g, a.lat, tile, g.p[0], t, syn0);
            load_tile<Real, R, false, SP>(vn, src, Ln);
        }
    }
    for (; tile < tiles; tile += gridDim.x) {
        Cx<Real> v[1 << R];
        LayCtx<R> L0;
        if constexpr (PF) {
            L0 = Ln;
#pragma unroll
            for (int q = 0; q < (1 << R); ++q) v[q] = vn[q];
            const uint64_t nt = tile + gridDim.x;
            if (nt < tiles) {
                lay_ctx<R, SP>(Ln, g, a.lat, nt, g.p[0], t, syn0);
                load_tile<Real, R, false, SP>(vn, src, Ln);
            }
        } else {
            lay_ctx<R, SP>(L0, g, a.lat, tile, g.p[0], t, syn0);
            load_tile<Real, R, false, SP>(v, src, L0);
        }
        if (a.part_z) accz += diag_norm_z<Real, R>(v, L0, a.lat, a.JB, a.hz);
        int cur = 0;
        for (int j = 0; j < g.nlay; ++j) {
            if (j > 0) exchange<Real, R>(v, lds, g.p[j - 1], g.p[j], t);
            butterflies<Real, R>(v, g.blo[j], g.bhi[j]);
            cur = j;
        }
        if (a.top) {
            LayCtx<R> Lm;
            lay_ctx<R, SP>(Lm, g, a.lat, tile, g.p[cur], t, true);
            mul_diag_x<Real, R>(v, Lm, a.lat, a.JA, a.hx, a.xscale, a.part_x ? &accx : nullptr);
            for (int j = g.nlay - 1; j >= 0; --j) {
                if (j != cur) {
                    exchange<Real, R>(v, lds, g.p[cur], g.p[j], t);
                    cur = j;
                }
                butterflies<Real, R>(v, g.blo[j], g.bhi[j]);
            }
        }
        if (cur != 0) exchange<Real, R>(v, lds, g.p[cur], g.p[0], t);
        if (lz) {
            lanczos_out<Real, R, SP>(v, x, reinterpret_cast<const Cx<Real> *>(a.p), reinterpret_cast<Cx<Real> *>(a.w),
                                 L0, a.lat, a.JB, a.hz, sig, alpha, cp, a.use_prev != 0, acc);
            continue;
        }
        if (a.final_pass) add_diag_z<Real, R, SP>(v, x, L0, a.lat, a.JB, a.hz, acc);
        store_tile<Real, R, false, SP>(v, dst, L0);
    }
    if (a.part) {
        const double s = block_sum(acc, red);
        if (t == 0) a.part[lb] = s;
    }
    if (a.part_w) {
        const double s = block_sum(acc, red);
        if (t == 0) a.part_w[lb] = s;
    }
    if (a.part_z) {
        const double s = block_sum(accz, red);
        if (t == 0) a.part_z[lb] = s;
    }
    if (a.part_x) {
        const double s = block_sum(accx, red);
        if (t == 0) a.part_x[lb] = s;
    }
}

// Deterministic sum of n partials by one block (every thread gets it).
__device__ double sum_parts(const double *p, int n, double *red) {
    double s = 0.0;
    for (int j = (int)threadIdx.x; j < n; j += (int)blockDim.x) s += p[j];
    return block_sum(s, red);
}

template <typename Real>
__global__ void __launch_bounds__(256) vec_kernel(VecArgs a) {
    __shared__ double red[8];
    const Cx<Real> *y = reinterpret_cast<const Cx<Real> *>(a.y);
    const Cx<Real> *u = reinterpret_cast<const Cx<Real> *>(a.u);
    const Cx<Real> *p = reinterpret_cast<const Cx<Real> *>(a.p);
    Cx<Real> *w = reinterpret_cast<Cx<Real> *>(a.w);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    if (a.mode == 1) {
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nelem; i += stride) {
            const Cx<Real> e = u[i];
            acc += (double)e.x * (double)e.x + (double)e.y * (double)e.y;
        }
    } else {
        const LanczosCoef ck = a.coef[a.k];
        const double sig = ck.sigma;
        const double alpha = sig * sig * sum_parts(a.apart, a.napart, red);
        const Real cy = (Real)sig, cu = (Real)(alpha * sig);
        const Real cp = a.use_prev ? (Real)(ck.beta * a.coef[a.k - 1].sigma) : (Real)0;
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nelem; i += stride) {
            const Cx<Real> ey = y[i], eu = u[i];
            Cx<Real> r{cy * ey.x - cu * eu.x, cy * ey.y - cu * eu.y};
            if (a.use_prev) {
                const Cx<Real> ep = p[i];
                r.x -= cp * ep.x;
                r.y -= cp * ep.y;
            }
            w[i] = r;
            acc += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
        }
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) scalar_kernel(ScalarArgs a) {
    __shared__ double red[8];
    if (a.mode == 1) {
        const double nn = sum_parts(a.wpart, a.nwpart, red);
        if (threadIdx.x == 0) {
            const double b = sqrt(nn);
            a.coef[0] = LanczosCoef{0.0, b, b > 1e-300 ? 1.0 / b : 0.0, 0.0};
        }
        return;
    }
    const double sig = a.coef[a.k].sigma;
    const double alpha = sig * sig * (sum_parts(a.apart, a.napart, red) + sum_parts(a.apart2, a.napart2, red));
    const double nn = sum_parts(a.wpart, a.nwpart, red);
    if (threadIdx.x == 0) {
        a.coef[a.k].alpha = alpha;
        const double b = sqrt(nn);
        a.coef[a.k + 1] = LanczosCoef{0.0, b, b > 1e-300 ? 1.0 / b : 0.0, 0.0};
    }
}

template <typename Real>
__global__ void __launch_bounds__(256) combine_kernel(CombineArgs a) {
    Cx<Real> *psi = reinterpret_cast<Cx<Real> *>(a.psi);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nelem; i += stride) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < a.m; ++j) {
            const Cx<Real> e = reinterpret_cast<const Cx<Real> *>(a.u[j])[i];
            re += a.cre[j] * (double)e.x - a.cim[j] * (double)e.y;
            im += a.cre[j] * (double)e.y + a.cim[j] * (double)e.x;
        }
        psi[i] = Cx<Real>{(Real)re, (Real)im};
    }
}

template <typename Real>
__global__ void __launch_bounds__(256) acc_kernel(AccArgs a) {
    Cx<Real> *g = reinterpret_cast<Cx<Real> *>(a.g);
    const Cx<Real> *u = reinterpret_cast<const Cx<Real> *>(a.u);
    const double c = a.s * a.coef[a.k].sigma;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nelem; i += stride) {
        const Cx<Real> e = u[i];
        double re = c * (double)e.x, im = c * (double)e.y;
        if (!a.first) {
            const Cx<Real> o = g[i];
            re += (double)o.x;
            im += (double)o.y;
        }
        g[i] = Cx<Real>{(Real)re, (Real)im};
    }
}

template <typename Real>
__global__ void __launch_bounds__(256) dot_kernel(DotArgs a) {
    __shared__ double red[8];
    const Cx<Real> *x = reinterpret_cast<const Cx<Real> *>(a.a);
    const Cx<Real> *y = reinterpret_cast<const Cx<Real> *>(a.b);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    double s0 = 0.0, s1 = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nelem; i += stride) {
        const Cx<Real> p = x[i], q = y[i];
        if (a.mode == 0) {  // conj(p) q
            s0 += (double)p.x * (double)q.x + (double)p.y * (double)q.y;
            s1 += (double)p.x * (double)q.y - (double)p.y * (double)q.x;
        } else {
            const double dr = (double)p.x - a.theta * (double)q.x, di = (double)p.y - a.theta * (double)q.y;
            s0 += dr * dr + di * di;
        }
    }
    const double r0 = block_sum(s0, red);
    const double r1 = block_sum(s1, red);
    if (threadIdx.x == 0) {
        a.part[2 * blockIdx.x] = r0;
        a.part[2 * blockIdx.x + 1] = r1;
    }
}

// ---------------------------------------------------------------- launchers

static std::mutex g_krylov_lds_mu;
static std::set<const void *> g_krylov_lds_done;

static hipError_t allow_lds(const void *fn, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_krylov_lds_mu);
    if (g_krylov_lds_done.count(fn)) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e == hipSuccess) g_krylov_lds_done.insert(fn);
    return e;
}

template <typename Real, int R, bool PF, bool SP>
static hipError_t do_ham_pf(const HamArgs &a, unsigned workers, size_t lds, hipStream_t s) {
    const void *fn = reinterpret_cast<const void *>(&ham_kernel<Real, R, PF, SP>);
    hipError_t e = allow_lds(fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ham_kernel<Real, R, PF, SP>), dim3(workers), dim3(1u << (a.geom.m - R)), lds, s, a);
    return hipGetLastError();
}

// Two register tiles fit without spilling up to 256 bytes of elements per
// thread, except complex64 at R = 5, whose 32 elements per tile need more
// index and syndrome registers than the other shapes.
template <typename Real, int R>
static hipError_t do_ham(const HamArgs &a, unsigned workers, size_t lds, hipStream_t s) {
    if (a.geom.m - R < 6 || a.geom.m - R > 9) return hipErrorInvalidConfiguration;  // launch bounds
    constexpr bool pf = (2 * sizeof(Real) << R) <= 256 && !(sizeof(Real) == 4 && R == 5);
    // groups in two runs of qubits take the kernel with their address map
    if (a.geom.hi) return do_ham_pf<Real, R, pf, true>(a, workers, lds, s);
    return do_ham_pf<Real, R, pf, false>(a, workers, lds, s);
}

hipError_t launch_ham(bool c128, int R, const HamArgs &a, unsigned workers, size_t lds, hipStream_t s) {
    if (c128) {
        switch (R) {
            case 2: return do_ham<double, 2>(a, workers, lds, s);
            case 3: return do_ham<double, 3>(a, workers, lds, s);
            case 4: return do_ham<double, 4>(a, workers, lds, s);
            case 5: return do_ham<double, 5>(a, workers, lds, s);
        }
    } else {
        switch (R) {
            case 2: return do_ham<float, 2>(a, workers, lds, s);
            case 3: return do_ham<float, 3>(a, workers, lds, s);
            case 4: return do_ham<float, 4>(a, workers, lds, s);
            case 5: return do_ham<float, 5>(a, workers, lds, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_vec(bool c128, const VecArgs &a, unsigned blocks, hipStream_t s) {
    if (c128)
        hipLaunchKernelGGL(vec_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(vec_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scalar(const ScalarArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(scalar_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_acc(bool c128, const AccArgs &a, unsigned blocks, hipStream_t s) {
    if (c128)
        hipLaunchKernelGGL(acc_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(acc_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dot(bool c128, const DotArgs &a, unsigned blocks, hipStream_t s) {
    if (c128)
        hipLaunchKernelGGL(dot_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(dot_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_combine(bool c128, const CombineArgs &a, unsigned blocks, hipStream_t s) {
    if (c128)
        hipLaunchKernelGGL(combine_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(combine_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace z2h
