// Exact solvers (the references of Sec. VII, extended past 2x2): the
// Hamiltonian of Eq. (effi) applied to a state, its ground energy by the
// Lanczos recurrence, and stepwise exact evolution exp(-i dt H(s_k)) by a
// Krylov (Lanczos) basis per step.  Every vector operation runs on the
// device; the host only sequences launches and works on the small
// tridiagonal matrices.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "z2h_runtime.h"
#include "z2h_solvers.h"

using namespace z2h;
using namespace z2h::rt;

namespace {

constexpr int kCheckEvery = 8;   // Lanczos iterations between convergence checks
static_assert(kHamWorkersMax <= kVecBlocks, "the |w|^2 partials of a fused pass fit the vector-kernel slots");

size_t state_bytes(const Plan &P) { return P.esize << P.n; }

int ham_workers(const GroupGeom &g) {
    const uint64_t tiles = 1ull << g.tiles_log2;
    return (int)std::min<uint64_t>(tiles, (uint64_t)kHamWorkersMax);
}

unsigned vec_blocks(const Plan &P) {
    const uint64_t need = ((1ull << P.n) + 255) / 256;
    return (unsigned)std::min<uint64_t>(need, (uint64_t)kVecBlocks);
}

// XCD-major order for the passes over the groups the plan selects, on
// grids of eight or more workers per CU (as the Trotter pass kernels).
static int ham_xcd(const Plan &P, int group, int workers) {
    return ((P.xcd >> group) & 1) && workers >= 8 * 256 ? 1 : 0;
}

// y = H x: passes over groups 0, 1, .., K-1, .., 1, 0 (one pass when K = 1).
// The last pass writes Re<x, y> partials to apart (if not null).
z2h_status ham_passes(const Plan &P, const void *x, void *y, const z2h_couplings &H, double *apart,
                      int *napart, hipStream_t s) {
    HamArgs a;
    memset(&a, 0, sizeof a);
    a.lat = P.lat;
    a.JA = H.JA;
    a.JB = H.JB;
    a.hx = H.hx;
    a.hz = H.hz;
    a.xscale = std::ldexp(1.0, -P.n);
    const int K = P.K, npass = 2 * K - 1;
    for (int i = 0; i < npass; ++i) {
        const int gi = i < K ? i : 2 * K - 2 - i;
        a.geom = P.geom[gi];
        a.src = i == 0 ? x : y;
        a.dst = y;
        a.top = gi == K - 1;
        a.final_pass = i == npass - 1;
        a.x = a.final_pass ? x : nullptr;
        a.part = a.final_pass ? apart : nullptr;
        const int w = ham_workers(a.geom);
        a.xcd = ham_xcd(P, gi, w);
        if (a.final_pass && napart) *napart = w;
        hipError_t e = launch_ham(P.c128, a.geom.R, a, (unsigned)w, obs_lds_bytes(P, a.geom, a.geom.R), s);
        if (e != hipSuccess) return fail(Z2H_ERR_HIP, "Hamiltonian pass failed: %s", hipGetErrorString(e));
    }
    return Z2H_OK;
}

// Scratch of the Lanczos recurrence inside a workspace.
struct LanczosWs {
    void *vec[kKrylovMax + 1];   // state-sized buffers
    double *apart, *apart_x, *wpart;
    LanczosCoef *coef;
};

size_t lanczos_carve(const Plan &P, int nvec, int ncoef, char *base, LanczosWs *L) {
    Carver c{base, 0};
    LanczosWs tmp;
    memset(&tmp, 0, sizeof tmp);
    for (int i = 0; i < nvec; ++i) tmp.vec[i] = c.take(state_bytes(P));
    tmp.apart = (double *)c.take(sizeof(double) * 2 * kVecBlocks);  // also the dot kernel's (Re, Im) pairs
    tmp.apart_x = (double *)c.take(sizeof(double) * kHamWorkersMax);
    tmp.wpart = (double *)c.take(sizeof(double) * kVecBlocks);
    tmp.coef = (LanczosCoef *)c.take(sizeof(LanczosCoef) * (size_t)ncoef);
    if (L) *L = tmp;
    return align256(c.off);
}

z2h_status norm_start(const Plan &P, const void *u, const LanczosWs &L, hipStream_t s) {
    VecArgs v;
    memset(&v, 0, sizeof v);
    v.u = u;
    v.nelem = 1ull << P.n;
    v.mode = 1;
    v.part = L.wpart;
    const unsigned nb = vec_blocks(P);
    hipError_t e = launch_vec(P.c128, v, nb, s);
    if (e == hipSuccess) {
        ScalarArgs sa;
        memset(&sa, 0, sizeof sa);
        sa.wpart = L.wpart;
        sa.nwpart = (int)nb;
        sa.mode = 1;
        sa.coef = L.coef;
        e = launch_scalar(sa, s);
    }
    if (e != hipSuccess) return fail(Z2H_ERR_HIP, "Lanczos start norm failed: %s", hipGetErrorString(e));
    return Z2H_OK;
}

z2h_status launch_scalar_k(const LanczosWs &L, int k, int napart, int napart2, int nwpart, hipStream_t s) {
    ScalarArgs sa;
    memset(&sa, 0, sizeof sa);
    sa.apart = L.apart;
    sa.napart = napart;
    sa.apart2 = napart2 ? L.apart_x : nullptr;
    sa.napart2 = napart2;
    sa.wpart = L.wpart;
    sa.nwpart = nwpart;
    sa.k = k;
    sa.mode = 0;
    sa.coef = L.coef;
    hipError_t e = launch_scalar(sa, s);
    if (e != hipSuccess) return fail(Z2H_ERR_HIP, "Lanczos coefficient kernel failed: %s", hipGetErrorString(e));
    return Z2H_OK;
}

// One Lanczos iteration k: w = sigma_k (H u - alpha_k u) - beta_k sigma_{k-1} p
// written to w; coef[k].alpha and coef[k+1] (beta, sigma).  With several
// groups the update is fused into the Hamiltonian's passes (alpha from the
// first and the top pass, w written by the last one); a one-group plan
// forms y = H u and updates in an elementwise kernel.
z2h_status lanczos_iter(const Plan &P, const z2h_couplings &H, int k, const void *u, const void *p, void *w,
                        void *y, const LanczosWs &L, hipStream_t s) {
    if (P.K > 1) {
        HamArgs a;
        memset(&a, 0, sizeof a);
        a.lat = P.lat;
        a.JA = H.JA;
        a.JB = H.JB;
        a.hx = H.hx;
        a.hz = H.hz;
        a.xscale = std::ldexp(1.0, -P.n);
        const int K = P.K, npass = 2 * K - 1;
        const int nz = ham_workers(P.geom[0]), nx = ham_workers(P.geom[K - 1]);
        for (int i = 0; i < npass; ++i) {
            const int gi = i < K ? i : 2 * K - 2 - i;
            a.geom = P.geom[gi];
            a.src = i == 0 ? u : y;
            a.dst = y;
            a.top = gi == K - 1;
            a.final_pass = i == npass - 1;
            a.part_z = i == 0 ? L.apart : nullptr;
            a.part_x = gi == K - 1 ? L.apart_x : nullptr;
            if (a.final_pass) {
                a.x = u;
                a.lz = 1;
                a.p = k > 0 ? p : nullptr;
                a.use_prev = k > 0;
                a.w = w;
                a.part_w = L.wpart;
                a.apart_z = L.apart;
                a.napart_z = nz;
                a.apart_x = L.apart_x;
                a.napart_x = nx;
                a.coef = L.coef;
                a.k = k;
            }
            a.xcd = ham_xcd(P, gi, ham_workers(a.geom));
            hipError_t e = launch_ham(P.c128, a.geom.R, a, (unsigned)ham_workers(a.geom),
                                      obs_lds_bytes(P, a.geom, a.geom.R), s);
            if (e != hipSuccess) return fail(Z2H_ERR_HIP, "Lanczos pass failed: %s", hipGetErrorString(e));
        }
        return launch_scalar_k(L, k, nz, nx, nz, s);
    }
    int napart = 0;
    z2h_status st = ham_passes(P, u, y, H, L.apart, &napart, s);
    if (st) return st;
    VecArgs v;
    memset(&v, 0, sizeof v);
    v.y = y;
    v.u = u;
    v.p = k > 0 ? p : nullptr;
    v.w = w;
    v.nelem = 1ull << P.n;
    v.apart = L.apart;
    v.napart = napart;
    v.k = k;
    v.use_prev = k > 0;
    v.mode = 0;
    v.coef = L.coef;
    v.part = L.wpart;
    const unsigned nb = vec_blocks(P);
    hipError_t e = launch_vec(P.c128, v, nb, s);
    if (e != hipSuccess) return fail(Z2H_ERR_HIP, "Lanczos update failed: %s", hipGetErrorString(e));
    return launch_scalar_k(L, k, napart, 0, (int)nb, s);
}

// Both pointers valid and the byte ranges [a, a + na) and [b, b + nb) disjoint.
z2h_status check_pair(const void *a, size_t sa, const void *b, size_t sb, const char *na, const char *nb) {
    z2h_status st = validate_state_ptr(a, na);
    if (!st) st = validate_state_ptr(b, nb);
    if (st) return st;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    if (x < y + sb && y < x + sa) return fail(Z2H_ERR_INVALID, "%s and %s overlap", na, nb);
    return Z2H_OK;
}

bool finite4(const z2h_couplings &c) {
    return std::isfinite(c.JA) && std::isfinite(c.JB) && std::isfinite(c.hx) && std::isfinite(c.hz);
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a[0..m) and off-diagonal b[1..m) (Sturm count from the pivots of
// the LDL^T factorisation of T - x I).
int sturm_count(const double *a, const double *b, int m, double x) {
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < m; ++i) {
        const double off = i > 0 ? b[i] * b[i] / q : 0.0;
        q = a[i] - x - off;
        if (q == 0.0) q = -1e-300;
        if (q < 0) ++cnt;
    }
    return cnt;
}

// Lowest eigenvalue by bisection inside the Gershgorin interval.
double tridiag_lowest(const double *a, const double *b, int m) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i]) : 0.0) + (i + 1 < m ? std::fabs(b[i + 1]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(a, b, m, mid) >= 1)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Eigen-decomposition of the symmetric tridiagonal T (diagonal a[0..m),
// off-diagonal b[1..m)) by cyclic Jacobi rotations: T = Q diag(lam) Q^T,
// Q row-major (column l is the eigenvector of lam[l]).
void tridiag_eigs(const double *a, const double *b, int m, std::vector<double> &lam, std::vector<double> &Q) {
    std::vector<double> A((size_t)m * m, 0.0);
    Q.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) {
        A[(size_t)i * m + i] = a[i];
        if (i > 0) A[(size_t)i * m + i - 1] = A[(size_t)(i - 1) * m + i] = b[i];
        Q[(size_t)i * m + i] = 1.0;
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                const double v = A[(size_t)i * m + j] * A[(size_t)i * m + j];
                tot += v;
                if (i != j) off += v;
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = A[(size_t)p * m + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
                // rotation angle that zeroes A[p][q]
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < m; ++k) {
                    const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                    A[(size_t)k * m + p] = c * akp - s * akq;
                    A[(size_t)k * m + q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {
                    const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
                    A[(size_t)p * m + k] = c * apk - s * aqk;
                    A[(size_t)q * m + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    const double qkp = Q[(size_t)k * m + p], qkq = Q[(size_t)k * m + q];
                    Q[(size_t)k * m + p] = c * qkp - s * qkq;
                    Q[(size_t)k * m + q] = s * qkp + c * qkq;
                }
            }
    }
    lam.resize((size_t)m);
    for (int l = 0; l < m; ++l) lam[l] = A[(size_t)l * m + l];
}

// Eigenvector of the lowest eigenvalue theta of T (diagonal a[0..m),
// off-diagonal b[1..m)) by inverse iteration: with the shift theta - delta
// just below the spectrum, T - shift is positive definite, so each solve is
// a stable LDL^T (Thomas) elimination.  The result has unit norm.
void tridiag_lowest_vector(const double *a, const double *b, int m, double theta, std::vector<double> &x) {
    double scale = 0.0;
    for (int i = 0; i < m; ++i) scale = std::max(scale, std::fabs(a[i]) + (i > 0 ? std::fabs(b[i]) : 0.0));
    const double shift = theta - 1e-10 * std::max(1.0, scale);
    x.assign((size_t)m, 1.0 / std::sqrt((double)m));
    std::vector<double> d((size_t)m), l((size_t)m), z((size_t)m);
    for (int it = 0; it < 4; ++it) {
        // factor (T - shift) = L D L^T and solve L D L^T x' = x
        d[0] = a[0] - shift;
        z[0] = x[0];
        for (int i = 1; i < m; ++i) {
            l[i] = b[i] / d[i - 1];
            d[i] = a[i] - shift - l[i] * b[i];
            z[i] = x[i] - l[i] * z[i - 1];
        }
        x[m - 1] = z[m - 1] / d[m - 1];
        for (int i = m - 2; i >= 0; --i) x[i] = z[i] / d[i] - l[i + 1] * x[i + 1];
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += x[i] * x[i];
        nrm = std::sqrt(nrm);
        for (int i = 0; i < m; ++i) x[i] /= nrm;
    }
}

// exp(-i tau T) e_1 = Q diag(exp(-i tau lam)) Q^T e_1 (m <= kKrylovMax).
void tridiag_expv(const double *a, const double *b, int m, double tau, std::complex<double> *out) {
    std::vector<double> lam, Q;
    tridiag_eigs(a, b, m, lam, Q);
    for (int j = 0; j < m; ++j) out[j] = 0.0;
    for (int l = 0; l < m; ++l) {
        const std::complex<double> ph(std::cos(tau * lam[l]), -std::sin(tau * lam[l]));
        const double w = Q[(size_t)0 * m + l];
        for (int j = 0; j < m; ++j) out[j] += Q[(size_t)j * m + l] * w * ph;
    }
}

// Sum of the dot kernel's per-block partials (fixed order): (Re, Im) in
// mode 0, the squared norm in mode 1.
z2h_status dot_host(const Plan &P, const void *x, const void *y, double theta, int mode, double *part, double out[2],
                    hipStream_t s) {
    DotArgs d;
    memset(&d, 0, sizeof d);
    d.a = x;
    d.b = y;
    d.theta = theta;
    d.mode = mode;
    d.nelem = 1ull << P.n;
    d.part = part;
    const unsigned nb = vec_blocks(P);
    hipError_t e = launch_dot(P.c128, d, nb, s);
    if (e != hipSuccess) return fail(Z2H_ERR_HIP, "dot kernel failed: %s", hipGetErrorString(e));
    std::vector<double> h(2 * (size_t)nb);
    HIP_TRY(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out[0] = out[1] = 0.0;
    for (unsigned i = 0; i < nb; ++i) {
        out[0] += h[2 * i];
        out[1] += h[2 * i + 1];
    }
    return Z2H_OK;
}

double sched_s_host(const z2h_schedule &S, int64_t k) {
    return S.sampling ? (double)(k + 1) / (double)S.steps : ((double)k + 0.5) / (double)S.steps;
}

}  // namespace

extern "C" {

z2h_status z2h_hamiltonian_apply(const z2h_plan *plan, const void *d_x, void *d_y, const z2h_couplings *H,
                                 void *stream) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        const Plan &P = plan->P;
        if (!H || !finite4(*H)) return fail(Z2H_ERR_INVALID, "couplings NULL or not finite");
        z2h_status st = check_pair(d_x, state_bytes(P), d_y, state_bytes(P), "d_x", "d_y");
        if (st) return st;
        if ((st = check_device_(P))) return st;
        return ham_passes(P, d_x, d_y, *H, nullptr, nullptr, (hipStream_t)stream);
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_hamiltonian_apply");
    }
}

z2h_status z2h_lanczos_sizes(const z2h_plan *plan, int32_t max_iter, size_t *ws_bytes) {
    if (!plan || !ws_bytes) return fail(Z2H_ERR_INVALID, "plan or ws_bytes is NULL");
    if (max_iter < 1 || max_iter > 100000) return fail(Z2H_ERR_INVALID, "max_iter %d out of [1, 100000]", max_iter);
    *ws_bytes = lanczos_carve(plan->P, 2, max_iter + 2, nullptr, nullptr);
    return Z2H_OK;
}

z2h_status z2h_lanczos_ground(const z2h_plan *plan, void *d_v, void *d_ws, size_t ws_bytes, const z2h_couplings *H,
                              int32_t max_iter, double tol, double *h_alpha, double *h_beta, int32_t *iters,
                              double *e0, void *stream) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        const Plan &P = plan->P;
        if (!H || !finite4(*H)) return fail(Z2H_ERR_INVALID, "couplings NULL or not finite");
        if (!e0 || !iters) return fail(Z2H_ERR_INVALID, "e0 or iters is NULL");
        if (max_iter < 1 || max_iter > 100000) return fail(Z2H_ERR_INVALID, "max_iter %d out of [1, 100000]", max_iter);
        if (!(tol >= 0.0)) return fail(Z2H_ERR_INVALID, "tol must be >= 0");
        z2h_status st = validate_state_ptr(d_v, "d_v");
        if (st) return st;
        if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(Z2H_ERR_INVALID, "d_ws NULL or not 256-byte aligned");
        const size_t need = lanczos_carve(P, 2, max_iter + 2, nullptr, nullptr);
        if (ws_bytes < need) return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
        if ((st = check_pair(d_v, state_bytes(P), d_ws, ws_bytes, "d_v", "d_ws"))) return st;
        if ((st = check_device_(P))) return st;
        hipStream_t s = (hipStream_t)stream;
        LanczosWs L;
        lanczos_carve(P, 2, max_iter + 2, (char *)d_ws, &L);
        void *u = d_v, *p = L.vec[0], *y = L.vec[1];
        if ((st = norm_start(P, u, L, s))) return st;
        std::vector<LanczosCoef> hc((size_t)max_iter + 2);
        std::vector<double> a, b;
        double theta = 0.0, prev = NAN;
        int done = 0;
        for (int k = 0; k < max_iter; ++k) {
            if ((st = lanczos_iter(P, *H, k, u, p, p, y, L, s))) return st;
            std::swap(u, p);  // the new vector was written over the previous one
            done = k + 1;
            if (done % kCheckEvery != 0 && done != max_iter) continue;
            HIP_TRY(hipMemcpyAsync(hc.data(), L.coef, sizeof(LanczosCoef) * (size_t)(done + 1), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (!(hc[0].beta > 0.0)) return fail(Z2H_ERR_NUMERIC, "start vector has zero norm");
            a.assign((size_t)done, 0.0);
            b.assign((size_t)done + 1, 0.0);
            for (int i = 0; i < done; ++i) {
                a[i] = hc[i].alpha;
                b[i] = i > 0 ? hc[i].beta : 0.0;
                if (!std::isfinite(a[i]) || !std::isfinite(b[i])) return fail(Z2H_ERR_NUMERIC, "non-finite Lanczos coefficient");
            }
            b[done] = hc[done].beta;
            // An invariant subspace (beta ~ 0) ends the recurrence: T is cut
            // there, and the vectors after it are not used.
            double scale = 0.0;
            for (int i = 0; i < done; ++i) scale = std::max(scale, std::fabs(a[i]) + b[i]);
            int cut = 0;
            for (int i = 1; i <= done && !cut; ++i)
                if (b[i] <= 1e-13 * std::max(scale, 1e-300)) cut = i;
            if (cut) {
                done = cut;
                theta = tridiag_lowest(a.data(), b.data(), done);
                break;
            }
            theta = tridiag_lowest(a.data(), b.data(), done);
            if (std::fabs(theta - prev) <= tol * std::max(1.0, std::fabs(theta))) break;
            prev = theta;
        }
        *iters = done;
        *e0 = theta;
        for (int i = 0; i < done; ++i) {
            if (h_alpha) h_alpha[i] = a[i];
            if (h_beta) h_beta[i] = b[i + 1];
        }
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_lanczos_ground");
    }
}

z2h_status z2h_exact_sizes(const z2h_plan *plan, int32_t krylov_dim, size_t *ws_bytes) {
    if (!plan || !ws_bytes) return fail(Z2H_ERR_INVALID, "plan or ws_bytes is NULL");
    if (krylov_dim < 1 || krylov_dim > kKrylovMax)
        return fail(Z2H_ERR_INVALID, "krylov_dim %d out of [1, %d]", krylov_dim, kKrylovMax);
    *ws_bytes = lanczos_carve(plan->P, krylov_dim + 1, krylov_dim + 2, nullptr, nullptr);
    return Z2H_OK;
}

z2h_status z2h_exact_evolve(const z2h_plan *plan, void *d_state, void *d_ws, size_t ws_bytes,
                            const z2h_schedule *sched, int32_t krylov_dim, double *err_est, void *stream) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        const Plan &P = plan->P;
        z2h_status st = validate_schedule(P, sched);
        if (st) return st;
        if (krylov_dim < 1 || krylov_dim > kKrylovMax)
            return fail(Z2H_ERR_INVALID, "krylov_dim %d out of [1, %d]", krylov_dim, kKrylovMax);
        const int m = krylov_dim;
        if ((st = validate_state_ptr(d_state, "d_state"))) return st;
        if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(Z2H_ERR_INVALID, "d_ws NULL or not 256-byte aligned");
        const size_t need = lanczos_carve(P, m + 1, m + 2, nullptr, nullptr);
        if (ws_bytes < need) return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
        if ((st = check_pair(d_state, state_bytes(P), d_ws, ws_bytes, "d_state", "d_ws"))) return st;
        if ((st = check_device_(P))) return st;
        hipStream_t s = (hipStream_t)stream;
        LanczosWs L;
        lanczos_carve(P, m + 1, m + 2, (char *)d_ws, &L);
        void *y = L.vec[m];
        const void *ub[kKrylovMax + 1];
        ub[0] = d_state;
        for (int j = 1; j <= m; ++j) ub[j] = L.vec[j - 1];
        std::vector<LanczosCoef> hc((size_t)m + 2);
        std::vector<double> a((size_t)m), b((size_t)m + 1);
        std::vector<std::complex<double>> e((size_t)m);
        double err = 0.0;
        const z2h_schedule &S = *sched;
        for (int64_t k = S.k_begin; k < S.k_end; ++k) {
            const double s0 = sched_s_host(S, k);
            const double sz = S.sZ ? S.sZ[k] : s0, sx = S.sX ? S.sX[k] : s0;
            z2h_couplings H;
            H.JA = S.start.JA + sx * (S.end.JA - S.start.JA);
            H.hx = S.start.hx + sx * (S.end.hx - S.start.hx);
            H.JB = S.start.JB + sz * (S.end.JB - S.start.JB);
            H.hz = S.start.hz + sz * (S.end.hz - S.start.hz);
            if (!finite4(H)) return fail(Z2H_ERR_INVALID, "step %lld: couplings not finite", (long long)k);
            if ((st = norm_start(P, d_state, L, s))) return st;
            for (int j = 0; j < m; ++j) {
                if ((st = lanczos_iter(P, H, j, ub[j], j > 0 ? ub[j - 1] : nullptr, (void *)ub[j + 1], y, L, s)))
                    return st;
            }
            HIP_TRY(hipMemcpyAsync(hc.data(), L.coef, sizeof(LanczosCoef) * (size_t)(m + 1), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            const double nrm = hc[0].beta;
            if (!(nrm > 0.0) || !std::isfinite(nrm)) return fail(Z2H_ERR_NUMERIC, "step %lld: state norm %g", (long long)k, nrm);
            for (int j = 0; j < m; ++j) {
                a[j] = hc[j].alpha;
                b[j] = j > 0 ? hc[j].beta : 0.0;
                if (!std::isfinite(a[j]) || !std::isfinite(b[j]))
                    return fail(Z2H_ERR_NUMERIC, "step %lld: non-finite Krylov coefficient", (long long)k);
            }
            b[m] = hc[m].beta;
            tridiag_expv(a.data(), b.data(), m, S.dt, e.data());
            err += nrm * b[m] * std::abs(e[m - 1]);
            CombineArgs c;
            memset(&c, 0, sizeof c);
            c.psi = d_state;
            c.m = m;
            c.nelem = 1ull << P.n;
            for (int j = 0; j < m; ++j) {
                c.u[j] = ub[j];
                const std::complex<double> cj = nrm * hc[j].sigma * e[j];
                c.cre[j] = cj.real();
                c.cim[j] = cj.imag();
            }
            hipError_t he = launch_combine(P.c128, c, vec_blocks(P), s);
            if (he != hipSuccess) return fail(Z2H_ERR_HIP, "Krylov combination failed: %s", hipGetErrorString(he));
        }
        if (err_est) *err_est = err;
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_exact_evolve");
    }
}

z2h_status z2h_lanczos_vector_sizes(const z2h_plan *plan, int32_t iters, size_t *ws_bytes) {
    if (!plan || !ws_bytes) return fail(Z2H_ERR_INVALID, "plan or ws_bytes is NULL");
    if (iters < 1 || iters > 4096) return fail(Z2H_ERR_INVALID, "iters %d out of [1, 4096]", iters);
    *ws_bytes = lanczos_carve(plan->P, 3, iters + 2, nullptr, nullptr);
    return Z2H_OK;
}

z2h_status z2h_lanczos_vector(const z2h_plan *plan, void *d_v, void *d_ws, size_t ws_bytes, const z2h_couplings *H,
                              const double *h_alpha, const double *h_beta, int32_t iters, double *energy,
                              double *residual, void *stream) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        const Plan &P = plan->P;
        if (!H || !finite4(*H)) return fail(Z2H_ERR_INVALID, "couplings NULL or not finite");
        if (iters < 1 || iters > 4096) return fail(Z2H_ERR_INVALID, "iters %d out of [1, 4096]", iters);
        if (!h_alpha || (iters > 1 && !h_beta)) return fail(Z2H_ERR_INVALID, "alpha or beta is NULL");
        z2h_status st = validate_state_ptr(d_v, "d_v");
        if (st) return st;
        if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(Z2H_ERR_INVALID, "d_ws NULL or not 256-byte aligned");
        const size_t need = lanczos_carve(P, 3, iters + 2, nullptr, nullptr);
        if (ws_bytes < need) return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
        if ((st = check_pair(d_v, state_bytes(P), d_ws, ws_bytes, "d_v", "d_ws"))) return st;
        for (int i = 0; i < iters; ++i)
            if (!std::isfinite(h_alpha[i]) || (i + 1 < iters && !std::isfinite(h_beta[i])))
                return fail(Z2H_ERR_INVALID, "coefficient %d not finite", i);
        if ((st = check_device_(P))) return st;
        // lowest eigenpair of T
        std::vector<double> b((size_t)iters + 1, 0.0), sv;
        for (int i = 1; i < iters; ++i) b[i] = h_beta[i - 1];
        const double theta = tridiag_lowest(h_alpha, b.data(), iters);
        tridiag_lowest_vector(h_alpha, b.data(), iters, theta, sv);
        hipStream_t s = (hipStream_t)stream;
        LanczosWs L;
        lanczos_carve(P, 3, iters + 2, (char *)d_ws, &L);
        void *u = d_v, *p = L.vec[0], *y = L.vec[1], *g = L.vec[2];
        // the same recurrence again (same kernels, so the same vectors),
        // accumulating g = sum_k s_k v_k
        if ((st = norm_start(P, u, L, s))) return st;
        const unsigned nb = vec_blocks(P);
        for (int k = 0; k < iters; ++k) {
            AccArgs a;
            memset(&a, 0, sizeof a);
            a.g = g;
            a.u = u;
            a.coef = L.coef;
            a.s = sv[k];
            a.k = k;
            a.first = k == 0;
            a.nelem = 1ull << P.n;
            hipError_t e = launch_acc(P.c128, a, nb, s);
            if (e != hipSuccess) return fail(Z2H_ERR_HIP, "Ritz accumulation failed: %s", hipGetErrorString(e));
            if (k + 1 < iters) {
                if ((st = lanczos_iter(P, *H, k, u, p, p, y, L, s))) return st;
                std::swap(u, p);
            }
        }
        double nn[2];
        if ((st = dot_host(P, g, g, 0.0, 0, L.apart, nn, s))) return st;
        if (!(nn[0] > 0.0) || !std::isfinite(nn[0])) return fail(Z2H_ERR_NUMERIC, "Ritz vector norm %g", nn[0]);
        CombineArgs c;
        memset(&c, 0, sizeof c);
        c.psi = d_v;
        c.u[0] = g;
        c.cre[0] = 1.0 / std::sqrt(nn[0]);
        c.m = 1;
        c.nelem = 1ull << P.n;
        hipError_t e = launch_combine(P.c128, c, nb, s);
        if (e != hipSuccess) return fail(Z2H_ERR_HIP, "normalisation failed: %s", hipGetErrorString(e));
        double rq = theta;
        if (energy || residual) {
            if ((st = ham_passes(P, d_v, y, *H, nullptr, nullptr, s))) return st;
            double hv[2], rr[2];
            if ((st = dot_host(P, d_v, y, 0.0, 0, L.apart, hv, s))) return st;
            rq = hv[0];
            if ((st = dot_host(P, y, d_v, rq, 1, L.apart, rr, s))) return st;
            if (residual) *residual = std::sqrt(rr[0]);
        }
        if (energy) *energy = rq;
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_lanczos_vector");
    }
}

z2h_status z2h_overlap(const z2h_plan *plan, const void *d_a, const void *d_b, void *d_ws, size_t ws_bytes,
                       double *re, double *im, void *stream) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        if (!re || !im) return fail(Z2H_ERR_INVALID, "re or im is NULL");
        z2h_status st = validate_state_ptr(d_a, "d_a");
        if (!st) st = validate_state_ptr(d_b, "d_b");
        if (st) return st;
        if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(Z2H_ERR_INVALID, "d_ws NULL or not 256-byte aligned");
        if (ws_bytes < sizeof(double) * 2 * kVecBlocks)
            return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, sizeof(double) * 2 * kVecBlocks);
        if ((st = check_device_(plan->P))) return st;
        double o[2];
        if ((st = dot_host(plan->P, d_a, d_b, 0.0, 0, (double *)d_ws, o, (hipStream_t)stream))) return st;
        *re = o[0];
        *im = o[1];
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_overlap");
    }
}

z2h_status z2h_tridiag_lowest(int32_t m, const double *alpha, const double *beta, double *out) {
    if (m < 1 || !alpha || !out || (m > 1 && !beta)) return fail(Z2H_ERR_INVALID, "bad tridiagonal arguments");
    std::vector<double> b((size_t)m + 1, 0.0);
    for (int i = 1; i < m; ++i) b[i] = beta[i - 1];
    *out = tridiag_lowest(alpha, b.data(), m);
    return Z2H_OK;
}

z2h_status z2h_tridiag_expv(int32_t m, const double *alpha, const double *beta, double tau, double *out_re,
                            double *out_im) {
    if (m < 1 || m > kKrylovMax || !alpha || !out_re || !out_im || (m > 1 && !beta))
        return fail(Z2H_ERR_INVALID, "bad tridiagonal arguments");
    std::vector<double> b((size_t)m + 1, 0.0);
    for (int i = 1; i < m; ++i) b[i] = beta[i - 1];
    std::vector<std::complex<double>> e((size_t)m);
    tridiag_expv(alpha, b.data(), m, tau, e.data());
    for (int j = 0; j < m; ++j) {
        out_re[j] = e[j].real();
        out_im[j] = e[j].imag();
    }
    return Z2H_OK;
}

}  // extern "C"
