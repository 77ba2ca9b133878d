// Adjoint gradient of the final energy with respect to the per-step
// schedule values (reverse evolution with the inverse passes).
//
// Forward: psi_M = prod_k [X_k^(1/2) Z_k X_k^(1/2)] psi_0 with Z_k =
// exp(-i dt H_Z(sZ[k])) and X_k^(1/2) = exp(-i dt/2 H_X(sX[k])).  With
// lambda = H psi_M carried backwards next to psi through the inverse of every
// pass, dL/dsZ[k] = 2 dt Im <lambda|dH_Z/ds|psi> at the z pass of step k and
// dL/dsX[k] = dt Im <lambda|dH_X/ds|psi> summed over the two x half-steps of
// step k (L = <psi_M|H|psi_M> / <psi_M|psi_M>; every pass is unitary, so no
// forward state needs to be stored).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "z2h_runtime.h"

using namespace z2h;
using namespace z2h::rt;

static size_t adj_ws_fixed(const Plan &P) {
    Carver c{nullptr, 0};
    for (int j = 0; j < 3; ++j) c.take(P.esize << P.n);           // psi, lambda, scratch
    size_t maxtiles = 1;
    for (int g = 0; g < P.K; ++g) maxtiles = std::max(maxtiles, (size_t)1 << P.geom[g].tiles_log2);
    c.take(sizeof(double) * maxtiles);                              // per-block partials
    c.take(sizeof(double) * kObsQ * obs_records(P));                // observable records
    c.take(sizeof(double) * kObsQ);
    return align256(c.off);
}

namespace z2h {
namespace rt {
size_t ws_adjoint_size(const Plan &P) { return adj_ws_fixed(P); }
}  // namespace rt
}  // namespace z2h

static z2h_status adj_launch(const Plan &P, AdjArgs &a, int group, hipStream_t s) {
    a.geom = P.geom[group];
    a.lat = P.lat;
    const unsigned nb = 1u << a.geom.tiles_log2;
    // the adjoint kernel exchanges whole elements whatever the group's
    // exchange in the Trotter passes: size its LDS for that
    GroupGeom ge = a.geom;
    ge.cx = 0;
    hipError_t e = launch_adj(P.c128, a, nb, lds_bytes(P, ge, ge.R), s);
    if (e != hipSuccess) return fail(Z2H_ERR_HIP, "adjoint kernel launch failed: %s", hipGetErrorString(e));
    return Z2H_OK;
}

extern "C" z2h_status z2h_adjoint(const z2h_plan *plan, const void *d_psi_final, void *d_ws, size_t ws_bytes,
                                  const z2h_schedule *sched, const z2h_couplings *lossH, double *d_gradZ,
                                  double *d_gradX, double *h_loss, void *stream) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        const Plan &P = plan->P;
        z2h_status st = validate_state_ptr(d_psi_final, "d_psi_final");
        if (st) return st;
        if ((st = validate_schedule(P, sched))) return st;
        if (!lossH || !d_gradZ || !d_gradX || !d_ws) return fail(Z2H_ERR_INVALID, "NULL argument");
        if ((uintptr_t)d_ws & 255) return fail(Z2H_ERR_INVALID, "d_ws not 256-byte aligned");
        const double *hc = &lossH->JA;
        for (int j = 0; j < 4; ++j)
            if (!std::isfinite(hc[j])) return fail(Z2H_ERR_INVALID, "loss couplings not finite");
        if (sched->k_begin != 0 || sched->k_end != sched->steps || sched->steps < 1)
            return fail(Z2H_ERR_INVALID, "the adjoint needs the whole ramp (k_begin = 0, k_end = steps >= 1)");
        if (sched->order != 0) return fail(Z2H_ERR_UNSUPPORTED, "the adjoint supports the x-z-x step order");
        if (sched->renorm) return fail(Z2H_ERR_INVALID, "the adjoint needs the unitary (renorm = 0) ramp");
        for (int g = 0; g < P.K; ++g)
            if (!P.geom[g].full || !adj_shape_ok(P.geom[g].R, P.geom[g].full))
                return fail(Z2H_ERR_UNSUPPORTED, "plan group %d has no adjoint kernel", g);
        const int S = (int)sched->steps;
        const int Kq0 = std::max(P.K, 2), nlev0 = 2 * (Kq0 - 1) * (S + 1) + 1;
        const size_t need = adj_ws_fixed(P) + 2 * align256(sizeof(double) * S) + align256(sizeof(double) * nlev0);
        if (ws_bytes < need) return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
        if ((st = check_device_(P))) return st;
        hipStream_t s = (hipStream_t)stream;
        const size_t sb = P.esize << P.n;
        Carver c{(char *)d_ws, 0};
        void *A = c.take(sb);
        void *B = c.take(sb);
        void *C = c.take(sb);
        size_t maxtiles = 1;
        for (int g = 0; g < P.K; ++g) maxtiles = std::max(maxtiles, (size_t)1 << P.geom[g].tiles_log2);
        double *part = (double *)c.take(sizeof(double) * maxtiles);
        double *rec = (double *)c.take(sizeof(double) * kObsQ * obs_records(P));
        double *obs_out = (double *)c.take(sizeof(double) * kObsQ);
        double *dsz = (double *)c.take(sizeof(double) * S);
        double *dsx = (double *)c.take(sizeof(double) * S);
        const int K = P.K, Kq = std::max(K, 2), Pp = 2 * (Kq - 1);
        const int nlev = Pp * (S + 1) + 1;
        double *level_sum = (double *)c.take(sizeof(double) * nlev);

        JobDev J = make_job(sched, 0);
        if (sched->sZ) HIP_TRY(hipMemcpyAsync(dsz, sched->sZ, sizeof(double) * S, hipMemcpyHostToDevice, s));
        if (sched->sX) HIP_TRY(hipMemcpyAsync(dsx, sched->sX, sizeof(double) * S, hipMemcpyHostToDevice, s));
        J.sZ = sched->sZ ? dsz : nullptr;
        J.sX = sched->sX ? dsx : nullptr;
        HIP_TRY(hipMemcpyAsync(A, d_psi_final, sb, hipMemcpyDeviceToDevice, s));

        // L and <psi|psi> of the final state
        ObsBuffers ob;
        memset(&ob, 0, sizeof ob);
        ob.scratch = C;
        ob.partZ = rec;
        ob.partX = rec + (size_t)obs_workers(P.geom[0]) * kObsQ;
        ob.out = obs_out;
        ob.H_inline[0] = lossH->JA;
        ob.H_inline[1] = lossH->JB;
        ob.H_inline[2] = lossH->hx;
        ob.H_inline[3] = lossH->hz;
        if ((st = run_observe(P, A, 1, ob, nullptr, 0, nullptr, 0, s))) return st;
        double hobs[kObsQ];
        HIP_TRY(hipMemcpyAsync(hobs, obs_out, sizeof hobs, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));  // also completes the schedule uploads
        const double L = hobs[1], N = hobs[0];
        if (!std::isfinite(L) || !(N > 0)) return fail(Z2H_ERR_NUMERIC, "final state has norm %g, energy %g", N, L);

        // lambda = H psi: diagonal part in the computational basis ...
        AdjArgs a;
        memset(&a, 0, sizeof a);
        a.job = J;
        a.mode = 2;
        a.A = A;
        a.B = B;
        a.no_transform = 1;
        a.op.basis = 0;
        a.dJ = -lossH->JB;
        a.dh = -lossH->hz;
        a.dscale = 1.0;
        if ((st = adj_launch(P, a, 0, s))) return st;
        // ... plus the Hadamard-basis part, through a transformed copy
        HIP_TRY(hipMemcpyAsync(C, A, sb, hipMemcpyDeviceToDevice, s));
        AdjArgs x;
        memset(&x, 0, sizeof x);
        x.job = J;
        x.A = C;
        x.B = nullptr;
        if (K == 1) {
            x.mode = 2;
            x.B = C;
            x.op.basis = 1;
            x.dJ = -lossH->JA;
            x.dh = -lossH->hx;
            x.dscale = std::ldexp(1.0, -P.n);
            if ((st = adj_launch(P, x, 0, s))) return st;
        } else {
            x.mode = 0;
            for (int g = 0; g < K - 1; ++g)
                if ((st = adj_launch(P, x, g, s))) return st;
            x.mode = 2;
            x.B = C;
            x.op.basis = 1;
            x.dJ = -lossH->JA;
            x.dh = -lossH->hx;
            x.dscale = std::ldexp(1.0, -P.n);
            if ((st = adj_launch(P, x, K - 1, s))) return st;
            x.mode = 0;
            x.B = nullptr;
            for (int g = K - 2; g >= 0; --g)
                if ((st = adj_launch(P, x, g, s))) return st;
        }
        hipError_t e = launch_axpy(P.c128, B, C, 1ull << P.n, s);
        if (e != hipSuccess) return fail(Z2H_ERR_HIP, "axpy launch failed: %s", hipGetErrorString(e));

        // reverse sweep over the forward levels
        for (int lev = nlev - 1; lev >= 0; --lev) {
            const LevelOp op = level_op_host(lev, Kq, S, 0, 0);
            if (op.kind == kIdle) continue;
            if (K == 1 && op.kind == kPlainH) continue;  // one-group plans transform inside the x pass
            AdjArgs r;
            memset(&r, 0, sizeof r);
            r.job = J;
            r.op = op;
            r.A = A;
            r.B = B;
            const int group = K == 1 ? 0 : op.group;
            if (op.kind == kPlainH) {
                r.mode = 0;
                if ((st = adj_launch(P, r, group, s))) return st;
                continue;
            }
            r.mode = 1;
            r.no_transform = (K == 1 && op.basis == 0) ? 1 : 0;
            // dH/ds in the level's basis
            if (op.basis == 0) {
                r.dJ = -(sched->end.JB - sched->start.JB);
                r.dh = -(sched->end.hz - sched->start.hz);
            } else {
                r.dJ = -(sched->end.JA - sched->start.JA);
                r.dh = -(sched->end.hx - sched->start.hx);
            }
            r.part = part;
            if ((st = adj_launch(P, r, group, s))) return st;
            AdjFinalArgs f;
            memset(&f, 0, sizeof f);
            f.part = part;
            f.np = 1 << P.geom[group].tiles_log2;
            f.out = level_sum + lev;
            e = launch_adj_final(f, s);
            if (e != hipSuccess) return fail(Z2H_ERR_HIP, "adjoint reduction failed: %s", hipGetErrorString(e));
        }
        AdjGradArgs gr;
        memset(&gr, 0, sizeof gr);
        gr.level_sum = level_sum;
        gr.gZ = d_gradZ;
        gr.gX = d_gradX;
        gr.S = S;
        gr.K = Kq;
        gr.P = Pp;
        gr.n = P.n;
        gr.dt = sched->dt;
        gr.inv_norm = 1.0 / N;
        e = launch_adj_grad(gr, s);
        if (e != hipSuccess) return fail(Z2H_ERR_HIP, "gradient assembly failed: %s", hipGetErrorString(e));
        if (h_loss) *h_loss = L;
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_adjoint");
    }
}
