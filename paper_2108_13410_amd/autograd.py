"""torch.autograd.Function for the final energy of a Trotterized ramp as a
function of its per-step schedule values (the adjoint of include/z2h.h).

forward: evolve psi_0 with schedule values sZ[k], sX[k] and return
L = <psi_M|H_loss|psi_M> (all in the HIP library); backward: z2h_adjoint
(reverse evolution, no stored intermediate states).
"""
from __future__ import annotations

import torch

from . import z2h


class EvolveEnergy(torch.autograd.Function):
    """L(sZ, sX) for a fixed lattice plan, ramp end points and dt.

    sZ, sX: float64 tensors of length M (CPU or CUDA); returns a float64
    scalar tensor on the same device as sZ.
    """

    @staticmethod
    def forward(ctx, sZ, sX, plan, c0, c1, dt, lossH, init=z2h.Z2H_INIT_PSI1):
        M = int(sZ.numel())
        sz_h = sZ.detach().to("cpu", torch.float64).contiguous().numpy()
        sx_h = sX.detach().to("cpu", torch.float64).contiguous().numpy()
        sizes = z2h.z2h_plan_sizes(plan)
        psi = z2h.alloc_state(plan)
        ws = z2h.alloc_bytes(max(sizes["ws_evolve"] + 32 * M + 1024, sizes["ws_observe"],
                                 sizes["ws_adjoint"] + 64 * M + 1024))
        sched = z2h.schedule(c0, c1, M, dt, sZ=sz_h, sX=sx_h)
        z2h.z2h_state_init(plan, psi, init)
        z2h.z2h_evolve(plan, psi, ws, sched)
        L = z2h.z2h_observe(plan, psi, ws, lossH)["energy"]
        ctx.plan, ctx.sched, ctx.lossH = plan, sched, lossH
        ctx.psi, ctx.ws, ctx.M = psi, ws, M
        ctx.dev = sZ.device
        return torch.tensor(L, dtype=torch.float64, device=sZ.device)

    @staticmethod
    def backward(ctx, gL):
        gZ = torch.empty(ctx.M, dtype=torch.float64, device="cuda")
        gX = torch.empty(ctx.M, dtype=torch.float64, device="cuda")
        z2h.z2h_adjoint(ctx.plan, ctx.psi, ctx.ws, ctx.sched, ctx.lossH, gZ, gX)
        g = gL.to("cuda", torch.float64)
        return (g * gZ).to(ctx.dev), (g * gX).to(ctx.dev), None, None, None, None, None, None
