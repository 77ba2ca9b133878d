"""z2h_evolve_noalloc (scratch in a fixed device array) against z2h_evolve
(scratch in the caller's workspace): the same kernels, so the states and
per-step norms agree bit for bit.  Two calls in a row, the second on a
smaller input; then z2h_evolve again, so that the fixed array's leftover
contents cannot leak into either path."""
import numpy as np
import pytest
import torch

from paper_2108_13410_amd import workloads, z2h

pytestmark = pytest.mark.gpu


def _pair(Lx, Ly, dtype, M, dt, c1, arrays=None, renorm=1):
    plan = z2h.z2h_plan_create(Lx, Ly, dtype)
    sz = z2h.z2h_plan_sizes(plan)
    kw = {}
    if arrays is not None:
        kw = dict(sZ=arrays[0], sX=arrays[1])
    sched = z2h.schedule(workloads.TORIC, c1, M, dt, renorm=renorm, **kw)
    a = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, a, z2h.Z2H_INIT_PSI1)
    b = a.clone()
    ws = z2h.alloc_bytes(sz["ws_evolve"] + 16 * M + 512)
    na = torch.zeros(M, dtype=torch.float64, device="cuda")
    nb = torch.zeros(M, dtype=torch.float64, device="cuda")
    z2h.z2h_evolve(plan, a, ws, sched, norms=na)
    z2h.z2h_evolve_noalloc(plan, b, sched, norms=nb)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(a), torch.view_as_real(b))
    assert torch.equal(na, nb)
    assert abs(float(na[-1]) - 1.0) < (1e-5 if dtype == z2h.Z2H_C64 else 1e-12)
    return plan, a


def test_noalloc_matches_workspace_path_two_calls():
    print("case noalloc 3x4 c64 M=40, then 3x3 c128 M=25 with schedule arrays", flush=True)
    _pair(3, 4, z2h.Z2H_C64, 40, 0.05, (1.0, 1.0, 0.3, 0.2))
    rng = np.random.default_rng(5)
    M = 25
    k = np.arange(M)
    sZ = (k + 0.5) / M + rng.normal(0, 0.01, M)
    sX = (k + 0.5) / M + rng.normal(0, 0.01, M)
    _pair(3, 3, z2h.Z2H_C128, M, 0.08, (1.0, 1.0, 0.25, 0.35), arrays=(sZ, sX), renorm=0)
    print("case noalloc 3x3 c64 M=30 after the larger calls", flush=True)
    _pair(3, 3, z2h.Z2H_C64, 30, 0.05, (1.0, 1.0, 0.4, 0.1))


def test_noalloc_rejects_oversize_scratch():
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    psi = z2h.alloc_state(plan)
    M = (z2h.Z2H_NOALLOC_SCRATCH_BYTES // 16) + 1
    s = np.full(M, 0.5)
    with pytest.raises(z2h.Z2HError) as err:
        z2h.z2h_evolve_noalloc(plan, psi, z2h.schedule(workloads.TORIC, (1, 1, .1, .1), M, 1e-3, sZ=s, sX=s))
    assert err.value.code == z2h.Z2H_ERR_UNSUPPORTED
