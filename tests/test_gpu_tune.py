"""Autotuner on the GPU: it picks one of its candidates, and every candidate
schedule evolves the state to the same result (oracle-checked default)."""
import numpy as np
import pytest
import torch

from paper_2108_13410_amd import z2h

from helpers import fidelity_loss, gpu_run

pytestmark = pytest.mark.gpu


def run_plan(plan, c0, c1, M, dt):
    sz = z2h.z2h_plan_sizes(plan)
    psi = z2h.alloc_state(plan)
    ws = z2h.alloc_bytes(max(sz["ws_evolve"], sz["ws_observe"]))
    z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
    z2h.z2h_evolve(plan, psi, ws, z2h.schedule(c0, c1, M, dt))
    torch.cuda.synchronize()
    return psi.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("dtype", [z2h.Z2H_C128, z2h.Z2H_C64])
def test_every_candidate_schedule_agrees(dtype, tmp_path):
    c0, c1, M, dt = (1, 1, 0, 0), (1, 1, 0.3, 0.3), 20, 0.05
    ref, _, _ = gpu_run(3, 3, dtype, c0, c1, M, dt)
    cands = z2h.z2h_tune_candidates(3, 3, dtype)
    for c in cands:
        print(f"case schedule {c} dtype={dtype}", flush=True)
        g = run_plan(z2h.z2h_plan_create_config(3, 3, dtype, c), c0, c1, M, dt)
        assert fidelity_loss(ref, g) < (1e-13 if dtype == z2h.Z2H_C128 else 1e-6), c
    cache = str(tmp_path / "tune.txt")
    best, ms = z2h.z2h_autotune(3, 3, dtype, 64, cache)
    print("autotune best", best, ms, flush=True)
    assert best in cands and ms > 0
    assert open(cache).read().split()[3] == best
