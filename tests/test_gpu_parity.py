"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances: complex128 fidelity loss <= 1e-12 with amplitudes within 1e-10;
complex64 fidelity loss <= 1e-5 with intensive observables within 1e-5
(energy per link, mean fields, loops, weight histogram).
"""
import numpy as np
import pytest

import oracle
from paper_2108_13410_amd import z2h

from helpers import (compare_observables, fidelity_loss, gpu_run, oracle_observables, oracle_run,
                     to_oracle_order)

pytestmark = pytest.mark.gpu

C128, C64 = z2h.Z2H_C128, z2h.Z2H_C64
TC = (1.0, 1.0, 0.0, 0.0)

_cache = {}


def _oracle(key, fn):
    if key not in _cache:
        _cache[key] = fn()
    return _cache[key]


def _check(Lx, Ly, dtype, g_psi, g_obs, o_psi, H):
    n = 2 * Lx * Ly
    o_lib = to_oracle_order(Lx, Ly, g_psi)
    loss = fidelity_loss(o_psi, o_lib)
    o_obs = oracle_observables(Lx, Ly, o_psi, H)
    if dtype == C128:
        assert loss <= 1e-12, loss
        assert np.max(np.abs(o_lib - o_psi)) <= 1e-10
        compare_observables(g_obs, o_obs, 1e-10, n)
    else:
        assert loss <= 1e-5, loss
        compare_observables(g_obs, o_obs, 1e-5, n)
    return loss


@pytest.mark.parametrize("dtype", [C128, C64])
def test_2x2_adiabatic_ramp(dtype):
    """2x2 torus, T = 10, M = 100, ramp from the toric code to (0.2, 0.2)."""
    c1 = (1.0, 1.0, 0.2, 0.2)
    print(f"case 2x2 dtype={dtype}", flush=True)
    g_psi, g_obs, _ = gpu_run(2, 2, dtype, TC, c1, 100, 0.1)
    o = _oracle(("2x2",), lambda: oracle_run(2, 2, TC, c1, 100, 0.1))
    _check(2, 2, dtype, g_psi, g_obs, o, c1)


@pytest.mark.parametrize("dtype", [C128, C64])
def test_3x3_point(dtype):
    """3x3 torus, one point (0.3, 0.3), T = 20, 1000 steps (full size)."""
    c1 = (1.0, 1.0, 0.3, 0.3)
    print(f"case 3x3 M=1000 dtype={dtype}", flush=True)
    g_psi, g_obs, norms = gpu_run(3, 3, dtype, TC, c1, 1000, 0.02, renorm=1 if dtype == C64 else 0)
    o = _oracle(("3x3",), lambda: oracle_run(3, 3, TC, c1, 1000, 0.02))
    _check(3, 3, dtype, g_psi, g_obs, o, c1)
    assert np.all(np.abs(norms - 1) < (1e-12 if dtype == C128 else 1e-5))


@pytest.mark.parametrize("dtype,mtb", [(C128, 8), (C64, 8), (C128, 10)])
def test_multigroup_schedules(dtype, mtb):
    """Small tiles force 3-4 transform groups (the 4x4 pass structure) at n = 18."""
    c1 = (1.0, 0.8, 0.35, 0.25)
    print(f"case 3x3 groups mtb={mtb} dtype={dtype}", flush=True)
    plan = z2h.z2h_plan_create(3, 3, dtype, mtb)
    assert z2h.z2h_plan_info(plan)["groups"] >= 3
    g_psi, g_obs, _ = gpu_run(3, 3, dtype, TC, c1, 30, 0.05, max_tile_bits=mtb)
    o = _oracle(("3x3-30",), lambda: oracle_run(3, 3, TC, c1, 30, 0.05))
    _check(3, 3, dtype, g_psi, g_obs, o, c1)


@pytest.mark.parametrize("Lx,Ly,dtype", [(2, 3, C128), (2, 3, C64), (3, 2, C128), (2, 4, C64)])
def test_rectangular(Lx, Ly, dtype):
    c1 = (0.9, 1.1, 0.4, 0.15)
    print(f"case {Lx}x{Ly} dtype={dtype}", flush=True)
    g_psi, g_obs, _ = gpu_run(Lx, Ly, dtype, TC, c1, 40, 0.1)
    o = _oracle((Lx, Ly, "rect"), lambda: oracle_run(Lx, Ly, TC, c1, 40, 0.1))
    _check(Lx, Ly, dtype, g_psi, g_obs, o, c1)


@pytest.mark.parametrize("order,sampling", [(1, 0), (0, 1), (1, 1)])
def test_order_and_sampling(order, sampling):
    c0, c1 = (1.0, 1.0, 0.05, 0.0), (0.5, 0.5, 0.5, 0.1)
    print(f"case order={order} sampling={sampling}", flush=True)
    for Lx, Ly in ((2, 2), (3, 3)):
        g_psi, g_obs, _ = gpu_run(Lx, Ly, C128, c0, c1, 25, 0.08, order=order, sampling=sampling)
        o = oracle_run(Lx, Ly, c0, c1, 25, 0.08, order=order, sampling=sampling)
        _check(Lx, Ly, C128, g_psi, g_obs, o, c1)


def test_schedule_arrays():
    """Per-step schedule values sZ, sX (the adjoint's parameters)."""
    rng = np.random.default_rng(13410)
    M = 20
    sZ = (np.arange(M) + 0.5) / M + rng.normal(0, 0.05, M)
    sX = (np.arange(M) + 0.5) / M + rng.normal(0, 0.05, M)
    c1 = (1.0, 1.0, 0.3, 0.3)
    for Lx, Ly in ((2, 2), (3, 3)):
        print(f"case arrays {Lx}x{Ly}", flush=True)
        g_psi, g_obs, _ = gpu_run(Lx, Ly, C128, TC, c1, M, 0.1, sZ=sZ, sX=sX)
        o = oracle_run(Lx, Ly, TC, c1, M, 0.1, sZ=sZ, sX=sX)
        _check(Lx, Ly, C128, g_psi, g_obs, o, c1)


@pytest.mark.parametrize("init", [z2h.Z2H_INIT_PSI1, z2h.Z2H_INIT_PSI1P, z2h.Z2H_INIT_ZERO, z2h.Z2H_INIT_PLUS])
def test_initial_states(init):
    """Eqs. (ini1), (ini2) and the product states, evolved a few steps."""
    c1 = (1.0, 1.0, 0.25, 0.3)
    for Lx, Ly in ((2, 2), (3, 3)):
        print(f"case init={init} {Lx}x{Ly}", flush=True)
        g_psi, g_obs, _ = gpu_run(Lx, Ly, C128, TC, c1, 6, 0.1, init=init)
        n = 2 * Lx * Ly
        if init == z2h.Z2H_INIT_PSI1:
            o0 = oracle.init_psi1(Lx, Ly)
        elif init == z2h.Z2H_INIT_PSI1P:
            o0 = oracle.init_psi1p(Lx, Ly)
        elif init == z2h.Z2H_INIT_ZERO:
            o0 = oracle.state(n)
            o0[0] = 1
        else:
            o0 = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
        o = oracle_run(Lx, Ly, TC, c1, 6, 0.1, init=o0)
        _check(Lx, Ly, C128, g_psi, g_obs, o, c1)


def test_split_ramp_equals_whole():
    """Checkpoint/resume: steps [0,k) then [k,M) reproduce the whole ramp."""
    c1 = (1.0, 1.0, 0.3, 0.3)
    a, _, _ = gpu_run(3, 3, C128, TC, c1, 40, 0.05)
    b, _, _ = gpu_run(3, 3, C128, TC, c1, 40, 0.05, chunks=[7, 23])
    assert fidelity_loss(a, b) < 1e-14
    assert np.max(np.abs(a - b)) < 1e-13


def test_zero_steps_is_identity():
    c1 = (1.0, 1.0, 0.3, 0.3)
    g_psi, g_obs, _ = gpu_run(3, 3, C128, TC, c1, 0, 0.1)
    o = oracle.init_psi1(3, 3)
    np.testing.assert_allclose(to_oracle_order(3, 3, g_psi), o, atol=1e-15)
    assert abs(g_obs["energy"] + 18) < 1e-12


def test_zero_field_is_a_phase_at_4x4_shape_small():
    """Zero field: only a global phase exp(+i(JA Ns + JB Np) T); observables stay
    at the toric-code values (checked on 3x3 with a 3-group schedule)."""
    c = (1.0, 0.7, 0.0, 0.0)
    g_psi, g_obs, _ = gpu_run(3, 3, C128, c, c, 50, 0.1, max_tile_bits=8)
    o0 = oracle.init_psi1(3, 3)
    ph = np.exp(1j * 1.7 * 9 * 5.0)
    np.testing.assert_allclose(to_oracle_order(3, 3, g_psi), ph * o0, atol=1e-12)
    assert abs(g_obs["energy"] + 1.7 * 9) < 1e-11
    assert abs(g_obs["xloop"][0] - 1) < 1e-12 and abs(g_obs["xloop"][1] - 1) < 1e-12


@pytest.mark.parametrize("dtype,cfg", [(C64, "split=12:4:12:0/6:3:11:5:2"), (C128, "split=12:4:12:0/6:3:12:6"),
                                       (C128, "split=9:3:10:0/9:3:11:2")])
def test_block_order_is_bitwise_neutral(dtype, cfg):
    """XCD-major block order (per group, ",xcd=<mask>") only renumbers the
    workgroups: every tile is computed by the same code and the norm
    partials are summed in tile order, so all masks give the same state bit
    for bit; the all-groups order is also checked against the oracle."""
    import torch
    c1 = (1.0, 0.9, 0.3, 0.25)
    M, dt = 40, 0.05
    states = []
    for mask in (0, 1, 2, 3):
        print(f"case 3x3 {cfg} xcd={mask} dtype={dtype}", flush=True)
        plan = z2h.z2h_plan_create_config(3, 3, dtype, f"{cfg},xcd={mask}")
        assert z2h.z2h_plan_describe(plan)["xcd"] == mask
        sizes = z2h.z2h_plan_sizes(plan)
        psi = z2h.alloc_state(plan)
        ws = z2h.alloc_bytes(sizes["ws_evolve"] + 16 * M + 1024)
        z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
        z2h.z2h_evolve(plan, psi, ws, z2h.schedule(TC, c1, M, dt, renorm=1 if dtype == C64 else 0))
        torch.cuda.synchronize()
        states.append(psi.cpu().numpy())
        z2h.z2h_plan_destroy(plan)
    for s in states[1:]:
        assert np.array_equal(s.view(np.uint8), states[0].view(np.uint8))
    o = _oracle(("3x3-xcd", M), lambda: oracle_run(3, 3, TC, c1, M, dt))
    loss = fidelity_loss(o, to_oracle_order(3, 3, states[3].astype(np.complex128)))
    assert loss <= (1e-12 if dtype == C128 else 1e-5), loss


@pytest.mark.parametrize("dtype,order", [(C64, 0), (C64, 1), (C128, 0)])
def test_component_exchange_bitwise(dtype, order):
    """2x5 torus (20 qubits), renormalised every step in complex64: layout
    changes that exchange the real and then the imaginary parts (":1c", half
    the LDS) move the same values as the element exchange, so the state and
    the per-step norms are the same bits as with one tile per block (and as
    two-tile blocks in complex64); order 1 adds half passes of mixed kind.
    Checked against the oracle as well."""
    import torch
    c1 = (1.0, 0.9, 0.3, 0.25)
    M, dt = 12, 0.1
    if dtype == C64:
        cfgs = ("split=10:5:11:0:1c/10:5:14:4:1c", "split=10:5:11:0/10:5:14:4", "split=10:5:11:0:2/10:5:14:4:2")
    else:
        cfgs = ("split=10:5:11:0:1c/10:5:13:3:1c", "split=10:5:11:0/10:5:13:3")
    states = []
    for cfg in cfgs:
        print(f"case 2x5 dtype={dtype} {cfg} order={order}", flush=True)
        plan = z2h.z2h_plan_create_config(2, 5, dtype, cfg)
        d = z2h.z2h_plan_describe(plan)
        assert [g["cx"] for g in d["groups"]] == ([1, 1] if ":1c" in cfg else [0, 0])
        sizes = z2h.z2h_plan_sizes(plan)
        psi = z2h.alloc_state(plan)
        ws = z2h.alloc_bytes(sizes["ws_evolve"] + 16 * M + 1024)
        norms = torch.zeros(M, dtype=torch.float64, device="cuda")
        z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
        z2h.z2h_evolve(plan, psi, ws, z2h.schedule(TC, c1, M, dt, renorm=1 if dtype == C64 else 0, order=order),
                       norms=norms)
        torch.cuda.synchronize()
        states.append((psi.cpu().numpy(), norms.cpu().numpy()))
        z2h.z2h_plan_destroy(plan)
    for s, nrm in states[1:]:
        assert np.array_equal(s.view(np.uint8), states[0][0].view(np.uint8))
        assert np.array_equal(nrm, states[0][1])
    o = _oracle(("2x5-cx", order), lambda: oracle_run(2, 5, TC, c1, M, dt, order=order))
    loss = fidelity_loss(o, to_oracle_order(2, 5, states[0][0].astype(np.complex128)))
    assert loss <= (1e-12 if dtype == C128 else 1e-5), loss


@pytest.mark.parametrize("dtype,order,cfg", [(C128, 0, "split=4:2:8:0/10:5:13:3:1c:h3@17/6:3:9:3"),
                                             (C64, 1, "split=4:2:8:0/10:5:14:4:1c:h3@17/6:3:10:4"),
                                             (C128, 1, "split=4:2:8:0/6:3:9:3:at8/10:5:13:3:1c"),
                                             (C64, 0, "split=4:2:8:0/6:3:10:4:at8/10:5:14:4:1c"),
                                             (C128, 0, "split=4:2:8:0/10:4:13:3:h3@17/6:3:9:3"),
                                             (C64, 1, "split=4:2:8:0/6:3:10:4:at8/10:4:13:3")])
def test_split_run_group(dtype, order, cfg):
    """2x5 torus (20 qubits) with a group in two runs of qubits, one of
    whose register windows holds bits of both runs: the middle group
    (qubits 4-10 and 17-19), or the last group (qubits 4-7 and 14-19, with
    the x-basis phase and the x-basis observables on it); groups of whole
    windows run the component-exchange kernels, the others (ten qubits in
    windows of four) the general pass kernel.  State and observables
    against the oracle."""
    c1 = (1.0, 0.8, 0.35, 0.25)
    M, dt = 12, 0.1
    print(f"case 2x5 {cfg} dtype={dtype} order={order}", flush=True)
    plan = z2h.z2h_plan_create_config(2, 5, dtype, cfg)
    assert any(g["hi"] for g in z2h.z2h_plan_describe(plan)["groups"])
    z2h.z2h_plan_destroy(plan)
    g_psi, g_obs, _ = gpu_run(2, 5, dtype, TC, c1, M, dt, config=cfg, order=order,
                              renorm=1 if dtype == C64 else 0)
    o = _oracle(("2x5-split", order), lambda: oracle_run(2, 5, TC, c1, M, dt, order=order))
    _check(2, 5, dtype, g_psi, g_obs, o, c1)


@pytest.mark.parametrize("dtype,M,order", [(C64, 600, 1), (C128, 530, 0)])
def test_precomputed_tables_across_chunks_bitwise(dtype, M, order):
    """z2h_evolve computes the phase tables of up to 1024 levels per launch
    ahead of the passes; z2h_evolve_noalloc lets every workgroup build its
    own. Over more than 1024 levels (two table chunks; order 0 adds the
    half passes of the z-x-z order) both give the same bits, states and
    per-step norms."""
    import torch
    print(f"case tables 3x3 dtype={dtype} M={M} order={order}", flush=True)
    c1 = (1.0, 1.0, 0.35, 0.25)
    plan = z2h.z2h_plan_create(3, 3, dtype)
    sz = z2h.z2h_plan_sizes(plan)
    sched = z2h.schedule(TC, c1, M, 0.02, renorm=1 if dtype == C64 else 0, order=order)
    a = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, a, z2h.Z2H_INIT_PSI1)
    b = a.clone()
    ws = z2h.alloc_bytes(sz["ws_evolve"])
    na = torch.zeros(M, dtype=torch.float64, device="cuda")
    nb = torch.zeros(M, dtype=torch.float64, device="cuda")
    z2h.z2h_evolve(plan, a, ws, sched, norms=na)
    z2h.z2h_evolve_noalloc(plan, b, sched, norms=nb)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(a), torch.view_as_real(b))
    assert torch.equal(na, nb)
    assert abs(float(na[-1]) - 1.0) < (1e-5 if dtype == C64 else 1e-12)
