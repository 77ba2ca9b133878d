"""Piecewise-linear paths with observable traces (z2h_path_evolve) against
the oracle: every trace sample equals the oracle's observables after the same
number of gate-level Trotter steps along the same legs (Sec. III, Fig. evo).
Legs are emulated on the oracle with explicit per-step schedule values, so
the oracle runs exactly the steps the path prescribes."""
import numpy as np
import pytest
import torch

import oracle
from helpers import compare_observables, oracle_observables, standard_loops_lib, to_oracle_order
from paper_2108_13410_amd import z2h

pytestmark = pytest.mark.gpu


def oracle_path(Lx, Ly, init, verts, steps, dt, sampling, order, every):
    """Observables of the oracle state at the path's sample points."""
    psi = {"psi1": oracle.init_psi1, "psi1p": oracle.init_psi1p}[init](Lx, Ly)
    out = [oracle_observables(Lx, Ly, psi, verts[0])]
    for i, M in enumerate(steps):
        if M <= 0:
            continue
        a, b = np.array(verts[i], float), np.array(verts[i + 1], float)
        e = every if every > 0 else M
        for k0 in range(0, M, e):
            k1 = min(M, k0 + e)
            ks = np.arange(k0, k1)
            s = (ks + 1.0) / M if sampling else (ks + 0.5) / M
            oracle.evolve(Lx, Ly, psi, tuple(a), tuple(b), k1 - k0, dt, sZ=s, sX=s, order=order)
            out.append(oracle_observables(Lx, Ly, psi, tuple(a + (k1 / M) * (b - a))))
    return psi, out


def trace_rows(trace):
    rows = []
    for r in trace.cpu().numpy():
        rows.append({"norm": r[0], "energy": r[1], "sumA": r[2], "sumB": r[3], "mx": r[4], "mz": r[5],
                     "zloop": list(r[6:14]), "xloop": list(r[14:22]), "dos": list(r[22:55])})
    return rows


def gpu_path(Lx, Ly, dtype, init, verts, steps, dt, sampling, order, every, renorm=0):
    plan = z2h.z2h_plan_create(Lx, Ly, dtype)
    sz = z2h.z2h_plan_sizes(plan)
    psi = z2h.alloc_state(plan)
    ws = z2h.alloc_bytes(max(sz["ws_evolve"], sz["ws_observe"]))
    z2h.z2h_state_init(plan, psi, {"psi1": z2h.Z2H_INIT_PSI1, "psi1p": z2h.Z2H_INIT_PSI1P}[init])
    path = z2h.make_path(verts, steps, dt, sampling=sampling, order=order, renorm=renorm, every=every)
    zl, xl = standard_loops_lib(Lx, Ly)
    tr = z2h.z2h_path_evolve(plan, psi, ws, path, zl, xl)
    return psi.cpu().numpy().astype(np.complex128), trace_rows(tr)


@pytest.mark.parametrize("sampling,order,init", [(1, 0, "psi1"), (0, 0, "psi1p"), (1, 1, "psi1")])
def test_path_trace_2x2_c128(sampling, order, init):
    verts = [(1, 1, 0, 0), (1, 1, 0.3, 0), (1, 1, 0.3, 0.2), (0.8, 1.1, 0.1, 0.4)]
    steps = [30, 17, 25]
    print(f"case path 2x2 c128 sampling={sampling} order={order} init={init}", flush=True)
    g_psi, g = gpu_path(2, 2, z2h.Z2H_C128, init, verts, steps, 0.1, sampling, order, 7)
    o_psi, o = oracle_path(2, 2, init, verts, steps, 0.1, sampling, order, 7)
    assert len(g) == len(o) == 1 + 5 + 3 + 4
    for a, b in zip(g, o):
        compare_observables(a, b, 1e-11, 8)
    assert oracle.fidelity_loss(to_oracle_order(2, 2, g_psi), o_psi) < 1e-12


def test_path_trace_3x3_c64_renorm():
    verts = [(0.5, 0.5, 0, 0), (0.5, 0.5, 0.4, 0), (0.5, 0.5, 0.4, 0.1), (0.5, 0.5, 0.0, 0.1)]
    steps = [40, 10, 40]
    print("case path 3x3 c64 renorm", flush=True)
    g_psi, g = gpu_path(3, 3, z2h.Z2H_C64, "psi1", verts, steps, 0.05, 1, 0, 9, renorm=1)
    o_psi, o = oracle_path(3, 3, "psi1", verts, steps, 0.05, 1, 0, 9)
    assert len(g) == len(o)
    for a, b in zip(g, o):
        compare_observables(a, b, 1e-5, 18)
    assert oracle.fidelity_loss(to_oracle_order(3, 3, g_psi), o_psi) < 1e-5


def test_untraced_path_equals_ramps():
    """A path observed only at leg ends is the same computation as its legs
    run as separate ramps (bitwise)."""
    import torch
    verts = [(1, 1, 0, 0), (1, 1, 0.25, 0.05), (1, 1, 0.1, 0.3)]
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C64)
    sz = z2h.z2h_plan_sizes(plan)
    ws = z2h.alloc_bytes(max(sz["ws_evolve"], sz["ws_observe"]))
    a = z2h.alloc_state(plan)
    b = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, a, z2h.Z2H_INIT_PSI1)
    z2h.z2h_state_init(plan, b, z2h.Z2H_INIT_PSI1)
    z2h.z2h_path_evolve(plan, a, ws, z2h.make_path(verts, [20, 30], 0.05, renorm=1))
    for i, M in enumerate((20, 30)):
        z2h.z2h_evolve(plan, b, ws, z2h.schedule(verts[i], verts[i + 1], M, 0.05, sampling=1, renorm=1))
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(a), torch.view_as_real(b))


def _single_path_trace(plan, path, init):
    psi = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, psi, init)
    sz = z2h.z2h_plan_sizes(plan)
    ws = z2h.alloc_bytes(max(sz["ws_evolve"], sz["ws_observe"]))
    tr = z2h.z2h_path_evolve(plan, psi, ws, path)
    torch.cuda.synchronize()
    return psi, tr.cpu().numpy()


@pytest.mark.parametrize("dtype", [z2h.Z2H_C128, z2h.Z2H_C64])
def test_paths_batched_equal_single(dtype):
    """z2h_paths_evolve on three 3x3 paths (different couplings and initial
    states, equal leg lengths) gives, path by path, exactly the samples and
    final states of separate z2h_path_evolve calls."""
    plan = z2h.z2h_plan_create(3, 3, dtype)
    renorm = 1 if dtype == z2h.Z2H_C64 else 0
    paths, inits = [], []
    for j, g in enumerate((0.2, 0.3, 0.45)):
        verts = [(0.5, 0.5, 0.0, 0.0), (0.5, 0.5, g, 0.0), (0.5, 0.5, g, 0.1), (0.5, 0.5, 0.0, 0.1)]
        paths.append(z2h.make_path(verts, [30, 10, 30], 0.05, sampling=1, renorm=renorm, every=10))
        inits.append(z2h.Z2H_INIT_PSI1 if j != 1 else z2h.Z2H_INIT_PSI1P)
    print(f"case batched paths dtype={dtype}", flush=True)
    states, trace = z2h.z2h_paths_evolve(plan, paths, inits=inits)
    torch.cuda.synchronize()
    tr = trace.cpu().numpy()
    n = 18
    for j, path in enumerate(paths):
        psi, ref = _single_path_trace(plan, path, inits[j])
        assert tr.shape[0] == ref.shape[0] == 1 + 3 + 1 + 3
        assert np.array_equal(tr[:, j, :], ref), (j, np.abs(tr[:, j, :] - ref).max())
        assert torch.equal(states[j << n:(j + 1) << n], psi)


def test_paths_batched_ragged_legs():
    """Legs of different length (the red paths' rise to lambda = r): the
    shorter path repeats its leg-end sample while the longer one runs on, and
    otherwise matches its own single-path trace bitwise."""
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    mk = lambda r, m: z2h.make_path([(0.5, 0.5, 0.0, 0.0), (0.5, 0.5, 0.3, 0.0), (0.5, 0.5, 0.3, r),
                                     (0.5, 0.5, 0.0, r)], [20, m, 20], 0.05, sampling=1, every=10)
    short, long_ = mk(0.05, 5), mk(0.15, 15)
    print("case batched paths, ragged legs", flush=True)
    states, trace = z2h.z2h_paths_evolve(plan, [short, long_])
    torch.cuda.synchronize()
    tr = trace.cpu().numpy()
    _, ref_s = _single_path_trace(plan, short, z2h.Z2H_INIT_PSI1)
    _, ref_l = _single_path_trace(plan, long_, z2h.Z2H_INIT_PSI1)
    assert tr.shape[0] == 1 + 2 + 2 + 2 and ref_l.shape[0] == 7 and ref_s.shape[0] == 6
    assert np.array_equal(tr[:, 1, :], ref_l)
    # short path: samples 0-2 (start, leg 1), leg 2 end twice, then leg 3
    assert np.array_equal(tr[:4, 0, :], ref_s[:4])
    assert np.array_equal(tr[4, 0, :], ref_s[3])
    assert np.array_equal(tr[5:, 0, :], ref_s[4:])


@pytest.mark.parametrize("Lx,Ly,every", [(2, 2, 7), (2, 3, 0)])
def test_paths_batched_small_lattices(Lx, Ly, every):
    """Batched paths on one-group plans (2x2: the LDS-resident kernel) and
    without intermediate samples (every = 0: one segment per leg) equal the
    single-path runs bitwise."""
    plan = z2h.z2h_plan_create(Lx, Ly, z2h.Z2H_C128)
    paths = [z2h.make_path([(1.0, 1.0, 0.0, 0.0), (1.0, 1.0, g, 0.1), (0.8, 1.0, g, 0.3)], [21, 14], 0.07,
                           sampling=0, every=every) for g in (0.2, 0.5)]
    print(f"case batched paths {Lx}x{Ly} every={every}", flush=True)
    states, trace = z2h.z2h_paths_evolve(plan, paths)
    torch.cuda.synchronize()
    tr = trace.cpu().numpy()
    n = 2 * Lx * Ly
    for j, path in enumerate(paths):
        psi, ref = _single_path_trace(plan, path, z2h.Z2H_INIT_PSI1)
        assert np.array_equal(tr[:, j, :], ref)
        assert torch.equal(states[j << n:(j + 1) << n], psi)
