"""GPU parity of the gate-level circuits (Sec. III with the ancilla; Eqs.
(ini1), (ini2)) through the C ABI.

- One Trotter step as the library's gate list, run gate by gate, in tile
  groups (register phases, layout changes through LDS) and in register
  groups, against the oracle's own gate-level circuit (paper numbering),
  from a random link state with the ancilla in |0>.
- The preparation circuits against psi_1 and psi_1'.
- A gate-level ramp against the fused Trotter path of the library and the
  oracle's Trotter evolution; the ancilla stays in |0>.
- 4x4 plus the ancilla (33 qubits, complex64, fused): two steps against the
  Trotter path on sampled amplitudes.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import circuit
from paper_2108_13410_amd import z2h

from helpers import index_map

pytestmark = pytest.mark.gpu
CDT = {z2h.Z2H_C128: torch.complex128, z2h.Z2H_C64: torch.complex64}


def lib_to_oracle_anc(Lx, Ly, psi_lib):
    """(n + 1)-qubit library-order state -> oracle order (ancilla bit n kept)."""
    n = 2 * Lx * Ly
    im = index_map(Lx, Ly).astype(np.int64)
    out = np.empty_like(psi_lib)
    out[im] = psi_lib[: 1 << n]
    out[im + (1 << n)] = psi_lib[1 << n:]
    return out


def oracle_to_lib_anc(Lx, Ly, psi_or):
    n = 2 * Lx * Ly
    im = index_map(Lx, Ly).astype(np.int64)
    return np.concatenate([psi_or[im], psi_or[im + (1 << n)]])


def run(nq, dtype, psi, gates, ngates, fuse):
    ws = z2h.alloc_bytes(z2h.z2h_gates_ws_bytes(nq))
    z2h.z2h_gates_run(nq, dtype, psi, ws, gates, ngates, fuse=fuse)
    torch.cuda.synchronize()


@pytest.mark.parametrize("Lx,Ly", [(2, 2), (2, 3), (3, 3)])
@pytest.mark.parametrize("fuse", [0, 1, 2])
@pytest.mark.parametrize("dtype,order", [(z2h.Z2H_C128, 0), (z2h.Z2H_C128, 1), (z2h.Z2H_C64, 0)])
def test_circuit_step_against_oracle_circuit(Lx, Ly, fuse, dtype, order):
    n = 2 * Lx * Ly
    cx, cz = (0.7, 0.4, 0.3, 0.2), (0.6, 0.9, 0.1, 0.45)
    dt = 0.37
    print(f"case circuit step {Lx}x{Ly} fuse={fuse} dtype={dtype} order={order}", flush=True)
    rng = np.random.default_rng(40 + n)
    x = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    x /= np.linalg.norm(x)
    x_or = circuit.with_ancilla(x)
    ref = circuit.apply(x_or, circuit.step_gates(Lx, Ly, cx, cz, dt, order))
    gates, ng = z2h.z2h_circuit_step(Lx, Ly, cx, cz, dt, order)
    psi = torch.tensor(oracle_to_lib_anc(Lx, Ly, x_or), dtype=CDT[dtype], device="cuda")
    run(n + 1, dtype, psi, gates, ng, fuse)
    got = lib_to_oracle_anc(Lx, Ly, psi.cpu().numpy().astype(np.complex128))
    tol = 1e-12 if dtype == z2h.Z2H_C128 else 2e-6
    assert np.abs(got - ref).max() < tol
    assert np.abs(got[1 << n:]).max() < tol  # ancilla back in |0>


@pytest.mark.parametrize("Lx,Ly", [(2, 3), (3, 3)])
@pytest.mark.parametrize("which", [z2h.Z2H_INIT_PSI1, z2h.Z2H_INIT_PSI1P])
@pytest.mark.parametrize("fuse", [0, 1, 2])
def test_preparation_circuits(Lx, Ly, which, fuse):
    n = 2 * Lx * Ly
    print(f"case prep {Lx}x{Ly} which={which} fuse={fuse}", flush=True)
    psi = torch.zeros(1 << (n + 1), dtype=torch.complex128, device="cuda")
    psi[0] = 1
    gates, ng = z2h.z2h_circuit_prep(Lx, Ly, which)
    run(n + 1, z2h.Z2H_C128, psi, gates, ng, fuse)
    got = lib_to_oracle_anc(Lx, Ly, psi.cpu().numpy())
    ref = oracle.init_psi1(Lx, Ly) if which == z2h.Z2H_INIT_PSI1 else oracle.init_psi1p(Lx, Ly)
    assert np.abs(got[: 1 << n] - ref).max() < 1e-13
    assert np.abs(got[1 << n:]).max() == 0


@pytest.mark.parametrize("fuse", [0, 1, 2])
def test_gate_level_ramp_equals_fused_trotter_path(fuse):
    """3x3, 12 steps of the ramp from psi_1 (prepared by the circuit of
    Eq. (ini1)): the gate-level run, the library's fused Trotter path and the
    oracle's Trotter evolution agree (1e-12), the ancilla stays in |0>."""
    Lx, Ly, n, M, dt = 3, 3, 18, 12, 0.1
    c0, c1 = (0.5, 0.5, 0.0, 0.0), (0.5, 0.5, 0.35, 0.25)
    print(f"case gate-level ramp fuse={fuse}", flush=True)
    psi = torch.zeros(1 << (n + 1), dtype=torch.complex128, device="cuda")
    psi[0] = 1
    ws = z2h.alloc_bytes(z2h.z2h_gates_ws_bytes(n + 1))
    gates, ng = z2h.z2h_circuit_prep(Lx, Ly, z2h.Z2H_INIT_PSI1)
    z2h.z2h_gates_run(n + 1, z2h.Z2H_C128, psi, ws, gates, ng, fuse=fuse)
    z2h.z2h_circuit_evolve(Lx, Ly, z2h.Z2H_C128, psi, ws, z2h.schedule(c0, c1, M, dt), fuse=fuse)
    plan = z2h.z2h_plan_create(Lx, Ly, z2h.Z2H_C128)
    phi = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, phi, z2h.Z2H_INIT_PSI1)
    sz = z2h.z2h_plan_sizes(plan)
    z2h.z2h_evolve(plan, phi, z2h.alloc_bytes(sz["ws_evolve"]), z2h.schedule(c0, c1, M, dt))
    torch.cuda.synchronize()
    g = psi.cpu().numpy()
    assert np.abs(g[: 1 << n] - phi.cpu().numpy()).max() < 1e-12
    assert np.abs(g[1 << n:]).max() < 1e-13
    ref = oracle.init_psi1(Lx, Ly)
    oracle.evolve(Lx, Ly, ref, c0, c1, M, dt)
    got = lib_to_oracle_anc(Lx, Ly, g)
    assert np.abs(got[: 1 << n] - ref).max() < 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("fuse", [1, 2])
def test_gate_level_4x4_with_ancilla_c128(fuse):
    """33 qubits in complex128 (128 GiB, with the 64 GiB Trotter-path state
    beside it): two steps of the 4x4 ramp from psi_1 against the complex128
    Trotter path on 2^16 sampled link amplitudes (1e-11 of the largest) and
    the ancilla half on 2^16 samples."""
    Lx, Ly, n, M, dt = 4, 4, 32, 200, 0.1
    c0, c1 = (0.5, 0.5, 0.0, 0.0), (0.5, 0.5, 0.4, 0.3)
    print(f"case gate-level 4x4 + ancilla c128 fuse={fuse}", flush=True)
    torch.cuda.empty_cache()
    plan = z2h.z2h_plan_create(Lx, Ly, z2h.Z2H_C128)
    phi = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, phi, z2h.Z2H_INIT_PSI1)
    psi = torch.zeros(1 << (n + 1), dtype=torch.complex128, device="cuda")
    psi[: 1 << n].copy_(phi)
    ws = z2h.alloc_bytes(z2h.z2h_gates_ws_bytes(n + 1))
    z2h.z2h_circuit_evolve(Lx, Ly, z2h.Z2H_C128, psi, ws, z2h.schedule(c0, c1, M, dt, k_end=2), fuse=fuse)
    sz = z2h.z2h_plan_sizes(plan)
    z2h.z2h_evolve(plan, phi, z2h.alloc_bytes(sz["ws_evolve"]), z2h.schedule(c0, c1, M, dt, k_end=2))
    torch.cuda.synchronize()
    rng = np.random.default_rng(10)
    idx = torch.tensor(rng.integers(0, 1 << n, 1 << 16), device="cuda")
    a, b = psi[idx].cpu().numpy(), phi[idx].cpu().numpy()
    scale = np.abs(b).max()
    assert np.abs(a - b).max() < 1e-11 * scale
    anc = psi[idx + (1 << n)].cpu().numpy()
    assert np.abs(anc).max() < 1e-11 * scale
    del psi, phi
    torch.cuda.empty_cache()


@pytest.mark.slow
@pytest.mark.parametrize("fuse", [1, 2])
def test_gate_level_4x4_with_ancilla(fuse):
    """33 qubits in complex64 (64 GiB), LDS or register gate groups: two
    steps of the 4x4 ramp from psi_1 against the Trotter path (complex64) on
    2^16 sampled link amplitudes and the ancilla half on 2^16 samples."""
    Lx, Ly, n, M, dt = 4, 4, 32, 200, 0.1
    c0, c1 = (0.5, 0.5, 0.0, 0.0), (0.5, 0.5, 0.4, 0.3)
    print(f"case gate-level 4x4 + ancilla c64 fuse={fuse}", flush=True)
    torch.cuda.empty_cache()
    plan = z2h.z2h_plan_create(Lx, Ly, z2h.Z2H_C64)
    phi = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, phi, z2h.Z2H_INIT_PSI1)
    psi = torch.zeros(1 << (n + 1), dtype=torch.complex64, device="cuda")
    psi[: 1 << n].copy_(phi)
    ws = z2h.alloc_bytes(z2h.z2h_gates_ws_bytes(n + 1))
    z2h.z2h_circuit_evolve(Lx, Ly, z2h.Z2H_C64, psi, ws, z2h.schedule(c0, c1, M, dt, k_end=2), fuse=fuse)
    sz = z2h.z2h_plan_sizes(plan)
    z2h.z2h_evolve(plan, phi, z2h.alloc_bytes(sz["ws_evolve"]), z2h.schedule(c0, c1, M, dt, k_end=2))
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    idx = torch.tensor(rng.integers(0, 1 << n, 1 << 16), device="cuda")
    a, b = psi[idx].cpu().numpy(), phi[idx].cpu().numpy()
    scale = np.abs(b).max()
    # complex64: about 2000 rounded gate applications per amplitude here, and
    # the fused path's own rounding
    assert np.abs(a - b).max() < 3e-5 * scale
    anc = psi[idx + (1 << n)].cpu().numpy()
    assert np.abs(anc).max() < 3e-5 * scale
    del psi, phi
    torch.cuda.empty_cache()


def random_gates(rng, nq, count):
    """A random gate list (oracle tuples and the library's array): one-qubit
    rotations, Hadamards, CNOTs both ways, a projection and a renormalisation
    in the middle, on qubits drawn from a few clusters so that consecutive
    gates share qubits and the fused executors form real groups."""
    clusters = [rng.choice(nq, size=min(nq, 6), replace=False) for _ in range(4)]
    ora, lib = [], []
    for i in range(count):
        cl = clusters[(i // 15) % len(clusters)]
        r = rng.random()
        if i == count // 2:
            q = int(rng.choice(cl))
            ora += [("P0", (q,)), ("NORM", ())]
            lib += [(z2h.Z2H_GATE_PROJ0, q, 0, 0.0), (z2h.Z2H_GATE_NORM, 0, 0, 0.0)]
        elif r < 0.35:
            c, t = (int(x) for x in rng.choice(cl, size=2, replace=False))
            ora.append(("CNOT", (c, t)))
            lib.append((z2h.Z2H_GATE_CNOT, c, t, 0.0))
        else:
            q, th = int(rng.choice(cl)), float(rng.uniform(-3, 3))
            kind = ("H", "RX", "RZ")[int(rng.integers(3))]
            ora.append((kind, (q,)) if kind == "H" else (kind, (q,), th))
            lib.append(({"H": z2h.Z2H_GATE_H, "RX": z2h.Z2H_GATE_RX, "RZ": z2h.Z2H_GATE_RZ}[kind], q, 0, th))
    arr = (z2h.z2h_gate * len(lib))()
    for a, (k, q0, q1, th) in zip(arr, lib):
        a.kind, a.q0, a.q1, a.theta = k, q0, q1, th
    return ora, arr, len(lib)


@pytest.mark.parametrize("nq", [5, 6, 9, 12, 14, 16])
@pytest.mark.parametrize("fuse", [0, 1, 2])
@pytest.mark.parametrize("dtype", [z2h.Z2H_C128, z2h.Z2H_C64])
def test_random_gate_lists(nq, fuse, dtype):
    """Random gate lists against the oracle's gate-by-gate application: every
    executor, layouts on low and high qubits, tiles smaller than a wave
    (fewer than 11 qubits) and the gate-by-gate fallback (5 qubits)."""
    rng = np.random.default_rng(1000 * nq + 10 * fuse + dtype)
    print(f"case random gates nq={nq} fuse={fuse} dtype={dtype}", flush=True)
    x = rng.normal(size=1 << nq) + 1j * rng.normal(size=1 << nq)
    x /= np.linalg.norm(x)
    ora, arr, ng = random_gates(rng, nq, 150)
    ref = circuit.apply(x, ora)
    psi = torch.tensor(x, dtype=CDT[dtype], device="cuda")
    run(nq, dtype, psi, arr, ng, fuse)
    got = psi.cpu().numpy().astype(np.complex128)
    tol = 1e-12 if dtype == z2h.Z2H_C128 else 5e-6
    assert np.abs(got - ref).max() < tol


def _lib_array(lib):
    arr = (z2h.z2h_gate * len(lib))()
    for a, (k, q0, q1, th) in zip(arr, lib):
        a.kind, a.q0, a.q1, a.theta = k, q0, q1, th
    return arr


@pytest.mark.parametrize("nq", [12, 15])
@pytest.mark.parametrize("fuse", [1, 2])
@pytest.mark.parametrize("dtype", [z2h.Z2H_C128, z2h.Z2H_C64])
def test_cnot_runs_and_hadamard_counts(nq, fuse, dtype):
    """Runs of CNOTs with one target (composed by the register kernels),
    including a control that cancels itself and a run that cancels
    completely, between odd and even numbers of Hadamards per group, against
    the oracle's gate-by-gate application."""
    H, RX, RZ, CX = z2h.Z2H_GATE_H, z2h.Z2H_GATE_RX, z2h.Z2H_GATE_RZ, z2h.Z2H_GATE_CNOT
    t, a, b, c = nq - 1, 1, 5, nq - 3
    lib = [(H, a, 0, 0.0), (H, b, 0, 0.0), (H, c, 0, 0.0),
           (CX, a, t, 0.0), (CX, b, t, 0.0), (CX, a, t, 0.0), (CX, c, t, 0.0),   # a cancels: mask b ^ c
           (RZ, t, 0, 0.7),
           (CX, c, t, 0.0), (CX, b, t, 0.0),
           (CX, b, a, 0.0), (CX, b, a, 0.0),                                     # cancels completely
           (H, a, 0, 0.0), (RX, b, 0, -0.4), (H, t, 0, 0.0),
           (CX, t, b, 0.0), (CX, a, b, 0.0), (RZ, b, 0, 1.3), (CX, a, b, 0.0), (CX, t, b, 0.0),
           (H, c, 0, 0.0), (H, b, 0, 0.0), (H, 0, 0, 0.0)]
    name = {H: "H", RX: "RX", RZ: "RZ", CX: "CNOT"}
    ora = [(name[k], (q0, q1)) if k == CX else ((name[k], (q0,)) if k == H else (name[k], (q0,), th))
           for k, q0, q1, th in lib]
    print(f"case CNOT runs nq={nq} fuse={fuse} dtype={dtype}", flush=True)
    rng = np.random.default_rng(7 + nq)
    x = rng.normal(size=1 << nq) + 1j * rng.normal(size=1 << nq)
    x /= np.linalg.norm(x)
    ref = circuit.apply(x, ora)
    psi = torch.tensor(x, dtype=CDT[dtype], device="cuda")
    run(nq, dtype, psi, _lib_array(lib), len(lib), fuse)
    got = psi.cpu().numpy().astype(np.complex128)
    tol = 1e-12 if dtype == z2h.Z2H_C128 else 2e-6
    assert np.abs(got - ref).max() < tol


@pytest.mark.slow
@pytest.mark.parametrize("fuse", [0, 1, 2])
def test_max_qubits_circuit_then_inverse(fuse):
    """34 qubits, the largest state the gate API accepts (complex64,
    128 GiB): a random circuit on qubits spread over the whole index
    (including the top qubit, 64 GiB apart) changes the state, and the
    inverse circuit (reversed, angles negated) restores 2^16 sampled
    amplitudes to 1e-4 of the largest."""
    nq = 34
    H, RX, RZ, CX = z2h.Z2H_GATE_H, z2h.Z2H_GATE_RX, z2h.Z2H_GATE_RZ, z2h.Z2H_GATE_CNOT
    rng = np.random.default_rng(34 + fuse)
    pool = [0, 1, 2, 5, 9, 14, 20, 27, 31, 32, 33]
    fwd = []
    for _ in range(40 if fuse else 12):
        if rng.random() < 0.4:
            c, t = (int(q) for q in rng.choice(pool, 2, replace=False))
            fwd.append((CX, c, t, 0.0))
        else:
            fwd.append(((H, RX, RZ)[int(rng.integers(3))], int(rng.choice(pool)), 0, float(rng.uniform(-2, 2))))
    inv = [(k, q0, q1, -th if k in (RX, RZ) else 0.0) for k, q0, q1, th in reversed(fwd)]
    print(f"case 34 qubits circuit and inverse fuse={fuse}", flush=True)
    torch.cuda.empty_cache()
    psi = torch.randn(1 << nq, dtype=torch.complex64, device="cuda")
    idx = torch.tensor(rng.integers(0, 1 << nq, 1 << 16), device="cuda")
    idx[:4] = torch.tensor([0, (1 << nq) - 1, 1 << 33, (1 << 33) - 1], device="cuda")
    before = psi[idx].cpu().numpy()
    ws = z2h.alloc_bytes(z2h.z2h_gates_ws_bytes(nq))
    z2h.z2h_gates_run(nq, z2h.Z2H_C64, psi, ws, _lib_array(fwd), len(fwd), fuse=fuse)
    mid = psi[idx].cpu().numpy()
    z2h.z2h_gates_run(nq, z2h.Z2H_C64, psi, ws, _lib_array(inv), len(inv), fuse=fuse)
    after = psi[idx].cpu().numpy()
    scale = np.abs(before).max()
    assert np.abs(mid - before).max() > 0.1 * scale
    assert np.abs(after - before).max() < 1e-4 * scale
    del psi
    torch.cuda.empty_cache()
