"""GPU parity of the exact solvers through the C ABI.

- H x (z2h_hamiltonian_apply) against the oracle's sparse H element by
  element at 2x2 .. 3x3, and on sampled rows (the row-by-row definition) at
  3x4 and 4x4, where the pass chain has three groups.
- Lanczos ground energies against the oracle's exact diagonalisation up to
  3x3 (including the paper's printed 3x3 energy) and, at 4x4, against closed
  forms (zero field; decoupled links) and the self-duality of Sec. III.
- Krylov stepwise exact evolution against the oracle's exact stepwise
  evolution, and the Trotter product's distance to it (second order in dt).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import ed
from paper_2108_13410_amd import z2h

from helpers import fidelity_loss, index_map, lib_to_oracle_bits, to_oracle_order

pytestmark = pytest.mark.gpu

CDT = {z2h.Z2H_C128: torch.complex128, z2h.Z2H_C64: torch.complex64}


def lib_idx_to_oracle(Lx, Ly, idx):
    perm = lib_to_oracle_bits(Lx, Ly)
    idx = np.asarray(idx, dtype=np.int64)
    out = np.zeros_like(idx)
    for b, pb in enumerate(perm):
        out |= ((idx >> b) & 1) << int(pb)
    return out


def oracle_idx_to_lib(Lx, Ly, idx):
    perm = lib_to_oracle_bits(Lx, Ly)
    idx = np.asarray(idx, dtype=np.int64)
    out = np.zeros_like(idx)
    for b, pb in enumerate(perm):
        out |= ((idx >> int(pb)) & 1) << b
    return out


def to_lib_order(Lx, Ly, psi_oracle):
    return psi_oracle[index_map(Lx, Ly).astype(np.int64)]


def random_state_gpu(n, dtype, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    v = torch.randn(1 << n, dtype=CDT[dtype], device="cuda", generator=g)
    return v.div_(torch.linalg.vector_norm(v))


@pytest.mark.parametrize("Lx,Ly", [(2, 2), (2, 3), (3, 3)])
@pytest.mark.parametrize("dtype", [z2h.Z2H_C128, z2h.Z2H_C64])
def test_hamiltonian_apply_full(Lx, Ly, dtype):
    """Every element of H x against the oracle's sparse H (1e-12 relative in
    complex128; complex64 rounds each of the n transform levels: 1e-5)."""
    n = 2 * Lx * Ly
    c = (0.7, 1.1, 0.3, -0.45)
    print(f"case H x {Lx}x{Ly} dtype={dtype}", flush=True)
    rng = np.random.default_rng(3)
    x_or = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    x_or /= np.linalg.norm(x_or)
    ref = ed.hamiltonian(Lx, Ly, c) @ x_or
    plan = z2h.z2h_plan_create(Lx, Ly, dtype)
    x = torch.tensor(to_lib_order(Lx, Ly, x_or), dtype=CDT[dtype], device="cuda")
    x0 = x.clone()
    y = z2h.alloc_state(plan)
    z2h.z2h_hamiltonian_apply(plan, x, y, c)
    torch.cuda.synchronize()
    got = to_oracle_order(Lx, Ly, y.cpu().numpy().astype(np.complex128))
    tol = 1e-12 if dtype == z2h.Z2H_C128 else 1e-5
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    assert torch.equal(x, x0)  # x is read only


@pytest.mark.parametrize("Lx,Ly,dtype,cfg", [
    (3, 4, z2h.Z2H_C128, None), (3, 4, z2h.Z2H_C64, None), (4, 4, z2h.Z2H_C64, None), (4, 4, z2h.Z2H_C128, None),
    (2, 5, z2h.Z2H_C128, "split=4:2:8:0/10:5:13:3:1c:h3@17/6:3:9:3"),
    (2, 5, z2h.Z2H_C64, "split=4:2:8:0/6:3:10:4:at8/10:5:14:4:1c"),
    (4, 4, z2h.Z2H_C128, "split=12:4:12:0/10:5:13:3:1c:h7@22/10:5:13:3:1c,xcd=7"),
    (2, 5, z2h.Z2H_C128, "split=4:2:8:0/10:4:13:3:h3@17/6:3:9:3"),
    (4, 4, z2h.Z2H_C128, "split=12:4:12:0/10:4:13:3:h7@22/10:4:13:3,xcd=7")])
def test_hamiltonian_apply_sampled_rows(Lx, Ly, dtype, cfg):
    """Three-group pass chains (3x4, 4x4, and groups in two runs of qubits
    with register windows across them): 4096 sampled rows, including the
    first and last index, against the row-by-row definition of H."""
    n = 2 * Lx * Ly
    c = (0.5, 0.8, 0.35, 0.2)
    print(f"case H x sampled {Lx}x{Ly} dtype={dtype} {cfg}", flush=True)
    torch.cuda.empty_cache()
    plan = z2h.z2h_plan_create_config(Lx, Ly, dtype, cfg) if cfg else z2h.z2h_plan_create(Lx, Ly, dtype)
    assert len(z2h.z2h_plan_describe(plan)["groups"]) >= 2
    x = random_state_gpu(n, dtype, 11)
    y = z2h.alloc_state(plan)
    z2h.z2h_hamiltonian_apply(plan, x, y, c)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    lib_rows = np.concatenate([[0, (1 << n) - 1], rng.integers(0, 1 << n, 4094)]).astype(np.int64)
    orc_rows = lib_idx_to_oracle(Lx, Ly, lib_rows)

    def fetch(idx_or):
        li = torch.tensor(oracle_idx_to_lib(Lx, Ly, idx_or), device="cuda")
        return x[li].cpu().numpy().astype(np.complex128)

    ref = ed.hamiltonian_rows(Lx, Ly, c, orc_rows, fetch)
    got = y[torch.tensor(lib_rows, device="cuda")].cpu().numpy().astype(np.complex128)
    scale = np.abs(ref).max()
    tol = 1e-12 if dtype == z2h.Z2H_C128 else 1e-5
    assert np.abs(got - ref).max() <= tol * scale
    del x, y
    torch.cuda.empty_cache()


def lanczos(Lx, Ly, dtype, c, max_iter=300, tol=1e-13):
    plan = z2h.z2h_plan_create(Lx, Ly, dtype)
    v = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, v, z2h.Z2H_INIT_PLUS)
    ws = z2h.alloc_bytes(z2h.z2h_lanczos_sizes(plan, max_iter))
    out = z2h.z2h_lanczos_ground(plan, v, ws, c, max_iter=max_iter, tol=tol)
    del v, ws
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("Lx,Ly,c", [
    (2, 2, (0.5, 0.5, 0.3, 0.25)),
    (2, 3, (1.0, 0.7, 0.2, 0.5)),
    (3, 3, (0.5, 0.5, 0.12, 0.0)),
    (3, 3, (0.5, 0.5, 0.3, 0.2)),
    (3, 3, (0.5, 0.5, 0.0, 0.0)),
])
def test_lanczos_against_ed(Lx, Ly, c):
    """Ground energies against the oracle's exact diagonalisation (1e-9).
    The (0.5, 0.5, 0.12, 0) point is the paper's printed 3x3 energy
    (-9.16003, Fig. topo); zero field ends in an invariant subspace."""
    print(f"case Lanczos {Lx}x{Ly} c={c}", flush=True)
    e0, it, a, b = lanczos(Lx, Ly, z2h.Z2H_C128, c)
    ref = ed.ground(Lx, Ly, c)[0]
    assert abs(e0 - ref) < 1e-9, (e0, ref, it)
    assert it == len(a) == len(b)
    if c[2] == 0 and c[3] == 0:
        assert it < 20 and abs(e0 + (c[0] + c[1]) * Lx * Ly) < 1e-12
    if Lx == 3 and c == (0.5, 0.5, 0.12, 0.0):
        assert abs(e0 - (-9.16003)) < 3e-4


def test_lanczos_c64():
    """Complex64 vectors (FP64 coefficients): 3x3 ground energy within 1e-5."""
    c = (0.5, 0.5, 0.25, 0.15)
    e0, it, _, _ = lanczos(3, 3, z2h.Z2H_C64, c, tol=1e-9)
    ref = ed.ground(3, 3, c)[0]
    assert abs(e0 - ref) < 1e-5 * abs(ref), (e0, ref, it)


@pytest.mark.slow
def test_lanczos_4x4_closed_forms_and_duality():
    """4x4 (2^32 amplitudes, complex128: 192 GiB of vectors):
    - zero field: E0 = -(JA + JB) 16;
    - JA = JB = 0: independent links, E0 = -32 sqrt(hx^2 + hz^2);
    - self-duality (Sec. III): E0(JA, JB, hx, hz) = E0(JB, JA, hz, hx), at a
      point with a unique, gapped ground state (both fields above the
      transition), where the recurrence converges in about a hundred steps."""
    print("case Lanczos 4x4 c128", flush=True)
    torch.cuda.empty_cache()
    e, _, _, _ = lanczos(4, 4, z2h.Z2H_C128, (0.5, 0.7, 0.0, 0.0), max_iter=64)
    assert abs(e + 1.2 * 16) < 1e-10, e
    e, _, _, _ = lanczos(4, 4, z2h.Z2H_C128, (0.0, 0.0, 0.3, 0.4), max_iter=64)
    assert abs(e + 32 * 0.5) < 1e-10, e
    e1, it1, _, _ = lanczos(4, 4, z2h.Z2H_C128, (0.5, 0.45, 0.6, 0.35), max_iter=160, tol=1e-12)
    e2, it2, _, _ = lanczos(4, 4, z2h.Z2H_C128, (0.45, 0.5, 0.35, 0.6), max_iter=160, tol=1e-12)
    print(f"4x4 E0(0.5, 0.45, 0.6, 0.35) = {e1:.12f} ({it1} it), dual {e2:.12f} ({it2} it)", flush=True)
    assert abs(e1 - e2) < 1e-9


def sched_with(c0, c1, M, dt, sampling=0, sZ=None, sX=None):
    return z2h.schedule(c0, c1, M, dt, sampling=sampling, sZ=sZ, sX=sX)


@pytest.mark.parametrize("Lx,Ly,variant", [(2, 2, "plain"), (2, 3, "plain"), (3, 3, "plain"), (2, 3, "arrays"),
                                           (3, 3, "right")])
def test_exact_evolve_against_oracle(Lx, Ly, variant):
    """Stepwise exact evolution of a ramp from psi_1 against the oracle's
    (expm_multiply) for midpoint and right-endpoint sampling and for
    explicit per-step schedule arrays: fidelity loss < 1e-12."""
    n = 2 * Lx * Ly
    c0, c1 = (0.5, 0.5, 0.0, 0.0), (0.5, 0.5, 0.35, 0.25)
    M, dt = 12, 0.1
    kw = {}
    if variant == "arrays":
        rng = np.random.default_rng(4)
        kw = dict(sZ=np.sort(rng.uniform(0, 1, M)), sX=np.sort(rng.uniform(0, 1, M)))
    if variant == "right":
        kw = dict(sampling=1)
    print(f"case exact evolve {Lx}x{Ly} {variant}", flush=True)
    plan = z2h.z2h_plan_create(Lx, Ly, z2h.Z2H_C128)
    psi = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
    ws = z2h.alloc_bytes(z2h.z2h_exact_sizes(plan, 16))
    err = z2h.z2h_exact_evolve(plan, psi, ws, sched_with(c0, c1, M, dt, **kw), krylov_dim=16)
    torch.cuda.synchronize()
    ref = ed.exact_stepwise_sparse(Lx, Ly, oracle.init_psi1(Lx, Ly), c0, c1, M, dt,
                                   sampling=kw.get("sampling", 0), sZ=kw.get("sZ"), sX=kw.get("sX"))
    got = to_oracle_order(Lx, Ly, psi.cpu().numpy())
    assert fidelity_loss(ref, got) < 1e-12
    assert np.abs(got - ref).max() < 1e-10
    assert 0 <= err < 1e-10


def test_trotter_distance_to_exact_is_second_order():
    """3x3 ramp, T = 2: the Trotter product (z2h_evolve) against the exact
    stepwise product (z2h_exact_evolve) with the same per-step couplings;
    the distance falls ~4x per halving of dt, and at M = 20 it equals the
    oracle's own Trotter-vs-exact distance."""
    c0, c1 = (0.5, 0.5, 0.0, 0.0), (0.5, 0.5, 0.4, 0.3)
    T = 2.0
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    sz = z2h.z2h_plan_sizes(plan)
    wsT = z2h.alloc_bytes(max(sz["ws_evolve"], sz["ws_observe"]))
    wsE = z2h.alloc_bytes(z2h.z2h_exact_sizes(plan, 16))
    dist = []
    for M in (20, 40, 80):
        a, b = z2h.alloc_state(plan), z2h.alloc_state(plan)
        z2h.z2h_state_init(plan, a, z2h.Z2H_INIT_PSI1)
        z2h.z2h_state_init(plan, b, z2h.Z2H_INIT_PSI1)
        z2h.z2h_evolve(plan, a, wsT, z2h.schedule(c0, c1, M, T / M))
        z2h.z2h_exact_evolve(plan, b, wsE, z2h.schedule(c0, c1, M, T / M), krylov_dim=16)
        torch.cuda.synchronize()
        dist.append(torch.linalg.vector_norm(a - b).item())
        if M == 20:
            p = oracle.init_psi1(3, 3)
            oracle.evolve(3, 3, p, c0, c1, M, T / M)
            q = ed.exact_stepwise_sparse(3, 3, oracle.init_psi1(3, 3), c0, c1, M, T / M)
            assert abs(dist[0] - np.linalg.norm(p - q)) < 1e-9 * max(1.0, dist[0])
    print("Trotter distance to exact at M = 20, 40, 80:", dist, flush=True)
    assert 3.7 < dist[0] / dist[1] < 4.3
    assert 3.85 < dist[1] / dist[2] < 4.15


def test_lanczos_vector_against_ed():
    """3x3 ground state at a gapped point (0.5, 0.5, 0.3, 0.2): the repeated
    recurrence's Ritz vector against the oracle's eigenvector (fidelity
    1 - 1e-10), its Rayleigh quotient against the ED energy (1e-10) and its
    residual |Hv - Ev|; z2h_overlap of the vector with itself is 1."""
    c = (0.5, 0.5, 0.3, 0.2)
    print("case Lanczos vector 3x3", flush=True)
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    v = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, v, z2h.Z2H_INIT_PLUS)
    ws = z2h.alloc_bytes(z2h.z2h_lanczos_sizes(plan, 300))
    e0, it, a, b = z2h.z2h_lanczos_ground(plan, v, ws, c, max_iter=300, tol=1e-13)
    del ws
    z2h.z2h_state_init(plan, v, z2h.Z2H_INIT_PLUS)
    E, res = z2h.z2h_lanczos_vector(plan, v, c, a, b)
    E_or, g_or = ed.ground_state(3, 3, c)
    g = to_oracle_order(3, 3, v.cpu().numpy())
    fid = abs(np.vdot(g_or, g)) ** 2
    print(f"3x3 E {E:.12f} (ED {E_or:.12f}), residual {res:.2e}, fidelity 1 - {1 - fid:.2e}, {it} it", flush=True)
    assert abs(E - E_or) < 1e-10 and abs(e0 - E_or) < 1e-9
    assert res < 1e-6
    assert fid > 1 - 1e-10
    assert abs(z2h.z2h_overlap(plan, v, v) - 1) < 1e-12


def test_adiabatic_fidelity_3x3():
    """psi_1 ramped to (0.5, 0.5, 0.3, 0.2) (T = 20, M = 1000, complex128):
    the fidelity |<g|psi_T>|^2 with the ground state there, all on the GPU
    (Trotter path, Lanczos vector, overlap), equals the oracle's (Trotter
    evolution, ED eigenvector) within 1e-9."""
    c0, c1, M, T = (0.5, 0.5, 0.0, 0.0), (0.5, 0.5, 0.3, 0.2), 1000, 20.0
    print("case adiabatic fidelity 3x3", flush=True)
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    g = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, g, z2h.Z2H_INIT_PLUS)
    ws = z2h.alloc_bytes(z2h.z2h_lanczos_sizes(plan, 300))
    _, _, a, b = z2h.z2h_lanczos_ground(plan, g, ws, c1, max_iter=300, tol=1e-13)
    z2h.z2h_state_init(plan, g, z2h.Z2H_INIT_PLUS)
    z2h.z2h_lanczos_vector(plan, g, c1, a, b)
    psi = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
    sz = z2h.z2h_plan_sizes(plan)
    z2h.z2h_evolve(plan, psi, z2h.alloc_bytes(sz["ws_evolve"]), z2h.schedule(c0, c1, M, T / M))
    F = abs(z2h.z2h_overlap(plan, g, psi)) ** 2
    ref = oracle.init_psi1(3, 3)
    oracle.evolve(3, 3, ref, c0, c1, M, T / M)
    _, g_or = ed.ground_state(3, 3, c1)
    F_or = abs(np.vdot(g_or, ref)) ** 2
    print(f"3x3 adiabatic fidelity {F:.12f} (oracle {F_or:.12f})", flush=True)
    assert abs(F - F_or) < 1e-9


@pytest.mark.slow
def test_lanczos_vector_4x4_and_adiabatic_fidelity():
    """4x4, complex64 (start vector plus three work vectors: 128 GiB): the
    ground state at the 4x4 ramp's end point (1, 1, 0.25, 0.25); its
    residual and Rayleigh quotient, then the fidelity of the Trotterized
    ramp (T = 20, M = 200, psi_1) with it."""
    from paper_2108_13410_amd import workloads
    job = workloads.point_4x4()
    c1 = job["c1"]
    print("case Lanczos vector 4x4 c64", flush=True)
    torch.cuda.empty_cache()
    plan = z2h.z2h_plan_create(4, 4, z2h.Z2H_C64)
    g = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, g, z2h.Z2H_INIT_PLUS)
    ws = z2h.alloc_bytes(z2h.z2h_lanczos_sizes(plan, 160))
    e0, it, a, b = z2h.z2h_lanczos_ground(plan, g, ws, c1, max_iter=160, tol=1e-9)
    del ws
    torch.cuda.empty_cache()
    z2h.z2h_state_init(plan, g, z2h.Z2H_INIT_PLUS)
    E, res = z2h.z2h_lanczos_vector(plan, g, c1, a, b)
    torch.cuda.empty_cache()
    psi = z2h.alloc_state(plan)
    z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
    sz = z2h.z2h_plan_sizes(plan)
    z2h.z2h_evolve(plan, psi, z2h.alloc_bytes(sz["ws_evolve"]),
                   z2h.schedule(job["c0"], c1, job["M"], job["T"] / job["M"], renorm=1))
    F = abs(z2h.z2h_overlap(plan, g, psi)) ** 2
    print(f"4x4 E0 {e0:.8f} ({it} it), Ritz {E:.8f}, residual {res:.2e}, adiabatic fidelity {F:.8f}", flush=True)
    assert abs(E - e0) < 1e-5 * abs(e0)
    assert res < 1e-3
    assert 0.0 < F <= 1.0 + 1e-5
    del g, psi
    torch.cuda.empty_cache()
