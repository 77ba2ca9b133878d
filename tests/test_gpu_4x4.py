"""4x4 torus (32 qubits, 2^32 amplitudes) and the multi-group pass schedule.

The FP64 oracle cannot hold a 4x4 state, so the full-size runs are pinned
by results that hold exactly at any size:
  - zero field: psi_1 only gains the phase exp(+i (JA Ns + JB Np) T);
  - JA = JB = 0 from |0...0>: a product of identical single-link states
    (closed form from 2x2 matrix exponentials);
  - self-duality (Sec. III): x-z-x from psi_1 and z-x-z from psi_1' with the
    couplings exchanged give the same energy, <X> and <Z> swapped;
  - complex64 against complex128 on the 4x4 ramp (T = 20, M = 200);
  - J_B = h_z = 0 from psi_1: dynamics diagonal in the Hadamard basis on
    the 2^15 plaquette-span codewords (sampled amplitudes as 32768-term
    sums, <B_p> by enumeration);
  - h_z = 0: the star sector and the 't Hooft loops stay at +1 through the
    full mixed dynamics.
The same 3-group pass structure is checked against the oracle element by
element at 3x4 and 2x7 (24 and 28 qubits).
"""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

import oracle
from paper_2108_13410_amd import workloads, z2h

from helpers import fidelity_loss, oracle_run, to_oracle_order

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
SX = np.array([[0, 1], [1, 0]], complex)
SZ = np.array([[1, 0], [0, -1]], complex)


class Run:
    """One 4x4 state on the GPU (32 or 64 GiB) with its workspace."""

    def __init__(self, dtype, Lx=4, Ly=4, cfg=None):
        self.plan = z2h.z2h_plan_create_config(Lx, Ly, dtype, cfg) if cfg else z2h.z2h_plan_create(Lx, Ly, dtype)
        sz = z2h.z2h_plan_sizes(self.plan)
        self.psi = z2h.alloc_state(self.plan)
        self.ws = z2h.alloc_bytes(max(sz["ws_evolve"] + 65536, sz["ws_observe"]))
        self.n = 2 * Lx * Ly
        self.Lx, self.Ly = Lx, Ly

    def ramp(self, c0, c1, M, dt, init=z2h.Z2H_INIT_PSI1, **kw):
        z2h.z2h_state_init(self.plan, self.psi, init)
        z2h.z2h_evolve(self.plan, self.psi, self.ws, z2h.schedule(c0, c1, M, dt, **kw))
        zl, xl = z2h.z2h_loop_masks(self.Lx, self.Ly)
        return z2h.z2h_observe(self.plan, self.psi, self.ws, c1, zl, xl)

    def sample(self, idx):
        t = torch.as_tensor(idx.astype(np.int64), device="cuda")
        return self.psi[t].cpu().numpy().astype(np.complex128)

    def free(self):
        del self.psi, self.ws
        torch.cuda.empty_cache()


def _shipped_4x4():
    """The 4x4 schedules of the shipped table, which bench.py times (strided
    groups in two runs of qubits)."""
    import os
    out = {}
    for line in open(os.path.join(os.path.dirname(z2h.__file__), "tuned_mi355x.txt")):
        f = line.split()
        if len(f) == 4 and f[0] == "32" and f[2] == "1":
            out[z2h.Z2H_C128 if f[1] == "1" else z2h.Z2H_C64] = f[3]
    return out


SHIPPED_4X4 = _shipped_4x4()
PLANS_4X4 = [(z2h.Z2H_C64, None), (z2h.Z2H_C128, None), (z2h.Z2H_C64, "shipped"), (z2h.Z2H_C128, "shipped")]


def _popcount(a):
    a = a.astype(np.uint64)
    c = np.zeros(a.shape, np.int64)
    for b in range(64):
        c += ((a >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return c


@pytest.mark.parametrize("dtype,plan", PLANS_4X4)
def test_4x4_zero_field_phase(dtype, plan):
    print(f"case 4x4 zero field dtype={dtype} plan={plan}", flush=True)
    r = Run(dtype, cfg=SHIPPED_4X4[dtype] if plan else None)
    JA, JB, M, dt = 1.0, 0.8, 4, 0.1
    ob = r.ramp((JA, JB, 0, 0), (JA, JB, 0, 0), M, dt)
    tol = 1e-12 if dtype == z2h.Z2H_C128 else 2e-6
    assert abs(ob["energy"] + 16 * (JA + JB)) < 16 * tol * 10
    assert abs(ob["norm"] - 1) < tol * 10
    assert abs(ob["xloop"][0] - 1) < tol * 10 and abs(ob["xloop"][1] - 1) < tol * 10
    assert abs(ob["zloop"][0] - 1) < tol * 10 and abs(ob["zloop"][1] - 1) < tol * 10
    # sampled amplitudes: closed form of Eq. (ini1) times the global phase
    rng = np.random.default_rng(1)
    idx = rng.integers(0, 1 << 32, 200000, dtype=np.uint64)
    st, pl = z2h.z2h_masks(4, 4)
    even = np.ones(idx.size, bool)
    for m in pl:
        even &= (_popcount(idx & np.uint64(int(m))) % 2) == 0
    ph = np.exp(1j * 16 * (JA + JB) * M * dt)
    ref = np.where(even, 2.0 ** (-(32 - 16 + 1) / 2), 0.0) * ph
    got = r.sample(idx)
    scale = 2.0 ** (-8.5)
    assert np.max(np.abs(got - ref)) < (1e-12 if dtype == z2h.Z2H_C128 else 1e-6) * scale
    r.free()


@pytest.mark.parametrize("dtype,plan", PLANS_4X4)
def test_4x4_product_state(dtype, plan):
    """JA = JB = 0 from |0...0>: each link evolves on its own (the planner's
    schedule and the shipped one, whose strided groups are two runs of
    qubits)."""
    print(f"case 4x4 product dtype={dtype} plan={plan}", flush=True)
    r = Run(dtype, cfg=SHIPPED_4X4[dtype] if plan else None)
    c0, c1, M, dt = (0, 0, 0.05, 0.3), (0, 0, 0.6, -0.1), 6, 0.2
    ob = r.ramp(c0, c1, M, dt, init=z2h.Z2H_INIT_ZERO)
    u = np.array([1, 0], complex)
    for k in range(M):
        s = (k + 0.5) / M
        hx = (1 - s) * c0[2] + s * c1[2]
        hz = (1 - s) * c0[3] + s * c1[3]
        half = sla.expm(0.5j * hx * dt * SX)
        u = half @ sla.expm(1j * hz * dt * SZ) @ half @ u
    rng = np.random.default_rng(2)
    idx = rng.integers(0, 1 << 32, 200000, dtype=np.uint64)
    w = _popcount(idx)
    ref = u[0] ** (32 - w) * u[1] ** w
    got = r.sample(idx)
    amax = np.max(np.abs(ref))
    tol = 1e-11 if dtype == z2h.Z2H_C128 else 2e-5
    assert np.max(np.abs(got - ref)) < tol * max(amax, abs(u[0]) ** 32)
    # closed-form observables of the product state
    mz = abs(u[0]) ** 2 - abs(u[1]) ** 2
    mx = 2 * (np.conj(u[0]) * u[1]).real
    otol = 1e-10 if dtype == z2h.Z2H_C128 else 1e-5
    assert abs(ob["mz"] - mz) < otol and abs(ob["mx"] - mx) < otol
    assert abs(ob["zloop"][2] - mz ** 4) < otol  # W1: 4 horizontal links
    r.free()


def test_4x4_self_duality():
    """Sec. III self-duality on the full 32-qubit state (complex128)."""
    print("case 4x4 duality c128", flush=True)
    r = Run(z2h.Z2H_C128)
    a0, a1 = (1.0, 0.7, 0.0, 0.0), (1.0, 0.7, 0.3, 0.2)
    b0, b1 = (0.7, 1.0, 0.0, 0.0), (0.7, 1.0, 0.2, 0.3)
    oa = r.ramp(a0, a1, 8, 0.15, init=z2h.Z2H_INIT_PSI1, order=0)
    ob = r.ramp(b0, b1, 8, 0.15, init=z2h.Z2H_INIT_PSI1P, order=1)
    assert abs(oa["energy"] - ob["energy"]) < 1e-10
    assert abs(oa["mx"] - ob["mz"]) < 1e-11 and abs(oa["mz"] - ob["mx"]) < 1e-11
    assert abs(oa["sumA"] - ob["sumB"]) < 1e-10 and abs(oa["sumB"] - ob["sumA"]) < 1e-10
    r.free()


def test_4x4_c64_against_c128():
    """The 4x4 ramp of the benchmark configuration: T = 20, M = 200 to
    (0.25, 0.25); complex64 (renormalized each step) against complex128."""
    cfg = workloads.point_4x4()
    M, dt = cfg["M"], cfg["T"] / cfg["M"]
    res = {}
    for dtype in (z2h.Z2H_C128, z2h.Z2H_C64):
        print(f"case 4x4 M=200 dtype={dtype}", flush=True)
        r = Run(dtype)
        res[dtype] = r.ramp(cfg["c0"], cfg["c1"], M, dt, renorm=1 if dtype == z2h.Z2H_C64 else 0)
        r.free()
    a, b = res[z2h.Z2H_C128], res[z2h.Z2H_C64]
    print("4x4 c128", a["energy"], a["norm"], " c64", b["energy"], b["norm"], flush=True)
    assert abs(a["norm"] - 1) < 1e-11
    assert abs(a["energy"] - b["energy"]) / 32 < 1e-5
    for k in ("mx", "mz"):
        assert abs(a[k] - b[k]) < 1e-5
    for j in range(4):
        assert abs(a["zloop"][j] - b["zloop"][j]) < 1e-5
    # variational: above the zero-field ground energy shifted by the fields
    assert a["energy"] > -2 * 16 - 0.25 * 64


@pytest.mark.parametrize("Lx,Ly,dtype,M", [(3, 4, z2h.Z2H_C128, 4), (3, 4, z2h.Z2H_C64, 4), (2, 7, z2h.Z2H_C128, 2)])
def test_three_group_schedule_against_oracle(Lx, Ly, dtype, M):
    """24 and 28 qubits: the multi-group pass structure of the 4x4 runs,
    element by element against the oracle."""
    print(f"case {Lx}x{Ly} dtype={dtype} M={M}", flush=True)
    c0, c1 = (1, 1, 0, 0), (1.0, 0.9, 0.4, 0.3)
    r = Run(dtype, Lx, Ly)
    assert z2h.z2h_plan_info(r.plan)["groups"] >= 2
    r.ramp(c0, c1, M, 0.12)
    g = r.psi.cpu().numpy().astype(np.complex128)
    r.free()
    o = oracle_run(Lx, Ly, c0, c1, M, 0.12)
    loss = fidelity_loss(o, to_oracle_order(Lx, Ly, g))
    assert loss < (1e-12 if dtype == z2h.Z2H_C128 else 1e-5), loss


def test_4x4_two_tile_schedule_bitwise():
    """The complex64 4x4 schedules with two 128-byte tiles per block, and
    with one tile per block and the component exchange (XCD-major order in
    every group), compute exactly what the planner's default schedule
    computes: blocks only regroup tiles and the renormalisation sums per-tile
    partials in the same order, so 6 Trotter steps of the 4x4 ramp leave
    bit-identical states (checked on 2^20 sampled amplitudes). The observables
    are FP64 sums whose partials follow each plan's own first-group tiling,
    so they agree to rounding (1e-13 relative)."""
    print("case 4x4 c64 two-tile and component-exchange schedules vs default", flush=True)
    cfg = "split=12:4:12:0/10:5:14:4:2/10:5:14:4:2"
    cfg_cx = "split=12:4:12:0/10:5:14:4:1c/10:5:14:4:1c,xcd=7"
    plans = [z2h.z2h_plan_create(4, 4, z2h.Z2H_C64), z2h.z2h_plan_create_config(4, 4, z2h.Z2H_C64, cfg),
             z2h.z2h_plan_create_config(4, 4, z2h.Z2H_C64, cfg_cx)]
    assert [g.get("pair", 1) for g in z2h.z2h_plan_describe(plans[1])["groups"]] == [1, 2, 2]
    assert [g["cx"] for g in z2h.z2h_plan_describe(plans[2])["groups"]] == [0, 1, 1]
    sz = z2h.z2h_plan_sizes(plans[0])
    ws = z2h.alloc_bytes(max(sz["ws_evolve"], sz["ws_observe"]))
    psi = z2h.alloc_state(plans[0])
    job = workloads.point_4x4()
    rng = np.random.default_rng(7)
    idx = torch.tensor(rng.integers(0, 1 << 32, 1 << 20), dtype=torch.int64, device="cuda")
    samples, obs = [], []
    for plan in plans:
        z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
        z2h.z2h_evolve(plan, psi, ws, z2h.schedule(job["c0"], job["c1"], job["M"], job["T"] / job["M"],
                                                   k_end=6, renorm=1))
        samples.append(torch.view_as_real(psi[idx]).cpu())
        obs.append(z2h.z2h_observe(plan, psi, ws, job["c1"]))
    for k in (1, 2):
        assert torch.equal(samples[0], samples[k])
        for key in ("energy", "norm", "mx", "mz"):
            assert abs(obs[0][key] - obs[k][key]) <= 1e-13 * max(1.0, abs(obs[0][key])), key


@pytest.mark.parametrize("dtype,cfg", [
    (z2h.Z2H_C64, "split=12:4:12:0/10:5:14:4:1c:h5/10:5:14:4:1c,xcd=1"),
    (z2h.Z2H_C64, "split=12:4:12:0/10:5:14:4:1c:h5@23/10:5:14:4:1c,xcd=1"),
    (z2h.Z2H_C64, "split=12:4:12:0/10:5:14:4:1c:h5@24/10:5:14:4:1c,xcd=7"),
    (z2h.Z2H_C128, "split=12:4:12:0/10:5:13:3:1c:h5/10:5:13:3:1c,xcd=3"),
    (z2h.Z2H_C128, "split=12:4:12:0/10:5:13:3:1c:h7@22/10:5:13:3:1c,xcd=3")])
def test_4x4_split_run_schedule(dtype, cfg):
    """4x4 schedules whose strided groups are two runs of qubits (":h"):
    the middle group 12-16 and 27-31 with the top group 17-26, or both
    groups in two runs with register windows across them (middle 12-16 and
    23-27, top 17-22 and 28-31; middle 12-16 and 24-28, top 17-23 and 29-31;
    complex128: middle 12-14 and 22-28, top 15-21 and 29-31).  The same transforms grouped differently round
    differently, so 6 Trotter steps of the 4x4 ramp are compared with the
    planner's default schedule to the precision's rounding on 2^20 sampled
    amplitudes, and the observables likewise."""
    print(f"case 4x4 split-run schedule dtype={dtype} {cfg}", flush=True)
    plans = [z2h.z2h_plan_create(4, 4, dtype), z2h.z2h_plan_create_config(4, 4, dtype, cfg)]
    d = z2h.z2h_plan_describe(plans[1])
    assert d["groups"][1]["hi"] > 0
    sz = z2h.z2h_plan_sizes(plans[0])
    ws = z2h.alloc_bytes(max(sz["ws_evolve"], sz["ws_observe"]))
    psi = z2h.alloc_state(plans[0])
    job = workloads.point_4x4()
    rng = np.random.default_rng(11)
    idx = torch.tensor(rng.integers(0, 1 << 32, 1 << 20), dtype=torch.int64, device="cuda")
    samples, obs = [], []
    for plan in plans:
        z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
        z2h.z2h_evolve(plan, psi, ws, z2h.schedule(job["c0"], job["c1"], job["M"], job["T"] / job["M"],
                                                   k_end=6, renorm=1 if dtype == z2h.Z2H_C64 else 0))
        samples.append(psi[idx].cpu().numpy().astype(np.complex128))
        obs.append(z2h.z2h_observe(plan, psi, ws, job["c1"]))
    del psi, ws
    torch.cuda.empty_cache()
    tol = 1e-12 if dtype == z2h.Z2H_C128 else 1e-5
    scale = np.max(np.abs(samples[0]))
    assert np.max(np.abs(samples[1] - samples[0])) <= tol * scale
    for key in ("energy", "norm", "mx", "mz"):
        assert abs(obs[0][key] - obs[1][key]) <= tol * max(1.0, abs(obs[0][key])), key


@pytest.mark.parametrize("dtype,cfg", [
    (z2h.Z2H_C64, "split=12:4:12:0/10:5:14:4:1c:h5@24/10:5:14:4:1c,xcd=7"),
    (z2h.Z2H_C128, "split=12:4:12:0/10:5:13:3:1c:h7@22/10:5:13:3:1c,xcd=7")])
def test_4x4_precomputed_tables_bitwise(dtype, cfg):
    """Phase tables computed ahead of the passes (fetched by each block
    before its tile) and tables built by every workgroup (",tables=0") give
    the same bits: 6 Trotter steps of the 4x4 ramp, 2^20 sampled amplitudes
    and the per-step norms."""
    print(f"case 4x4 precomputed tables dtype={dtype}", flush=True)
    plans = [z2h.z2h_plan_create_config(4, 4, dtype, cfg), z2h.z2h_plan_create_config(4, 4, dtype, cfg + ",tables=0")]
    assert [z2h.z2h_plan_describe(p)["tables"] for p in plans] == [1, 0]
    sz = [z2h.z2h_plan_sizes(p) for p in plans]
    assert sz[0]["ws_evolve"] > sz[1]["ws_evolve"]
    ws = z2h.alloc_bytes(sz[0]["ws_evolve"])
    psi = z2h.alloc_state(plans[0])
    job = workloads.point_4x4()
    rng = np.random.default_rng(17)
    idx = torch.tensor(rng.integers(0, 1 << 32, 1 << 20), dtype=torch.int64, device="cuda")
    samples, norms = [], []
    for plan in plans:
        nrm = torch.zeros(6, dtype=torch.float64, device="cuda")
        z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
        z2h.z2h_evolve(plan, psi, ws, z2h.schedule(job["c0"], job["c1"], job["M"], job["T"] / job["M"], k_end=6,
                                                   renorm=1 if dtype == z2h.Z2H_C64 else 0), norms=nrm)
        samples.append(torch.view_as_real(psi[idx]).cpu())
        norms.append(nrm.cpu())
    del psi, ws
    torch.cuda.empty_cache()
    assert torch.equal(samples[0], samples[1])
    assert torch.equal(norms[0], norms[1])


def _plaquette_codewords():
    """The 2^15 sums (XOR) of plaquette masks of the 4x4 torus (library
    numbering): 15 of the 16 plaquettes are independent, the product of all
    is the identity."""
    st, pl = z2h.z2h_masks(4, 4)
    words = np.zeros(1, np.uint64)
    for m in pl[:15]:
        words = np.concatenate([words, words ^ np.uint64(int(m))])
    assert np.unique(words).size == 1 << 15
    return words, pl


@pytest.mark.parametrize("dtype", [z2h.Z2H_C128, z2h.Z2H_C64])
def test_4x4_x_diagonal_dynamics(dtype):
    """J_B = h_z = 0 from psi_1 (Eq. (ini1)): only the star and x-field terms
    act, both diagonal in the Hadamard basis.  There psi_1 is the uniform
    superposition of the 2^15 plaquette-span codewords x (all stars even), so
    step k multiplies x by exp(+i dt (J_A N_s + h_x (n - 2 w(x)))) at s_k.
    Closed forms at the full 32 qubits: sampled amplitudes as 32768-term
    sums, <B_p> by enumerating the codewords, <A_v> = 1, <Z> = 0, <X>
    constant."""
    print(f"case 4x4 x-diagonal dtype={dtype}", flush=True)
    r = Run(dtype)
    n, ns, M, dt = 32, 16, 6, 0.2
    c0, c1 = (0.8, 0.0, 0.1, 0.0), (1.1, 0.0, 0.55, 0.0)
    ob = r.ramp(c0, c1, M, dt, renorm=0)
    words, pl = _plaquette_codewords()
    w = _popcount(words)

    def phase(wt):
        ph = np.zeros(wt.shape)
        for k in range(M):
            s = (k + 0.5) / M
            JA = (1 - s) * c0[0] + s * c1[0]
            hx = (1 - s) * c0[2] + s * c1[2]
            ph += dt * (JA * ns + hx * (n - 2 * wt))
        return ph

    amp = 2.0 ** (-7.5) * np.exp(1j * phase(w))          # Hadamard-basis amplitudes
    rng = np.random.default_rng(5)
    idx = rng.integers(0, 1 << 32, 48, dtype=np.uint64)
    sign = 1 - 2 * (_popcount(idx[:, None] & words[None, :]) & 1)
    ref = 2.0 ** (-16) * (sign * amp[None, :]).sum(axis=1)
    got = r.sample(idx)
    amax = 2.0 ** (-8.5)
    tol = 1e-11 if dtype == z2h.Z2H_C128 else 2e-5
    assert np.max(np.abs(got - ref)) < tol * amax
    # observables
    otol = 1e-10 if dtype == z2h.Z2H_C128 else 2e-5
    ph_w = phase(w)
    sumB = 0.0
    for m in pl:
        shifted = words ^ np.uint64(int(m))
        sumB += np.mean(np.cos(phase(_popcount(shifted)) - ph_w))
    mx = np.mean(1 - 2 * (_popcount(words[:, None] & (np.uint64(1) << np.arange(n, dtype=np.uint64))[None, :]) & 1))
    assert abs(ob["sumA"] - ns) < otol * ns
    assert abs(ob["mz"]) < otol
    assert abs(ob["mx"] - mx) < otol
    assert abs(ob["sumB"] - sumB) < otol * ns
    assert abs(ob["energy"] - (-c1[0] * ob["sumA"] - c1[2] * n * ob["mx"])) < otol * n
    r.free()


@pytest.mark.parametrize("plan", [None, "shipped"])
def test_4x4_star_sector_conserved(plan):
    """h_z = 0 (Sec. IV): every term commutes with the stars and with the
    't Hooft loops, and psi_1 is their +1 eigenstate, so through the full
    mixed dynamics <A_v> = 1 and <V_1> = <V_2> = 1 at 32 qubits (complex64,
    renormalised each step)."""
    print(f"case 4x4 star sector c64 plan={plan}", flush=True)
    r = Run(z2h.Z2H_C64, cfg=SHIPPED_4X4[z2h.Z2H_C64] if plan else None)
    ob = r.ramp((1.0, 1.0, 0.0, 0.0), (0.9, 1.2, 0.45, 0.0), 10, 0.15, renorm=1)
    assert abs(ob["sumA"] - 16) < 16 * 2e-5
    assert abs(ob["xloop"][0] - 1) < 2e-5 and abs(ob["xloop"][1] - 1) < 2e-5
    assert 0.2 < ob["mx"] < 1.0 and ob["sumB"] < 16 - 1e-3  # the dynamics did move the state
    r.free()
