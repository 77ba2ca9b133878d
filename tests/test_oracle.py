"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here touches a GPU or the HIP library.  Each test names the passage
or the closed form it checks.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import bound, ed

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SX = np.array([[0, 1], [1, 0]], complex)
SZ = np.array([[1, 0], [0, -1]], complex)


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return np.array(rows)


def _rand_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


# ------------------------------------------------------------------ lattice

@pytest.mark.parametrize("Lx,Ly", [(2, 2), (2, 3), (3, 3), (4, 4), (3, 5)])
def test_lattice_incidence(Lx, Ly):
    """Sec. II: every star and plaquette has four links; every link lies on two
    stars and two plaquettes; a star and a plaquette share 0 or 2 links (they
    commute); the product of all stars (all plaquettes) is the identity."""
    st, pl = oracle.masks(Lx, Ly)
    n = 2 * Lx * Ly
    for m in list(st) + list(pl):
        assert bin(int(m)).count("1") == 4
    for l in range(n):
        assert sum(int(m) >> l & 1 for m in st) == 2
        assert sum(int(m) >> l & 1 for m in pl) == 2
    for a in st:
        for b in pl:
            assert bin(int(a) & int(b)).count("1") in (0, 2)
    acc_s = acc_p = 0
    for a, b in zip(st, pl):
        acc_s ^= int(a)
        acc_p ^= int(b)
    assert acc_s == 0 and acc_p == 0


def test_paper_plaquette_numbering():
    """Appendix, Eq. (cmt12): on the 3x3 lattice the plaquettes next to link 4
    are {1,10,4,13} and {4,11,7,14} (1-based)."""
    _, pl = oracle.masks(3, 3)
    sets = [sorted(l + 1 for l in range(18) if int(m) >> l & 1) for m in pl]
    assert [1, 4, 10, 13] in sets
    assert [4, 7, 11, 14] in sets
    assert sum(1 for s in sets if 4 in s) == 2


def test_loops_commute_and_pair():
    """Sec. IV: the noncontractible loops commute with every star and
    plaquette; V1 anticommutes with W2 and V2 with W1."""
    for Lx, Ly in [(2, 2), (3, 3), (3, 4)]:
        st, pl = oracle.masks(Lx, Ly)
        lp = oracle.loops(Lx, Ly)
        for zname in ("W1", "W2"):
            for a in st:
                assert bin(lp[zname] & int(a)).count("1") % 2 == 0
        for xname in ("V1", "V2"):
            for b in pl:
                assert bin(lp[xname] & int(b)).count("1") % 2 == 0
        assert bin(lp["V1"] & lp["W2"]).count("1") % 2 == 1
        assert bin(lp["V2"] & lp["W1"]).count("1") % 2 == 1
        assert bin(lp["V1"] & lp["W1"]).count("1") % 2 == 0
        assert bin(lp["V2"] & lp["W2"]).count("1") % 2 == 0


# ------------------------------------------------------------------ spectrum

def _closed_form_spectrum(Ns, Np, JA, JB):
    vals = []
    for a in range(0, Ns + 1, 2):
        for b in range(0, Np + 1, 2):
            e = -JA * (Ns - 2 * a) - JB * (Np - 2 * b)
            vals += [e] * (4 * math.comb(Ns, a) * math.comb(Np, b))
    return np.sort(np.array(vals))


@pytest.mark.parametrize("Lx,Ly,JA,JB", [(2, 2, 1.0, 1.0), (2, 2, 1.0, 0.7), (2, 3, 0.6, 1.0)])
def test_zero_field_spectrum(Lx, Ly, JA, JB):
    """Toric code at zero field: E = -JA(Ns-2a) - JB(Np-2b) with an even number
    a (b) of violated stars (plaquettes), degeneracy 4 C(Ns,a) C(Np,b); the
    ground level -(JA Ns + JB Np) is 4-fold (Sec. IV)."""
    ev = ed.spectrum(Lx, Ly, (JA, JB, 0, 0))
    ref = _closed_form_spectrum(Lx * Ly, Lx * Ly, JA, JB)
    assert ev.size == ref.size
    np.testing.assert_allclose(np.sort(ev), ref, atol=1e-10)
    assert np.sum(np.abs(ev - ev.min()) < 1e-9) == 4


def test_ed_energy_matches_observables():
    """<psi|H|psi> from the sparse Hamiltonian equals the oracle's term-by-term
    Pauli expectations on a random state."""
    c = (0.9, 1.1, 0.3, 0.25)
    psi = _rand_state(8, 1)
    H = ed.hamiltonian(2, 2, c)
    e = np.vdot(psi, H @ psi).real
    ob = oracle.observe(2, 2, psi, c)
    assert abs(ob["norm"] - 1) < 1e-13
    assert abs(ob["energy"] - e) < 1e-12


# ------------------------------------------------------------------ states

@pytest.mark.parametrize("Lx,Ly", [(2, 2), (2, 3), (3, 3)])
def test_psi1_closed_form(Lx, Ly):
    """Eq. (ini1): psi_1 is the equal superposition of every configuration with
    all plaquettes even: 2^(n-Np+1) amplitudes of 2^(-(n-Np+1)/2).  It is a
    +1 eigenstate of every star, plaquette and 't Hooft loop (Sec. IV)."""
    n, Np = 2 * Lx * Ly, Lx * Ly
    psi = oracle.init_psi1(Lx, Ly)
    nz = np.abs(psi) > 1e-12
    assert nz.sum() == 2 ** (n - Np + 1)
    np.testing.assert_allclose(psi[nz], 2.0 ** (-(n - Np + 1) / 2), atol=1e-14)
    st, pl = oracle.masks(Lx, Ly)
    for m in pl:
        assert abs(oracle.expect_z(psi, m) - 1) < 1e-12
    for m in st:
        assert abs(oracle.expect_x(psi, m) - 1) < 1e-12
    lp = oracle.loops(Lx, Ly)
    assert abs(oracle.expect_x(psi, lp["V1"]) - 1) < 1e-12
    assert abs(oracle.expect_x(psi, lp["V2"]) - 1) < 1e-12
    # energy of the zero-field ground level
    ob = oracle.observe(Lx, Ly, psi, (1, 1, 0, 0))
    assert abs(ob["energy"] + 2 * Np) < 1e-11


@pytest.mark.parametrize("Lx,Ly", [(2, 2), (2, 3), (3, 3)])
def test_psi1p_is_sum_of_sectors(Lx, Ly):
    """Sec. IV: psi_1' = (psi_1 + W1 psi_1 + W2 psi_1 + W1 W2 psi_1)/2 with the
    four sector states orthonormal."""
    p1 = oracle.init_psi1(Lx, Ly)
    lp = oracle.loops(Lx, Ly)
    p2 = oracle.apply_z_string(p1, lp["W1"])
    p3 = oracle.apply_z_string(p1, lp["W2"])
    p4 = oracle.apply_z_string(p2, lp["W2"])
    G = np.array([[np.vdot(a, b) for b in (p1, p2, p3, p4)] for a in (p1, p2, p3, p4)])
    np.testing.assert_allclose(G, np.eye(4), atol=1e-12)
    p1p = oracle.init_psi1p(Lx, Ly)
    np.testing.assert_allclose(p1p, (p1 + p2 + p3 + p4) / 2, atol=1e-13)


# ------------------------------------------------------------------ gates

def test_rotation_convention():
    """Eq. (gate1) with R_a(theta) = exp(-i theta sigma^a / 2): compare the
    oracle's single-qubit gates with scipy's matrix exponential."""
    rng = np.random.default_rng(3)
    for l in range(3):
        th = rng.uniform(-2, 2)
        psi = _rand_state(3, 10 + l)
        for gate, P in ((oracle.rx, SX), (oracle.rz, SZ)):
            out = psi.copy()
            gate(out, l, th)
            U1 = sla.expm(-0.5j * th * P)
            U = np.kron(np.kron(np.eye(2 ** (2 - l)), U1), np.eye(2 ** l))
            np.testing.assert_allclose(out, U @ psi, atol=1e-14)


def test_pauli_string_exponentials():
    """exp(i theta P) for Z and X strings against the dense matrix exponential."""
    n = 6
    rng = np.random.default_rng(4)
    for mask in (0b000111, 0b101010, 0b110011):
        th = rng.uniform(-2, 2)
        for fn, P1 in ((oracle.exp_z, SZ), (oracle.exp_x, SX)):
            P = np.array([[1.0]])
            for l in reversed(range(n)):
                P = np.kron(P, P1 if mask >> l & 1 else np.eye(2))
            psi = _rand_state(n, mask)
            out = psi.copy()
            fn(out, mask, th)
            np.testing.assert_allclose(out, sla.expm(1j * th * P) @ psi, atol=1e-13)


# ------------------------------------------------------------------ the step

@pytest.mark.parametrize("order", [0, 1])
def test_step_equals_grouped_exponentials(order):
    """Sec. III, Eqs. (decom), (gate1): the five-factor step with each factor
    expanded into single-term exponentials equals exp(-iHX t/2) exp(-iHZ t)
    exp(-iHX t/2) (HX = star + x-field terms, HZ = plaquette + z-field terms)
    exactly, because every summand inside a factor commutes."""
    rng = np.random.default_rng(5 + order)
    cx = (0.8, 0.0, 0.37, 0.0)
    cz = (0.0, 1.3, 0.0, 0.21)
    dt = 0.31
    psi = _rand_state(8, 42)
    out = psi.copy()
    oracle.trotter_step(2, 2, out, cx, cz, dt, order)
    U = ed.grouped_step_dense(2, 2, cx, cz, dt, order)
    np.testing.assert_allclose(out, U @ psi, atol=1e-13)
    del rng


def test_step_local_error_is_third_order():
    """Second-order Trotter-Suzuki (Sec. III, Eq. T2S3): the one-step error
    against exp(-iH t) scales as t^3."""
    c = (0.5, 0.5, 0.4, 0.3)
    H = ed.hamiltonian(2, 2, c).toarray()
    psi = _rand_state(8, 7)
    errs = []
    for t in (0.2, 0.1, 0.05):
        out = psi.copy()
        oracle.trotter_step(2, 2, out, c, c, t)
        errs.append(np.linalg.norm(out - sla.expm(-1j * t * H) @ psi))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 7.0 < r1 < 9.0 and 7.5 < r2 < 8.5


def test_zero_field_evolution_is_a_global_phase():
    """At zero field every term commutes and psi_1 is an eigenstate with
    E = -(JA Ns + JB Np): the evolution is exactly the phase exp(+i(JA Ns +
    JB Np) T)."""
    for Lx, Ly, M, dt in ((2, 2, 50, 0.1), (3, 3, 5, 0.2)):
        JA, JB = 1.0, 0.6
        psi0 = oracle.init_psi1(Lx, Ly)
        psi = psi0.copy()
        oracle.evolve(Lx, Ly, psi, (JA, JB, 0, 0), (JA, JB, 0, 0), M, dt)
        ph = np.exp(1j * (JA + JB) * Lx * Ly * M * dt)
        np.testing.assert_allclose(psi, ph * psi0, atol=1e-12)


def test_product_state_closed_form():
    """JA = JB = 0 from |0...0>: the links evolve independently, each by the
    product over steps of R_x(-hx dt) R_z(-2 hz dt) R_x(-hx dt) with the
    ramped fields; amplitudes are alpha^(n-w) beta^w."""
    Lx, Ly = 2, 3
    n = 12
    c0 = (0.0, 0.0, 0.1, 0.4)
    c1 = (0.0, 0.0, 0.7, -0.2)
    M, dt = 17, 0.23
    psi = oracle.state(n)
    psi[0] = 1
    oracle.evolve(Lx, Ly, psi, c0, c1, M, dt)
    u = np.array([1, 0], complex)
    for k in range(M):
        s = (k + 0.5) / M
        hx = (1 - s) * c0[2] + s * c1[2]
        hz = (1 - s) * c0[3] + s * c1[3]
        half = sla.expm(0.5j * hx * dt * SX)
        u = half @ sla.expm(1j * hz * dt * SZ) @ half @ u
    w = np.array([bin(i).count("1") for i in range(1 << n)])
    ref = u[0] ** (n - w) * u[1] ** w
    np.testing.assert_allclose(psi, ref, atol=1e-13)


def test_self_duality():
    """Sec. III: Hadamards on every link plus the lattice map star <-> plaquette
    turn H(JA,JB,hx,hz) into H(JB,JA,hz,hx) and psi_1 into psi_1'.  Hence the
    x-z-x step from psi_1 and the z-x-z step from psi_1' with the couplings
    exchanged give the same energy, with <sigma^x> and <sigma^z> swapped."""
    Lx, Ly, M, dt = 2, 3, 30, 0.15
    a0, a1 = (1.0, 0.7, 0.0, 0.0), (1.0, 0.7, 0.3, 0.2)
    b0, b1 = (0.7, 1.0, 0.0, 0.0), (0.7, 1.0, 0.2, 0.3)
    p = oracle.init_psi1(Lx, Ly)
    q = oracle.init_psi1p(Lx, Ly)
    oracle.evolve(Lx, Ly, p, a0, a1, M, dt, order=0)
    oracle.evolve(Lx, Ly, q, b0, b1, M, dt, order=1)
    op = oracle.observe(Lx, Ly, p, a1)
    oq = oracle.observe(Lx, Ly, q, b1)
    assert abs(op["energy"] - oq["energy"]) < 1e-12
    assert abs(op["mx"] - oq["mz"]) < 1e-12
    assert abs(op["mz"] - oq["mx"]) < 1e-12
    assert abs(op["sumA"] - oq["sumB"]) < 1e-12


def test_trotter_error_is_second_order_in_dt():
    """Global error of the ramp against the exact stepwise evolution falls
    ~4x per halving of dt at fixed T (second-order method)."""
    c0, c1 = (1, 1, 0, 0), (1, 1, 0.4, 0.3)
    T = 2.0
    errs = []
    for M in (10, 20, 40):
        psi0 = oracle.init_psi1(2, 2)
        psi = psi0.copy()
        oracle.evolve(2, 2, psi, c0, c1, M, T / M)
        ex = ed.exact_stepwise(2, 2, psi0, c0, c1, M, T / M)
        errs.append(np.linalg.norm(psi - ex))
    assert 3.6 < errs[0] / errs[1] < 4.4
    assert 3.8 < errs[1] / errs[2] < 4.2


def test_hamiltonian_rows_equal_sparse_matrix():
    """Row-by-row H x (used at sizes the sparse matrix cannot reach) equals
    the sparse H of the same couplings on every row."""
    for Lx, Ly in ((2, 2), (2, 3)):
        n = 2 * Lx * Ly
        x = _rand_state(n, 9)
        c = (0.7, 1.1, 0.3, -0.45)
        ref = ed.hamiltonian(Lx, Ly, c) @ x
        got = ed.hamiltonian_rows(Lx, Ly, c, np.arange(1 << n), lambda i: x[i])
        assert np.abs(got - ref).max() < 1e-13


def test_ground_state_vector_product_form():
    """JA = JB = 0: the ground state is the product over links of the lowest
    eigenvector of -hx X - hz Z (amplitudes alpha^(n-w) beta^w)."""
    Lx, Ly, n = 2, 3, 12
    hx, hz = 0.3, 0.4
    E0, v = ed.ground_state(Lx, Ly, (0.0, 0.0, hx, hz))
    w1, u1 = np.linalg.eigh(-hx * SX.real - hz * SZ.real)
    assert abs(E0 - n * w1[0]) < 1e-10
    a, b = u1[:, 0]
    w = np.array([bin(i).count("1") for i in range(1 << n)])
    ref = a ** (n - w) * b ** w
    assert abs(abs(np.vdot(ref, v)) - 1) < 1e-10


def test_sparse_exact_stepwise_equals_dense():
    """The sparse exact evolution (expm_multiply) and the dense one (expm)
    are two algorithms for the same product of exponentials."""
    for Lx, Ly, M, dt in ((2, 2, 7, 0.3), (2, 2, 3, 1.1)):
        psi0 = _rand_state(2 * Lx * Ly, 5)
        c0, c1 = (1.0, 0.8, 0.1, 0.0), (0.6, 1.0, 0.5, 0.3)
        a = ed.exact_stepwise(Lx, Ly, psi0, c0, c1, M, dt, sampling=1)
        b = ed.exact_stepwise_sparse(Lx, Ly, psi0, c0, c1, M, dt, sampling=1)
        assert np.abs(a - b).max() < 1e-12


def test_sparse_exact_stepwise_product_state():
    """JA = JB = 0 from |0...0> at 3x3, with separate schedule values for the
    x field (sX) and the z field (sZ): every link evolves by
    exp(-i dt (-hx X - hz Z)) per step, amplitudes alpha^(n-w) beta^w."""
    Lx, Ly, n, M, dt = 3, 3, 18, 6, 0.3
    c0, c1 = (0.0, 0.0, 0.2, 0.5), (0.0, 0.0, 0.9, -0.1)
    rng = np.random.default_rng(2)
    sZ, sX = rng.uniform(0, 1, M), rng.uniform(0, 1, M)
    psi0 = oracle.state(n)
    psi0[0] = 1
    psi = ed.exact_stepwise_sparse(Lx, Ly, psi0, c0, c1, M, dt, sZ=sZ, sX=sX)
    u = np.array([1, 0], complex)
    for k in range(M):
        hx = (1 - sX[k]) * c0[2] + sX[k] * c1[2]
        hz = (1 - sZ[k]) * c0[3] + sZ[k] * c1[3]
        u = sla.expm(1j * dt * (hx * SX + hz * SZ)) @ u
    w = np.array([bin(i).count("1") for i in range(1 << n)])
    assert np.abs(psi - u[0] ** (n - w) * u[1] ** w).max() < 1e-12


def test_sparse_exact_stepwise_zero_field_phase():
    """Zero field at 3x3: psi_1 only gains exp(+i (JA Ns + JB Np) T)."""
    JA, JB, M, dt = 0.5, 0.9, 4, 0.37
    psi0 = oracle.init_psi1(3, 3)
    psi = ed.exact_stepwise_sparse(3, 3, psi0, (JA, JB, 0, 0), (JA, JB, 0, 0), M, dt)
    assert np.abs(psi - np.exp(1j * (JA + JB) * 9 * M * dt) * psi0).max() < 1e-12


def test_norm_conserved():
    psi = oracle.init_psi1(3, 3)
    oracle.evolve(3, 3, psi, (1, 1, 0, 0), (1, 1, 0.3, 0.3), 20, 0.1)
    assert abs(np.vdot(psi, psi).real - 1) < 1e-13


def test_small_adiabatic_run_against_ed():
    """2x2, T = 10, M = 100 ramp to (0.2, 0.2) (Sec. VII-style comparison):
    the final energy lies above the exact ground energy (variational bound)
    and within the adiabatic error of it; the Trotterized and the exact
    stepwise runs agree to O(dt^2)."""
    c0, c1 = (1, 1, 0, 0), (1, 1, 0.2, 0.2)
    H = ed.hamiltonian(2, 2, c1).toarray()
    e0 = np.linalg.eigvalsh(H)[0]
    psi0 = oracle.init_psi1(2, 2)
    psi = psi0.copy()
    oracle.evolve(2, 2, psi, c0, c1, 100, 0.1)
    E = oracle.observe(2, 2, psi, c1)["energy"]
    assert E >= e0 - 1e-12
    assert E - e0 < 5e-2
    ex = ed.exact_stepwise(2, 2, psi0, c0, c1, 100, 0.1)
    Eex = np.vdot(ex, H @ ex).real
    assert abs(E - Eex) < 5e-4
    assert oracle.fidelity_loss(psi, ex) < 1e-4


def test_sector_conservation_on_field_axes():
    """Sec. IV: the 't Hooft loops V1, V2 commute with H when hz = 0, so
    psi_1 keeps <V1> = <V2> = 1 along the g axis; dually the Wilson loops
    W1, W2 commute with H when hx = 0, so psi_1' keeps <W1> = <W2> = 1."""
    lp = oracle.loops(3, 3)
    p = oracle.init_psi1(3, 3)
    oracle.evolve(3, 3, p, (1, 1, 0, 0), (1, 1, 0.4, 0.0), 8, 0.2)
    assert abs(oracle.expect_x(p, lp["V1"]) - 1) < 1e-12
    assert abs(oracle.expect_x(p, lp["V2"]) - 1) < 1e-12
    q = oracle.init_psi1p(3, 3)
    oracle.evolve(3, 3, q, (1, 1, 0, 0), (1, 1, 0.0, 0.4), 8, 0.2)
    assert abs(oracle.expect_z(q, lp["W1"]) - 1) < 1e-12
    assert abs(oracle.expect_z(q, lp["W2"]) - 1) < 1e-12


@pytest.mark.slow
def test_paper_printed_energies():
    """Fig. topo caption (Sec. IV): 3x3 torus with JA = JB = 1/2.  The printed
    adiabatic energies at p = 0.12 and 0.50 lie within 3e-4 above the exact
    ground energy of Eq. (effi) at (g, lambda) = (p, 0); the ground energy at
    (0, p) is the same by self-duality."""
    rows = _read_golden("paper_energies.txt")
    for p, E, Ep in rows:
        e0 = ed.ground(3, 3, (0.5, 0.5, p, 0.0))[0]
        e0d = ed.ground(3, 3, (0.5, 0.5, 0.0, p))[0]
        assert abs(e0 - e0d) < 1e-8
        for val in (E, Ep):
            if p < 0.2 and val == Ep:
                continue  # E' at p = 0.12 is the other topological sector (history dependent)
            assert -1e-6 < val - e0 < 3e-4


# ------------------------------------------------------------------ DOS

def test_weight_histogram_brute_force():
    """Sec. V: the DOS of Ztilde = -sum Z is |psi|^2 binned by the number w of
    links with sigma^z = -1.  For psi_1 on 2x2 it is the count of
    even-plaquette configurations of weight w over 32."""
    psi = oracle.init_psi1(2, 2)
    hist = oracle.weight_hist(psi)
    st, pl = oracle.masks(2, 2)
    ref = np.zeros(9)
    for i in range(256):
        if all(bin(i & int(m)).count("1") % 2 == 0 for m in pl):
            ref[bin(i).count("1")] += 1 / 32
    np.testing.assert_allclose(hist, ref, atol=1e-14)


# ------------------------------------------------------------------ bound

def test_trotter_bound_table():
    """Table contrast_tab: the closed-form bound reproduces every printed
    epsilon; the step-by-step sum of Eq. (target) agrees with it to O(1/N);
    epsilon(n0=10)/epsilon(800) is exactly (800/10)^2."""
    rows = _read_golden("trotter_bound_table.txt")
    p, r = 0.5, 0.05
    for n, dg, dt, eps in rows:
        cf = bound.closed_form(p, r, dg, dt)
        assert abs(cf - eps) <= 0.5e-5 + 1e-12
        sm = bound.summed(p, r, dg, dt)
        assert abs(sm - cf) / cf < 1e-4
    e10 = bound.closed_form(p, r, rows[0][1], rows[0][2])
    e800 = bound.closed_form(p, r, rows[3][1], rows[3][2])
    assert abs(e10 / e800 - 6400) < 1e-6


# ------------------------------------------------------------------ gate-level circuits (Sec. III)

from oracle import circuit  # noqa: E402


def test_circuit_gates_against_expm():
    """Each gate's matrix and the ancilla gadget against scipy's expm: on
    links with the ancilla in |0>, CNOTs - R_z(theta) - CNOTs equals
    exp(-i theta/2 Z_links) and returns the ancilla to |0>."""
    n = 5
    rng = np.random.default_rng(21)
    x = _rand_state(n, 22)
    for name, M in (("RX", lambda t: sla.expm(-0.5j * t * SX)), ("RZ", lambda t: sla.expm(-0.5j * t * SZ))):
        th = rng.uniform(-2, 2)
        got = circuit.apply(x, [(name, (2,), th)])
        ref = np.einsum("ij,ajb->aib", M(th), x.reshape(1 << (n - 3), 2, 4)).reshape(-1)
        assert np.abs(got - ref).max() < 1e-14
    links, anc, th = [0, 2, 3], 4, 0.83
    y = circuit.apply(x[: 1 << 4].copy().tolist() + [0] * (1 << 4), circuit._gadget(anc, links, th))
    zs = np.ones(1 << 4)
    for i in range(1 << 4):
        zs[i] = (-1) ** sum((i >> l) & 1 for l in links)
    ref = np.exp(-0.5j * th * zs) * x[: 1 << 4]
    assert np.abs(y[: 1 << 4] - ref).max() < 1e-14
    assert np.abs(y[1 << 4:]).max() < 1e-15


@pytest.mark.parametrize("Lx,Ly", [(2, 2), (2, 3)])
@pytest.mark.parametrize("order", [0, 1])
def test_circuit_step_equals_algebraic_step(Lx, Ly, order):
    """Sec. III: one gate-level step with the ancilla in |0> equals the
    oracle's Trotter step (Pauli-string exponentials, pinned above) on the
    links, and leaves the ancilla in |0>."""
    n = 2 * Lx * Ly
    x = _rand_state(n, 30 + order)
    cx, cz = (0.7, 0.4, 0.3, 0.2), (0.6, 0.9, 0.1, 0.45)
    got = circuit.apply(circuit.with_ancilla(x), circuit.step_gates(Lx, Ly, cx, cz, 0.37, order))
    ref = x.copy()
    oracle.trotter_step(Lx, Ly, ref, cx, cz, 0.37, order)
    assert np.abs(got[: 1 << n] - ref).max() < 1e-13
    assert np.abs(got[1 << n:]).max() < 1e-14


@pytest.mark.parametrize("Lx,Ly", [(2, 2), (2, 3)])
def test_preparation_circuits(Lx, Ly):
    """Eqs. (ini1) and (ini2) at gate level give psi_1 and psi_1'."""
    n = 2 * Lx * Ly
    zero = np.zeros(1 << (n + 1), complex)
    zero[0] = 1
    p1 = circuit.apply(zero, circuit.prep_gates(Lx, Ly, "psi1"))
    p2 = circuit.apply(zero, circuit.prep_gates(Lx, Ly, "psi1p"))
    assert np.abs(p1[: 1 << n] - oracle.init_psi1(Lx, Ly)).max() < 1e-14
    assert np.abs(p2[: 1 << n] - oracle.init_psi1p(Lx, Ly)).max() < 1e-14
    assert np.abs(p1[1 << n:]).max() == 0 and np.abs(p2[1 << n:]).max() == 0


def test_circuit_gate_count():
    """Per step: n rotations in each of the three field layers, and in each
    of the two stabilizer halves 4 + 1 + 4 gates per plaquette gadget and
    4 + 9 + 4 per star gadget: 3n + 2 (9 Np + 17 Ns) = 522 at 3x3."""
    for Lx, Ly in ((2, 2), (3, 3), (4, 4)):
        n, nv = 2 * Lx * Ly, Lx * Ly
        assert len(circuit.step_gates(Lx, Ly, (1, 1, 0.1, 0.1), (1, 1, 0.1, 0.1), 0.1)) == 3 * n + 2 * 26 * nv
    assert 3 * 18 + 2 * 26 * 9 == 522


# ------------------------------------------------------------------ schedule branches of the ramp (Sec. III, Appendix)

def _single_link_ramp(c0, c1, M, dt, sx_of, sz_of):
    """Closed form of one decoupled link (JA = JB = 0): per step the x-field
    half, the full z-field factor and the x-field half again (Sec. III), with
    the x field taken at sx_of(k) and the z field at sz_of(k).  Matrices come
    from scipy's expm of the 2x2 Pauli generators, not from the oracle."""
    u = np.array([1, 0], complex)
    for k in range(M):
        sx, sz = sx_of(k), sz_of(k)
        hx = (1 - sx) * c0[2] + sx * c1[2]
        hz = (1 - sz) * c0[3] + sz * c1[3]
        half = sla.expm(0.5j * hx * dt * SX)
        u = half @ sla.expm(1j * hz * dt * SZ) @ half @ u
    return u


def _product_amplitudes(u, n):
    w = np.array([bin(i).count("1") for i in range(1 << n)])
    return u[0] ** (n - w) * u[1] ** w


def test_right_endpoint_sampling_closed_form():
    """Appendix, Eq. (target): the paper's ramp takes g = n dg for n = 1..N,
    i.e. step k (0-based) uses s_k = (k + 1)/M.  JA = JB = 0 from |0...0>:
    every link follows the single-link product at those s_k.  Midpoint or
    left-end sampling moves the fields by dg/2 or dg per step and fails by
    far more than the tolerance."""
    Lx, Ly, n = 2, 3, 12
    c0, c1 = (0.0, 0.0, 0.1, 0.4), (0.0, 0.0, 0.9, -0.3)
    M, dt = 13, 0.31
    psi = oracle.state(n)
    psi[0] = 1
    oracle.evolve(Lx, Ly, psi, c0, c1, M, dt, sampling=1)
    right = _product_amplitudes(_single_link_ramp(c0, c1, M, dt, lambda k: (k + 1) / M, lambda k: (k + 1) / M), n)
    assert np.abs(psi - right).max() < 1e-13
    for wrong in (lambda k: k / M, lambda k: (k + 0.5) / M):
        other = _product_amplitudes(_single_link_ramp(c0, c1, M, dt, wrong, wrong), n)
        assert np.abs(psi - other).max() > 1e-3


def test_per_step_schedule_arrays_closed_form():
    """Per-step schedule values (the adjoint's free parameters): the x-type
    couplings of step k sit at sX[k] and the z-type ones at sZ[k].  JA = JB = 0
    from |0...0> pins the fields: h_x at sX[k], h_z at sZ[k] (the swapped
    assignment fails)."""
    Lx, Ly, n = 2, 3, 12
    c0, c1 = (0.0, 0.0, 0.2, 0.5), (0.0, 0.0, 0.8, -0.4)
    M, dt = 11, 0.27
    rng = np.random.default_rng(17)
    sZ, sX = rng.uniform(-0.2, 1.2, M), rng.uniform(-0.2, 1.2, M)
    psi = oracle.state(n)
    psi[0] = 1
    oracle.evolve(Lx, Ly, psi, c0, c1, M, dt, sZ=sZ, sX=sX)
    ref = _product_amplitudes(_single_link_ramp(c0, c1, M, dt, lambda k: sX[k], lambda k: sZ[k]), n)
    assert np.abs(psi - ref).max() < 1e-13
    swapped = _product_amplitudes(_single_link_ramp(c0, c1, M, dt, lambda k: sZ[k], lambda k: sX[k]), n)
    assert np.abs(psi - swapped).max() > 1e-3


def test_per_step_schedule_arrays_stabilizer_phase():
    """Zero fields, per-step schedule values: psi_1 (Eq. (ini1)) is a +1
    eigenstate of every A_v and B_p, so step k multiplies it by
    exp(+i dt (JA(sX[k]) Ns + JB(sZ[k]) Np)).  Pins that the star coupling
    follows sX and the plaquette coupling sZ."""
    Lx, Ly = 2, 3
    nv = Lx * Ly
    c0, c1 = (0.3, 1.4, 0.0, 0.0), (1.1, -0.2, 0.0, 0.0)
    M, dt = 9, 0.21
    rng = np.random.default_rng(18)
    sZ, sX = rng.uniform(0, 1, M), rng.uniform(0, 1, M)
    psi0 = oracle.init_psi1(Lx, Ly)
    psi = psi0.copy()
    oracle.evolve(Lx, Ly, psi, c0, c1, M, dt, sZ=sZ, sX=sX)
    ang = sum(dt * nv * (((1 - sX[k]) * c0[0] + sX[k] * c1[0]) + ((1 - sZ[k]) * c0[1] + sZ[k] * c1[1]))
              for k in range(M))
    assert np.abs(psi - np.exp(1j * ang) * psi0).max() < 1e-13
    bad = sum(dt * nv * (((1 - sZ[k]) * c0[0] + sZ[k] * c1[0]) + ((1 - sX[k]) * c0[1] + sX[k] * c1[1]))
              for k in range(M))
    assert np.abs(psi - np.exp(1j * bad) * psi0).max() > 1e-3


@pytest.mark.parametrize("sampling", [0, 1])
def test_schedule_arrays_equal_to_linear_schedule_are_the_default(sampling):
    """sZ = sX = the default sampling points reproduces the default run bit
    for bit (same couplings, same arithmetic), for both samplings."""
    Lx, Ly, M, dt = 2, 3, 15, 0.2
    c0, c1 = (1.0, 0.8, 0.0, 0.1), (0.7, 1.0, 0.45, 0.3)
    k = np.arange(M, dtype=np.float64)
    s = (k + 1) / M if sampling else (k + 0.5) / M
    a = oracle.init_psi1(Lx, Ly)
    b = a.copy()
    oracle.evolve(Lx, Ly, a, c0, c1, M, dt, sampling=sampling)
    oracle.evolve(Lx, Ly, b, c0, c1, M, dt, sZ=s, sX=s.copy(), sampling=sampling)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("sampling", [0, 1])
@pytest.mark.parametrize("order", [0, 1])
def test_circuit_ramp_equals_oracle_ramp(sampling, order):
    """The gate-level ramp (ancilla gadgets, Sec. III) equals the oracle's
    Pauli-exponential ramp at 2x2 for both samplings and both orders, with
    the ancilla back in |0>; the two share no code."""
    Lx, Ly, n, M, dt = 2, 2, 8, 7, 0.33
    c0, c1 = (1.0, 0.6, 0.0, 0.2), (0.8, 1.0, 0.5, 0.35)
    x = oracle.init_psi1(Lx, Ly)
    got = circuit.evolve(Lx, Ly, circuit.with_ancilla(x), c0, c1, M, dt, sampling=sampling, order=order)
    ref = x.copy()
    oracle.evolve(Lx, Ly, ref, c0, c1, M, dt, sampling=sampling, order=order)
    assert np.abs(got[: 1 << n] - ref).max() < 1e-13
    assert np.abs(got[1 << n:]).max() < 1e-14


def test_circuit_ramp_right_endpoint_closed_form():
    """Gate-level ramp with JA = JB = 0 from |0...0> (plus the ancilla) at
    s_k = (k + 1)/M: the decoupled-link closed form."""
    Lx, Ly, n, M, dt = 2, 2, 8, 6, 0.4
    c0, c1 = (0.0, 0.0, 0.3, -0.2), (0.0, 0.0, 0.7, 0.6)
    x = oracle.state(n + 1)
    x[0] = 1
    got = circuit.evolve(Lx, Ly, x, c0, c1, M, dt, sampling=1)
    ref = _product_amplitudes(_single_link_ramp(c0, c1, M, dt, lambda k: (k + 1) / M, lambda k: (k + 1) / M), n)
    assert np.abs(got[: 1 << n] - ref).max() < 1e-13
    assert np.abs(got[1 << n:]).max() < 1e-14
