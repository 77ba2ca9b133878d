"""Adjoint gradient (reverse evolution) against central FP64 finite
differences of the oracle, step 1e-6, through torch.autograd."""
import numpy as np
import pytest
import torch

import oracle
from paper_2108_13410_amd import workloads, z2h
from paper_2108_13410_amd.autograd import EvolveEnergy

pytestmark = pytest.mark.gpu


def oracle_loss(Lx, Ly, c0, c1, dt, sZ, sX, lossH):
    psi = oracle.init_psi1(Lx, Ly)
    oracle.evolve(Lx, Ly, psi, c0, c1, len(sZ), dt, sZ=sZ, sX=sX)
    return oracle.observe(Lx, Ly, psi, lossH)["energy"] / oracle.observe(Lx, Ly, psi, lossH)["norm"]


def fd(Lx, Ly, c0, c1, dt, sZ, sX, lossH, kind, k, h=1e-6):
    a, b = sZ.copy(), sX.copy()
    arr = a if kind == 0 else b
    arr[k] += h
    lp = oracle_loss(Lx, Ly, c0, c1, dt, a, b, lossH)
    arr[k] -= 2 * h
    lm = oracle_loss(Lx, Ly, c0, c1, dt, a, b, lossH)
    return (lp - lm) / (2 * h)


def adjoint_grad(Lx, Ly, dtype, c0, c1, dt, sZ, sX, lossH, mtb=0):
    plan = z2h.z2h_plan_create(Lx, Ly, dtype, mtb)
    tz = torch.tensor(sZ, dtype=torch.float64, requires_grad=True)
    tx = torch.tensor(sX, dtype=torch.float64, requires_grad=True)
    L = EvolveEnergy.apply(tz, tx, plan, c0, c1, dt, lossH)
    L.backward()
    return L.item(), tz.grad.numpy(), tx.grad.numpy()


def test_adjoint_2x2_all_entries():
    """One-workgroup plan: every one of the 2M gradient entries against FD."""
    rng = np.random.default_rng(5)
    M, dt = 12, 0.2
    c0, c1, H = (1.0, 0.8, 0.0, 0.0), (0.7, 1.0, 0.45, 0.3), (0.9, 1.1, 0.35, 0.25)
    sZ = (np.arange(M) + 0.5) / M + rng.normal(0, 0.05, M)
    sX = (np.arange(M) + 0.5) / M + rng.normal(0, 0.05, M)
    L, gZ, gX = adjoint_grad(2, 2, z2h.Z2H_C128, c0, c1, dt, sZ, sX, H)
    assert abs(L - oracle_loss(2, 2, c0, c1, dt, sZ, sX, H)) < 1e-12
    for k in range(M):
        for kind, g in ((0, gZ), (1, gX)):
            ref = fd(2, 2, c0, c1, dt, sZ, sX, H, kind, k)
            assert abs(g[k] - ref) < 1e-7 * max(1.0, abs(ref)), (kind, k, g[k], ref)


def test_adjoint_plans_agree():
    """Two- and three-group pass schedules give the same gradient."""
    rng = np.random.default_rng(6)
    M, dt = 10, 0.15
    c0, c1, H = (1, 1, 0, 0), (1, 1, 0.3, 0.3), (1, 1, 0.3, 0.3)
    sZ = (np.arange(M) + 0.5) / M + rng.normal(0, 0.01, M)
    sX = (np.arange(M) + 0.5) / M + rng.normal(0, 0.01, M)
    a = adjoint_grad(3, 3, z2h.Z2H_C128, c0, c1, dt, sZ, sX, H)
    b = adjoint_grad(3, 3, z2h.Z2H_C128, c0, c1, dt, sZ, sX, H, mtb=10)
    assert abs(a[0] - b[0]) < 1e-12
    np.testing.assert_allclose(a[1], b[1], atol=1e-11)
    np.testing.assert_allclose(a[2], b[2], atol=1e-11)


@pytest.mark.parametrize("dtype,cfg", [(z2h.Z2H_C128, "split=10:5:11:0/10:5:13:3:1c"),
                                       (z2h.Z2H_C64, "split=10:5:11:0:1c/10:5:14:4:1c")])
def test_adjoint_component_exchange_plan(dtype, cfg):
    """2x5 torus: a plan whose Trotter passes use the component exchange
    (half the LDS) gives the gradient of the same plan with element
    exchanges; the adjoint's own kernels size their LDS for whole elements."""
    print(f"case adjoint 2x5 dtype={dtype} {cfg}", flush=True)
    rng = np.random.default_rng(8)
    M, dt = 6, 0.15
    c0, c1, H = (1, 1, 0, 0), (1, 0.9, 0.35, 0.25), (1, 0.9, 0.35, 0.25)
    sZ = (np.arange(M) + 0.5) / M + rng.normal(0, 0.01, M)
    sX = (np.arange(M) + 0.5) / M + rng.normal(0, 0.01, M)
    out = []
    for c in (cfg, cfg.replace(":1c", "")):
        plan = z2h.z2h_plan_create_config(2, 5, dtype, c)
        tz = torch.tensor(sZ, dtype=torch.float64, requires_grad=True)
        tx = torch.tensor(sX, dtype=torch.float64, requires_grad=True)
        L = EvolveEnergy.apply(tz, tx, plan, c0, c1, dt, H)
        L.backward()
        out.append((L.item(), tz.grad.numpy(), tx.grad.numpy()))
    assert out[0][0] == out[1][0]
    np.testing.assert_array_equal(out[0][1], out[1][1])
    np.testing.assert_array_equal(out[0][2], out[1][2])
    assert np.all(np.isfinite(out[0][1])) and np.abs(out[0][1]).max() > 0


@pytest.mark.parametrize("cfg", ["split=4:2:8:0/10:5:13:3:1c:h3@17/6:3:9:3",
                                 "split=4:2:8:0/6:3:9:3:at8/10:5:13:3:1c"])
def test_adjoint_split_run_plan(cfg):
    """2x5 torus, complex128: plans with a group in two runs of qubits (the
    middle group, or the last group with the x-basis phase) give the
    gradient of a plan with contiguous groups, to rounding."""
    print(f"case adjoint 2x5 {cfg}", flush=True)
    rng = np.random.default_rng(9)
    M, dt = 6, 0.15
    c0, c1, H = (1, 1, 0, 0), (1, 0.9, 0.35, 0.25), (1, 0.9, 0.35, 0.25)
    sZ = (np.arange(M) + 0.5) / M + rng.normal(0, 0.01, M)
    sX = (np.arange(M) + 0.5) / M + rng.normal(0, 0.01, M)
    out = []
    for c in (cfg, "split=10:5:11:0/10:5:13:3:1c"):
        plan = z2h.z2h_plan_create_config(2, 5, z2h.Z2H_C128, c)
        tz = torch.tensor(sZ, dtype=torch.float64, requires_grad=True)
        tx = torch.tensor(sX, dtype=torch.float64, requires_grad=True)
        L = EvolveEnergy.apply(tz, tx, plan, c0, c1, dt, H)
        L.backward()
        out.append((L.item(), tz.grad.numpy(), tx.grad.numpy()))
    assert abs(out[0][0] - out[1][0]) < 1e-12
    np.testing.assert_allclose(out[0][1], out[1][1], atol=1e-11)
    np.testing.assert_allclose(out[0][2], out[1][2], atol=1e-11)
    assert np.abs(out[0][1]).max() > 0


@pytest.mark.slow
def test_adjoint_3x3_config():
    """3x3 torus, M = 200 (T = 20), two schedule values per step from the
    linear schedule plus N(0, 0.01) noise; loss <H1> at (0.3, 0.3); 10
    seeded entries against central FD (step 1e-6) of the FP64 oracle."""
    M, T = 200, 20.0
    c0, c1 = workloads.TORIC, workloads.point(0.3, 0.3)
    sZ, sX = workloads.adjoint_angles(M)
    L, gZ, gX = adjoint_grad(3, 3, z2h.Z2H_C128, c0, c1, T / M, sZ, sX, c1)
    assert abs(L - oracle_loss(3, 3, c0, c1, T / M, sZ, sX, c1)) < 1e-10
    worst = 0.0
    for kind, k in workloads.fd_indices(M):
        g = (gZ if kind == 0 else gX)[k]
        ref = fd(3, 3, c0, c1, T / M, sZ, sX, c1, kind, k)
        err = abs(g - ref) / max(1.0, abs(ref))
        worst = max(worst, err)
        print(f"entry ({kind},{k}) adjoint {g:.10e} fd {ref:.10e} rel {err:.2e}", flush=True)
        assert err < 1e-6
    print("worst relative error", worst)
