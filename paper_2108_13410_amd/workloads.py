"""Seeded synthetic workloads (inputs only: lattices, couplings, step counts,
schedule perturbations).  Shared by the tests, the benchmark and the oracle
checks; holds none of the method's arithmetic.

The paper studies synthetic lattice Hamiltonians only (no dataset); these
generators produce the configurations the benchmark and the parity tests
use:

  point_2x2   2x2 torus, ramp from the toric code to (hx, hz) = (0.2, 0.2),
              T = 10, M = 100 (complex128)
  point_3x3   3x3 torus, ramp to (0.3, 0.3), T = 20, M = 1000
  scan_3x3    32 x 32 grid of (hx, hz) on [0, 0.6]^2, 3x3, T = 20, M = 1000
  mixed       2x2, 2x3 and 3x3 tori, (hx, hz) ~ U[0, 0.6]^2, M ~ U{200..1000},
              T = 20 (seeded)
  adjoint     3x3, M = 200, T = 20, per-step schedule values (k + 1/2)/M plus
              N(0, 0.01) noise (seeded)
  point_4x4   4x4 torus, ramp to (0.25, 0.25), T = 20, M = 200
"""
from __future__ import annotations

import numpy as np

SEED = 13410
TORIC = (1.0, 1.0, 0.0, 0.0)  # JA, JB, hx, hz at s = 0


def point(hx, hz, JA=1.0, JB=1.0):
    return (JA, JB, float(hx), float(hz))


def point_2x2():
    return dict(Lx=2, Ly=2, c0=TORIC, c1=point(0.2, 0.2), T=10.0, M=100)


def point_3x3():
    return dict(Lx=3, Ly=3, c0=TORIC, c1=point(0.3, 0.3), T=20.0, M=1000)


def point_4x4(M=200):
    return dict(Lx=4, Ly=4, c0=TORIC, c1=point(0.25, 0.25), T=20.0, M=M)


def scan_3x3(side=32, hmax=0.6, M=1000, T=20.0):
    """Grid of (hx, hz), endpoints included, hz fastest."""
    h = np.linspace(0.0, hmax, side)
    jobs = []
    for hx in h:
        for hz in h:
            jobs.append(dict(Lx=3, Ly=3, c0=TORIC, c1=point(hx, hz), T=T, M=M))
    return jobs


def mixed(count_each=32, seed=SEED, T=20.0, mlo=200, mhi=1000):
    rng = np.random.default_rng(seed)
    jobs = []
    for (Lx, Ly) in ((2, 2), (2, 3), (3, 3)):
        for _ in range(count_each):
            hx, hz = rng.uniform(0.0, 0.6, 2)
            M = int(rng.integers(mlo, mhi + 1))
            jobs.append(dict(Lx=Lx, Ly=Ly, c0=TORIC, c1=point(hx, hz), T=T, M=M))
    return jobs


def adjoint_angles(M=200, sigma=0.01, seed=SEED):
    rng = np.random.default_rng(seed)
    base = (np.arange(M) + 0.5) / M
    return base + rng.normal(0.0, sigma, M), base + rng.normal(0.0, sigma, M)


def fd_indices(M=200, count=10, seed=SEED):
    """Indices (kind, k) of the schedule values checked by finite differences:
    kind 0 = z-type value sZ[k], 1 = x-type value sX[k]."""
    rng = np.random.default_rng(seed + 1)
    flat = rng.choice(2 * M, size=count, replace=False)
    return [(int(f) // M, int(f) % M) for f in flat]
