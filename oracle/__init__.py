"""FP64 CPU oracle for the Trotterized toric-code evolution.

TEST INFRASTRUCTURE ONLY: this package checks the HIP library; it is never on
the product path.  Only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it.  It shares no code with the HIP
library (own lattice, own link numbering, gate-by-gate application of the
paper's circuit factors).

Contents
  - ctypes wrapper around ``z2h_oracle.c`` (state preparation, Trotter step,
    Pauli expectations), built into ``liboracle.so`` by ``oracle/build.py``;
  - ``ed``: sparse Hamiltonian, exact diagonalisation and exact stepwise
    evolution with NumPy/SciPy (Sec. VII comparison with ED);
  - ``bound``: the Trotter error bound of the Appendix.

Parity status of every function is listed in the module docstrings; all of
them are pinned by tests under ``tests/test_oracle*.py``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# Z2H_ORACLE_LIB names another build of the C core (the sanitizer build run
# by the CPU tests); default: the in-tree build.
_LIB_PATH = os.environ.get("Z2H_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def lib():
    """Load liboracle.so, building it with gcc if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        c_int, c_i64, c_u64, c_dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        P = ctypes.c_void_p
        L.or_link.argtypes = [c_int, c_int, c_int, c_int, c_int]
        L.or_link.restype = c_i64
        L.or_masks.argtypes = [c_int, c_int, P, P]
        L.or_masks.restype = c_int
        for name in ("or_h",):
            getattr(L, name).argtypes = [c_int, P, c_int]
        L.or_rx.argtypes = [c_int, P, c_int, c_dbl]
        L.or_rz.argtypes = [c_int, P, c_int, c_dbl]
        L.or_exp_z.argtypes = [c_int, P, c_u64, c_dbl]
        L.or_exp_x.argtypes = [c_int, P, c_u64, c_dbl]
        L.or_init_psi1.argtypes = [c_int, c_int, P]
        L.or_init_psi1.restype = c_int
        L.or_init_psi1p.argtypes = [c_int, c_int, P]
        L.or_init_psi1p.restype = c_int
        L.or_trotter_step.argtypes = [c_int, c_int, P, P, P, c_dbl, c_int]
        L.or_evolve.argtypes = [c_int, c_int, P, P, P, c_i64, c_dbl, P, P, c_int, c_int]
        L.or_evolve.restype = c_int
        L.or_expect_z.argtypes = [c_int, P, c_u64]
        L.or_expect_z.restype = c_dbl
        L.or_expect_x.argtypes = [c_int, P, c_u64]
        L.or_expect_x.restype = c_dbl
        L.or_observe.argtypes = [c_int, c_int, P, P, P]
        L.or_observe.restype = c_int
        L.or_weight_hist.argtypes = [c_int, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c4(c):
    a = np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(4))
    return a


# ------------------------------------------------------------------ lattice

def link(Lx, Ly, x, y, d):
    """Oracle index of link h(x,y) (d=0) or v(x,y) (d=1)."""
    return int(lib().or_link(Lx, Ly, x, y, d))


def masks(Lx, Ly):
    """(stars, plaquettes) as uint64 arrays indexed by vertex y*Lx + x."""
    st = np.zeros(Lx * Ly, np.uint64)
    pl = np.zeros(Lx * Ly, np.uint64)
    if lib().or_masks(Lx, Ly, _p(st), _p(pl)) != 0:
        raise ValueError("bad lattice")
    return st, pl


def loops(Lx, Ly):
    """Noncontractible loops of Sec. IV (masks in oracle numbering).

    W1 = prod_x Z on h(x,0) and W2 = prod_y Z on v(0,y) are the Wilson loops
    around the two cycles; V1 = prod_x X on v(x,0) and V2 = prod_y X on h(0,y)
    are the 't Hooft loops crossing them.
    """
    W1 = sum(1 << link(Lx, Ly, x, 0, 0) for x in range(Lx))
    W2 = sum(1 << link(Lx, Ly, 0, y, 1) for y in range(Ly))
    V1 = sum(1 << link(Lx, Ly, x, 0, 1) for x in range(Lx))
    V2 = sum(1 << link(Lx, Ly, 0, y, 0) for y in range(Ly))
    return {"W1": W1, "W2": W2, "V1": V1, "V2": V2}


# ------------------------------------------------------------------ states

def state(n):
    return np.zeros(1 << n, np.complex128)


def init_psi1(Lx, Ly):
    """psi_1 of Eq. (ini1)."""
    psi = state(2 * Lx * Ly)
    lib().or_init_psi1(Lx, Ly, _p(psi))
    return psi


def init_psi1p(Lx, Ly):
    """psi_1' of Eq. (ini2)."""
    psi = state(2 * Lx * Ly)
    lib().or_init_psi1p(Lx, Ly, _p(psi))
    return psi


def apply_x_string(psi, mask):
    """X_mask psi (pure permutation, for building the sector states of Sec. IV)."""
    idx = np.arange(psi.size, dtype=np.uint64)
    return psi[idx ^ np.uint64(mask)]


def apply_z_string(psi, mask):
    idx = np.arange(psi.size, dtype=np.uint64) & np.uint64(mask)
    par = np.zeros(psi.size, np.int64)
    m = int(mask)
    while m:
        b = m & -m
        par ^= ((idx & np.uint64(b)) != 0).astype(np.int64)
        m ^= b
    return psi * (1 - 2 * par)


# ------------------------------------------------------------------ gates

def rx(psi, l, theta):
    lib().or_rx(int(np.log2(psi.size)), _p(psi), l, theta)


def rz(psi, l, theta):
    lib().or_rz(int(np.log2(psi.size)), _p(psi), l, theta)


def exp_z(psi, mask, theta):
    lib().or_exp_z(int(np.log2(psi.size)), _p(psi), mask, theta)


def exp_x(psi, mask, theta):
    lib().or_exp_x(int(np.log2(psi.size)), _p(psi), mask, theta)


def trotter_step(Lx, Ly, psi, cx, cz, dt, order=0):
    """One step of Sec. III in place; cx/cz = couplings (JA,JB,hx,hz) for the
    x-type and z-type terms."""
    lib().or_trotter_step(Lx, Ly, _p(psi), _p(_c4(cx)), _p(_c4(cz)), dt, order)


def evolve(Lx, Ly, psi, c0, c1, M, dt, sZ=None, sX=None, sampling=0, order=0):
    """Adiabatic ramp c(s) = (1-s) c0 + s c1 over M steps of dt, in place."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous
    sZa = None if sZ is None else np.ascontiguousarray(sZ, dtype=np.float64)
    sXa = None if sX is None else np.ascontiguousarray(sX, dtype=np.float64)
    rc = lib().or_evolve(Lx, Ly, _p(psi), _p(_c4(c0)), _p(_c4(c1)), int(M), float(dt),
                         None if sZa is None else _p(sZa), None if sXa is None else _p(sXa),
                         int(sampling), int(order))
    if rc != 0:
        raise ValueError("or_evolve rejected its arguments")
    return psi


# ------------------------------------------------------------------ observables

def expect_z(psi, mask):
    return float(lib().or_expect_z(int(np.log2(psi.size)), _p(psi), int(mask)))


def expect_x(psi, mask):
    return float(lib().or_expect_x(int(np.log2(psi.size)), _p(psi), int(mask)))


def observe(Lx, Ly, psi, c):
    """dict(norm, energy, sumA, sumB, mx, mz) -- raw sums for the given state."""
    out = np.zeros(6)
    lib().or_observe(Lx, Ly, _p(psi), _p(_c4(c)), _p(out))
    return dict(zip(("norm", "energy", "sumA", "sumB", "mx", "mz"), out.tolist()))


def weight_hist(psi):
    """Distribution of |psi|^2 over Hamming weight w (Ztilde = 2w - n, Sec. V)."""
    n = int(np.log2(psi.size))
    out = np.zeros(n + 1)
    lib().or_weight_hist(n, _p(psi), _p(out))
    return out


def fidelity_loss(a, b):
    """1 - |<a|b>|^2 / (<a|a><b|b>): ignores a global phase."""
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    ov = np.vdot(a, b)
    return float(1.0 - abs(ov) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))
