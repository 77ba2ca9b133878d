"""Exact diagonalisation and exact stepwise evolution (Sec. VII), NumPy/SciPy.

TEST INFRASTRUCTURE ONLY.  Builds the Hamiltonian of Eq. (effi) with general
couplings c = (JA, JB, hx, hz),

    H = -JA sum_v A_v - JB sum_p B_p - hx sum_l X_l - hz sum_l Z_l,

as a sparse matrix in the oracle's basis (bit l of the index = link l, 0 is
sigma^z = +1), from the oracle's own star/plaquette masks.

Pinned by: the closed-form toric-code spectrum at zero field (degeneracies
included), the paper's printed 3x3 energies (Fig. topo caption), and the
self-duality of the model (Sec. III).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import masks


def _parity(idx, mask):
    v = idx & np.uint64(mask)
    par = np.zeros(idx.shape, np.int64)
    m = int(mask)
    while m:
        b = m & -m
        par ^= ((v & np.uint64(b)) != 0).astype(np.int64)
        m ^= b
    return par


def hamiltonian_parts(Lx, Ly):
    """Dict of the four sparse operators sum_v A_v, sum_p B_p, sum_l X_l, sum_l Z_l."""
    n = 2 * Lx * Ly
    N = 1 << n
    st, pl = masks(Lx, Ly)
    idx = np.arange(N, dtype=np.uint64)
    diagB = np.zeros(N)
    for m in pl:
        diagB += 1 - 2 * _parity(idx, m)
    diagZ = np.zeros(N)
    for l in range(n):
        diagZ += 1 - 2 * ((idx >> np.uint64(l)) & np.uint64(1)).astype(np.int64)

    def xsum(mlist):
        rows = np.concatenate([idx for _ in mlist])
        cols = np.concatenate([idx ^ np.uint64(m) for m in mlist])
        data = np.ones(rows.size)
        return sp.csr_matrix((data, (rows.astype(np.int64), cols.astype(np.int64))), shape=(N, N))

    return {
        "A": xsum([int(m) for m in st]),
        "B": sp.diags(diagB).tocsr(),
        "X": xsum([1 << l for l in range(n)]),
        "Z": sp.diags(diagZ).tocsr(),
    }


def hamiltonian(Lx, Ly, c, parts=None):
    """Sparse H(c) of Eq. (effi) with couplings c = (JA, JB, hx, hz)."""
    P = parts if parts is not None else hamiltonian_parts(Lx, Ly)
    JA, JB, hx, hz = (float(v) for v in c)
    return (-JA * P["A"] - JB * P["B"] - hx * P["X"] - hz * P["Z"]).tocsr()


def hamiltonian_rows(Lx, Ly, c, rows, fetch):
    """Entries (H x)_r for the oracle-basis indices r in `rows`, from the
    definition of Eq. (effi) row by row: the plaquette and z-field terms are
    diagonal, a star or an x field flips its links, so

        (H x)_r = [-JB sum_p (-1)^{par(r & p)} - hz sum_l (1 - 2 r_l)] x_r
                  - JA sum_v x_{r ^ v} - hx sum_l x_{r ^ 2^l}.

    fetch(idx) must return x at the oracle-basis indices idx (int64 array).
    Any lattice size: only the sampled rows and their neighbours are read."""
    n = 2 * Lx * Ly
    st, pl = masks(Lx, Ly)
    JA, JB, hx, hz = (float(v) for v in c)
    r = np.asarray(rows, dtype=np.uint64)
    dZ = np.zeros(r.shape)
    for m in pl:
        dZ += 1 - 2 * _parity(r, m)
    wz = np.zeros(r.shape)
    for l in range(n):
        wz += 1 - 2 * ((r >> np.uint64(l)) & np.uint64(1)).astype(np.int64)
    out = (-JB * dZ - hz * wz) * fetch(r.astype(np.int64))
    for m in st:
        out = out - JA * fetch((r ^ np.uint64(int(m))).astype(np.int64))
    for l in range(n):
        out = out - hx * fetch((r ^ np.uint64(1 << l)).astype(np.int64))
    return out


def spectrum(Lx, Ly, c):
    """All eigenvalues by dense diagonalisation (small lattices only)."""
    H = hamiltonian(Lx, Ly, c).toarray()
    return np.linalg.eigvalsh(H)


def ground(Lx, Ly, c, k=1):
    """Lowest k eigenvalues: dense for n <= 12, Lanczos above."""
    n = 2 * Lx * Ly
    if n <= 12:
        return np.sort(spectrum(Lx, Ly, c))[:k]
    H = hamiltonian(Lx, Ly, c)
    vals = spla.eigsh(H, k=k, which="SA", tol=1e-12, return_eigenvectors=False)
    return np.sort(vals)


def ground_state(Lx, Ly, c):
    """(E0, unit ground-state vector) by scipy's Lanczos (eigsh), for a
    non-degenerate ground state; the vector's global phase is arbitrary."""
    H = hamiltonian(Lx, Ly, c)
    vals, vecs = spla.eigsh(H, k=1, which="SA", tol=1e-13)
    v = vecs[:, 0].astype(np.complex128)
    return float(vals[0]), v / np.linalg.norm(v)


def exact_stepwise(Lx, Ly, psi0, c0, c1, M, dt, sampling=0):
    """prod_k expm(-i dt H(c(s_k))) psi0: the evolution the Trotter steps
    approximate, with the same per-step parameter values s_k (dense expm,
    small lattices only)."""
    parts = hamiltonian_parts(Lx, Ly)
    dense = {k: v.toarray() for k, v in parts.items()}
    c0 = np.asarray(c0, float)
    c1 = np.asarray(c1, float)
    psi = np.array(psi0, np.complex128)
    for k in range(M):
        s = (k + 1) / M if sampling else (k + 0.5) / M
        c = (1 - s) * c0 + s * c1
        H = -c[0] * dense["A"] - c[1] * dense["B"] - c[2] * dense["X"] - c[3] * dense["Z"]
        psi = sla.expm(-1j * dt * H) @ psi
    return psi


def exact_stepwise_sparse(Lx, Ly, psi0, c0, c1, M, dt, sampling=0, sZ=None, sX=None):
    """The same product of exact exponentials as exact_stepwise, applied with
    scipy's expm_multiply to the sparse H (reaches 3x3).  sZ / sX (optional
    arrays of M values) replace s_k for the plaquette/z-field and the
    star/x-field couplings of step k."""
    P = hamiltonian_parts(Lx, Ly)
    c0 = np.asarray(c0, float)
    c1 = np.asarray(c1, float)
    psi = np.array(psi0, np.complex128)
    for k in range(M):
        s = (k + 1) / M if sampling else (k + 0.5) / M
        sz = s if sZ is None else sZ[k]
        sx = s if sX is None else sX[k]
        cz = (1 - sz) * c0 + sz * c1
        cx = (1 - sx) * c0 + sx * c1
        H = (-cx[0] * P["A"] - cz[1] * P["B"] - cx[2] * P["X"] - cz[3] * P["Z"]).tocsr()
        psi = spla.expm_multiply(-1j * dt * H, psi)
    return psi


def grouped_step_dense(Lx, Ly, cx, cz, dt, order=0):
    """The Trotter step as a product of three matrix exponentials (dense):
    exp(-i HX dt/2) exp(-i HZ dt) exp(-i HX dt/2) with HX the star and x-field
    terms and HZ the plaquette and z-field terms (order 0), or the same with
    the roles of HX and HZ exchanged (order 1)."""
    parts = {k: v.toarray() for k, v in hamiltonian_parts(Lx, Ly).items()}
    HX = -cx[0] * parts["A"] - cx[2] * parts["X"]
    HZ = -cz[1] * parts["B"] - cz[3] * parts["Z"]
    if order == 0:
        h = sla.expm(-0.5j * dt * HX)
        return h @ sla.expm(-1j * dt * HZ) @ h
    h = sla.expm(-0.5j * dt * HZ)
    return h @ sla.expm(-1j * dt * HX) @ h
