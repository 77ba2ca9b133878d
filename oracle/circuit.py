"""The paper's circuits gate by gate, with the ancilla, in NumPy (FP64).

TEST INFRASTRUCTURE ONLY.  Written from Sec. III (the Trotter step: Eq.
(gate1) for the fields, the ancilla gadgets U_1 R_z U_1^dagger for a
plaquette and U_2^dagger R_z U_2 for a star) and from Eqs. (ini1), (ini2)
(state preparation with a projected ancilla), in the oracle's own link
numbering (the paper's), with the ancilla as qubit n.

A gate is a tuple (name, qubits, angle): ("H", (q,)), ("RX", (q,), theta),
("RZ", (q,), theta), ("CNOT", (control, target)), ("P0", (q,)) for the
projection on |0>, ("NORM", ()) for renormalisation.  R_a(theta) =
exp(-i theta sigma^a / 2), time order = list order.

Pinned by tests/test_oracle.py: one circuit step from any link state with
the ancilla in |0> equals the oracle's algebraic Trotter step and returns the
ancilla to |0>; the preparation circuits give psi_1 and psi_1'; each gate
and the ancilla gadget agree with scipy's expm; the gate count follows from
the circuit's structure.
"""
from __future__ import annotations

import numpy as np

from . import masks

_H = np.array([[1, 1], [1, -1]], complex) / np.sqrt(2)


def _rx(theta):
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]])


def _rz(theta):
    return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)])


def _links(mask):
    m = int(mask)
    return [l for l in range(64) if m >> l & 1]


def _gadget(anc, links, theta):
    """Parity of the links onto the ancilla, R_z(theta) there, parity back:
    on links with the ancilla in |0> this is exp(-i theta/2 Z_links)."""
    g = [("CNOT", (l, anc)) for l in links]
    return g + [("RZ", (anc,), theta)] + [("CNOT", (l, anc)) for l in links]


def _stabilizer_half(Lx, Ly, cx, cz, dt):
    st, pl = masks(Lx, Ly)
    anc = 2 * Lx * Ly
    g = []
    # exp(i JB B_p dt/2) = U_1 R_z(-JB dt)_a U_1^dagger for each plaquette
    for p in pl:
        g += _gadget(anc, _links(p), -cz[1] * dt)
    # exp(i JA A_v dt/2) = U_2^dagger R_z(-JA dt) U_2, U_2 = CNOTs after Hadamards
    for v in st:
        ls = _links(v)
        g += [("H", (l,)) for l in ls] + _gadget(anc, ls, -cx[0] * dt) + [("H", (l,)) for l in ls]
    return g


def step_gates(Lx, Ly, cx, cz, dt, order=0):
    """Gates of one Trotter step of Sec. III in time order (first acts first)."""
    n = 2 * Lx * Ly
    half = _stabilizer_half(Lx, Ly, cx, cz, dt)
    if order == 0:
        # exp(-iH_1 dt/2): R_x(-hx dt); exp(-iH_3 dt): R_z(-2 hz dt)   (Eq. (gate1))
        xh = [("RX", (l,), -cx[2] * dt) for l in range(n)]
        zf = [("RZ", (l,), -2 * cz[3] * dt) for l in range(n)]
        return xh + half + zf + half + xh
    zh = [("RZ", (l,), -cz[3] * dt) for l in range(n)]
    xf = [("RX", (l,), -2 * cx[2] * dt) for l in range(n)]
    return zh + half + xf + half + zh


def prep_gates(Lx, Ly, which="psi1"):
    """Eq. (ini1) (which = "psi1") or Eq. (ini2) ("psi1p") from |0...0>."""
    st, pl = masks(Lx, Ly)
    n = 2 * Lx * Ly
    anc = n
    g = []
    if which == "psi1":
        g += [("H", (l,)) for l in range(n)]
        for p in pl:
            ls = _links(p)
            g += [("CNOT", (l, anc)) for l in ls] + [("P0", (anc,))] + [("CNOT", (l, anc)) for l in ls]
    else:
        for v in st:
            ls = _links(v)
            g += [("H", (l,)) for l in ls] + [("CNOT", (l, anc)) for l in ls] + [("P0", (anc,))]
            g += [("CNOT", (l, anc)) for l in ls] + [("H", (l,)) for l in ls]
    return g + [("NORM", ())]


def _one_qubit(psi, q, M):
    nq = int(np.log2(psi.size))
    v = psi.reshape(1 << (nq - q - 1), 2, 1 << q)
    return np.einsum("ij,ajb->aib", M, v).reshape(-1)


def apply(psi, gates):
    """Apply gates to psi (n + 1 qubits, bit q of the index = qubit q); returns
    the new state."""
    psi = np.array(psi, np.complex128)
    idx = np.arange(psi.size, dtype=np.int64)
    for gate in gates:
        name, qs = gate[0], gate[1]
        if name == "H":
            psi = _one_qubit(psi, qs[0], _H)
        elif name == "RX":
            psi = _one_qubit(psi, qs[0], _rx(gate[2]))
        elif name == "RZ":
            psi = _one_qubit(psi, qs[0], _rz(gate[2]))
        elif name == "CNOT":
            c, t = qs
            i = idx[((idx >> c) & 1 == 1) & ((idx >> t) & 1 == 0)]
            j = i | (1 << t)
            psi[i], psi[j] = psi[j].copy(), psi[i].copy()
        elif name == "P0":
            psi[(idx >> qs[0]) & 1 == 1] = 0
        elif name == "NORM":
            nrm = np.linalg.norm(psi)
            if nrm > 0:
                psi = psi / nrm
        else:
            raise ValueError(name)
    return psi


def with_ancilla(psi_links):
    """Links state (n qubits) with the ancilla (qubit n) in |0>."""
    out = np.zeros(2 * psi_links.size, np.complex128)
    out[: psi_links.size] = psi_links
    return out


def evolve(Lx, Ly, psi, c0, c1, M, dt, sampling=0, order=0):
    """The ramp of Sec. III at gate level (n + 1 qubits), per-step couplings
    c(s_k) with s_k = (k + 1/2)/M (sampling 0) or (k + 1)/M (sampling 1)."""
    c0 = np.asarray(c0, float)
    c1 = np.asarray(c1, float)
    for k in range(M):
        s = (k + 1) / M if sampling else (k + 0.5) / M
        c = (1 - s) * c0 + s * c1
        psi = apply(psi, step_gates(Lx, Ly, c, c, dt, order))
    return psi
