"""Trotter error bound of the Appendix (test utility, not a kernel).

TEST INFRASTRUCTURE ONLY.  Takes the Appendix's steps in order: the norm
estimates of Eq. (EachTerm), (cmt12), (cmt13) for the 3x3 lattice, the
second-order commutator bound of Eq. (T2S3) with W1 and W2 of Eqs. (W1), (W2),
summed over the N steps of the ramp g = n*dg, n = 1..N at fixed lambda = r
(Eq. (target)).  ``closed_form`` is the paper's final expression after the
sums of Eq. (g^1).

Pinned by the epsilon column of Table contrast_tab.
"""
from __future__ import annotations


def norms(g, lam):
    """Norm estimates of Eqs. (EachTerm), (cmt12), (cmt13) on the 3x3 torus."""
    return {
        "H1": 18 * g, "H2": 9.0, "H3": 18 * lam,
        "12": 18 * g, "23": 18 * lam, "13": 36 * g * lam,
    }


def per_step(g, lam, dt):
    """(dt^3/6) W1 + (dt^3/12) W2 for one step at parameters (g, lam)."""
    a = norms(g, lam)
    W1 = a["H2"] * (a["12"] + a["13"]) + a["H3"] * (a["12"] + a["13"] + a["23"])
    W2 = a["H1"] * (a["12"] + a["13"]) + a["H2"] * a["23"]
    return dt ** 3 / 6 * W1 + dt ** 3 / 12 * W2


def summed(p, r, dg, dt):
    """Eq. (target): sum of the per-step bound over g = n dg, n = 1..N, N = p/dg."""
    import numpy as np
    N = int(round(p / dg))
    g = np.arange(1, N + 1, dtype=np.float64) * dg
    return float(np.sum(per_step(g, r, dt)))


def closed_form(p, r, dg, dt):
    """Final expression of the Appendix / Sec. VI with N = p/dg."""
    N = p / dg
    return dt ** 3 * N * (13.5 * p + 54 * p * r * r + 54 * p * r + 54 * r * r
                          + 9 * p * p + 18 * p * p * r + 13.5 * r)
