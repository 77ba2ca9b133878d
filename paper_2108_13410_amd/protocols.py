"""The paper's parameter paths (inputs only: vertices and step counts).

Couplings are (JA, JB, hx, hz) with the paper's star and plaquette coupling
1/2 (Sec. II, Eq. (effi)), hx = g and hz = lambda.  Steps follow the paper's
protocol (Sec. VI): dg = 1e-5 per Trotter step of dt = 0.02 along every leg
(a leg that changes g or lambda by d takes d / dg steps), parameter values
taken at the end of each step.

  topo_paths(p)       Fig. topo: psi_1 along the g axis to P(p, 0), then the
                      straight blue line to P'(0, p); and psi_1' along the
                      lambda axis to P'(0, p), then the blue line back to P.
  red_path(p, r)      Figs. sec_order, dos_sec: psi_1 to P(p, 0), up to
                      R(p, r), then along lambda = r to R'(0, r).
  dual_path(q)        Fig. dual_evo: psi_1' along the lambda axis to (0, q),
                      across to (q, q), then down the dual line to O.
  refined_red_path    the red path with n times finer steps (Sec. VI,
                      Table contrast_tab), and refinement_metrics for the
                      table's delta_n and alpha_n.
"""
from __future__ import annotations

import numpy as np

J = 0.5
DG = 1e-5
DT = 0.02


def pt(g, lam):
    return (J, J, float(g), float(lam))


def _steps(verts):
    out = []
    for a, b in zip(verts[:-1], verts[1:]):
        d = max(abs(b[2] - a[2]), abs(b[3] - a[3]))
        out.append(int(round(d / DG)))
    return out


def path(points):
    verts = [pt(*q) for q in points]
    return verts, _steps(verts)


def topo_paths(p):
    return {"E": ("psi1", *path([(0, 0), (p, 0), (0, p)])),
            "E'": ("psi1p", *path([(0, 0), (0, p), (p, 0)]))}


def red_path(p, r):
    return ("psi1", *path([(0, 0), (p, 0), (p, r), (0, r)]))


def dual_path(q=0.5):
    return ("psi1p", *path([(0, 0), (0, q), (q, q), (0, 0)]))


def refined_red_path(p, r, n):
    """The red path with the step refinement of Sec. VI: dg = 1e-4 / n and
    dt = 0.2 / n per step on every leg (n = 10 is the protocol above).
    Returns (init, vertices, steps, dt)."""
    dg = 1e-4 / n
    verts = [pt(0, 0), pt(p, 0), pt(p, r), pt(0, r)]
    steps = []
    for a, b in zip(verts[:-1], verts[1:]):
        d = max(abs(b[2] - a[2]), abs(b[3] - a[3]))
        steps.append(int(round(d / dg)))
    return "psi1", verts, steps, 0.2 / n


def refinement_metrics(E_ref, E_n):
    """Table contrast_tab: delta_n = sum over the grid of |E_n0(g) - E_n(g)|
    (1-norm), alpha_n = its maximum."""
    d = np.abs(np.asarray(E_ref, float) - np.asarray(E_n, float))
    return float(d.sum()), float(d.max())


def second_derivative(x, E, w=10):
    """d2E/dx2 at interior samples from least-squares quadratics over 2w+1
    neighbouring samples (x uniform).  Returns (x_mid, d2)."""
    x = np.asarray(x, float)
    E = np.asarray(E, float)
    xs = np.arange(-w, w + 1) * (x[1] - x[0])
    V = np.vander(xs, 3)                      # columns x^2, x, 1
    coef = np.linalg.pinv(V)[0]               # weights giving the x^2 coefficient
    d2 = 2.0 * np.convolve(E, coef[::-1], mode="valid")
    return x[w:len(x) - w], d2


def extremum_in(x, d2, lo, hi, kind="min"):
    """Abscissa of the smallest (largest) d2 value with lo < x < hi."""
    sel = (x > lo) & (x < hi)
    i = np.argmin(d2[sel]) if kind == "min" else np.argmax(d2[sel])
    return float(x[sel][i]), float(d2[sel][i])
