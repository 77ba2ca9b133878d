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
  dos_study           the Ztilde distributions of Figs. dos_sec and
                      dos_dual, and dos_maxima to count their maxima.
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


def dos_maxima(dos, n, interior=False, rel=0.01):
    """Ztilde = 2w - n of the local maxima of a weight distribution dos[w]
    (w = 0..n) over the weights it occupies, counting only peaks of at least
    rel times the largest entry; interior=True leaves out the two end points
    of the occupied range."""
    d = [float(x) for x in dos[: n + 1]]
    top = max(d)
    occ = [w for w in range(n + 1) if d[w] > 1e-12]
    out = []
    for i, w in enumerate(occ):
        left = d[occ[i - 1]] if i > 0 else -1.0
        right = d[occ[i + 1]] if i + 1 < len(occ) else -1.0
        if d[w] > left and d[w] > right and d[w] >= rel * top:
            if interior and (i == 0 or i == len(occ) - 1):
                continue
            out.append(2 * w - n)
    return out


def dos_study(z2h, plan, rs=None, dual_q=0.7, dual_g=(0.65, 0.30), every=1000):
    """Figs. dos_sec and dos_dual (Sec. V) on the plan's lattice: red paths
    P(0.5, 0) -> R(0.5, r) -> R'(0, r) for each r, run together and read at
    g = 0.19 on the last leg; the dual line (0, 0) -> (0, q) -> (q, q) -> O
    read at the g values given.  Returns ({r: dos}, {g: dos}), dos[w] = weight
    of Hamming weight w (Ztilde = 2w - n)."""
    n = plan.n
    rs = rs or [round(0.01 * k, 2) for k in range(1, 20)]
    paths = []
    for r in rs:
        _, verts, steps = red_path(0.5, r)
        paths.append(z2h.make_path(verts, steps, DT, sampling=1, every=every))
    _, tr = z2h.z2h_paths_evolve(plan, paths)
    tr = tr.cpu().numpy()
    per = int(round(0.01 / DG)) // every if every else 0   # samples per 0.01 in g
    last = steps[-1] // every                              # samples on the last leg (g from 0.5 to 0)
    k = int(round((0.5 - 0.19) / 0.01)) * per - 1
    red = {r: tr[-last + k, j, 22:23 + n] for j, r in enumerate(rs)}
    _, dverts, dsteps = dual_path(dual_q)
    _, dtr = z2h.z2h_paths_evolve(plan, [z2h.make_path(dverts, dsteps, DT, sampling=1, every=every)],
                                  inits=[z2h.Z2H_INIT_PSI1P])
    dtr = dtr.cpu().numpy()
    dlast = dsteps[-1] // every
    dual = {g: dtr[-dlast + int(round((dual_q - g) / 0.01)) * per - 1, 0, 22:23 + n] for g in dual_g}
    return red, dual


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
