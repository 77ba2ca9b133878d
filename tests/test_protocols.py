"""Host-side helpers of the paper's protocols (paper_2108_13410_amd/protocols.py):
path construction and the post-processing of traces (CPU only)."""
import numpy as np

from paper_2108_13410_amd import protocols as pr


def test_paths_follow_the_protocol_step():
    """Sec. VI: dg = 1e-5 per step, so a leg changing g or lambda by d has
    d / dg steps; the refined path divides dg and dt by n / 10."""
    _, verts, steps = pr.red_path(0.5, 0.05)
    assert steps == [50000, 5000, 50000] and verts[0] == (0.5, 0.5, 0.0, 0.0)
    _, verts, steps, dt = pr.refined_red_path(0.5, 0.05, 200)
    assert steps == [1000000, 100000, 1000000] and abs(dt - 1e-3) < 1e-18
    _, _, steps = pr.dual_path(0.5)
    assert steps == [50000, 50000, 50000]


def test_second_derivative_exact_on_quadratics():
    x = np.linspace(0, 1, 201)
    E = 3.0 * x ** 2 - 2.0 * x + 1.0
    xm, d2 = pr.second_derivative(x, E, 10)
    assert len(xm) == len(x) - 20 and np.allclose(d2, 6.0, atol=1e-8)
    g, v = pr.extremum_in(xm, -((xm - 0.3) ** 2), 0.1, 0.9, "max")
    assert abs(g - 0.3) < 1e-12


def test_refinement_metrics():
    d, a = pr.refinement_metrics([1.0, 2.0, 3.0], [1.0, 2.5, 2.0])
    assert d == 1.5 and a == 1.0


def test_dos_maxima():
    """Ztilde = 2w - n of local maxima of at least 1 % of the top bin; the
    interior variant ignores the ends of the occupied range."""
    n = 6
    d = np.array([0.3, 0.1, 0.2, 0.35, 0.05, 0.001, 0.002])
    assert pr.dos_maxima(d, n) == [-6, 0]             # w = 0 and w = 3; the tail bump at w = 6 is below 1 %
    assert pr.dos_maxima(d, n, interior=True) == [0]
    assert pr.dos_maxima(np.array([0, 0, 0.5, 0.2, 0.4, 0, 0]), n) == [-2, 2]
