"""CPU checks of the learned-closure data pipeline: the 2x coarse-graining
is the exact L2 projection of the fine element polynomials (reproduces
parent-degree polynomials, preserves integrals), and fields without
sub-filter content produce no SGS stress."""
import numpy as np
import pytest

from paper_2110_00853_amd import learned as Lp
from paper_2110_00853_amd import workloads as W


def test_projection_reproduces_parent_polynomials():
    P = Lp.projection_matrix()
    xi = W.gll_points(4)
    xl, xr = (xi - 1) / 2, (xi + 1) / 2
    for p in range(5):
        f = np.concatenate([xl ** p, xr ** p])
        assert np.allclose(P @ f, xi ** p, atol=1e-13)


def test_projection_preserves_integral():
    P = Lp.projection_matrix()
    xi = W.gll_points(4)
    xg, wg = np.polynomial.legendre.leggauss(8)
    rng = np.random.default_rng(0)
    f = rng.normal(size=10)
    Lint = Lp._lagrange(xi, xg)
    child = 0.5 * (wg @ Lint @ f[:5] + wg @ Lint @ f[5:])       # each child is half the parent
    parent = wg @ Lint @ (P @ f)
    assert parent == pytest.approx(child, rel=1e-13)


def test_coarse_grain_3d_exact_for_low_degree_fields():
    g = {"N": 4, "ne": [4, 2, 6], "lo": [0.0, 0.0, 0.0], "hi": [400.0, 200.0, 600.0], "periodic": [1, 1, 0]}
    gc = dict(g, ne=[2, 1, 3])
    xf = W.node_coords(g)
    xc = W.node_coords(gc)
    # degree <= 4 per coarse element in each direction (here a global polynomial)
    fun = lambda x: 1.0 + 0.01 * x[0] - 2e-5 * x[1] * x[2] + 1e-9 * x[0] ** 2 * x[2] ** 2
    assert np.allclose(Lp.coarse_grain(fun(xf), g["ne"]), fun(xc), rtol=1e-12)


def test_no_sgs_stress_without_subfilter_content():
    """Constant density and linear velocity: products are quadratic, so the
    filtered product equals the product of filtered fields and tau = 0."""
    g = {"N": 4, "ne": [2, 2, 2], "lo": [0.0, 0.0, 0.0], "hi": [400.0, 400.0, 400.0], "periodic": [1, 1, 0]}
    x = W.node_coords(g)
    n = x.shape[1]
    u = np.stack([0.01 * x[2], 0.02 * x[0] - 1.0, 0.005 * x[1]])
    T = np.full(n, 290.0)
    Y = W.state_from_primitives(np.full(n, 1.1 * 287.0 * 290.0), T, u[0], u[1], u[2], np.zeros(n), g=0.0)
    Yc, ruu, rth, rthu = Lp.filtered(Y, np.zeros(n), g["ne"], g=0.0)
    m = Yc[1:4]
    for q, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        assert np.allclose(ruu[q] - m[a] * m[b] / Yc[0], 0.0, atol=1e-10 * np.abs(ruu[q]).max())
