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


def test_heldout_box_interior_reproduces_full_grid_inputs(oracle_lib, tmp_path):
    """Closure inputs and targets recomputed on a stored box's interior
    elements equal those of the whole coarse grid at the same nodes (BR1
    gradients reach face neighbours only), up to the box's float32 storage."""
    import sys
    import os

    sys.path.insert(0, os.path.dirname(__file__))
    from test_learned_gain import box_samples

    cf = W.case("bubble_32", ne=(16, 16, 16))
    cc = W.case("bubble_32", ne=(8, 8, 8))
    Yf, _, _ = W.perturbed_state(cf, seed=31, amp_u=4.0, amp_T=1.0)
    zf = W.node_coords(cf["grid"])[2]
    snap = Lp.filtered(Yf, zf, cf["grid"]["ne"])
    Yc = snap[0]
    Gd = oracle_lib.Grid(cc["grid"])
    grad, _ = oracle_lib.Model(Gd, dict(cc["model"], closure="smag")).gradients(Yc)
    gu, gth = grad[:3], grad[-1]
    h = 6400.0 / 8
    Delta = float(np.cbrt((h / 4) ** 3))
    tau, q = Lp.sgs_fluxes(*snap)
    T_full, mask = Lp.targets_from_fluxes(Yc[0], tau, q, gu, gth, Delta)
    assert mask.sum() > 1000
    box = Lp.heldout_box(snap, mask, cc["grid"])
    path = str(tmp_path / "box.npz")
    np.savez(path, Delta=np.float64(Delta), **{"box_%s" % k: v for k, v in box.items()})
    X, T, _ = box_samples(np.load(path), cc["model"]["Cs"], cc["model"]["Prt"])
    # the same nodes on the full grid
    st = box["start"]
    ez, ey, ex = np.meshgrid(*[np.arange(st[d] + 1, st[d] + 5) for d in (2, 1, 0)], indexing="ij")
    nodes = ((((ez * 8 + ey) * 8 + ex).ravel())[:, None] * 125 + np.arange(125)[None]).ravel()
    m = mask[nodes]
    assert np.allclose(T, T_full[nodes][m], rtol=0, atol=2e-3 * np.abs(T_full[nodes][m]).max())
    gu_full = gu[:, :, nodes][:, :, m].reshape(9, -1).T
    assert np.allclose(X[:, :9], gu_full, rtol=0, atol=1e-5 * np.abs(gu_full).max())
