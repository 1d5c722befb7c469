"""Pins of the oracle's exponential modal filter (Sect. 5.4, eq.
exponential_filter): each Legendre mode of an element's deviation from the
background is scaled by sigma(n) = exp(-alpha ((n - Nc)/(N - Nc))^s) per
direction (the modes evaluated here with numpy's Legendre series, not the
oracle's), the background and the unmasked variables are untouched, and the
element integrals (mass) do not change."""
import numpy as np
import pytest
from numpy.polynomial import legendre as L

from paper_2110_00853_amd import workloads as W

GRID = {"N": 4, "ne": [2, 2, 2], "lo": [0.0, 0.0, 0.0], "hi": [400.0, 300.0, 500.0], "periodic": [1, 1, 0]}
Q = 5


def _mode_field(a, b, c):
    """P_a(xi) P_b(eta) P_c(zeta) on every element's nodes (node i + 5 j + 25 k)."""
    xi = W.gll_points(4)
    Pa = L.legval(xi, np.eye(Q)[a])
    Pb = L.legval(xi, np.eye(Q)[b])
    Pc = L.legval(xi, np.eye(Q)[c])
    loc = (Pc[:, None, None] * Pb[None, :, None] * Pa[None, None, :]).reshape(-1)
    return np.tile(loc, int(np.prod(GRID["ne"])))


def _sigma(n, order, alpha, Nc=0, N=4):
    return 1.0 if n <= Nc else np.exp(-alpha * ((n - Nc) / (N - Nc)) ** order)


@pytest.fixture
def model(oracle_lib):
    c = {"grid": GRID, "model": {"nvar": 5, "closure": "const", "nu": 75.0, "g": 9.81}, "ic": {"kind": "bubble"}}
    Y, Yref, _ = W.perturbed_state(c, seed=2)
    return oracle_lib.Model(oracle_lib.Grid(GRID), c["model"], Yref), Y, Yref


@pytest.mark.parametrize("order,alpha,Nc", [(64, 36.0, 0), (8, 36.0, 0), (4, 10.0, 1), (2, 5.0, 2)])
def test_modes_are_scaled_by_sigma(model, order, alpha, Nc):
    M, _, Yref = model
    for (a, b, c) in [(0, 0, 0), (4, 0, 0), (0, 3, 0), (0, 0, 2), (1, 4, 3), (4, 4, 4), (2, 1, 0)]:
        f = _mode_field(a, b, c)
        Y = Yref.copy()
        Y[1] += 0.7 * f
        Y[4] += 50.0 * f
        out = M.exp_filter(Y, mask=0b10010, order=order, alpha=alpha, Nc=Nc)
        s = _sigma(a, order, alpha, Nc) * _sigma(b, order, alpha, Nc) * _sigma(c, order, alpha, Nc)
        assert np.allclose(out[1], Yref[1] + 0.7 * s * f, rtol=0, atol=1e-13)
        assert np.allclose(out[4], Yref[4] + 50.0 * s * f, rtol=1e-15, atol=2e-9)


def test_paper_filter_removes_the_top_mode(model):
    """s = 64, alpha = 36: mode 4 scaled by exp(-36) ~ 2e-16, modes up to 2
    kept to within 1e-30, mode 3 by exp(-36 (3/4)^64) ~ 1 - 4e-7."""
    assert _sigma(4, 64, 36.0) == pytest.approx(np.exp(-36.0), rel=1e-15)
    assert 1.0 - _sigma(3, 64, 36.0) == pytest.approx(36.0 * 0.75 ** 64, rel=1e-6)
    M, _, Yref = model
    Y = Yref.copy()
    Y[2] += _mode_field(4, 0, 0) + _mode_field(0, 2, 0)
    out = M.exp_filter(Y, mask=0b00100)
    assert np.allclose(out[2], _mode_field(0, 2, 0), atol=1e-14)


def test_background_unmasked_variables_and_mass_are_kept(model, oracle_lib):
    M, Y, Yref = model
    assert np.array_equal(M.exp_filter(Yref, mask=0b11111), Yref)
    out = M.exp_filter(Y, mask=0b10001, order=4, alpha=20.0)
    assert np.array_equal(out[1:4], Y[1:4])
    assert np.abs(out[0] - Y[0]).max() > 1e-6  # it did act
    wJ = oracle_lib.Grid(GRID).wJ()
    ne = int(np.prod(GRID["ne"]))
    for v in (0, 4):
        before = (wJ * Y[v]).reshape(ne, -1).sum(1)
        after = (wJ * out[v]).reshape(ne, -1).sum(1)
        assert np.abs(after - before).max() <= 1e-14 * np.abs(before).max()
