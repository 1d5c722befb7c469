"""Pins of the oracle's GLL nodes, weights and differentiation matrix
(Sect. 3.1: tensor-product Lagrange basis on Legendre-Gauss-Lobatto points,
derivatives through the 1-D matrix along each reference direction)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_n4_closed_form(oracle_lib):
    ref = np.loadtxt(os.path.join(GOLDEN, "gll_n4.txt"))
    xi, w, _ = oracle_lib.gll(4)
    # within one unit in the last place of the closed forms
    assert np.allclose(xi, ref[:, 0], rtol=0, atol=2.3e-16)
    assert np.allclose(w, ref[:, 1], rtol=0, atol=2.3e-16)
    assert xi[3] == pytest.approx(np.sqrt(3.0 / 7.0), abs=2.3e-16)
    assert xi[2] == 0.0 and xi[0] == -1.0 and xi[4] == 1.0


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8])
def test_quadrature_exact_to_degree_2N_minus_1(oracle_lib, N):
    xi, w, _ = oracle_lib.gll(N)
    for p in range(2 * N):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert np.dot(w, xi ** p) == pytest.approx(exact, abs=1e-14)
    # degree 2N is not integrated exactly by an (N+1)-point Lobatto rule
    assert abs(np.dot(w, xi ** (2 * N)) - 2.0 / (2 * N + 1)) > 1e-6


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 8])
def test_D_exact_for_polynomials_up_to_N(oracle_lib, N):
    xi, _, D = oracle_lib.gll(N)
    for p in range(N + 1):
        d = D @ xi ** p
        exact = p * xi ** (p - 1) if p > 0 else np.zeros_like(xi)
        assert np.max(np.abs(d - exact)) < 4e-14 * max(1, N * N)
    # one degree higher cannot be represented
    d = D @ xi ** (N + 1)
    assert np.max(np.abs(d - (N + 1) * xi ** N)) > 1e-3


@pytest.mark.parametrize("N", [2, 4, 7])
def test_D_matches_library_lagrange_derivative(oracle_lib, N):
    """D_ij = l_j'(x_i), with l_j fitted through the nodes by numpy."""
    xi, _, D = oracle_lib.gll(N)
    from numpy.polynomial import Polynomial

    for j in range(N + 1):
        e = np.zeros(N + 1)
        e[j] = 1.0
        lj = Polynomial.fit(xi, e, N, domain=[-1, 1], window=[-1, 1])
        assert np.allclose(D[:, j], lj.deriv()(xi), atol=1e-11)


@pytest.mark.parametrize("N", [1, 3, 4, 6])
def test_D_annihilates_constants_and_sbp(oracle_lib, N):
    """Row sums vanish (diagonal = minus off-diagonal sum) and the GLL
    summation-by-parts identity W D + D^T W = diag(-1, 0, ..., 0, 1) holds,
    which makes the weak and strong DG forms coincide."""
    xi, w, D = oracle_lib.gll(N)
    assert np.max(np.abs(D.sum(axis=1))) < 1e-14 * (N + 1) ** 2
    W = np.diag(w)
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1.0, 1.0
    assert np.max(np.abs(W @ D + D.T @ W - B)) < 5e-15 * (N + 1) ** 2
