"""Pins of the LSRK54 integrator (Sect. 3.2: Carpenter & Kennedy low-storage
explicit Runge-Kutta family; five stages, fourth order, 2N storage)."""
from fractions import Fraction

import numpy as np
import pytest

from paper_2110_00853_amd import workloads as W


def butcher(A, B):
    """Butcher tableau of the 2N-storage scheme dQ = A_s dQ + k_s,
    Y += B_s dQ, k_s = dt F(Y after stage s-1)."""
    s = len(A)
    q = np.zeros(s)
    y = np.zeros(s)
    a = np.zeros((s, s))
    for i in range(s):
        a[i] = y
        q = A[i] * q
        q[i] += 1.0
        y = y + B[i] * q
    return a, y


def test_order_conditions(oracle_lib):
    A, B, Cc = oracle_lib.lsrk54_coeffs()
    a, b = butcher(A, B)
    c = a.sum(axis=1)
    assert np.allclose(c, Cc, atol=1e-15)
    cond = [
        (b.sum(), 1.0), (b @ c, 1 / 2), (b @ c ** 2, 1 / 3), (b @ a @ c, 1 / 6),
        (b @ c ** 3, 1 / 4), (b @ (c * (a @ c)), 1 / 8), (b @ a @ c ** 2, 1 / 12), (b @ a @ a @ c, 1 / 24),
    ]
    for val, exact in cond:
        assert val == pytest.approx(exact, abs=1e-15)
    # stability polynomial 1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/200
    assert b @ a @ a @ a @ c == pytest.approx(1 / 200, abs=1e-15)


def test_coefficients_are_the_published_rationals(oracle_lib):
    A, B, Cc = oracle_lib.lsrk54_coeffs()
    assert A[0] == 0.0 and Cc[0] == 0.0
    assert B[0] == float(Fraction(1432997174477, 9575080441755))
    assert Cc[1] == B[0]


def test_empirical_temporal_order(oracle_lib):
    """Advance a smooth state over a fixed interval with dt, dt/2, dt/4 and a
    fine reference: the error falls at fourth order."""
    g = {"N": 4, "ne": [2, 2, 1], "lo": [0.0, 0.0, 0.0], "hi": [4000.0, 4000.0, 2000.0], "periodic": [1, 1, 1]}
    G = oracle_lib.Grid(g)
    Y0, _ = W.isentropic_vortex(g, 0.0, center=(2000.0, 2000.0), L=600.0)
    M = oracle_lib.Model(G, {"nvar": 5, "closure": "none", "g": 0.0})
    T = 6.0
    ref, _ = M.steps(Y0, T / 768, 768)
    errs = []
    for n in (24, 48, 96):
        Y, _ = M.steps(Y0, T / n, n)
        errs.append(np.abs(Y[1] - ref[1]).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 3.8), (errs, orders)
