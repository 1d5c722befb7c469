"""Pins of the oracle's Vreman eddy viscosity (Sect. 4.2, eq. vreman-sgs):
closed forms for pure shear, solid-body rotation and isotropic dilatation,
the second principal invariant of beta computed another way, invariance
under rotations of the axes for an isotropic mixing length, and the
Richardson stability factor."""
import numpy as np
import pytest

CS = 0.18


def test_pure_shear_has_no_eddy_viscosity(oracle_lib):
    # a single velocity-gradient entry: beta has rank one, B_beta = 0
    for (i, j) in [(0, 2), (1, 0), (2, 1)]:
        gu = np.zeros((3, 3))
        gu[i, j] = 0.37
        assert oracle_lib.vreman(gu, 0.0, CS, [50.0, 60.0, 40.0]) == 0.0


def test_solid_rotation_closed_form(oracle_lib):
    w = 0.8
    gu = np.array([[0.0, -w, 0.0], [w, 0.0, 0.0], [0.0, 0.0, 0.0]])
    d = [50.0, 30.0, 70.0]
    # beta = diag(d2^2 w^2, d1^2 w^2, 0), B = d1^2 d2^2 w^4, u_ij u_ij = 2 w^2
    expect = 2.5 * CS ** 2 * d[0] * d[1] * w / np.sqrt(2.0)
    assert oracle_lib.vreman(gu, 0.0, CS, d) == pytest.approx(expect, rel=1e-14)


def test_isotropic_dilatation_closed_form(oracle_lib):
    a = 0.05
    d = np.array([50.0, 30.0, 70.0])
    d2 = d * d
    expect = 2.5 * CS ** 2 * a * np.sqrt((d2[0] * d2[1] + d2[0] * d2[2] + d2[1] * d2[2]) / 3.0)
    assert oracle_lib.vreman(a * np.eye(3), 0.0, CS, d) == pytest.approx(expect, rel=1e-14)


def test_second_invariant_of_beta_another_way(oracle_lib):
    rng = np.random.default_rng(4)
    for _ in range(50):
        gu = rng.normal(size=(3, 3)) * 0.1
        d = rng.uniform(20.0, 80.0, 3)
        beta = (gu * d[None, :] ** 2) @ gu.T          # sum_m d_m^2 u_i,m u_j,m
        B = 0.5 * (np.trace(beta) ** 2 - np.trace(beta @ beta))
        expect = 2.5 * CS ** 2 * np.sqrt(max(B, 0.0) / np.sum(gu * gu))
        assert oracle_lib.vreman(gu, 0.0, CS, d) == pytest.approx(expect, rel=1e-12)


def test_rotation_invariance_for_isotropic_mixing_length(oracle_lib):
    rng = np.random.default_rng(5)
    for _ in range(20):
        gu = rng.normal(size=(3, 3)) * 0.1
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        a = oracle_lib.vreman(gu, 0.0, CS, [40.0] * 3)
        b = oracle_lib.vreman(q @ gu @ q.T, 0.0, CS, [40.0] * 3)
        assert b == pytest.approx(a, rel=1e-12)


def test_richardson_factor(oracle_lib):
    rng = np.random.default_rng(6)
    gu = rng.normal(size=(3, 3)) * 0.05
    S = 0.5 * (gu + gu.T)
    SS = 2.0 * np.sum(S * S)
    base = oracle_lib.vreman(gu, 0.0, CS, [50.0] * 3, Prt=1 / 3, richardson=True)
    assert base == oracle_lib.vreman(gu, 0.0, CS, [50.0] * 3)
    # unstable stratification leaves it alone; stable damps it by (1 - Ri/Pr)^(1/4)
    assert oracle_lib.vreman(gu, -1e-4, CS, [50.0] * 3, Prt=1 / 3, richardson=True) == base
    N2 = 0.1 * SS
    fb = (1.0 - (N2 / SS) * 3.0) ** 0.25
    assert oracle_lib.vreman(gu, N2, CS, [50.0] * 3, Prt=1 / 3, richardson=True) == pytest.approx(base * fb, rel=1e-13)
    assert oracle_lib.vreman(gu, SS, CS, [50.0] * 3, Prt=1 / 3, richardson=True) == 0.0
