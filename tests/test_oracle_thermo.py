"""Pins of the oracle's thermodynamics (Sect. 2.5-2.7: moist internal energy,
equation of state, saturation adjustment with the closed-form saturation
vapour pressure)."""
import os

import numpy as np
import pytest
from scipy.integrate import quad

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def table1():
    out = {}
    for line in open(os.path.join(GOLDEN, "table1_constants.txt")):
        if line.strip() and not line.startswith("#"):
            name, val = line.split()[:2]
            out[name] = float(val)
    return out


K = table1()
G_ = 9.81
P_TR = 611.657


def test_dry_temperature_and_pressure_follow_table1(oracle_lib):
    """Dry air: I = c_vd (T - T_0) and p = rho R_d T."""
    rng = np.random.default_rng(3)
    n = 50
    rho = rng.uniform(0.5, 1.3, n)
    u = rng.uniform(-20, 20, (3, n))
    T = rng.uniform(220, 320, n)
    z = rng.uniform(0, 5000, n)
    e = K["c_vd"] * (T - K["T_0"]) + G_ * z + 0.5 * (u ** 2).sum(0)
    Y = np.vstack([rho, rho * u, rho * e])
    T_o, p_o, ql, _ = oracle_lib.thermo_nodes(Y, z, G_)
    assert np.allclose(T_o, T, rtol=1e-13)
    assert np.allclose(p_o, rho * K["R_d"] * T, rtol=1e-13)
    assert np.all(ql == 0)


def test_saturation_pressure_at_triple_point(oracle_lib):
    assert oracle_lib.pvsat(K["T_0"]) == pytest.approx(P_TR, rel=1e-15)


@pytest.mark.parametrize("T", [250.0, 273.16, 285.0, 300.0, 310.0])
def test_saturation_pressure_integrates_clausius_clapeyron(oracle_lib, T):
    """ln(p*/p_tr) = int_{T_0}^{T} L_v(s) / (R_v s^2) ds with
    L_v(s) = L_v0 + (c_pv - c_pl)(s - T_0), integrated numerically."""
    cpv = K["c_vv"] + K["R_v"]
    Lv = lambda s: K["L_v0"] + (cpv - K["c_vl"]) * (s - K["T_0"])
    val, _ = quad(lambda s: Lv(s) / (K["R_v"] * s * s), K["T_0"], T, epsabs=0.0, epsrel=1e-12, limit=200)
    assert oracle_lib.pvsat(T) == pytest.approx(P_TR * np.exp(val), rel=1e-12)


def _I(T, rho, qt, ql):
    qv = qt - ql
    Iv0 = K["L_v0"] - K["R_v"] * K["T_0"]
    d = T - K["T_0"]
    return (1 - qt) * K["c_vd"] * d + qv * (K["c_vv"] * d + Iv0) + ql * K["c_vl"] * d


def test_unsaturated_closed_form(oracle_lib):
    rho, qt, T = 1.1, 5e-3, 295.0
    I = _I(T, rho, qt, 0.0)
    T_o, ql = oracle_lib.saturation_adjust(rho, qt, I)
    assert ql == 0.0
    assert T_o == pytest.approx(T, abs=1e-11)


@pytest.mark.parametrize("T,rho,excess", [(290.0, 1.15, 2e-3), (280.0, 1.2, 5e-4), (300.0, 1.0, 1e-5),
                                          (274.0, 0.9, 3e-3)])
def test_saturated_round_trip(oracle_lib, T, rho, excess):
    """Equilibrium state (T, rho, q_t) -> I by the definition of moist internal
    energy -> saturation adjustment recovers T and q_l."""
    qvs = oracle_lib.pvsat(T) / (rho * K["R_v"] * T)
    qt = qvs + excess
    I = _I(T, rho, qt, excess)
    T_o, ql = oracle_lib.saturation_adjust(rho, qt, I)
    assert T_o == pytest.approx(T, abs=1e-10)
    assert ql == pytest.approx(excess, abs=1e-12)


def test_moist_pressure_and_virtual_temperature(oracle_lib):
    """p = rho R_m T with R_m = R_d (1 - q_t) + R_v q_v (eq. R_m), and theta_v
    = T (p0/p)^(R_d/c_pd) R_m / R_d."""
    T, rho, excess = 288.0, 1.1, 1e-3
    qvs = oracle_lib.pvsat(T) / (rho * K["R_v"] * T)
    qt = qvs + excess
    I = _I(T, rho, qt, excess)
    z = np.array([100.0])
    Y = np.array([[rho], [0.0], [0.0], [0.0], [rho * (I + G_ * 100.0)], [rho * qt]])
    T_o, p_o, ql, thv = oracle_lib.thermo_nodes(Y, z, G_)
    Rm = K["R_d"] * (1 - qt) + K["R_v"] * qvs
    # equivalent form of eq. R_m: R_d [1 + (eps - 1) q_t - eps q_c]
    eps = K["R_v"] / K["R_d"]
    assert Rm == pytest.approx(K["R_d"] * (1 + (eps - 1) * qt - eps * excess), rel=1e-14)
    assert p_o[0] == pytest.approx(rho * Rm * T, rel=1e-12)
    kappa = K["R_d"] / (K["c_vd"] + K["R_d"])
    assert thv[0] == pytest.approx(T * (1e5 / p_o[0]) ** kappa * Rm / K["R_d"], rel=1e-12)
