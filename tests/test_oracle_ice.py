"""Pins of the oracle's ice phase (Sect. 2.5 and 2.7, Table 1): the
Clausius-Clapeyron saturation pressure over ice (triple point, slope L_s/(R_v
T^2) with L_s(T) = L_v0 + L_f0 + (c_pv - c_vi)(T - T_0)), the liquid
fraction, and the saturation adjustment with ice: at the returned
temperature the equilibrium internal energy, recomputed here from Table 1,
equals the input one, vapour sits at the mixed saturation value, and the
condensate splits by the liquid fraction; above freezing the result is the
liquid-only one."""
import numpy as np
import pytest

RD, RV, CVD, CVV, CVL, CVI = 287.0, 462.0, 717.5, 1397.5, 4181.0, 2100.0
T0, LV0, LF0 = 273.16, 2.5008e6, 0.3336e6
CPV = CVV + RV
IV0 = LV0 - RV * T0


def test_triple_point_and_clausius_clapeyron_slopes(oracle_lib):
    assert oracle_lib.pvsat_ice(T0) == oracle_lib.pvsat(T0) == 611.657
    for T in (200.0, 235.0, 260.0, 272.0):
        h = 1e-4 * T
        slope_i = (np.log(oracle_lib.pvsat_ice(T + h)) - np.log(oracle_lib.pvsat_ice(T - h))) / (2 * h)
        Ls = LV0 + LF0 + (CPV - CVI) * (T - T0)
        assert slope_i == pytest.approx(Ls / (RV * T * T), rel=1e-7)
        slope_l = (np.log(oracle_lib.pvsat(T + h)) - np.log(oracle_lib.pvsat(T - h))) / (2 * h)
        Lv = LV0 + (CPV - CVL) * (T - T0)
        assert slope_l == pytest.approx(Lv / (RV * T * T), rel=1e-7)
        # below the triple point ice saturates at a lower vapour pressure
        assert oracle_lib.pvsat_ice(T) < oracle_lib.pvsat(T)


def test_liquid_fraction(oracle_lib):
    assert oracle_lib.liquid_fraction(280.0) == 1.0 and oracle_lib.liquid_fraction(273.15) == 1.0
    assert oracle_lib.liquid_fraction(233.0) == 0.0 and oracle_lib.liquid_fraction(200.0) == 0.0
    assert oracle_lib.liquid_fraction(253.075) == pytest.approx(0.5, abs=1e-15)


def _istar(T, qt, qv, ql, qi):
    return (1 - qt) * CVD * (T - T0) + qv * (CVV * (T - T0) + IV0) + ql * CVL * (T - T0) + qi * (CVI * (T - T0) - LF0)


@pytest.mark.parametrize("T_target", [262.0, 250.0, 240.0, 228.0, 268.0])
def test_saturation_adjustment_with_ice(oracle_lib, T_target):
    rho, qt = 0.8, 6e-3
    # I of a saturated state at T_target, built here from Table 1
    lam = min(1.0, max(0.0, (T_target - 233.0) / (273.15 - 233.0)))
    pv = lam * oracle_lib.pvsat(T_target) + (1 - lam) * oracle_lib.pvsat_ice(T_target)
    qv = pv / (rho * RV * T_target)
    assert qv < qt
    qc = qt - qv
    I = _istar(T_target, qt, qv, lam * qc, (1 - lam) * qc)
    T, ql, qi = oracle_lib.saturation_adjust_phase(rho, qt, I, ice=True)
    assert T == pytest.approx(T_target, abs=1e-9)
    assert ql == pytest.approx(lam * qc, abs=1e-15) and qi == pytest.approx((1 - lam) * qc, abs=1e-15)
    # without ice the same energy gives a warmer, all-liquid state
    Tl, qll, qil = oracle_lib.saturation_adjust_phase(rho, qt, I, ice=False)
    assert qil == 0.0
    if lam < 1.0:
        assert Tl < T  # latent heat of fusion not released
    assert _istar(Tl, qt, qt - qll, qll, 0.0) == pytest.approx(I, abs=1e-7 * abs(I))


def test_above_freezing_and_unsaturated_states_are_unchanged(oracle_lib):
    rho, qt = 1.1, 1.5e-2
    for I in (2.0e4, 4.0e4, 6.0e4):
        a = oracle_lib.saturation_adjust_phase(rho, qt, I, ice=True)
        b = oracle_lib.saturation_adjust_phase(rho, qt, I, ice=False)
        if a[0] >= 273.15:
            assert a == b
    # unsaturated cold air: no condensate, T from the dry-plus-vapour energy
    T, ql, qi = oracle_lib.saturation_adjust_phase(0.9, 1e-5, -3.0e4, ice=True)
    assert ql == 0.0 and qi == 0.0
    assert T == pytest.approx(T0 + (-3.0e4 - 1e-5 * IV0) / ((1 - 1e-5) * CVD + 1e-5 * CVV), rel=1e-15)
