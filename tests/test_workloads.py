"""Checks of the seeded input generators against closed forms (hydrostatic
balance of the background profiles, Sect. 5.1 eq. pressureDistrib and
Sect. 5.4 eq. pressure_hs_brunt / density_hs_brunt)."""
import numpy as np
import pytest

from paper_2110_00853_amd import workloads as W

G_ = 9.81
RD = 287.0


@pytest.mark.parametrize("prof", ["isothermal", "neutral", "constant_N"])
def test_background_is_hydrostatic(prof):
    z = np.linspace(0.0, 6000.0, 601)
    f = getattr(W, prof)
    p, T = f(z)
    assert p[0] == pytest.approx(1e5, rel=1e-15)
    rho = p / (RD * T)
    dz = 1e-3
    dpdz = (f(z + dz)[0] - f(z - dz)[0]) / (2 * dz)
    assert np.allclose(dpdz, -rho * G_, rtol=1e-7)


def test_neutral_background_has_uniform_enthalpy():
    """c_pd T + g z is constant for uniform potential temperature."""
    z = np.linspace(0.0, 5000.0, 101)
    p, T = W.neutral(z)
    h = 1004.5 * T + G_ * z
    assert np.ptp(h) < 1e-9 * h[0]


def test_constant_N_buoyancy_frequency():
    z = np.linspace(0.0, 15000.0, 151)
    p, T = W.constant_N(z, Nbv=0.01)
    th = T * (1e5 / p) ** (287.0 / 1004.5)
    dz = 1e-2
    dth = (np.log(W.constant_N(z + dz)[1] * (1e5 / W.constant_N(z + dz)[0]) ** (287.0 / 1004.5))
           - np.log(W.constant_N(z - dz)[1] * (1e5 / W.constant_N(z - dz)[0]) ** (287.0 / 1004.5))) / (2 * dz)
    assert np.allclose(G_ * dth, 1e-4, rtol=1e-6)


def test_moist_profile_hydrostatic_and_cloudy_top():
    z = np.array([0.0, 100.0, 300.0, 500.0, 520.0, 1000.0, 2000.0, 3000.0])
    p, T, qt = W.moist_hydrostatic(z)
    Y = W.state_from_primitives(p, T, 0 * z, 0 * z, 0 * z, z, qt=qt)
    rho = Y[0]
    # trapezoidal dp/dz against -rho g between levels
    dpdz = np.diff(p) / np.diff(z)
    mid = -0.5 * (rho[1:] + rho[:-1]) * G_
    assert np.allclose(dpdz, mid, rtol=2e-3)
    # the mixed-layer top is supersaturated, so condensate is present there
    qvs = W.pvsat(T) / (rho * 462.0 * T)
    assert qt[4] > qvs[4]


def test_coordinates_layout_and_counts():
    g = {"N": 4, "ne": [3, 2, 2], "lo": [0, 0, 0], "hi": [300.0, 200.0, 400.0], "periodic": [1, 1, 0]}
    x = W.node_coords(g)
    assert x.shape == (3, W.n_nodes(g))
    # node 1 of element 0 lies at i = 1 along x, element 1 is the x-neighbour
    assert x[0, 1] == pytest.approx(50.0 * (1 - np.sqrt(3 / 7)))
    assert x[0, 125] == pytest.approx(100.0)
    assert x[1, 125 * 3] == pytest.approx(100.0)
    assert x[2, 125 * 6] == pytest.approx(200.0)
