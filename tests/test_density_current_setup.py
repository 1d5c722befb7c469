"""Host checks of the density-current set-up (Sect. 5.2) and of the front
diagnostic (the front-location table of App. B), without a GPU."""
import numpy as np

from paper_2110_00853_amd import diagnostics as D
from paper_2110_00853_amd import workloads as W


def test_initial_cold_bubble_follows_the_stated_perturbation():
    c = W.case("density_current")
    assert c["grid"]["ne"] == [128, 1, 32] and c["grid"]["periodic"] == [0, 1, 0]
    # 50 m effective resolution: 200 m elements at N = 4
    h = (np.array(c["grid"]["hi"]) - np.array(c["grid"]["lo"])) / np.array(c["grid"]["ne"])
    assert np.allclose(h / 4, 50.0)
    xyz = W.node_coords(c["grid"])
    Y, Yref, dt = W.initial_state(c, xyz=xyz)
    dth = D.potential_temperature(Y, xyz[2]) - D.potential_temperature(Yref, xyz[2])
    r = np.sqrt((xyz[0] / 4000.0) ** 2 + ((xyz[2] - 3000.0) / 2000.0) ** 2)
    expect = np.where(r <= 1.0, -7.5 * (1.0 + np.cos(np.pi * r)), 0.0)
    assert np.abs(dth - expect).max() < 1e-9
    # background of uniform theta = 300 K, at rest
    assert np.abs(D.potential_temperature(Yref, xyz[2]) - 300.0).max() < 1e-9
    assert np.all(Y[1:4] == 0.0)
    assert 0.03 < dt < 0.05


def test_front_location_of_a_known_surface_profile():
    # theta' = -3 + x / 2500 along the ground crosses -1 K at x = 5000 m,
    # between bottom nodes; above the ground theta' = -5 K everywhere (must
    # not count)
    c = W.case("density_current", ne=(16, 1, 4), hi=(12800.0, 200.0, 3200.0))
    xyz = W.node_coords(c["grid"])
    z = xyz[2]
    p, T = W.neutral(z)
    thp = np.where(z <= 0.0, -3.0 + xyz[0] / 2500.0, -5.0)
    Tp = T + thp * (p / 1.0e5) ** (287.0 / 1004.5)
    zero = np.zeros_like(z)
    Y = W.state_from_primitives(p, Tp, zero, zero, zero, z)
    x = D.front_location(Y, xyz)
    assert abs(x - 5000.0) < 1e-6
    # a profile that is cold everywhere along the ground puts the front at the far wall
    Y2 = W.state_from_primitives(p, T - 2.0 * (p / 1.0e5) ** (287.0 / 1004.5), zero, zero, zero, z)
    assert D.front_location(Y2, xyz) == xyz[0].max()
    # and one that is nowhere cold puts it at the near wall
    assert D.front_location(W.state_from_primitives(p, T, zero, zero, zero, z), xyz) == 0.0
