"""Pins of the oracle's mesh and metric terms (Sect. 3.1 mapping; Sect. 5.3
terrain-following warp; eq. agnesi)."""
import numpy as np
import pytest

from paper_2110_00853_amd import workloads as W


def _cart(ne=(3, 2, 4), hi=(900.0, 400.0, 1600.0)):
    return {"N": 4, "ne": list(ne), "lo": [0.0, 0.0, 0.0], "hi": list(hi), "periodic": [1, 1, 0]}


def _warp(ne=(6, 2, 5)):
    return {"N": 4, "ne": list(ne), "lo": [0.0, 0.0, 0.0], "hi": [1500.0, 500.0, 1600.0],
            "periodic": [1, 1, 0], "topo": 1, "topo_h": 400.0, "topo_a": 300.0, "topo_xc": 750.0}


def test_cartesian_metrics_closed_form(oracle_lib):
    g = _cart()
    G = oracle_lib.Grid(g)
    Ja, J = G.metrics()
    h = np.array(g["hi"]) / np.array(g["ne"])
    assert np.allclose(J, h.prod() / 8.0, rtol=1e-13)
    for d in range(3):
        for c in range(3):
            exp = (h.prod() / h[d] / 4.0) if c == d else 0.0
            assert np.allclose(Ja[d, c], exp, rtol=1e-13, atol=1e-9)
    # integration weights sum to the box volume
    assert G.wJ().sum() == pytest.approx(np.prod(g["hi"]), rel=1e-13)


def test_coordinates_match_mesh_definition(oracle_lib):
    for g in (_cart(), _warp()):
        G = oracle_lib.Grid(g)
        assert np.allclose(G.coords(), W.node_coords(g), rtol=0, atol=1e-9)


def test_warped_metric_identities_and_volume(oracle_lib):
    g = _warp()
    G = oracle_lib.Grid(g)
    Ja, J = G.metrics()
    assert np.all(J > 0)
    # sum_d D_d (J a^d) = 0: for this x-z warp the cross-product metrics
    # reduce to D_xi D_zeta z - D_zeta D_xi z, which commute, so only
    # round-off of a doubly differentiated coordinate remains
    res = G.metric_identity()
    _, _, D = oracle_lib.gll(4)
    dn = np.abs(D).sum(axis=1).max()
    assert np.max(np.abs(res)) < 1e-14 * np.abs(Ja).max() * dn * dn
    # volume under a lid: L_y * int (z_top - z_sfc(x)) dx, with the Agnesi
    # integral h a [atan((x - xc)/a)] over the box
    a, hm, xc = g["topo_a"], g["topo_h"], g["topo_xc"]
    Lx, Ly, zt = g["hi"]
    ridge = hm * a * (np.arctan((Lx - xc) / a) - np.arctan((0 - xc) / a))
    vol = Ly * (zt * Lx - ridge)
    assert G.wJ().sum() == pytest.approx(vol, rel=2e-4)
    # surface follows the ridge, lid stays flat
    xyz = G.coords()
    zb = xyz[2][np.isclose(W.node_coords({**g, "topo": 0})[2], 0.0)]
    xb = xyz[0][np.isclose(W.node_coords({**g, "topo": 0})[2], 0.0)]
    assert np.allclose(zb, hm * a * a / ((xb - xc) ** 2 + a * a), rtol=1e-12)
    assert np.allclose(xyz[2].max(), zt)


def test_dense_kronecker_operators_match_sum_factorisation(oracle_lib):
    g = _warp(ne=(2, 1, 2))
    Ja1, J1 = oracle_lib.Grid(g).metrics()
    Ja2, J2 = oracle_lib.Grid(g, dense=True).metrics()
    assert np.allclose(J1, J2, rtol=1e-13)
    assert np.allclose(Ja1, Ja2, rtol=1e-12, atol=1e-9)
