"""Invariants the discrete method fixes, checked on the oracle: free-stream
preservation, hydrostatic rest, conservation of mass and total energy to
round-off (Sect. 6), mirror/permutation symmetry, and the brute-force dense
Kronecker operators against sum factorisation (Sect. 3.1)."""
import os

import numpy as np
import pytest

from paper_2110_00853_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

CART = {"N": 4, "ne": [3, 2, 3], "lo": [0.0, 0.0, 0.0], "hi": [600.0, 400.0, 600.0], "periodic": [1, 1, 1]}
WARP = {"N": 4, "ne": [4, 2, 3], "lo": [0.0, 0.0, 0.0], "hi": [1000.0, 500.0, 900.0], "periodic": [1, 1, 1],
        "topo": 1, "topo_h": 150.0, "topo_a": 200.0, "topo_xc": 500.0}


def _flux_scale(Y, h):
    rho = Y[0]
    u = Y[1:4] / rho
    p = 1e5
    return np.array([np.abs(Y[1:4]).max(), p, p, p, np.abs(Y[4] * u).max() + p * np.abs(u).max()]) * 2 / h


@pytest.mark.parametrize("grid", [CART, WARP], ids=["cartesian", "warped"])
@pytest.mark.parametrize("closure", ["none", "const", "smag"])
@pytest.mark.parametrize("nvar", [5, 6])
def test_free_stream_preserved(oracle_lib, grid, closure, nvar):
    G = oracle_lib.Grid(grid)
    Y = W.free_stream_state(grid, qt=None if nvar == 5 else 6e-3)
    M = oracle_lib.Model(G, {"nvar": nvar, "closure": closure, "nu": 75.0, "g": 0.0, "richardson": True})
    R = M.rhs(Y)
    h = min(np.array(grid["hi"]) / np.array(grid["ne"]))
    sc = _flux_scale(Y, h)
    for v in range(5):
        assert np.abs(R[v]).max() < 1e-12 * sc[v], v
    if nvar == 6:
        assert np.abs(R[5]).max() < 1e-12 * sc[0]


@pytest.mark.parametrize("closure", ["const", "smag"])
def test_hydrostatic_rest_stays_at_rest(oracle_lib, closure):
    """Neutral (uniform potential temperature) hydrostatic background with
    itself as reference state, free-slip adiabatic walls top and bottom: the
    tendency vanishes (h_tot is uniform, so even constant-nu diffusion has
    nothing to act on)."""
    g = dict(CART, periodic=[1, 1, 0], hi=[600.0, 400.0, 1500.0])
    G = oracle_lib.Grid(g)
    Y = W.neutral_rest_state(g)
    M = oracle_lib.Model(G, {"nvar": 5, "closure": closure, "nu": 75.0, "g": 9.81, "richardson": True}, Y)
    R = M.rhs(Y)
    rho_g = Y[0].max() * 9.81
    assert np.abs(R[0]).max() == 0.0
    assert np.abs(R[1:4]).max() <= 1e-12 * rho_g
    assert np.abs(R[4]).max() <= 1e-12 * rho_g * 300.0


def _drift(M, Y, dt, nsteps):
    I0 = M.integrals(Y)
    Y1, _ = M.steps(Y, dt, nsteps)
    I1 = M.integrals(Y1)
    return (I1 - I0) / I0, Y1


def test_conservation_periodic_box_smagorinsky(oracle_lib):
    """Periodic, gravity-free, source-free box with the Smagorinsky-Lilly
    closure: mass and total energy drift at round-off over 100 steps."""
    bound = float(open(os.path.join(GOLDEN, "conservation_bound.txt")).read().split()[-1])
    g = CART
    c = {"grid": g, "model": {"nvar": 5, "closure": "smag", "Cs": 0.21, "g": 0.0}, "ic": {"kind": "bubble"}}
    Y, _, speed = W.perturbed_state(c, seed=4, amp_u=8.0, amp_T=3.0)
    G = oracle_lib.Grid(g)
    M = oracle_lib.Model(G, c["model"])
    rel, Y1 = _drift(M, Y, W.cfl_dt(g, speed), 100)
    assert np.abs(Y1 - Y).max() > 1e-3            # the state did evolve
    assert abs(rel[0]) < 10 * bound and abs(rel[4]) < 10 * bound


def test_conservation_closed_box_with_gravity_moist(oracle_lib):
    """Moist state, gravity, free-slip adiabatic walls on all sides of the
    vertical, Smagorinsky + Richardson: mass, total water and total energy are
    conserved to round-off (the paper's 1 h moist bubble check, shortened)."""
    bound = float(open(os.path.join(GOLDEN, "conservation_bound.txt")).read().split()[-1])
    g = {"N": 4, "ne": [2, 2, 3], "lo": [0.0, 0.0, 0.0], "hi": [400.0, 400.0, 600.0], "periodic": [0, 1, 0]}
    c = {"grid": g, "model": {"nvar": 6, "closure": "smag", "Cs": 0.21, "richardson": True, "g": 9.81},
         "ic": {"kind": "moist"}}
    Y, Yref, speed = W.perturbed_state(c, seed=5, amp_u=3.0, amp_T=1.0, amp_q=2e-3)
    G = oracle_lib.Grid(g)
    M = oracle_lib.Model(G, c["model"], Yref)
    rel, Y1 = _drift(M, Y, W.cfl_dt(g, speed), 50)
    assert np.abs(Y1 - Y).max() > 1e-4
    for v in (0, 4, 5):
        assert abs(rel[v]) < 10 * bound, (v, rel)


def _mirror_x(Y, g):
    ne = g["ne"]
    Q = 5
    A = Y.reshape(Y.shape[0], ne[2], ne[1], ne[0], Q, Q, Q)
    B = A[:, :, :, ::-1, :, :, ::-1].copy()
    B[1] = -B[1]
    return B.reshape(Y.shape)


def _swap_xy(Y, g):
    ne = g["ne"]
    Q = 5
    A = Y.reshape(Y.shape[0], ne[2], ne[1], ne[0], Q, Q, Q)
    B = A.transpose(0, 1, 3, 2, 4, 6, 5).copy()
    B[[1, 2]] = B[[2, 1]]
    return B.reshape(Y.shape)


def test_mirror_and_permutation_symmetry(oracle_lib):
    """R commutes with the mirror x -> L - x (u -> -u) and with exchanging x
    and y, on a symmetric box with walls in z and the Smagorinsky closure."""
    g = {"N": 4, "ne": [3, 3, 2], "lo": [0.0, 0.0, 0.0], "hi": [600.0, 600.0, 400.0], "periodic": [1, 1, 0]}
    c = {"grid": g, "model": {"nvar": 5, "closure": "smag", "Cs": 0.21, "richardson": True, "g": 9.81},
         "ic": {"kind": "bubble"}}
    Y, Yref, _ = W.perturbed_state(c, seed=6)
    G = oracle_lib.Grid(g)
    M = oracle_lib.Model(G, c["model"], Yref)
    R = M.rhs(Y)
    scale = np.abs(R).max(axis=1, keepdims=True)
    Rm = M.rhs(_mirror_x(Y, g))
    assert np.max(np.abs(Rm - _mirror_x(R, g)) / scale) < 1e-10
    Rs = M.rhs(_swap_xy(Y, g))
    assert np.max(np.abs(Rs - _swap_xy(R, g)) / scale) < 1e-10


def test_dense_kronecker_rhs_matches(oracle_lib):
    """The tendency with explicit (N+1)^3 x (N+1)^3 Kronecker derivative
    matrices equals the sum-factorised one (warped, moist, Smagorinsky)."""
    g = dict(WARP, ne=[2, 1, 2], periodic=[1, 1, 0])
    c = {"grid": g, "model": {"nvar": 6, "closure": "smag", "richardson": True, "g": 9.81,
                              "sfc_flux": {"theta_flux": 8e-3, "qt_flux": 5.2e-5},
                              "subsidence": {"w0": 5e-3, "z_top": 900.0}, "f_cor": 1e-4, "u_g": -10.0,
                              "sponge": {"z_s": 500.0, "z_top": 900.0, "alpha": 0.5, "gamma": 2.0,
                                         "u_relax": (10.0, 0.0, 0.0)}},
         "ic": {"kind": "moist"}}
    Y, Yref, _ = W.perturbed_state(c, seed=7)
    R1 = oracle_lib.Model(oracle_lib.Grid(g), c["model"], Yref).rhs(Y)
    R2 = oracle_lib.Model(oracle_lib.Grid(g, dense=True), c["model"], Yref).rhs(Y)
    scale = np.abs(R1).max(axis=1, keepdims=True)
    assert np.max(np.abs(R1 - R2) / scale) < 1e-11
