"""Closed-form pins of the oracle's source terms and prescribed wall fluxes.

Each test builds a state whose flux divergence vanishes (a uniform state in a
periodic box, or at rest with walls) and reads the tendency that the source
alone leaves, against the closed form from the paper:
  * Coriolis on an f-plane with a geostrophic wind (momentum balance, Sect. 2;
    the f-plane form with u_g, v_g is the reading of the term);
  * the Rayleigh sponge, App. A eq. sponge, read as alpha sin^gamma(pi zeta / 2),
    zeta = (z - z_s)/(z_top - z_s): tau_s(z_top) = alpha, tau_s = 0 at and
    below z_s, alpha/2 at zeta = 1/2 for gamma = 2;
  * large-scale subsidence w_s = -w0 sin(pi z / z_top) acting on h_tot and q_t
    (the BOMEX forcing of Sect. 5.6, with a synthetic profile);
  * prescribed surface fluxes at the bottom wall (App. A): the tendency of the
    face nodes is J^s/(J w_N) x the upward flux, and its integral over the
    domain is the bottom area x the flux.
"""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def table1():
    out = {}
    with open(os.path.join(HERE, "golden", "table1_constants.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, val = line.split()[:2]
                out[name] = float(val)
    return out


C1 = table1()
RD, RV, CVD, CVV, T0, LV0 = C1["R_d"], C1["R_v"], C1["c_vd"], C1["c_vv"], C1["T_0"], C1["L_v0"]
IV0 = LV0 - RV * T0
CPD = CVD + RD   # reading: c_pd = c_vd + R_d


def uniform_state(n, rho, u, T, qt=None):
    """Conserved variables of a uniform (unsaturated) state, g = 0."""
    q = 0.0 if qt is None else qt
    I = (1 - q) * CVD * (T - T0) + q * (CVV * (T - T0) + IV0)
    e = I + 0.5 * float(np.dot(u, u))
    rows = [rho, rho * u[0], rho * u[1], rho * u[2], rho * e] + ([rho * qt] if qt is not None else [])
    return np.array([np.full(n, r) for r in rows])


def test_coriolis_geostrophic_closed_form(oracle_lib):
    """Uniform flow in a periodic box: only the Coriolis term is left,
    R_rho u = f (rho v - rho v_g), R_rho v = -f (rho u - rho u_g)."""
    g = {"N": 4, "ne": [2, 2, 2], "lo": [0.0] * 3, "hi": [600.0] * 3, "periodic": [1, 1, 1]}
    G = oracle_lib.Grid(g)
    rho, u = 1.07, np.array([-7.0, 2.5, 0.0])
    Y = uniform_state(G.nnodes, rho, u, 295.0)
    base = {"nvar": 5, "closure": "none", "g": 0.0}
    f, ug, vg = 1e-4, -10.0, 1.0
    R0 = oracle_lib.Model(G, base).rhs(Y)
    R = oracle_lib.Model(G, dict(base, f_cor=f, u_g=ug, v_g=vg)).rhs(Y)
    ex_u = f * (rho * u[1] - rho * vg)
    ex_v = -f * (rho * u[0] - rho * ug)
    assert np.allclose(R[1] - R0[1], ex_u, rtol=1e-9, atol=0)
    assert np.allclose(R[2] - R0[2], ex_v, rtol=1e-9, atol=0)
    for v in (0, 3, 4):
        assert np.array_equal(R[v], R0[v])
    # and the free stream itself is at rest to round-off
    assert np.abs(R0).max() < 1e-9


def test_sponge_profile_closed_form(oracle_lib):
    """Uniform horizontal flow between free-slip walls: the sponge leaves
    -tau_s(z) (rho u - rho u_relax) with tau_s = alpha at the lid, 0 at and
    below z_s, alpha/2 half-way (gamma = 2), and alpha sin^2(pi zeta/2)
    in general."""
    g = {"N": 4, "ne": [2, 1, 2], "lo": [0.0] * 3, "hi": [400.0, 200.0, 1000.0], "periodic": [1, 1, 0]}
    G = oracle_lib.Grid(g)
    z = G.coords()[2]
    rho, u = 1.1, np.array([12.0, -3.0, 0.0])
    Y = uniform_state(G.nnodes, rho, u, 300.0)
    alpha, urel = 0.5, np.array([10.0, 0.0, 0.0])
    base = {"nvar": 5, "closure": "none", "g": 0.0}
    sponge = {"z_s": 500.0, "z_top": 1000.0, "alpha": alpha, "gamma": 2.0, "u_relax": list(urel)}
    R0 = oracle_lib.Model(G, base).rhs(Y)
    R = oracle_lib.Model(G, dict(base, sponge=sponge)).rhs(Y)
    tau = -(R[1] - R0[1]) / (rho * (u[0] - urel[0]))
    assert np.allclose(tau[z == 1000.0], alpha, rtol=1e-12)
    assert np.all(tau[z <= 500.0] == 0.0)
    assert np.allclose(tau[z == 750.0], alpha / 2, rtol=1e-12)   # the middle GLL node of the top element
    zeta = np.clip((z - 500.0) / 500.0, 0.0, None)
    assert np.allclose(tau, alpha * np.sin(0.5 * np.pi * zeta) ** 2, rtol=1e-10, atol=1e-14)
    tau_v = -(R[2] - R0[2]) / (rho * (u[1] - urel[1]))
    assert np.allclose(tau_v, tau, rtol=1e-10, atol=1e-14)
    assert np.array_equal(R[3], R0[3]) and np.array_equal(R[0], R0[0])


@pytest.mark.parametrize("nvar", [5, 6])
def test_subsidence_closed_form(oracle_lib, nvar):
    """Air at rest, uniform density, T and q_t linear in z, zero viscosity:
    the energy and water tendencies are the subsidence terms alone,
    -rho w_s d h_tot/dz and -rho w_s d q_t/dz, w_s = -w0 sin(pi z/z_top)."""
    sp = pytest.importorskip("sympy")
    g = {"N": 4, "ne": [1, 1, 3], "lo": [0.0] * 3, "hi": [300.0, 300.0, 1500.0], "periodic": [1, 1, 0]}
    G = oracle_lib.Grid(g)
    z = G.coords()[2]
    rho, Ta, gT, qa, beta = 1.1, 300.0, -6e-3, 8e-3, -2e-6
    zs = sp.symbols("z")
    T = Ta + gT * zs
    q = (qa + beta * zs) if nvar == 6 else sp.Integer(0)
    I = (1 - q) * CVD * (T - T0) + q * (CVV * (T - T0) + IV0)
    h = I + (RD * (1 - q) + RV * q) * T                  # e_tot + p/rho at rest, g = 0
    e_fn = sp.lambdify(zs, I, "numpy")
    dh_fn = sp.lambdify(zs, sp.diff(h, zs), "numpy")
    rows = [np.full(z.size, rho), 0 * z, 0 * z, 0 * z, rho * e_fn(z)]
    if nvar == 6:
        rows.append(rho * (qa + beta * z))
    Y = np.array(rows)
    w0, ztop = 5e-3, 1500.0
    base = {"nvar": nvar, "closure": "const", "nu": 0.0, "g": 0.0}
    R0 = oracle_lib.Model(G, base).rhs(Y)
    R = oracle_lib.Model(G, dict(base, subsidence={"w0": w0, "z_top": ztop})).rhs(Y)
    ws = -w0 * np.sin(np.pi * z / ztop)
    assert np.allclose(R[4] - R0[4], -rho * ws * dh_fn(z), rtol=1e-9, atol=1e-12)
    if nvar == 6:
        assert np.allclose(R[5] - R0[5], -rho * ws * beta, rtol=1e-9, atol=1e-18)
    assert np.abs(R0[4]).max() < 1e-9 and np.abs(R0[0]).max() < 1e-12


@pytest.mark.parametrize("nvar", [5, 6])
def test_surface_flux_closed_form(oracle_lib, nvar):
    """Uniform air at rest with zero viscosity and prescribed bottom fluxes:
    only the bottom face nodes change, by (J^s/(J w_N)) x upward flux, with
    J^s/(J w_N) = 2/(h_z w_N) = 20/h_z; the energy flux is
    rho (c_pd theta_flux + L_v0 q_flux), mass and water rho q_flux (moist
    only).  The domain integral of the tendency is the bottom area x flux."""
    g = {"N": 4, "ne": [2, 2, 2], "lo": [0.0] * 3, "hi": [500.0, 400.0, 600.0], "periodic": [1, 1, 0]}
    G = oracle_lib.Grid(g)
    z = G.coords()[2]
    rho = 1.15
    Y = uniform_state(G.nnodes, rho, np.zeros(3), 299.0, qt=6e-3 if nvar == 6 else None)
    thf, qf = 8e-3, 5.2e-5
    base = {"nvar": nvar, "closure": "const", "nu": 0.0, "g": 0.0}
    R0 = oracle_lib.Model(G, base).rhs(Y)
    R = oracle_lib.Model(G, dict(base, sfc_flux={"theta_flux": thf, "qt_flux": qf})).rhs(Y)
    dR = R - R0
    bottom = z == 0.0
    lift = 20.0 / 300.0
    up_e = rho * (CPD * thf + (LV0 * qf if nvar == 6 else 0.0))
    assert np.allclose(dR[4][bottom], lift * up_e, rtol=1e-12)
    assert np.all(dR[4][~bottom] == 0.0)
    if nvar == 6:
        assert np.allclose(dR[0][bottom], lift * rho * qf, rtol=1e-12)
        assert np.allclose(dR[5][bottom], lift * rho * qf, rtol=1e-12)
    else:
        assert np.all(dR[0] == 0.0)
    wJ = G.wJ()
    area = 500.0 * 400.0
    assert np.sum(wJ * dR[4]) == pytest.approx(area * up_e, rel=1e-12)
    for v in (1, 2, 3):
        assert np.all(dR[v] == 0.0)
