"""Closed-form pins of the oracle's diffusive flux F2 and BR1 auxiliary
gradient (Sect. 3.1 BR1 lift; Sect. 4 eq. strain_rate, stress_tensor,
diff_moisture_flux, Diffusivity, diff_energy_flux; the d_qt (x) rho u term of
the momentum balance, Sect. 2).

Fields that are polynomials of degree <= N in z and constant in x and y are
reproduced exactly by the nodal interpolant, continuous across faces, so
BR1 returns their exact gradient and F2 has a closed form at every node:
  rho tau = -2 rho nu S;  rho d_qt = -rho D_t grad q_t, D_t = nu / Pr_t;
  momentum flux rho tau_ij + (rho d_qt)_j u_i;
  energy flux sum_i u_i rho tau_ij - rho D_t d h_tot / d x_j;
  water flux (rho d_qt)_j.
An element-wise constant field isolates the BR1 lift: with collocated GLL
quadrature the gradient at a face node is J^s/(J w_N) (g* - g^-) n with the
centred g* = (g^- + g^+)/2, i.e. 10/h (g^+ - g^-)/2 x 2 = difference over h/10
on a Cartesian mesh (w_N = 1/10), and zero on a wall face (g* = g^-).
"""
import os

import numpy as np
import pytest

from paper_2110_00853_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def table1():
    out = {}
    with open(os.path.join(HERE, "golden", "table1_constants.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, val = line.split()[:2]
                out[name] = float(val)
    return out


GRID = {"N": 4, "ne": [2, 2, 3], "lo": [0.0, 0.0, 0.0], "hi": [400.0, 400.0, 600.0], "periodic": [1, 1, 0]}


def _moist_linear_state(z, u0, alpha, v0, w0, rho0, T, q0, beta):
    """rho, T uniform; u = (u0 + alpha z, v0, w0); q_t = q0 + beta z
    (unsaturated): conserved variables from the Sect. 2.5 energies."""
    c = table1()
    Rd, Rv, cvd, cvv, T0, Lv0 = c["R_d"], c["R_v"], c["c_vd"], c["c_vv"], c["T_0"], c["L_v0"]
    n = z.size
    q = q0 + beta * z
    ux = u0 + alpha * z
    I = (1 - q) * cvd * (T - T0) + q * (cvv * (T - T0) + Lv0 - Rv * T0)
    e = I + 0.5 * (ux ** 2 + v0 ** 2 + w0 ** 2)
    rho = np.full(n, rho0)
    Y = np.array([rho, rho * ux, rho * v0 + 0 * z, rho * w0 + 0 * z, rho * e, rho * q])
    dhdz = (beta * ((cvv - cvd) * (T - T0) + Lv0 - Rv * T0 + (Rv - Rd) * T) + alpha * ux)
    return Y, ux, q, dhdz


@pytest.mark.parametrize("closure", ["const", "smag"])
def test_diffusive_flux_closed_form_moist(oracle_lib, closure):
    """Every word of F2 for a shear flow with a linear total-water profile:
    the water flux, the momentum carried by the diffusing water, the energy
    flux u.(rho tau) and the enthalpy diffusion, with both closures (the
    Smagorinsky viscosity of the pure shear is (C_s Delta)^2 |alpha|)."""
    G = oracle_lib.Grid(GRID)
    z = G.coords()[2]
    u0, alpha, v0, w0, rho0, T, q0, beta = 3.0, 0.02, -1.5, 0.7, 1.05, 291.0, 4e-3, 2e-6
    Y, ux, q, dhdz = _moist_linear_state(z, u0, alpha, v0, w0, rho0, T, q0, beta)
    Prt = 0.4
    if closure == "const":
        nu = 35.0
        model = {"nvar": 6, "closure": "const", "nu": nu, "Prt": Prt, "g": 0.0}
    else:
        Cs = 0.2
        Delta = (200.0 / 4 * 200.0 / 4 * 200.0 / 4) ** (1 / 3)
        nu = (Cs * Delta) ** 2 * alpha
        model = {"nvar": 6, "closure": "smag", "Cs": Cs, "Prt": Prt, "richardson": False, "g": 0.0}
    M = oracle_lib.Model(G, model)
    _, F2 = M.gradients(Y)
    Dt = nu / Prt
    rd_z = -rho0 * Dt * beta
    rtau_xz = -rho0 * nu * alpha
    exp = np.zeros((6, 3, z.size))
    exp[0, 2] = rd_z
    exp[1, 2] = rtau_xz + rd_z * ux
    exp[3, 0] = rtau_xz
    exp[2, 2] = rd_z * v0
    exp[3, 2] = rd_z * w0
    exp[4, 0] = w0 * rtau_xz
    exp[4, 2] = ux * rtau_xz - rho0 * Dt * dhdz
    exp[5, 2] = rd_z
    scale = np.abs(exp).max(axis=(1, 2))
    for v in range(6):
        err = np.abs(F2[v] - exp[v]).max() / scale[v]
        assert err < 1e-10, (v, err)


@pytest.mark.parametrize("mutation", [0, 5])
def test_momentum_carried_by_diffusing_water(oracle_lib, mutation):
    """The d_qt (x) rho u term alone (no shear): F2 of rho u_i along z is
    (rho d_qt)_z u_i.  The planted mistake that drops it fails."""
    G = oracle_lib.Grid(GRID)
    z = G.coords()[2]
    Y, ux, q, dhdz = _moist_linear_state(z, 4.0, 0.0, 2.0, 0.0, 1.1, 288.0, 5e-3, 3e-6)
    M = oracle_lib.Model(G, {"nvar": 6, "closure": "const", "nu": 20.0, "Prt": 1.0 / 3.0, "g": 0.0})
    oracle_lib.set_mutation(mutation)
    try:
        _, F2 = M.gradients(Y)
    finally:
        oracle_lib.set_mutation(0)
    rd_z = -1.1 * 60.0 * 3e-6
    ok = np.allclose(F2[1, 2], rd_z * 4.0, rtol=1e-11) and np.allclose(F2[2, 2], rd_z * 2.0, rtol=1e-11)
    assert ok == (mutation == 0)


@pytest.mark.parametrize("mutation", [0, 6])
def test_br1_lift_of_elementwise_constant_field(oracle_lib, mutation):
    """u_x constant in each element (jumps at every face): the BR1 gradient
    is zero inside, (c_nbr - c_own) 10/h at the face nodes of periodic faces
    (summed over the faces a node lies on), and zero at wall faces.  The
    planted doubled lift fails."""
    g = {"N": 4, "ne": [3, 2, 3], "lo": [0.0, 0.0, 0.0], "hi": [900.0, 500.0, 600.0], "periodic": [1, 1, 0]}
    G = oracle_lib.Grid(g)
    xyz = G.coords()
    ne, Q, nn = g["ne"], 5, xyz.shape[1]
    h = [(g["hi"][a] - g["lo"][a]) / ne[a] for a in range(3)]
    rng = np.random.default_rng(5)
    c = rng.uniform(-3, 3, size=ne[0] * ne[1] * ne[2])
    e_of = np.repeat(np.arange(c.size), Q ** 3)
    ux = c[e_of]
    rho, T = np.full(nn, 1.0), np.full(nn, 290.0)
    Y = W.state_from_primitives(rho * 287.0 * T, T, ux, np.zeros(nn), np.zeros(nn), xyz[2], g=0.0)
    M = oracle_lib.Model(G, {"nvar": 5, "closure": "const", "nu": 10.0, "g": 0.0})
    oracle_lib.set_mutation(mutation)
    try:
        grad, _ = M.gradients(Y)
    finally:
        oracle_lib.set_mutation(0)
    loc = np.tile(np.arange(Q ** 3), c.size)
    ijk = [loc % Q, (loc // Q) % Q, loc // (Q * Q)]
    e = e_of
    ec = [e % ne[0], (e // ne[0]) % ne[1], e // (ne[0] * ne[1])]
    exp = np.zeros((3, nn))
    for d in range(3):
        for side, node in ((-1, 0), (1, Q - 1)):
            on = ijk[d] == node
            nb = [a.copy() for a in ec]
            nb[d] = nb[d] + side
            wall = ((nb[d] < 0) | (nb[d] >= ne[d])) & (not g["periodic"][d])
            nb[d] = nb[d] % ne[d]
            en = nb[0] + ne[0] * (nb[1] + ne[1] * nb[2])
            jump = np.where(wall, 0.0, c[en] - c[e]) * side   # (g^+ - g^-) n_d
            exp[d] += np.where(on, jump * 10.0 / h[d], 0.0)
    ok = np.allclose(grad[0], exp, rtol=0, atol=1e-12 * np.abs(exp).max())
    assert ok == (mutation == 0)
