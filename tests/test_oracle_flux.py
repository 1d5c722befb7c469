"""Pins of the oracle's numerical flux, auxiliary gradient and closure
(Sect. 3.1 eq. nonviscFlux and the BR1 gradient; Sect. 4 eq. smago and
eq. richardson)."""
import numpy as np
import pytest

from paper_2110_00853_amd import workloads as W


def _state(rng, nvar=5):
    rho = rng.uniform(0.8, 1.2)
    u = rng.uniform(-30, 30, 3)
    T = rng.uniform(260, 310)
    qt = 8e-3 if nvar == 6 else None
    Y = W.state_from_primitives(np.array([rho * 287.0 * T]), np.array([T]), *[np.array([c]) for c in u],
                                np.array([0.0]), qt=None if qt is None else np.array([qt]), g=0.0)
    return Y[:, 0]


@pytest.mark.parametrize("nvar", [5, 6])
def test_rusanov_antisymmetry(oracle_lib, nvar):
    """F*(Y-, Y+, n) = -F*(Y+, Y-, -n): the two elements sharing a face see
    equal and opposite fluxes (conservation)."""
    rng = np.random.default_rng(1)
    for _ in range(10):
        Ym, Yp = _state(rng, nvar), _state(rng, nvar)
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        a = oracle_lib.rusanov(Ym, Yp, n)
        b = oracle_lib.rusanov(Yp, Ym, -n)
        assert np.allclose(a, -b, rtol=1e-14, atol=1e-12)


def test_rusanov_consistency_mass_flux(oracle_lib):
    """With equal states the dissipation vanishes and the mass component is
    the plain normal momentum rho u.n."""
    rng = np.random.default_rng(2)
    Y = _state(rng)
    n = np.array([0.6, 0.0, 0.8])
    f = oracle_lib.rusanov(Y, Y, n)
    assert f[0] == pytest.approx(np.dot(Y[1:4], n), rel=1e-15)


def test_rusanov_dissipation_is_half_max_wave_speed(oracle_lib):
    """Two states of equal velocity and pressure, different density: the
    mass-flux difference from the centred part is (1/2) lambda (rho- - rho+),
    lambda = max(|u.n| + c) of the two sides."""
    p, u = 9.0e4, np.array([10.0, 0.0, 0.0])
    T1, T2 = 280.0, 300.0
    Y1 = W.state_from_primitives(np.array([p]), np.array([T1]), *[np.array([c]) for c in u], np.array([0.0]), g=0)[:, 0]
    Y2 = W.state_from_primitives(np.array([p]), np.array([T2]), *[np.array([c]) for c in u], np.array([0.0]), g=0)[:, 0]
    n = np.array([1.0, 0.0, 0.0])
    f = oracle_lib.rusanov(Y1, Y2, n)
    lam = 10.0 + np.sqrt(1.4 * 287.0 * T2)
    centred = 0.5 * (Y1[1] + Y2[1])
    assert f[0] - centred == pytest.approx(0.5 * lam * (Y1[0] - Y2[0]), rel=1e-12)


def test_br1_gradient_exact_for_linear_fields(oracle_lib):
    """A globally linear velocity (continuous across faces, so every lift
    vanishes) has the exact constant gradient, also on the warped mesh."""
    for topo in (0, 1):
        g = {"N": 4, "ne": [3, 2, 3], "lo": [0.0, 0.0, 0.0], "hi": [600.0, 400.0, 900.0],
             "periodic": [0, 0, 0], "topo": topo, "topo_h": 150.0, "topo_a": 200.0, "topo_xc": 300.0}
        G = oracle_lib.Grid(g)
        x = G.coords()
        B = np.array([[0.01, -0.02, 0.005], [0.003, 0.004, -0.01], [-0.007, 0.002, 0.006]])
        u = np.array([1.0, -2.0, 0.5])[:, None] + B @ x
        rho = np.full(x.shape[1], 1.1)
        T = np.full(x.shape[1], 290.0)
        Y = W.state_from_primitives(rho * 287.0 * T, T, u[0], u[1], u[2], x[2], g=0.0)
        M = oracle_lib.Model(G, {"nvar": 5, "closure": "const", "nu": 10.0, "g": 0.0})
        grad, _ = M.gradients(Y)
        for i in range(3):
            for j in range(3):
                assert np.allclose(grad[i, j], B[i, j], atol=1e-13)


def test_smagorinsky_pure_shear_closed_form(oracle_lib):
    """u = (alpha z, 0, 0): |S|^2 = alpha^2, nu = (Cs Delta)^2 |alpha| f_b with
    f_b = (1 - Ri/Pr_t)^(1/4), Ri = N^2/alpha^2; f_b = 1 for Ri <= 0; nu = 0
    beyond the critical Richardson number Pr_t."""
    alpha, Cs, Delta, Prt = 0.02, 0.21, 50.0, 1.0 / 3.0
    gu = np.zeros((3, 3))
    gu[0, 2] = alpha
    base = (Cs * Delta) ** 2 * alpha
    assert oracle_lib.smagorinsky(gu, 0.0, Cs, Delta, Prt, True) == pytest.approx(base, rel=1e-15)
    assert oracle_lib.smagorinsky(gu, -1e-4, Cs, Delta, Prt, True) == pytest.approx(base, rel=1e-15)
    N2 = 1e-4
    fb = (1 - N2 / alpha ** 2 / Prt) ** 0.25
    assert oracle_lib.smagorinsky(gu, N2, Cs, Delta, Prt, True) == pytest.approx(base * fb, rel=1e-14)
    assert oracle_lib.smagorinsky(gu, N2, Cs, Delta, Prt, False) == pytest.approx(base, rel=1e-15)
    assert oracle_lib.smagorinsky(gu, 2e-4, Cs, Delta, Prt, True) == 0.0
    assert oracle_lib.smagorinsky(np.zeros((3, 3)), N2, Cs, Delta, Prt, True) == 0.0
    # a pure rotation has no strain
    rot = np.array([[0, -0.3, 0], [0.3, 0, 0], [0, 0, 0]])
    assert oracle_lib.smagorinsky(rot, 0.0, Cs, Delta, Prt, True) == 0.0


def test_shear_closure_through_the_gradient_pipeline(oracle_lib):
    """Linear shear flow on a mesh: F2 momentum flux rho tau_xz = -rho nu alpha
    with the Smagorinsky nu of the closed form (no stratification)."""
    g = {"N": 4, "ne": [2, 2, 3], "lo": [0.0, 0.0, 0.0], "hi": [400.0, 400.0, 600.0], "periodic": [1, 1, 0]}
    G = oracle_lib.Grid(g)
    x = G.coords()
    alpha = 0.01
    n = x.shape[1]
    rho, T = 1.0, 300.0
    Y = W.state_from_primitives(np.full(n, rho * 287.0 * T), np.full(n, T), alpha * x[2], np.zeros(n),
                                np.zeros(n), x[2], g=0.0)
    M = oracle_lib.Model(G, {"nvar": 5, "closure": "smag", "Cs": 0.2, "richardson": False, "g": 0.0})
    _, F2 = M.gradients(Y)
    Delta = (200.0 / 4 * 200.0 / 4 * 200.0 / 4) ** (1 / 3)
    nu = (0.2 * Delta) ** 2 * alpha
    assert np.allclose(F2[1, 2], -rho * nu * alpha, rtol=1e-10)
    assert np.allclose(F2[3, 0], -rho * nu * alpha, rtol=1e-10)
    assert np.allclose(F2[0], 0.0)
