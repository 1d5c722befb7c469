"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
identical seeded inputs (tolerances: tendency 1e-11 relative per variable in
the max norm, state after 100 LSRK54 steps 1e-9)."""
import numpy as np
import pytest

import oracle
from paper_2110_00853_amd import binding as B
from paper_2110_00853_amd import workloads as W
from parity import hmin, rhs_errors, state_errors

pytestmark = pytest.mark.gpu

RHS_TOL = 1e-11
STEP_TOL = 1e-9


def _small(name, ne, hi, **grid_kw):
    c = W.case(name, ne=ne, hi=hi)
    c["grid"].update(grid_kw)
    return c


SMALL_CASES = {
    # the 4^3-element bubble itself (constant nu, walls in z)
    "bubble_4": W.case("bubble_4"),
    # Smagorinsky + Richardson on a ragged element count, 200 m elements
    "smag_ragged": _small("bubble_32", (5, 3, 7), (1000.0, 600.0, 1400.0)),
    # moist, surface fluxes, subsidence, Coriolis
    "moist": _small("moist_64", (4, 4, 6), (400.0, 400.0, 3000.0)),
    # warped terrain-following mesh with sponge
    "warped": _small("agnesi_96", (6, 2, 5), (1500.0, 500.0, 1600.0), topo_a=300.0, topo_xc=750.0, topo_h=200.0),
    # one element, periodic in every direction (its own neighbour), no gravity
    "single_periodic": _small("bubble_32", (1, 1, 1), (200.0, 200.0, 200.0), periodic=[1, 1, 1]),
    # inviscid (no gradient pass)
    "inviscid": _small("bubble_4", (3, 2, 2), (1500.0, 1000.0, 1000.0)),
    # one element layer: bottom and top walls on the same element, Smagorinsky
    "one_layer": _small("bubble_32", (3, 2, 1), (600.0, 400.0, 200.0)),
    # moist on a warped mesh (moist and metric terms together)
    "moist_warped": _small("moist_64", (4, 2, 5), (1500.0, 500.0, 3000.0), topo=1, topo_a=300.0, topo_xc=750.0,
                           topo_h=200.0),
    # moist inviscid: no carried temperature, saturation adjustment at every
    # node and face node of the tendency pass
    "moist_inviscid": _small("moist_64", (3, 2, 4), (300.0, 200.0, 2000.0)),
    # Vreman closure with the Richardson factor, anisotropic elements
    "vreman": _small("bubble_32", (5, 3, 7), (1000.0, 450.0, 1400.0), ),
    # Vreman on a moist warped mesh
    "vreman_moist_warped": _small("moist_64", (4, 2, 5), (1500.0, 500.0, 3000.0), topo=1, topo_a=300.0,
                                  topo_xc=750.0, topo_h=200.0),
    # Roe and HLLC numerical fluxes (dry): flat ragged mesh with Vreman, warped mesh, inviscid
    "roe": _small("bubble_32", (5, 3, 7), (1000.0, 450.0, 1400.0)),
    "hllc": _small("bubble_32", (5, 3, 7), (1000.0, 450.0, 1400.0)),
    "roe_warped": _small("agnesi_96", (6, 2, 5), (1500.0, 500.0, 1600.0), topo_a=300.0, topo_xc=750.0,
                         topo_h=200.0),
    "hllc_warped": _small("agnesi_96", (6, 2, 5), (1500.0, 500.0, 1600.0), topo_a=300.0, topo_xc=750.0,
                          topo_h=200.0),
    "hllc_inviscid": _small("bubble_4", (3, 2, 2), (1500.0, 1000.0, 1000.0)),
}
SMALL_CASES["roe"]["model"].update(closure="vreman", Cs=0.18, flux="roe")
SMALL_CASES["hllc"]["model"].update(closure="vreman", Cs=0.18, flux="hllc")
SMALL_CASES["roe_warped"]["model"].update(flux="roe")
SMALL_CASES["hllc_warped"]["model"].update(flux="hllc")
SMALL_CASES["hllc_inviscid"]["model"].update(closure="none", flux="hllc")
SMALL_CASES["vreman"]["model"].update(closure="vreman", Cs=0.18)
SMALL_CASES["vreman_moist_warped"]["model"].update(closure="vreman", Cs=0.18)
SMALL_CASES["single_periodic"]["model"]["g"] = 0.0
SMALL_CASES["inviscid"]["model"]["closure"] = "none"
SMALL_CASES["moist_inviscid"]["model"]["closure"] = "none"


def _state(c, seed=11):
    if c.get("name") == "bubble_4" and c["grid"]["ne"] == [4, 4, 4]:
        Y, Yref, _ = W.initial_state(c)
        return Y, Yref
    Y, Yref, _ = W.perturbed_state(c, seed=seed, amp_u=6.0, amp_T=2.0, amp_q=1.5e-3)
    if c["model"].get("g", 9.81) == 0.0:
        Yref = None
    return Y, Yref


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available()
    B.load()
    return torch


@pytest.mark.parametrize("name", list(SMALL_CASES))
def test_grid_geometry_matches_oracle(dev, name):
    c = SMALL_CASES[name]
    g = B.Grid(c["grid"])
    og = oracle.Grid(c["grid"])
    assert np.allclose(g.coords(), og.coords(), rtol=0, atol=1e-9)
    Ja, J = g.metrics()
    oJa, oJ = og.metrics()
    assert np.allclose(J, oJ, rtol=1e-12)
    assert np.allclose(Ja, oJa, rtol=1e-12, atol=1e-12 * np.abs(oJa).max())
    assert np.allclose(g.wJ(), og.wJ(), rtol=1e-12)


@pytest.mark.parametrize("name", list(SMALL_CASES))
def test_rhs_fp64_matches_oracle(dev, name):
    c = SMALL_CASES[name]
    Y, Yref = _state(c)
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref)
    Yd = m.new_state(Y)
    Rd = m.new_state()
    m.rhs(Yd, Rd)
    dev.cuda.synchronize()
    Rg = m.tendency_to_numpy(Rd)
    Rref = oracle.Model(oracle.Grid(c["grid"]), c["model"], Yref).rhs(Y)
    err = rhs_errors(Rg, Rref, Y, hmin(c["grid"]))
    print(name, "rhs errors per variable", err)
    assert np.all(np.isfinite(Rg))
    assert np.all(err < RHS_TOL), err


@pytest.mark.parametrize("name", ["bubble_4", "moist", "warped", "moist_warped", "moist_inviscid", "vreman",
                                  "vreman_moist_warped", "roe", "hllc", "roe_warped", "hllc_inviscid"])
def test_lsrk_step_matches_oracle(dev, name):
    c = SMALL_CASES[name]
    Y, Yref = _state(c)
    _, _, speed = W.perturbed_state(c, seed=11, amp_u=6.0, amp_T=2.0, amp_q=1.5e-3)
    dt = W.cfl_dt(c["grid"], speed)
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref)
    Ya, Yb, dQ = m.new_state(Y), m.new_state(), m.new_state()
    nsteps = 3
    for _ in range(nsteps):
        m.lsrk_step(Ya, Yb, dQ, 0.0, dt)
        Ya, Yb = Yb, Ya
    dev.cuda.synchronize()
    Yg = m.to_numpy(Ya)
    Yo, _ = oracle.Model(oracle.Grid(c["grid"]), c["model"], Yref).steps(Y, dt, nsteps)
    err = state_errors(Yg, Yo)
    print(name, "state errors after", nsteps, "steps", err)
    assert np.all(err < 1e-10), err


@pytest.mark.parametrize("name", ["bubble_4", "smag_ragged", "moist", "warped", "moist_inviscid", "roe", "hllc"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lsrk144_step_matches_oracle(dev, name, precision):
    """LSRK144 (fourteen fused stages, new state back in the input buffer)
    against the oracle's: FP64 at 1e-10 after 3 steps; FP32-bulk at 2e-3
    (measured at most 2.5e-4: FP32 flux arithmetic on deviations stored in
    FP32 from the background)."""
    c = SMALL_CASES[name]
    Y, Yref = _state(c)
    _, _, speed = W.perturbed_state(c, seed=11, amp_u=6.0, amp_T=2.0, amp_q=1.5e-3)
    dt = 2.0 * W.cfl_dt(c["grid"], speed)
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref, precision=precision)
    Ya, Yb, dQ = m.new_state(Y), m.new_state(), m.new_state()
    nsteps = 3
    for _ in range(nsteps):
        m.lsrk144_step(Ya, Yb, dQ, 0.0, dt)
    dev.cuda.synchronize()
    Yg = m.to_numpy(Ya).astype(np.float64)
    Yo, _ = oracle.Model(oracle.Grid(c["grid"]), c["model"], Yref).steps(Y, dt, nsteps, scheme="lsrk144")
    err = state_errors(Yg, Yo)
    print(name, precision, "LSRK144 state errors after", nsteps, "steps", err)
    assert np.all(err < (1e-10 if precision == "fp64" else 2e-3)), err


def test_bubble_4_hundred_steps(dev):
    """The 4^3-element dry bubble: state after 100 LSRK54 steps within 1e-9."""
    c = W.case("bubble_4")
    Y, Yref, dt = W.initial_state(c)
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref)
    Ya, Yb, dQ = m.new_state(Y), m.new_state(), m.new_state()
    for _ in range(100):
        m.lsrk_step(Ya, Yb, dQ, 0.0, dt)
        Ya, Yb = Yb, Ya
    dev.cuda.synchronize()
    Yg = m.to_numpy(Ya)
    Yo, _ = oracle.Model(oracle.Grid(c["grid"]), c["model"], Yref).steps(Y, dt, 100)
    err = state_errors(Yg, Yo)
    change = np.array([np.abs(Yo[v] - Y[v]).max() for v in range(5)])
    print("100-step state errors", err, "relative to the change", err * np.abs(Yo).max(axis=1) / change)
    assert np.all(err < STEP_TOL), err


def test_moist_hundred_steps(dev):
    """The small moist case (saturated nodes, surface fluxes, subsidence,
    Coriolis) after 100 LSRK54 steps within 1e-9: the temperature the
    tendency pass hands to the next stage must not drift from the oracle's
    saturation adjustment."""
    c = SMALL_CASES["moist"]
    Y, Yref = _state(c)
    _, _, speed = W.perturbed_state(c, seed=11, amp_u=6.0, amp_T=2.0, amp_q=1.5e-3)
    dt = W.cfl_dt(c["grid"], speed)
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref)
    Ya, Yb, dQ = m.new_state(Y), m.new_state(), m.new_state()
    for _ in range(100):
        m.lsrk_step(Ya, Yb, dQ, 0.0, dt)
        Ya, Yb = Yb, Ya
    dev.cuda.synchronize()
    Yg = m.to_numpy(Ya)
    Yo, _ = oracle.Model(oracle.Grid(c["grid"]), c["model"], Yref).steps(Y, dt, 100)
    _, _, ql, _ = oracle.thermo_nodes(Yo, W.node_coords(c["grid"])[2], c["model"].get("g", 9.81))
    err = state_errors(Yg, Yo)
    print("moist 100-step state errors", err, "saturated nodes at the end:", int(np.sum(ql > 0)))
    assert np.sum(ql > 0) > 0
    assert np.all(err < STEP_TOL), err


def test_diagnostics_match_oracle_integrals(dev):
    c = SMALL_CASES["moist"]
    Y, Yref = _state(c)
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref)
    d = m.diagnostics(m.new_state(Y), dt=0.1)
    ref = oracle.Model(oracle.Grid(c["grid"]), c["model"], Yref).integrals(Y)
    assert d["mass"] == pytest.approx(ref[0], rel=1e-14)
    assert d["energy"] == pytest.approx(ref[4], rel=1e-14)
    assert d["water"] == pytest.approx(ref[5], rel=1e-14)
    assert d["ke"] == pytest.approx(ref[6], rel=1e-13)
    T, p, ql, thv = oracle.thermo_nodes(Y, oracle.Grid(c["grid"]).coords()[2], 9.81)
    assert d["T_min"] == pytest.approx(T.min(), rel=1e-12)
    assert d["T_max"] == pytest.approx(T.max(), rel=1e-12)
    assert d["n_nonfinite"] == 0 and d["status"] == B.CM_OK


def test_nonfinite_state_is_reported(dev):
    c = SMALL_CASES["inviscid"]
    Y, Yref = _state(c)
    Y = Y.copy()
    Y[4, 17] = np.nan
    Y[2, 3] = np.inf
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref)
    d = m.diagnostics(m.new_state(Y))
    assert d["status"] == B.CM_ERR_NONFINITE and d["n_nonfinite"] == 2


def test_conservation_on_gpu_closed_box(dev):
    """Mass and total energy conserved to round-off over 50 steps on the GPU
    (moist, walls in z, Smagorinsky + Richardson, no surface fluxes)."""
    c = _small("moist_64", (3, 3, 4), (300.0, 300.0, 2000.0))
    for key in ("sfc_flux", "subsidence"):
        c["model"].pop(key, None)
    Y, Yref, speed = W.perturbed_state(c, seed=3, amp_u=4.0, amp_T=1.0, amp_q=1e-3)
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref)
    Ya, Yb, dQ = m.new_state(Y), m.new_state(), m.new_state()
    d0 = m.diagnostics(Ya)
    for _ in range(50):
        m.lsrk_step(Ya, Yb, dQ, 0.0, W.cfl_dt(c["grid"], speed))
        Ya, Yb = Yb, Ya
    d1 = m.diagnostics(Ya)
    for k in ("mass", "energy", "water"):
        assert abs(d1[k] - d0[k]) / abs(d0[k]) < 1e-14, (k, d0[k], d1[k])
    assert np.abs(m.to_numpy(Ya) - Y).max() > 1e-4


def test_fp32_bulk_rhs_error_is_stated(dev):
    """FP32-bulk tendency against the FP64 oracle: error stated, bounded at
    1e-3 (measured at most 1.2e-4, moist)."""
    for name in ("smag_ragged", "moist", "warped", "moist_warped"):
        c = SMALL_CASES[name]
        Y, Yref = _state(c)
        g = B.Grid(c["grid"])
        m = B.Model(g, c["model"], Yref, precision="fp32")
        Yd = m.new_state(Y)
        Rd = m.new_state()
        m.rhs(Yd, Rd)
        dev.cuda.synchronize()
        Rg = m.tendency_to_numpy(Rd).astype(np.float64)
        Rref = oracle.Model(oracle.Grid(c["grid"]), c["model"], Yref).rhs(Y)
        err = rhs_errors(Rg, Rref, Y, hmin(c["grid"]))
        print(name, "fp32-bulk rhs errors per variable", err)
        assert np.all(np.isfinite(Rg)) and np.all(err < 1e-3), err


@pytest.mark.parametrize("name", ["smag_ragged", "moist", "warped"])
def test_fp32_state_storage_round_trip(dev, name):
    """FP32-bulk storage holds float(Y - Y_bg): importing the background
    gives exact zeros, and a state comes back within float rounding of its
    deviation from the background (not of its full value); FP64 storage
    round-trips exactly."""
    c = SMALL_CASES[name]
    Y, Yref = _state(c)
    assert Yref is not None
    g = B.Grid(c["grid"])
    m32 = B.Model(g, c["model"], Yref, precision="fp32")
    assert bool((m32.new_state(Yref) == 0).all())
    back = m32.to_numpy(m32.new_state(Y))
    # float rounding of the deviation, plus the FP64 subtraction and addition
    bound = 2.0 ** -24 * np.abs(Y - Yref) + 2.0 ** -51 * np.abs(Y)
    assert np.all(np.abs(back - Y) <= bound)
    assert np.abs(Y - Yref).max() > 1e-3      # a real deviation was stored
    m64 = B.Model(g, c["model"], Yref)
    assert np.array_equal(m64.to_numpy(m64.new_state(Y)), Y)


def test_state_padding_contract(dev):
    """State buffers hold element runs of 160 slots: the padding of an input
    is never read (NaN there changes nothing), and outputs get zeros in
    slots 125..127 and leave 128..159 untouched."""
    torch = dev
    c = SMALL_CASES["smag_ragged"]
    Y, Yref = _state(c)
    g = B.Grid(c["grid"])
    assert g.state_stride == 160 * g.n_elem and g.srun == 160
    m = B.Model(g, c["model"], Yref)
    Yd = m.new_state(Y)
    R0 = m.new_state()
    m.rhs(Yd, R0)
    Ynan = Yd.clone().view(m.nvar, g.n_elem, 160)
    Ynan[:, :, 125:] = float("nan")
    R1 = torch.full((m.nvar, g.state_stride), float("nan"), dtype=torch.float64, device=Yd.device)
    m.rhs(Ynan.view(m.nvar, g.state_stride), R1)
    Ya = torch.full_like(R1, float("nan"))
    dQ = torch.full_like(R1, float("nan"))
    m.lsrk_step(Ynan.view(m.nvar, g.state_stride), Ya, dQ, 0.0, 0.01)
    torch.cuda.synchronize()
    r0 = R0.view(m.nvar, g.n_elem, 160).cpu().numpy()
    r1 = R1.view(m.nvar, g.n_elem, 160).cpu().numpy()
    assert np.array_equal(r0[:, :, :125], r1[:, :, :125])      # bit-identical tendency
    for T in (R1, Ya, dQ):
        a = T.view(m.nvar, g.n_elem, 160).cpu().numpy()
        assert np.all(np.isfinite(a[:, :, :125]))
        assert np.all(a[:, :, 125:128] == 0.0)
        assert np.all(np.isnan(a[:, :, 128:]))


def test_moist_model_rejects_roe_and_hllc(dev):
    c = SMALL_CASES["moist"]
    g = B.Grid(c["grid"])
    for flux in ("roe", "hllc"):
        with pytest.raises(B.CMError) as ei:
            B.Model(g, dict(c["model"], flux=flux))
        assert ei.value.status == B.CM_ERR_UNSUPPORTED


def _cold_moist_state(c, seed=12):
    """A cold moist state for the ice phase: pressure of an isothermal 250 K
    column, temperature falling from 280 K at the ground to 225 K at 3 km
    with smooth +-3 K and velocity perturbations, total water about twice
    the vapour that saturates over liquid, so that condensate forms all
    liquid, on the liquid-fraction ramp (233-273.15 K) and all ice."""
    xyz = W.node_coords(c["grid"])
    z = xyz[2]
    rng = np.random.default_rng(seed)
    p, T = W.isothermal(z, 250.0)
    zero = np.zeros_like(z)
    Yref = W.state_from_primitives(p, T, zero, zero, zero, z, qt=np.full_like(z, 1.0e-3))
    noise = lambda: W._smooth_noise(xyz, c["grid"], rng)  # noqa: E731
    Tp = 280.0 - 55.0 * z / 3000.0 + 3.0 * noise()
    qs = W.pvsat(Tp) / ((p - W.pvsat(Tp)) / (287.0 * Tp) * 462.0 * Tp)
    qt = qs * (2.0 + 0.5 * noise())
    Y = W.state_from_primitives(p, Tp, 5.0 * noise(), 5.0 * noise(), 5.0 * noise(), z, qt=qt)
    return Y, Yref


ICE_CASES = {
    "ice": _small("moist_64", (4, 3, 4), (400.0, 300.0, 3000.0)),
    "ice_warped": _small("moist_64", (4, 2, 4), (1500.0, 500.0, 3000.0), topo=1, topo_a=300.0, topo_xc=750.0,
                         topo_h=200.0),
    "ice_inviscid": _small("moist_64", (3, 2, 4), (300.0, 200.0, 3000.0)),
}
for _c in ICE_CASES.values():
    _c["model"]["ice"] = True
ICE_CASES["ice_inviscid"]["model"]["closure"] = "none"


@pytest.mark.parametrize("name", list(ICE_CASES))
def test_ice_phase_rhs_and_steps_match_oracle(dev, name):
    c = ICE_CASES[name]
    Y, Yref = _cold_moist_state(c)
    # the state holds condensate on both sides of the liquid-fraction ramp
    T, _, qc, _ = oracle.thermo_nodes(Y, W.node_coords(c["grid"])[2], 9.81, ice=True)
    assert (qc > 0).mean() > 0.3 and T.min() < 233.0 and T.max() > 273.15
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref)
    om = oracle.Model(oracle.Grid(c["grid"]), c["model"], Yref)
    Yd, Rd = m.new_state(Y), m.new_state()
    m.rhs(Yd, Rd)
    dev.cuda.synchronize()
    err = rhs_errors(m.tendency_to_numpy(Rd), om.rhs(Y), Y, hmin(c["grid"]))
    print(name, "ice-phase rhs errors", err)
    assert np.all(err < RHS_TOL), err
    dt = W.cfl_dt(c["grid"], 360.0)
    Ya, Yb, dQ = m.new_state(Y), m.new_state(), m.new_state()
    for _ in range(3):
        m.lsrk_step(Ya, Yb, dQ, 0.0, dt)
        Ya, Yb = Yb, Ya
    dev.cuda.synchronize()
    Yo, _ = om.steps(Y, dt, 3)
    serr = state_errors(m.to_numpy(Ya), Yo)
    print(name, "ice-phase state errors after 3 steps", serr)
    assert np.all(serr < 1e-10), serr
    # without the ice phase the same state evolves differently
    Rl = oracle.Model(oracle.Grid(c["grid"]), dict(c["model"], ice=False), Yref).rhs(Y)
    assert np.abs(Rl - om.rhs(Y)).max() > 1e-6 * np.abs(Rl).max()


def test_ice_phase_rejects_the_learned_closure(dev):
    c = ICE_CASES["ice"]
    g = B.Grid(c["grid"])
    with pytest.raises(B.CMError) as ei:
        B.Model(g, dict(c["model"], closure="mlp"))
    assert ei.value.status == B.CM_ERR_UNSUPPORTED
