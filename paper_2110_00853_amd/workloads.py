"""Seeded synthetic workloads: meshes, model settings and initial states.

This module is the only code that feeds both the GPU library and the CPU
oracle.  It builds *inputs*: node coordinates from the mesh definition, and
prognostic states from prescribed primitive profiles (pressure, temperature,
velocity, total water).  It holds none of the right-hand-side arithmetic and
imports neither the GPU binding nor the oracle.

State layout: float64 array [nvar, n_nodes], variables (rho, rho u, rho v,
rho w, rho e_tot[, rho q_t]); node order element-major, element = ex + ne0*(ey
+ ne1*ez), node = i + Q*(j + Q*k) with i along x.

Constants are Table 1 of the paper (Sect. 2.5) plus the stated readings for
g, p0, c_pd = c_vd + R_d and the triple-point pressure of water.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# Table 1 and readings (kept private to this module)
_RD, _RV = 287.0, 462.0
_CVD, _CVV, _CVL = 717.5, 1397.5, 4181.0
_T0 = 273.16
_LV0 = 2.5008e6
_G = 9.81
_P0 = 1.0e5
_CPD = _CVD + _RD
_CPV = _CVV + _RV
_PTR = 611.657
_IV0 = _LV0 - _RV * _T0
_KAPPA = _RD / _CPD


# --------------------------------------------------------------------------
# mesh
# --------------------------------------------------------------------------
def gll_points(N: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points on [-1, 1]: +-1 and the roots of P_N'."""
    from numpy.polynomial import legendre as L

    c = np.zeros(N + 1)
    c[N] = 1.0
    inner = np.sort(np.real(L.legroots(L.legder(c)))) if N > 1 else np.array([])
    pts = np.concatenate([[-1.0], inner, [1.0]])
    if N % 2 == 0:
        pts[N // 2] = 0.0
    return pts


def n_nodes(grid: dict) -> int:
    Q = grid.get("N", 4) + 1
    ne = grid["ne"]
    return int(ne[0] * ne[1] * ne[2] * Q ** 3)


def node_coords(grid: dict) -> np.ndarray:
    """Node coordinates [3, n_nodes] from the brick mesh and optional warp.

    Terrain following (Gal-Chen & Somerville linear decay): z = zh + z_sfc(x)
    (z_top - zh)/(z_top - z_lo), with the Agnesi ridge z_sfc = h a^2/((x -
    x_c)^2 + a^2) (Sect. 5.4, eq. agnesi).
    """
    N = grid.get("N", 4)
    Q = N + 1
    ne = grid["ne"]
    lo, hi = np.asarray(grid["lo"], float), np.asarray(grid["hi"], float)
    h = (hi - lo) / np.asarray(ne, float)
    xi = gll_points(N)
    s = (1.0 + xi) / 2.0
    ex = np.arange(ne[0])
    ey = np.arange(ne[1])
    ez = np.arange(ne[2])
    # axes ordered [ez, ey, ex, k, j, i]
    X = lo[0] + (ex[None, None, :, None, None, None] + s[None, None, None, None, None, :]) * h[0]
    Y = lo[1] + (ey[None, :, None, None, None, None] + s[None, None, None, None, :, None]) * h[1]
    Z = lo[2] + (ez[:, None, None, None, None, None] + s[None, None, None, :, None, None]) * h[2]
    shape = (ne[2], ne[1], ne[0], Q, Q, Q)
    X, Y, Z = (np.broadcast_to(a, shape).reshape(-1).copy() for a in (X, Y, Z))
    if grid.get("topo", 0) == 1:
        r = X - grid["topo_xc"]
        zs = grid["topo_h"] * grid["topo_a"] ** 2 / (r * r + grid["topo_a"] ** 2)
        Z = Z + zs * (hi[2] - Z) / (hi[2] - lo[2])
    return np.stack([X, Y, Z])


def min_node_spacing(grid: dict) -> float:
    N = grid.get("N", 4)
    xi = gll_points(N)
    h = (np.asarray(grid["hi"], float) - np.asarray(grid["lo"], float)) / np.asarray(grid["ne"], float)
    return float(np.min(h) * np.min(np.diff(xi)) / 2.0)


# --------------------------------------------------------------------------
# state construction from primitive fields
# --------------------------------------------------------------------------
def pvsat(T):
    """Saturation vapour pressure over liquid (closed-form Clausius-Clapeyron,
    constant heat capacities); used only to build moist initial states."""
    dc = _CPV - _CVL
    return _PTR * (T / _T0) ** (dc / _RV) * np.exp((_LV0 - dc * _T0) / _RV * (1.0 / _T0 - 1.0 / T))


def state_from_primitives(p, T, u, v, w, z, qt=None, g=_G):
    """Conserved state from pressure, temperature, velocity (and total water).

    Moist air is put in equilibrium: q_l = max(0, q_t - q_v*) with the density
    that makes p = rho R_m T hold for the saturated vapour pressure.
    """
    p, T, u, v, w, z = (np.asarray(a, float) for a in (p, T, u, v, w, z))
    ke = 0.5 * (u * u + v * v + w * w)
    if qt is None:
        rho = p / (_RD * T)
        I = _CVD * (T - _T0)
        e = ke + g * z + I
        return np.stack([rho, rho * u, rho * v, rho * w, rho * e])
    qt = np.asarray(qt, float)
    rho_u = p / ((_RD * (1.0 - qt) + _RV * qt) * T)      # unsaturated guess
    qvs_u = pvsat(T) / (rho_u * _RV * T)
    sat = qt > qvs_u
    rho_s = (p - pvsat(T)) / (_RD * (1.0 - qt) * T)
    rho = np.where(sat, rho_s, rho_u)
    qv = np.where(sat, pvsat(T) / (rho * _RV * T), qt)
    ql = qt - qv
    I = (1.0 - qt) * _CVD * (T - _T0) + qv * (_CVV * (T - _T0) + _IV0) + ql * _CVL * (T - _T0)
    e = ke + g * z + I
    return np.stack([rho, rho * u, rho * v, rho * w, rho * e, rho * qt])


def sound_speed_dry(T):
    return np.sqrt(_CPD / _CVD * _RD * np.asarray(T, float))


def cfl_dt(grid: dict, speed_max: float, cfl: float = 0.4) -> float:
    """Time step cfl * (minimum GLL node spacing) / max(|u| + c).

    The paper states no time-step rule.  A Courant number of 0.4 on the
    minimum GLL spacing is used: 0.8 is unstable for the 3-D N=4 operator
    with LSRK54 (it diverges within ten steps on the 4^3 bubble)."""
    return cfl * min_node_spacing(grid) / speed_max


# --------------------------------------------------------------------------
# background profiles
# --------------------------------------------------------------------------
def isothermal(z, T_iso=300.0, g=_G):
    """Isothermal hydrostatic profile: p = p0 exp(-g z / (R_d T))."""
    z = np.asarray(z, float)
    return _P0 * np.exp(-g * z / (_RD * T_iso)), np.full_like(z, T_iso)


def neutral(z, theta0=300.0, g=_G):
    """Uniform potential temperature (eq. pressureDistrib)."""
    z = np.asarray(z, float)
    p = _P0 * (1.0 - g * z / (_CPD * theta0)) ** (_CPD / _RD)
    T = theta0 * (p / _P0) ** _KAPPA
    return p, T


def constant_N(z, theta_sfc=300.0, Nbv=0.01, p_sfc=1.0e5, g=_G):
    """Constant Brunt-Vaisala background (eq. pressure_hs_brunt; density by the
    ideal-gas law with T = theta (p/p_sfc)^(R_d/c_pd))."""
    z = np.asarray(z, float)
    theta = theta_sfc * np.exp(Nbv * Nbv / g * z)
    p = p_sfc * (1.0 + g * g / (_CPD * theta_sfc * Nbv * Nbv) * (np.exp(-z * Nbv * Nbv / g) - 1.0)) ** (_CPD / _RD)
    T = theta * (p / p_sfc) ** _KAPPA
    return p, T


def _moist_T_from_thetal(p, thl, qt, T_guess=None, half_width=None, iters=100):
    """Temperature from liquid-water potential temperature at pressure p:
    the root of T - Pi theta_l - L_v0 q_l(T)/c_pd by bisection (bracket
    [Pi theta_l, Pi theta_l + L_v0 q_t/c_pd + 1], or T_guess +- half_width)."""
    Pi = (p / _P0) ** _KAPPA
    if T_guess is None:
        lo = Pi * thl
        hi = lo + _LV0 * qt / _CPD + 1.0
    else:
        lo, hi = T_guess - half_width, T_guess + half_width

    def resid(T):
        ps = pvsat(T)
        qv = ps * _RD * (1.0 - qt) / ((p - ps) * _RV)   # p_v*/(rho_s R_v T), rho_s = (p - p_v*)/(R_d (1-q_t) T)
        ql = np.maximum(qt - qv, 0.0)
        return T - Pi * thl - _LV0 * ql / _CPD

    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        r = resid(mid)
        lo = np.where(r < 0.0, mid, lo)
        hi = np.where(r < 0.0, hi, mid)
    return 0.5 * (lo + hi)


def shallow_cumulus_profiles(zq):
    """Synthetic shallow-convection profiles (liquid potential temperature and
    total water) at heights zq: well mixed to 520 m (298.7 K, 17 g/kg), then a
    stable layer with d theta/dz = 3.85 K/km and q_t falling linearly to 5 g/kg
    at 3 km."""
    zq = np.asarray(zq, float)
    thl = np.where(zq <= 520.0, 298.7, 298.7 + 3.85e-3 * (zq - 520.0))
    qt = np.where(zq <= 520.0, 17.0e-3, 17.0e-3 + (5.0e-3 - 17.0e-3) * (zq - 520.0) / (3000.0 - 520.0))
    return thl, qt


def moist_hydrostatic(z, g=_G, p_sfc=_P0, nsub=4):
    """Integrate dp/dz = -rho g for the shallow-cumulus profiles (RK4 over the
    sorted unique node heights, nsub substeps per interval); returns p, T, q_t
    at every height in z."""
    z = np.asarray(z, float)
    levels, inv = np.unique(np.concatenate([[0.0], z]), return_inverse=True)

    def dpdz(zz, pp):
        thl, qt = shallow_cumulus_profiles(np.array([zz]))
        T = _moist_T_from_thetal(np.array([pp]), thl, qt)
        Y = state_from_primitives(np.array([pp]), T, 0 * T, 0 * T, 0 * T, np.array([zz]), qt=qt, g=g)
        return -Y[0, 0] * g

    pl = np.zeros_like(levels)
    pl[0] = p_sfc
    p = p_sfc
    for a in range(1, levels.size):
        z0, z1 = levels[a - 1], levels[a]
        hstep = (z1 - z0) / nsub
        zz = z0
        for _ in range(nsub):
            k1 = dpdz(zz, p)
            k2 = dpdz(zz + hstep / 2, p + hstep / 2 * k1)
            k3 = dpdz(zz + hstep / 2, p + hstep / 2 * k2)
            k4 = dpdz(zz + hstep, p + hstep * k3)
            p = p + hstep / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            zz += hstep
        pl[a] = p
    thl_l, qt_l = shallow_cumulus_profiles(levels)
    T_l = _moist_T_from_thetal(pl, thl_l, qt_l)
    idx = inv[1:]
    return pl[idx], T_l[idx], qt_l[idx]


# --------------------------------------------------------------------------
# model / grid settings of the benchmark cases
# --------------------------------------------------------------------------
def _grid(ne, hi, periodic=(1, 1, 0), lo=(0.0, 0.0, 0.0), **kw):
    g = {"N": 4, "ne": list(ne), "lo": list(lo), "hi": list(hi), "periodic": list(periodic)}
    g.update(kw)
    return g


CASES = {
    # dry bubble, 4^3 elements on a 2 km cube, constant nu = 75
    "bubble_4": {
        "grid": _grid((4, 4, 4), (2000.0, 2000.0, 2000.0)),
        "model": {"nvar": 5, "closure": "const", "nu": 75.0, "Prt": 1.0 / 3.0, "g": _G},
        "ic": {"kind": "bubble", "center": (1000.0, 1000.0, 500.0)},
    },
    # dry bubble at scale, 32^3 elements on a 6.4 km cube, Smagorinsky-Lilly + Ri
    "bubble_32": {
        "grid": _grid((32, 32, 32), (6400.0, 6400.0, 6400.0)),
        "model": {"nvar": 5, "closure": "smag", "Cs": 0.21, "Prt": 1.0 / 3.0, "richardson": True, "g": _G},
        "ic": {"kind": "bubble", "center": (3200.0, 3200.0, 500.0)},
    },
    # moist shallow convection, 64x64x30 elements on 6.4 x 6.4 x 3 km
    "moist_64": {
        "grid": _grid((64, 64, 30), (6400.0, 6400.0, 3000.0)),
        "model": {"nvar": 6, "closure": "smag", "Cs": 0.21, "Prt": 1.0 / 3.0, "richardson": True, "g": _G,
                  "f_cor": 1.0e-4, "u_g": -10.0, "v_g": 0.0,
                  "sfc_flux": {"theta_flux": 8.0e-3, "qt_flux": 5.2e-5},
                  "subsidence": {"w0": 5.0e-3, "z_top": 3000.0}},
        "ic": {"kind": "moist", "seed": 20211001},
    },
    # flow over an Agnesi hill on a warped mesh, 96x16x50 elements, 24 x 4 x 16 km
    "agnesi_96": {
        "grid": _grid((96, 16, 50), (24000.0, 4000.0, 16000.0), topo=1, topo_h=400.0, topo_a=1000.0,
                      topo_xc=12000.0),
        "model": {"nvar": 5, "closure": "smag", "Cs": 0.21, "Prt": 1.0 / 3.0, "richardson": True, "g": _G,
                  "sponge": {"z_s": 11000.0, "z_top": 16000.0, "alpha": 0.5, "gamma": 2.0,
                             "u_relax": (10.0, 0.0, 0.0)}},
        "ic": {"kind": "agnesi", "u0": 10.0, "Nbv": 0.01},
    },
    # 2.5-D density current (Sect. 5.2): [0, 25.6 km] x one 200 m element
    # (periodic) x [0, 6.4 km], free-slip walls in x and z, 50 m effective
    # resolution (200 m elements, N = 4), constant nu = 75 m^2/s with
    # Pr = 1 (the classical set-up the front-location table quotes)
    "density_current": {
        "grid": _grid((128, 1, 32), (25600.0, 200.0, 6400.0), periodic=(0, 1, 0)),
        "model": {"nvar": 5, "closure": "const", "nu": 75.0, "Prt": 1.0, "g": _G},
        "ic": {"kind": "density_current", "theta0": 300.0, "theta_c": -15.0, "center": (0.0, 3000.0),
               "radii": (4000.0, 2000.0)},
    },
}
CASES["learned_32"] = copy.deepcopy(CASES["bubble_32"])
CASES["learned_32"]["model"]["closure"] = "mlp"


def case(name: str, ne=None, hi=None, **model_overrides) -> dict:
    """A copy of a named case, optionally on a different element count/box."""
    c = copy.deepcopy(CASES[name])
    c["name"] = name
    if ne is not None:
        c["grid"]["ne"] = list(ne)
    if hi is not None:
        c["grid"]["hi"] = list(hi)
    c["model"].update(model_overrides)
    return c


# --------------------------------------------------------------------------
# initial states
# --------------------------------------------------------------------------
def _smooth_noise(xyz, grid, rng, nmodes=3):
    """Smooth random-phase field, periodic over the box, unit amplitude."""
    lo, hi = np.asarray(grid["lo"], float), np.asarray(grid["hi"], float)
    L = hi - lo
    f = np.zeros(xyz.shape[1])
    for _ in range(nmodes):
        k = rng.integers(1, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        a = rng.uniform(0.5, 1.0)
        f += a * np.prod([np.cos(2 * np.pi * k[d] * (xyz[d] - lo[d]) / L[d] + ph[d]) for d in range(3)], axis=0)
    return f / nmodes


def bubble_state(grid: dict, center, r0=500.0, dtheta=1.0, T_iso=300.0, g=_G, xyz=None):
    """Isothermal background plus a cosine-bell potential-temperature bubble
    dtheta (1 + cos(pi r/r0)) applied at fixed pressure."""
    xyz = node_coords(grid) if xyz is None else xyz
    z = xyz[2]
    p, T = isothermal(z, T_iso, g)
    r = np.sqrt(sum((xyz[d] - center[d]) ** 2 for d in range(3)))
    dth = np.where(r <= r0, dtheta * (1.0 + np.cos(np.pi * r / r0)), 0.0)
    Tp = T + dth * (p / _P0) ** _KAPPA
    zero = np.zeros_like(z)
    Y = state_from_primitives(p, Tp, zero, zero, zero, z, g=g)
    Yref = state_from_primitives(p, T, zero, zero, zero, z, g=g)
    return Y, Yref, float(np.max(sound_speed_dry(Tp)))


def density_current_state(grid: dict, theta0=300.0, theta_c=-15.0, center=(0.0, 3000.0),
                          radii=(4000.0, 2000.0), g=_G, xyz=None):
    """Neutral hydrostatic background (uniform theta0) plus the cold bubble
    dtheta = theta_c/2 (1 + cos(pi r)) for r <= 1, r = |((x - x_c)/r_x,
    (z - z_c)/r_z)| (Sect. 5.2, eq. densityCurrentEqn, reading the printed
    radius as the usual elliptic distance), applied at fixed pressure; the
    flow starts at rest."""
    xyz = node_coords(grid) if xyz is None else xyz
    z = xyz[2]
    p, T = neutral(z, theta0, g)
    r = np.sqrt(((xyz[0] - center[0]) / radii[0]) ** 2 + ((z - center[1]) / radii[1]) ** 2)
    dth = np.where(r <= 1.0, 0.5 * theta_c * (1.0 + np.cos(np.pi * r)), 0.0)
    Tp = T + dth * (p / _P0) ** _KAPPA
    zero = np.zeros_like(z)
    Y = state_from_primitives(p, Tp, zero, zero, zero, z, g=g)
    Yref = state_from_primitives(p, T, zero, zero, zero, z, g=g)
    return Y, Yref, float(np.max(sound_speed_dry(T)))


def perturbed_state(c: dict, seed: int = 0, amp_u=5.0, amp_T=1.0, amp_q=1.0e-3, xyz=None):
    """Background of case c plus smooth random velocity / temperature (and
    moisture) perturbations: a generic state for parity tests."""
    grid, model = c["grid"], c["model"]
    xyz = node_coords(grid) if xyz is None else xyz
    g = model.get("g", _G)
    rng = np.random.default_rng(seed)
    z = xyz[2]
    kind = c["ic"]["kind"]
    qt = None
    if kind == "moist":
        p, T, qt = moist_hydrostatic(z, g=g)
    elif kind == "agnesi":
        p, T = constant_N(z, Nbv=c["ic"]["Nbv"], g=g)
    else:
        p, T = isothermal(z, 300.0, g)
    zero = np.zeros_like(z)
    Yref = state_from_primitives(p, T, zero, zero, zero, z, qt=qt, g=g)
    u = amp_u * _smooth_noise(xyz, grid, rng)
    v = amp_u * _smooth_noise(xyz, grid, rng)
    w = amp_u * _smooth_noise(xyz, grid, rng)
    Tp = T + amp_T * _smooth_noise(xyz, grid, rng)
    qp = None
    if qt is not None:
        qp = np.clip(qt + amp_q * _smooth_noise(xyz, grid, rng), 1e-4, None)
    if kind == "agnesi":
        u = u + c["ic"]["u0"]
    Y = state_from_primitives(p, Tp, u, v, w, z, qt=qp, g=g)
    speed = float(np.max(np.sqrt(u * u + v * v + w * w) + sound_speed_dry(Tp)))
    return Y, Yref, speed


def initial_state(c: dict, xyz=None):
    """Initial state, reference (background) state and stable time step of
    a named case.  Returns (Y, Yref, dt)."""
    grid, model = c["grid"], c["model"]
    xyz = node_coords(grid) if xyz is None else xyz
    g = model.get("g", _G)
    ic = c["ic"]
    z = xyz[2]
    zero = np.zeros_like(z)
    if ic["kind"] == "bubble":
        Y, Yref, cmax = bubble_state(grid, ic["center"], dtheta=ic.get("dtheta", 1.0), g=g, xyz=xyz)
        return Y, Yref, cfl_dt(grid, cmax)
    if ic["kind"] == "density_current":
        Y, Yref, cmax = density_current_state(grid, ic["theta0"], ic["theta_c"], ic["center"], ic["radii"],
                                              g=g, xyz=xyz)
        return Y, Yref, cfl_dt(grid, cmax)
    if ic["kind"] == "moist":
        p, T, qt = moist_hydrostatic(z, g=g)
        u = np.full_like(z, model.get("u_g", 0.0))
        Yref = state_from_primitives(p, T, zero, zero, zero, z, qt=qt, g=g)
        rng = np.random.default_rng(ic["seed"])
        low = z < 1600.0
        n = z.size
        dth = np.where(low, rng.uniform(-0.1, 0.1, n), 0.0)
        dq = np.where(low, rng.uniform(-0.025e-3, 0.025e-3, n), 0.0)
        thl, qt0 = shallow_cumulus_profiles(z)
        qtp = qt0 + dq
        Tp = T.copy()
        if low.any():
            # perturbations change T by well under a kelvin: bisection in T +- 1 K
            Tp[low] = _moist_T_from_thetal(p[low], thl[low] + dth[low], qtp[low], T_guess=T[low],
                                           half_width=1.0, iters=32)
        Y = state_from_primitives(p, Tp, u, zero, zero, z, qt=qtp, g=g)
        cmax = float(np.max(np.abs(u) + sound_speed_dry(Tp)))
        return Y, Yref, cfl_dt(grid, cmax)
    if ic["kind"] == "agnesi":
        p, T = constant_N(z, Nbv=ic["Nbv"], g=g)
        u = np.full_like(z, ic["u0"])
        Yref = state_from_primitives(p, T, zero, zero, zero, z, g=g)
        Y = state_from_primitives(p, T, u, zero, zero, z, g=g)
        cmax = float(np.max(np.abs(u) + sound_speed_dry(T)))
        return Y, Yref, cfl_dt(grid, cmax)
    raise ValueError(ic["kind"])


def neutral_rest_state(grid: dict, theta0=300.0, g=_G):
    """Hydrostatic rest state of uniform potential temperature."""
    xyz = node_coords(grid)
    z = xyz[2]
    p, T = neutral(z, theta0, g)
    zero = np.zeros_like(z)
    Y = state_from_primitives(p, T, zero, zero, zero, z, g=g)
    return Y


def free_stream_state(grid: dict, rho=1.1, u=(12.0, -7.0, 3.0), T=290.0, qt=None):
    """Uniform density, velocity and temperature everywhere (gravity off)."""
    n = n_nodes(grid)
    p = np.full(n, rho * (_RD if qt is None else _RD * (1 - qt) + _RV * qt) * T)
    z = np.zeros(n)
    q = None if qt is None else np.full(n, qt)
    return state_from_primitives(p, np.full(n, T), np.full(n, u[0]), np.full(n, u[1]), np.full(n, u[2]),
                                 z, qt=q, g=0.0)


def isentropic_vortex(grid: dict, t: float, center=(5000.0, 5000.0), L=500.0, umax=60.0,
                      U=(30.0, 0.0), T_inf=300.0, rho_inf=1.0, xyz=None):
    """Isentropic vortex translated by the uniform flow U (no gravity, no
    viscosity): u_theta = umax' r e^{(1-r^2)/2} with r in units of L, and
    T = T_inf - (2 pi umax'... )^2 ... from c_p dT/dr = u_theta^2 / r, with
    density from the isentrope rho ~ T^(1/(gamma-1)).  Exact solution of the
    compressible Euler equations for any time t."""
    xyz = node_coords(grid) if xyz is None else xyz
    lo, hi = np.asarray(grid["lo"], float), np.asarray(grid["hi"], float)
    Lx, Ly = hi[0] - lo[0], hi[1] - lo[1]
    xc = lo[0] + (center[0] - lo[0] + U[0] * t) % Lx
    yc = lo[1] + (center[1] - lo[1] + U[1] * t) % Ly
    dx = xyz[0] - xc
    dy = xyz[1] - yc
    dx = dx - Lx * np.round(dx / Lx)
    dy = dy - Ly * np.round(dy / Ly)
    r2 = (dx * dx + dy * dy) / (L * L)
    amp = umax * np.exp(0.5 * (1.0 - r2))
    u = U[0] - amp * dy / L
    v = U[1] + amp * dx / L
    A = umax * umax / (2.0 * _CPD)
    T = T_inf - A * np.exp(1.0 - r2)
    gam = _CPD / _CVD
    rho = rho_inf * (T / T_inf) ** (1.0 / (gam - 1.0))
    p = rho * _RD * T
    z = np.zeros_like(u)
    Y = state_from_primitives(p, T, u, v, z, z, g=0.0)
    cmax = float(np.max(np.sqrt(u * u + v * v) + sound_speed_dry(T)))
    return Y, cmax
