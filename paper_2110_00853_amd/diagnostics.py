"""Host-side diagnostics of a dry state (not on the time-stepping path).

front_location: the density-current front at the ground (Sect. 5.2; the
front-location table of App. B): the largest x on the bottom boundary where
the potential-temperature perturbation is at most -1 K, interpolated
linearly between the bottom nodes on either side of the -1 K crossing.
"""
from __future__ import annotations

import numpy as np

# Table 1 and the readings the library uses (c_pd = c_vd + R_d, p0, g)
_RD, _CVD, _T0, _P0 = 287.0, 717.5, 273.16, 1.0e5
_CPD = _CVD + _RD


def potential_temperature(Y: np.ndarray, z: np.ndarray, g: float = 9.81) -> np.ndarray:
    """theta = T (p0/p)^(R_d/c_pd) of a dry state [5, n] (rho, rho u, rho v,
    rho w, rho e_tot) at heights z: I = e_tot - |u|^2/2 - g z, T = T_0 +
    I/c_vd, p = rho R_d T."""
    rho = Y[0]
    e = Y[4] / rho
    ke = 0.5 * (Y[1] ** 2 + Y[2] ** 2 + Y[3] ** 2) / (rho * rho)
    T = _T0 + (e - ke - g * z) / _CVD
    p = rho * _RD * T
    return T * (_P0 / p) ** (_RD / _CPD)


def front_location(Y: np.ndarray, xyz: np.ndarray, theta0: float = 300.0, level: float = -1.0,
                   g: float = 9.81) -> float:
    """x of the theta' = level crossing furthest from the cold pool's origin
    along the ground (node-ordered state [5, n] and coordinates [3, n]).
    Bottom nodes with equal x (element interfaces, the periodic y nodes) are
    averaged before the crossing is located."""
    zmin = xyz[2].min()
    bottom = np.abs(xyz[2] - zmin) <= 1e-9 * max(1.0, abs(zmin))
    x = xyz[0, bottom]
    th = potential_temperature(Y[:, bottom], xyz[2, bottom], g) - theta0
    xs, inv = np.unique(np.round(x, 6), return_inverse=True)
    tm = np.bincount(inv, weights=th) / np.bincount(inv)
    cold = np.nonzero(tm <= level)[0]
    if cold.size == 0:
        return float(xs[0])
    i = cold[-1]
    if i + 1 >= xs.size:
        return float(xs[-1])
    # linear interpolation between the last cold node and its neighbour
    f = (level - tm[i]) / (tm[i + 1] - tm[i])
    return float(xs[i] + f * (xs[i + 1] - xs[i]))
