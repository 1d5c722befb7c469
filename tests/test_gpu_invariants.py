"""Invariants the discrete method fixes, checked on the GPU path itself (no
oracle involved): a uniform free stream keeps a zero tendency on flat and
warped meshes, dry and moist, for every closure; a neutral hydrostatic rest
state with itself as reference stays at rest; both also at the full 32^3
benchmark size in the launch configuration bench.py times."""
import numpy as np
import pytest

from paper_2110_00853_amd import binding as B
from paper_2110_00853_amd import workloads as W

pytestmark = pytest.mark.gpu

CART = {"N": 4, "ne": [3, 2, 3], "lo": [0.0, 0.0, 0.0], "hi": [600.0, 400.0, 600.0], "periodic": [1, 1, 1]}
WARP = {"N": 4, "ne": [4, 2, 3], "lo": [0.0, 0.0, 0.0], "hi": [1000.0, 500.0, 900.0], "periodic": [1, 1, 1],
        "topo": 1, "topo_h": 150.0, "topo_a": 200.0, "topo_xc": 500.0}
FULL = {"N": 4, "ne": [32, 32, 32], "lo": [0.0, 0.0, 0.0], "hi": [10000.0, 10000.0, 10000.0],
        "periodic": [1, 1, 1]}


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available()
    B.load()
    return torch


def _flux_scale(Y, h):
    u = Y[1:4] / Y[0]
    p = 1e5
    return np.array([np.abs(Y[1:4]).max(), p, p, p, np.abs(Y[4] * u).max() + p * np.abs(u).max()]) * 2 / h


def _rhs(torch, grid, model, Y, Yref=None, precision="fp64"):
    g = B.Grid(grid)
    m = B.Model(g, model, Yref, precision=precision)
    Yd = m.new_state(Y)
    Rd = m.new_state()
    m.rhs(Yd, Rd)
    torch.cuda.synchronize()
    return m.tendency_to_numpy(Rd).astype(np.float64)


CASES = [(g, c, n) for g in ("cartesian", "warped") for c in ("none", "const", "smag") for n in (5, 6)]
CASES.append(("full_32", "smag", 5))  # the benchmark's own model at its size


@pytest.mark.parametrize("gname,closure,nvar", CASES)
def test_free_stream_preserved(torch, gname, closure, nvar):
    grid = {"cartesian": CART, "warped": WARP, "full_32": FULL}[gname]
    Y = W.free_stream_state(grid, qt=None if nvar == 5 else 6e-3)
    model = {"nvar": nvar, "closure": closure, "nu": 75.0, "g": 0.0, "richardson": True}
    R = _rhs(torch, grid, model, Y)
    h = min(np.array(grid["hi"]) / np.array(grid["ne"]))
    sc = _flux_scale(Y, h)
    for v in range(5):
        assert np.abs(R[v]).max() < 1e-12 * sc[v], (v, np.abs(R[v]).max(), sc[v])
    if nvar == 6:
        assert np.abs(R[5]).max() < 1e-12 * sc[0]


@pytest.mark.parametrize("closure", ["const", "smag"])
@pytest.mark.parametrize("size", ["small", "full_32"])
def test_hydrostatic_rest_stays_at_rest(torch, closure, size):
    if size == "small":
        g = dict(CART, periodic=[1, 1, 0], hi=[600.0, 400.0, 1500.0])
    else:
        g = dict(FULL, periodic=[1, 1, 0])
    Y = W.neutral_rest_state(g)
    model = {"nvar": 5, "closure": closure, "nu": 75.0, "g": 9.81, "richardson": True}
    R = _rhs(torch, g, model, Y, Y)
    rho_g = Y[0].max() * 9.81
    assert np.abs(R[0]).max() == 0.0
    assert np.abs(R[1:4]).max() <= 1e-12 * rho_g
    assert np.abs(R[4]).max() <= 1e-12 * rho_g * 300.0


@pytest.mark.parametrize("size", ["small", "full_32"])
def test_fp32_bulk_rest_state_stays_at_rest(torch, size):
    """FP32-bulk stores deviations from the background: the neutral rest
    state imported as its own background is stored as zeros, so the mass
    tendency vanishes exactly and the momentum tendencies to the FP64 model's
    bound (the FP64 thermodynamics of the float-rounded background against
    the reference computed from it); the energy tendency keeps only the FP32
    rounding of the diffusive flux of h_tot."""
    if size == "small":
        g = dict(CART, periodic=[1, 1, 0], hi=[600.0, 400.0, 1500.0])
    else:
        g = dict(FULL, periodic=[1, 1, 0])
    Y = W.neutral_rest_state(g)
    model = {"nvar": 5, "closure": "const", "nu": 75.0, "g": 9.81, "richardson": True}
    R = _rhs(torch, g, model, Y, Y, precision="fp32")
    rho_g = Y[0].max() * 9.81
    print(size, "fp32 rest-state tendency maxima", np.abs(R).max(axis=1))
    assert np.abs(R[0]).max() == 0.0
    assert np.abs(R[1:4]).max() <= 1e-12 * rho_g
    assert np.abs(R[4]).max() <= 1e-4 * rho_g * 300.0
