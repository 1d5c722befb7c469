"""Parity at the full benchmark sizes, in the configuration bench.py times:
the FP64 tendency of every node against the oracle (dry bubble 32^3,
moist shallow convection 64x64x30, warped Agnesi flow 96x16x50), and the
FP32-bulk tendency error against the same oracle (stated, bounded).

The FP64 bar is 1e-11 relative per variable, or four times the oracle's own
movement under one-ulp input perturbations where that is larger (the moist
momentum tendencies, whose floor is about 1.2e-11)."""
import numpy as np
import pytest

import oracle
from paper_2110_00853_amd import binding as B
from paper_2110_00853_amd import workloads as W
from parity import hmin, rhs_errors, rounding_floor

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["bubble_32", "agnesi_96", "moist_64"])
def test_full_size_rhs_matches_oracle(name):
    import torch

    c = W.case(name)
    Y, Yref, dt = W.initial_state(c)
    Rref, floor = rounding_floor(oracle.Model(oracle.Grid(c["grid"]), c["model"], Yref).rhs, Y, hmin(c["grid"]))
    tol = np.maximum(1e-11, 4.0 * floor)
    g = B.Grid(c["grid"])
    out = {}
    for prec in ("fp64", "fp32"):
        m = B.Model(g, c["model"], Yref, precision=prec)
        Yd = m.new_state(Y)
        Rd = m.new_state()
        m.rhs(Yd, Rd)
        torch.cuda.synchronize()
        out[prec] = rhs_errors(m.to_numpy(Rd).astype(np.float64), Rref, Y, hmin(c["grid"]))
        del m, Yd, Rd
    print(name, "full-size rhs errors fp64", out["fp64"], "oracle 1-ulp floor", floor, "fp32-bulk", out["fp32"])
    assert np.all(out["fp64"] < tol), (out["fp64"], tol)
    assert np.all(np.isfinite(out["fp32"])) and np.all(out["fp32"] < 5e-2), out["fp32"]
