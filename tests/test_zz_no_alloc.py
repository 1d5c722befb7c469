"""The allocation-free diagnostics entry point (cm_diagnostics_noalloc,
static per-device workspace) against cm_diagnostics (model-owned workspace)
through the C ABI: two calls in a row, the second on a smaller grid, so the
workspace still holds the first call's records.  The two entry points run the
same reduction with the same block count, so every field must agree bit for
bit (compensated FP64 integrals, extrema, CFL, non-finite count)."""
import numpy as np
import pytest

from paper_2110_00853_amd import binding as B
from paper_2110_00853_amd import workloads as W

pytestmark = pytest.mark.gpu


def _both(name, ne, hi, seed, dt, precision="fp64", plant_nan=False):
    import torch

    c = W.case(name, ne=ne, hi=hi)
    Y, Yref, _ = W.perturbed_state(c, seed=seed, amp_u=6.0, amp_T=2.0, amp_q=1.5e-3)
    if plant_nan:
        Y = Y.copy()
        Y[1, 17] = np.nan
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref, precision=precision)
    Yd = m.new_state(Y)
    torch.cuda.synchronize()
    print("noalloc diagnostics:", name, ne, precision, "nodes", g.n_nodes, flush=True)
    ref = m.diagnostics(Yd, dt)
    new = m.diagnostics(Yd, dt, noalloc=True)
    return ref, new


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_diagnostics_match_twice_second_smaller(precision):
    # 1.05M nodes: the first pass runs the maximum 2047 blocks
    big = _both("bubble_32", (21, 20, 20), (4200.0, 4000.0, 4000.0), seed=3, dt=0.05, precision=precision)
    # 6,000 nodes on a moist model: 24 blocks, the rest of the workspace stale
    small = _both("moist_64", (4, 3, 4), (400.0, 300.0, 2000.0), seed=5, dt=0.02, precision=precision)
    for ref, new in (big, small):
        assert ref["status"] == B.CM_OK and new["status"] == B.CM_OK
        for k in ref:
            assert new[k] == ref[k], (k, new[k], ref[k])
    assert small[0]["mass"] != big[0]["mass"] and small[0]["water"] != 0.0


def test_noalloc_diagnostics_report_nonfinite_like_the_model_path():
    ref, new = _both("bubble_4", (3, 2, 2), (1500.0, 1000.0, 1000.0), seed=7, dt=0.0, plant_nan=True)
    assert ref["status"] == new["status"] == B.CM_ERR_NONFINITE
    assert ref["n_nonfinite"] == new["n_nonfinite"] == 1
    for k in ref:
        if k != "status":
            assert new[k] == ref[k], (k, new[k], ref[k])
