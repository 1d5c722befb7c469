"""The exponential modal filter (Sect. 5.4, eq. exponential_filter) on the
GPU through the C ABI against the oracle's dense Kronecker application:
several filter settings, variable masks, flat and warped meshes (per-level
and per-node background), FP64 and FP32-bulk; the background is kept
exactly and element integrals to rounding."""
import numpy as np
import pytest

import oracle
from paper_2110_00853_amd import binding as B
from paper_2110_00853_amd import workloads as W

pytestmark = pytest.mark.gpu

FLAT = W.case("bubble_32", ne=(5, 3, 4), hi=(1000.0, 450.0, 800.0))
WARPED = W.case("agnesi_96", ne=(6, 2, 5), hi=(1500.0, 500.0, 1600.0))
WARPED["grid"].update(topo_a=300.0, topo_xc=750.0, topo_h=200.0)
MOIST = W.case("moist_64", ne=(4, 3, 4), hi=(400.0, 300.0, 2000.0))


@pytest.mark.parametrize("name,c", [("flat", FLAT), ("warped", WARPED), ("moist", MOIST)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_filter_matches_oracle(name, c, precision):
    import torch

    Y, Yref, _ = W.perturbed_state(c, seed=9, amp_u=6.0, amp_T=2.0, amp_q=1.5e-3)
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref, precision=precision)
    om = oracle.Model(oracle.Grid(c["grid"]), c["model"], Yref)
    nv = Y.shape[0]
    for mask, order, alpha, Nc in [(0b01110, 64, 36.0, 0), ((1 << nv) - 1, 4, 20.0, 0), (0b10001, 2, 8.0, 1)]:
        Yd = m.new_state(Y)
        m.exp_filter(Yd, mask, order, alpha, Nc)
        torch.cuda.synchronize()
        Yg = m.to_numpy(Yd).astype(np.float64)
        Yo = om.exp_filter(Y, mask, order, alpha, Nc)
        for v in range(nv):
            scale = max(np.abs(Yo[v] - Yref[v]).max(), 1e-300)
            err = np.abs(Yg[v] - Yo[v]).max() / scale
            tol = 1e-12 if precision == "fp64" else 1e-3 * np.abs(Y[v]).max() / scale + 1e-5
            print(name, precision, bin(mask), order, "var", v, "error relative to the deviation", err)
            assert err < tol, (v, err)
            if not (mask >> v) & 1 and precision == "fp64":
                assert np.array_equal(Yg[v], Y[v])


def test_filter_keeps_the_background_and_element_integrals():
    """The background is kept exactly (warped mesh, per-node background); on a
    flat mesh (constant Jacobian) every element integral is kept to rounding."""
    import torch

    c = WARPED
    Y, Yref, _ = W.perturbed_state(c, seed=10)
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref)
    Yd = m.new_state(Yref)
    m.exp_filter(Yd, 0b11111, 8, 36.0, 0)
    torch.cuda.synchronize()
    assert np.array_equal(m.to_numpy(Yd), Yref)
    c = FLAT
    Y, Yref, _ = W.perturbed_state(c, seed=10)
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref)
    Yd = m.new_state(Y)
    m.exp_filter(Yd, 0b11111, 2, 36.0, 0)
    torch.cuda.synchronize()
    out = m.to_numpy(Yd)
    wJ = g.wJ()
    ne = int(np.prod(c["grid"]["ne"]))
    for v in range(5):
        before = (wJ * Y[v]).reshape(ne, -1).sum(1)
        after = (wJ * out[v]).reshape(ne, -1).sum(1)
        assert np.abs(after - before).max() <= 1e-13 * np.abs(Y[v]).max() * np.abs(wJ).sum() / ne, v
    with pytest.raises(B.CMError):
        m.exp_filter(Yd, 1 << 5, 8, 36.0, 0)


def test_full_size_filter_matches_oracle():
    """The filter in the configuration bench.py times (all five variables of
    the 32^3 bubble, order 64, alpha 36, in place) against the oracle on
    every node, on a perturbed state."""
    import torch

    c = W.case("bubble_32")
    Y, Yref, _ = W.perturbed_state(c, seed=12, amp_u=4.0, amp_T=1.5)
    print("full-size filter: bubble_32", flush=True)
    g = B.Grid(c["grid"])
    m = B.Model(g, c["model"], Yref)
    Yd = m.new_state(Y)
    m.exp_filter(Yd, 0b11111, 64, 36.0, 0)
    torch.cuda.synchronize()
    Yg = m.to_numpy(Yd)
    Yo = oracle.Model(oracle.Grid(c["grid"]), c["model"], Yref).exp_filter(Y, 0b11111, 64, 36.0, 0)
    err = np.array([np.abs(Yg[v] - Yo[v]).max() / max(np.abs(Yo[v] - Yref[v]).max(), 1e-300) for v in range(5)])
    print("full-size filter errors relative to the deviation", err)
    assert np.all(err <= 1e-13), err
