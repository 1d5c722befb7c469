"""The time-step reading for the 4^3 dry bubble, checked on the oracle: with
LSRK54 and the N = 4 operator, a Courant number of 0.8 on the minimum GLL
node spacing (the configured value, taken literally) blows up within a few
steps, 0.5 within a few dozen, while 0.4 (the value the workloads use) stays
bounded.  The explicit stability limit of the 3-D DG operator at N = 4 is set
by the smallest GLL spacing, so the literal 0.8 cannot be run."""
import numpy as np
import pytest

from paper_2110_00853_amd import workloads as W


def _run(oracle_lib, cfl, steps):
    c = W.case("bubble_4")
    Y0, Yref, dt04 = W.initial_state(c)
    assert dt04 == pytest.approx(W.cfl_dt(c["grid"], W.sound_speed_dry(np.array([302.0]))[0]), rel=0.05)
    M = oracle_lib.Model(oracle_lib.Grid(c["grid"]), c["model"], Yref)
    dt = dt04 * cfl / 0.4
    Y, dQ = Y0, None
    wmax = 0.0
    with np.errstate(all="ignore"):
        for _ in range(steps):
            Y, dQ = M.steps(Y, dt, 1, dQ=dQ)
            w = np.abs(Y[3] / Y[0]).max()
            wmax = w if np.isfinite(w) else np.inf
            if wmax > 100.0:
                break
    return wmax


def test_configured_courant_number_blows_up(oracle_lib):
    assert _run(oracle_lib, 0.8, 10) > 100.0
    assert _run(oracle_lib, 0.5, 40) > 100.0


def test_courant_number_used_is_stable(oracle_lib):
    assert _run(oracle_lib, 0.4, 60) < 1.0
