"""What the trained closure network gains over Smagorinsky-Lilly, a priori,
on data it was never trained on: boxes of the coarse-grained resolved bubble
at t = 650 s (training used 100-600 s) and of a +3 K bubble (training saw
only the 2 K one).  The boxes hold the filtered state and the SGS fluxes
(from the FP64 resolved run); the closure inputs are recomputed here by the
oracle's BR1 gradients, on the box's interior elements, whose face
neighbours all lie in the box.  The network's raw outputs (bfloat16
operands, as deployed, with the deployed fallback rule) are compared with the
outputs Smagorinsky-Lilly implies, o1 = softplus^-1(nu_SL / (Delta^2 |S|)),
o2 = softplus^-1(Pr_t - 0.1), against the SGS targets.  The a-posteriori
comparison (theta and w errors of coarse runs against the filtered resolved
run) is produced by `python -m paper_2110_00853_amd.learned`."""
import os

import numpy as np
import pytest

import oracle
from paper_2110_00853_amd import learned

HERE = os.path.join(os.path.dirname(__file__), "..", "paper_2110_00853_amd", "data")
WEIGHTS = os.path.join(HERE, "mlp_bubble64_to_32.npz")
HELDOUT = os.path.join(HERE, "heldout_bubble3K_64_to_32.npz")
G = 9.81


def _softplus_inv(y):
    return np.log(np.expm1(y))


def box_samples(z, Cs, Prt):
    """Raw closure inputs [n, 12] and targets [n, 2] on the usable interior
    nodes of a stored box, with the inputs from the oracle."""
    grid = {"N": 4, "ne": [int(v) for v in z["box_ne"]], "lo": [float(v) for v in z["box_lo"]],
            "hi": [float(v) for v in z["box_hi"]], "periodic": [0, 0, 0]}
    Y = z["box_Y"].astype(np.float64)
    inner = z["box_inner"]
    Gd = oracle.Grid(grid)
    model = {"nvar": 5, "closure": "smag", "Cs": Cs, "Prt": Prt, "richardson": True, "g": G}
    grad, _ = oracle.Model(Gd, model).gradients(Y)
    zc = Gd.coords()[2]
    _, _, _, thv = oracle.thermo_nodes(Y, zc, G)
    gu = grad[:3][:, :, inner]
    gth = grad[-1][:, inner]
    N2 = G / thv[inner] * gth[2]
    h = (np.array(grid["hi"]) - np.array(grid["lo"])) / np.array(grid["ne"])
    Delta = float(np.cbrt(np.prod(h / 4.0)))
    assert Delta == pytest.approx(float(z["Delta"]), rel=1e-12)
    nu = np.array([oracle.smagorinsky(gu[:, :, n], N2[n], Cs, Delta, Prt, True) for n in range(N2.size)])
    raw = np.concatenate([gu.reshape(9, -1), N2[None], np.full((1, N2.size), Delta),
                          ((nu / (0.1 * Delta)) ** 2)[None]]).T
    T, mask = learned.targets_from_fluxes(Y[0, inner], z["box_tau"].astype(np.float64),
                                          z["box_q"].astype(np.float64), gu, gth, Delta)
    return raw[mask], T[mask], Delta


def _compare(params, norm, X, T, Delta, Prt):
    mean, std, lo, hi = norm[:12], norm[12:24], norm[24:36], norm[36:48]
    Xn = (X - mean) / std
    out = oracle.mlp_forward(params, Xn, bf16=True)
    gu = X[:, :9].reshape(-1, 3, 3)
    S = 0.5 * (gu + gu.transpose(0, 2, 1))
    Smag = np.sqrt(2.0 * np.sum(S * S, axis=(1, 2)))
    nu_sl = 0.1 * Delta * np.sqrt(X[:, 11])
    sl = np.stack([_softplus_inv(np.clip(nu_sl / (Delta * Delta * Smag), 1e-4, 10.0)),
                   np.full(X.shape[0], _softplus_inv(Prt - 0.1))], axis=1)
    # deployed fallback: an input outside the training range widened by 10 %
    # (an input constant in training passes at its training value)
    c, hw = 0.5 * (lo + hi), 0.5 * (hi - lo)
    tol = np.ldexp(1.0 + np.abs(mean / std), -20)
    fb = np.any(np.abs(Xn - c) > 1.1 * hw + tol, axis=1)
    pred = np.where(fb[:, None], sl, out)
    return np.mean((pred - T) ** 2, axis=0), np.mean((sl - T) ** 2, axis=0), fb.mean()


@pytest.mark.parametrize("which", ["t650", "bubble3K"])
def test_trained_network_beats_smagorinsky_on_held_out_data(which):
    path = WEIGHTS if which == "t650" else HELDOUT
    if not (os.path.exists(WEIGHTS) and os.path.exists(path)):
        pytest.skip("trained weights or held-out data not present")
    w = np.load(WEIGHTS)
    if "box_Y" not in np.load(path):
        pytest.skip("no held-out box in the data file")
    params, norm = w["params"].astype(np.float64), w["norm"].astype(np.float64)
    Cs, Prt = float(w["Cs"]), float(w["Prt"])
    X, T, Delta = box_samples(np.load(path), Cs, Prt)
    mse_net, mse_sl, fbr = _compare(params, norm, X, T, Delta, Prt)
    print("%s: held-out nodes %d  fallback %.4f  MSE network %s  MSE Smagorinsky %s"
          % (which, X.shape[0], fbr, mse_net, mse_sl))
    assert X.shape[0] > 1000
    assert np.all(np.isfinite(mse_net))
    assert mse_net[0] < mse_sl[0]   # eddy viscosity
