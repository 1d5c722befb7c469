"""What the trained closure network gains over Smagorinsky-Lilly, a priori:
on held-out nodes of the coarse-grained high-resolution bubble (the
evaluation snapshot, not trained on), the network's raw outputs (evaluated
with bf16 operands, as deployed, through the CPU reference forward) are
closer to the SGS targets than the outputs Smagorinsky-Lilly implies,
o1 = softplus^-1(nu_SL / (Delta^2 |S|)), o2 = softplus^-1(Pr_t - 0.1), with
the deployed fallback rule applied.  The a-posteriori comparison (theta and
w errors of coarse runs against the filtered resolved run) is produced by
`python -m paper_2110_00853_amd.learned`."""
import os

import numpy as np
import pytest

import oracle

DATA = os.path.join(os.path.dirname(__file__), "..", "paper_2110_00853_amd", "data", "mlp_bubble64_to_32.npz")


def _softplus_inv(y):
    return np.log(np.expm1(y))


def test_trained_network_beats_smagorinsky_on_held_out_nodes():
    if not os.path.exists(DATA):
        pytest.skip("trained weights not present")
    z = np.load(DATA)
    if "X_holdout" not in z:
        pytest.skip("weights file holds no held-out samples")
    params, norm = z["params"].astype(np.float64), z["norm"].astype(np.float64)
    X, T = z["X_holdout"], z["T_holdout"]
    Delta, Prt = float(z["Delta"]), float(z["Prt"])
    mean, std, lo, hi = norm[:12], norm[12:24], norm[24:36], norm[36:48]
    Xn = (X - mean) / std
    out = oracle.mlp_forward(params, Xn, bf16=True)
    # Smagorinsky-Lilly in the raw-output space
    gu = X[:, :9].reshape(-1, 3, 3)
    S = 0.5 * (gu + gu.transpose(0, 2, 1))
    Smag = np.sqrt(2.0 * np.sum(S * S, axis=(1, 2)))
    nu_sl = 0.1 * Delta * np.sqrt(X[:, 11])
    sl = np.stack([_softplus_inv(np.clip(nu_sl / (Delta * Delta * Smag), 1e-4, 10.0)),
                   np.full(X.shape[0], _softplus_inv(Prt - 0.1))], axis=1)
    # deployed fallback: an input outside the training range widened by 10 %
    c, hw = 0.5 * (lo + hi), 0.5 * (hi - lo)
    fb = np.any(np.abs(Xn - c) > 1.1 * hw, axis=1)
    pred = np.where(fb[:, None], sl, out)
    mse_net = np.mean((pred - T) ** 2, axis=0)
    mse_sl = np.mean((sl - T) ** 2, axis=0)
    print("held-out nodes %d  fallback %.4f  MSE network %s  MSE Smagorinsky %s"
          % (X.shape[0], fb.mean(), mse_net, mse_sl))
    assert np.all(np.isfinite(mse_net))
    assert mse_net.sum() < mse_sl.sum()
    assert mse_net[0] < mse_sl[0]   # eddy viscosity
