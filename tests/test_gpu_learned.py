"""The learned closure end to end at small scale on the GPU: resolved run,
coarse-graining, SGS targets, training with the MFMA kernels (two seeds),
the a-posteriori comparison with Smagorinsky, the held-out box, and the
held-out-bubble run from the saved weights (errors are reported; the
full-scale comparison is recorded by `python -m paper_2110_00853_amd.learned`)."""
import numpy as np
import pytest

from paper_2110_00853_amd import learned

pytestmark = pytest.mark.gpu


def test_pipeline_small(tmp_path):
    npz = str(tmp_path / "w.npz")
    r = learned.run_pipeline(fine_ne=16, t_train=(10.0, 20.0, 30.0), t_eval=40.0, t_holdout=50.0,
                             train_steps=200, batch=4096, seeds=(0, 1), out_npz=npz)
    print({k: v for k, v in r.items() if k not in ("params", "norm", "losses")})
    assert r["train_samples"] > 200
    first, last = r["losses"][0][1], r["losses"][-1][1]
    assert np.isfinite(last) and last < first
    for name in ("smagorinsky", "learned", "learned_no_fallback", "learned_seed1"):
        assert np.isfinite(r[name]["theta_rel_l2"]) and np.isfinite(r[name]["w_rel_l2"])
    assert 0.0 <= r["learned"]["fallback_fraction"] <= 1.0
    z = np.load(npz)
    assert z["box_Y"].shape == (5, 6 ** 3 * 125) and z["box_tau"].shape[2] == 4 ** 3 * 125
    h = learned.run_heldout(npz, fine_ne=16, t_eval=20.0, out_npz=str(tmp_path / "h.npz"))
    print({k: v for k, v in h.items()})
    assert np.isfinite(h["learned"]["theta_rel_l2"]) and h["dtheta"] == 1.5
