"""The learned closure end to end at small scale on the GPU: resolved run,
coarse-graining, SGS targets, training with the MFMA kernels, and the
a-posteriori comparison with Smagorinsky (errors are reported; the
full-scale comparison is recorded by `python -m paper_2110_00853_amd.learned`)."""
import numpy as np
import pytest

from paper_2110_00853_amd import learned

pytestmark = pytest.mark.gpu


def test_pipeline_small():
    r = learned.run_pipeline(fine_ne=16, t_train=(10.0, 20.0, 30.0), t_eval=40.0, train_steps=200, batch=4096)
    print({k: v for k, v in r.items() if k not in ("params", "norm", "losses")})
    assert r["train_samples"] > 200
    first, last = r["losses"][0][1], r["losses"][-1][1]
    assert np.isfinite(last) and last < first
    for name in ("smagorinsky", "learned", "learned_no_fallback"):
        assert np.isfinite(r[name]["theta_rel_l2"]) and np.isfinite(r[name]["w_rel_l2"])
    assert 0.0 <= r["learned"]["fallback_fraction"] <= 1.0
