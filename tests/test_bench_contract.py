"""Host-side parts of bench.py: the one-GPU guard, the algorithmic byte
counts behind the roofline, and the rule that the counter-derived traffic is
reported only for the kernel source it was measured on."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_node():
    # dry FP64: gradient pass Y + F2 (5 + 9 words), tendency pass Y, F2, dQ
    # read and dQ, Y_new written (first stage without the dQ read)
    assert bench.alg_bytes(5, 9, 8) == (112, 192, 232)
    grad, first, other = bench.alg_bytes(5, 9, 8)
    assert grad + other == 344
    assert (first + 4 * other) / 5 == 224
    # FP32-bulk halves every figure; moist adds a variable and three flux words
    assert bench.alg_bytes(5, 9, 4) == (56, 96, 116)
    assert bench.alg_bytes(6, 12, 8) == (144, 240, 288)


def test_traffic_is_reported_only_for_the_profiled_source(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel source")
    sha = hashlib.sha256(b"kernel source").hexdigest()
    prof = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(prof))
    assert bench.measured_traffic("bubble_32") is None  # no summary
    prof.write_text(json.dumps({"kernel_source_sha256": sha, "hbm_bytes_per_launch": 1.5e9}))
    assert bench.measured_traffic("bubble_32") == 1.5e9
    assert bench.measured_traffic("moist_64") is None  # taken on another workload
    assert bench.measured_traffic("bubble_32", "16,16,16") is None  # other element counts
    src.write_bytes(b"kernel source, changed")
    assert bench.measured_traffic("bubble_32") is None  # stale summary
