"""The committed profiler summaries describe the committed kernels: the
counter figures the benchmark's roofline line reports (calibrated HBM bytes
per launch of the dominant kernel) carry the hash of the kernel source they
were taken on, and the summaries name the commands that made them."""
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def test_traffic_counters_match_the_kernel_source():
    with open(os.path.join(ROOT, "paper_1005_0088_amd", "csrc", "kernels.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    with open(os.path.join(PROFILES, "traffic_cubic3d_24x4_mixed_bf16x3.json")) as f:
        t = json.load(f)
    assert t["kernels_hip_sha256_16"] == sha, "counters taken on another kernels.hip: retake them"
    assert t["dispatches"] > 0 and t["read_bytes_per_launch"] > 0 and t["write_bytes_per_launch"] > 0
    assert 1.9 < t["calibration_fetch_factor"] < 2.1 and 0.9 < t["calibration_write_factor"] < 1.1


def test_summaries_name_their_commands():
    names = [n for n in os.listdir(PROFILES) if n.endswith(".md")]
    assert {"kernels_cubic3d_24x4_mixed_bf16x3.md", "traffic_cubic3d_24x4_mixed_bf16x3.md",
            "bandwidth_cubic3d_24x4_mixed_bf16x3.md", "mfma_util_cubic3d_24x4_mixed_bf16x3.md"} <= set(names)
    for n in names:
        with open(os.path.join(PROFILES, n)) as f:
            text = f.read()
        assert "rocprofv3" in text and "bench.py" in text, n
