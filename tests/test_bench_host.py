"""bench.py host logic without a GPU: the one-GPU rule, the contract fields of
the CPU baseline and the gating of the committed traffic figures by the hash
of the device code."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_cpu_baseline_reports_the_contract_fields():
    if not os.path.exists(os.path.join(ROOT, "oracle", "liborc.so")):
        pytest.skip("oracle not built")
    c = bench.cpu_baseline(0.2)
    assert set(("value", "unit", "cores", "kind", "sample")) <= set(c)
    assert c["kind"] == "oracle" and c["unit"] == "MLUPS" and c["value"] > 0 and c["cores"] >= 1


def test_traffic_is_reported_only_for_the_profiled_device_code():
    h = bench.kernel_source_hash()
    assert len(h) == 16
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        t = json.load(fh)
    key = "lb_step_periodic8192_f32"
    assert key in t and t[key]["bytes_per_launch"] >= t[key]["algorithmic_bytes_per_launch"]
    got = bench.measured_traffic(key, 8192 * 8192)
    assert got == (t[key]["bytes_per_launch"] if t[key]["kernel_source_sha"] == h else None)
    assert bench.measured_traffic("no such workload", 1) is None
