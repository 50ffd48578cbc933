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


def test_cpu_baseline_uses_the_cpu_share(monkeypatch):
    """The oracle runs on OMP_NUM_THREADS threads when that is set (the host's
    CPU share), and `cores` reports the threads it used."""
    if not os.path.exists(os.path.join(ROOT, "oracle", "liborc.so")):
        pytest.skip("oracle not built")
    from oracle import oracle as O

    before = O.threads()
    monkeypatch.setenv("OMP_NUM_THREADS", "2")
    try:
        c = bench.cpu_baseline(0.2)
    finally:
        O.set_threads(before)
    assert c["cores"] == 2
    assert c["samples"][0]["threads"] == 2 and c["samples"][1]["threads"] == 1


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


def _csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "c_counter_collection.csv"), "w") as fh:
        fh.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for i, (k, c, v) in enumerate(rows):
            fh.write(f'{i},"{k}","{c}",{v}\n')


def test_pmc_summary_scales_the_counters_by_the_copy(tmp_path):
    """A copy of 2 GiB that FETCH_SIZE reports as 1 GiB gives a read scale of
    2; the step's bytes are then 2 x fetch + 1 x write, in KiB x 1024."""
    d = str(tmp_path)
    copy = "(anonymous namespace)::k_copy(unsigned int __vector(4) const*, unsigned int __vector(4)*, long long, long long)"
    # the copy probe's 2 GiB dispatches calibrate; other kernels of the run
    # (torch's fill and copies of other sizes) are ignored
    _csv(os.path.join(d, "cfetch"), [(copy, "FETCH_SIZE", 1048576.0)] * 3 + [("fill", "FETCH_SIZE", 5.0),
                                                                            ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 2.0)])
    _csv(os.path.join(d, "cwrite"), [(copy, "WRITE_SIZE", 2097152.0)] * 3)
    for st, code in (("f32", 0), ("f16", 1)):
        k = f"void (anonymous namespace)::k_step<{code}, false, (anonymous namespace)::Head>(...)"
        _csv(os.path.join(d, f"{st}fetch"), [(k, "FETCH_SIZE", 100.0), (k, "FETCH_SIZE", 300.0),
                                            ("k_init", "FETCH_SIZE", 9e9)])
        _csv(os.path.join(d, f"{st}write"), [(k, "WRITE_SIZE", 50.0)])
    t = bench.pmc_summary(d, n=64)
    e = t["lb_step_periodic64_f32"]
    assert e["fetch_scale"] == 2.0 and e["write_scale"] == 1.0
    assert e["bytes_per_launch"] == 1024 * (200.0 * 2 + 50.0)
    assert e["algorithmic_bytes_per_launch"] == 144 * 64 * 64
    assert t["lb_step_periodic64_f16"]["algorithmic_bytes_per_launch"] == 72 * 64 * 64
    assert e["kernel_source_sha"] == bench.kernel_source_hash()
