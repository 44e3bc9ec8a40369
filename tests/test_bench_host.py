"""Host logic of bench.py (no GPU): the one-GPU refusal, the workload key
that gates a replayed counter record, and the record's parsing and gating."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workload_key_orders_the_knobs_and_drops_timings():
    class A:
        workload, layout, batch, images_per_pass = "resnet20", "slice", 64, 16
    a = bench.workload_key(A, {"ks_batch": 32, "conv_outs": 8, "timings": {"x": 1}})
    b = bench.workload_key(A, {"conv_outs": 8, "ks_batch": 32})
    assert a == b == 'resnet20/slice/batch64/pass16/{"conv_outs": 8, "ks_batch": 32}'


def test_traffic_record_is_read_only_for_its_sources_and_workload(tmp_path, monkeypatch):
    h = bench.kernel_source_hash("conv_contract")
    assert len(h) == 16 and h == bench.kernel_source_hash("conv_contract")
    prof = tmp_path / "profiles"
    prof.mkdir()
    key = 'resnet20/slice/batch64/pass16/{"conv_outs": 8}'
    (prof / "conv_contract_traffic.md").write_text(
        "# record\n\n```\n"
        f"sources_sha256_16: {h}\nworkload_key: {key}\n"
        "fetch_bytes_per_launch: 3.0e9\nwrite_bytes_per_launch: 0.5e9\n"
        "traffic_bytes_per_launch: 3.5e9\nalg_bytes_per_launch: 3400000000\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the kernel's sources are read from the repository, the record from tmp_path
    monkeypatch.setattr(bench, "kernel_source_hash", lambda cls: h)
    got = bench.measured_traffic("conv_contract", key)
    assert got == {"bytes_per_launch": 3.5e9, "fetch_bytes_per_launch": 3.0e9, "write_bytes_per_launch": 0.5e9}
    assert bench.measured_traffic("conv_contract", key.replace("pass16", "pass64")) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda cls: "0" * 16)
    assert bench.measured_traffic("conv_contract", key) is None
    assert bench.measured_traffic("kip", key) is None
