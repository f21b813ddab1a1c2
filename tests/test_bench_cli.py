"""bench.py's host-side contract, without a GPU: more than one GPU is refused
with a message, and the counter traffic of a profiled kernel is reported only
while the kernel source still has the digest it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_traffic_only_for_the_measured_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    rec = {"kernel": "k", "bytes_per_launch": 12345, "kernel_source_sha256_16": "0123456789abcdef",
           "launch_block_x_seg_rows": [256, 32]}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_pass2_f64_4x2048.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE",
                        str(prof / "traffic_{kernel}_{storage}_4x2048.json"))
    monkeypatch.setattr(bench, "source_digest", lambda: "0123456789abcdef")
    assert bench.measured_traffic("pass2", "f64") == 12345
    assert bench.measured_traffic("pass2", "f64", (256, 32)) == 12345
    assert bench.measured_traffic("pass2", "f64", [256, 37]) is None  # another launch shape
    assert bench.measured_traffic("step", "f64") is None      # no file
    monkeypatch.setattr(bench, "source_digest", lambda: "fedcba9876543210")
    assert bench.measured_traffic("pass2", "f64") is None     # kernel changed since


def test_valu_roofline_from_the_measured_source(tmp_path, monkeypatch):
    # the VALU issue rate of a launch: instructions per launch from the
    # counter record, over the live launch time, against 614.4 G/s (1024
    # SIMDs at 2.4 GHz, one wave64 instruction per 4 cycles)
    sys.path.insert(0, ROOT)
    import bench
    assert abs(bench.VALU_PEAK_GIPS - 256 * 4 * 2.4e9 / 4 / 1e9) < 1e-9
    rec = {"kernel": "k", "bytes_per_launch": 1, "valu_insts_per_launch": 30720000,
           "kernel_source_sha256_16": "0123456789abcdef"}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_pass2_f16_4x2048.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE",
                        str(prof / "traffic_{kernel}_{storage}_4x2048.json"))
    monkeypatch.setattr(bench, "source_digest", lambda: "0123456789abcdef")
    v = bench.valu_roofline("pass2", "f16", 0.1)      # 30.72 M instructions in 100 us
    assert v["achieved"] == 307.2 and v["frac"] == 0.5 and v["insts_per_launch"] == 30720000
    assert bench.valu_roofline("pass2", "f32", 0.1) is None    # no file
    monkeypatch.setattr(bench, "source_digest", lambda: "fedcba9876543210")
    assert bench.valu_roofline("pass2", "f16", 0.1) is None    # kernel changed since
