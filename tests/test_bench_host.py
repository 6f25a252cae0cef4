"""Host-side checks of the benchmark script's contract (no GPU)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_lookup_checks_the_sources(tmp_path, monkeypatch):
    """A committed traffic figure is reported only while the kernel sources it
    was taken on are unchanged; workloads without one report none."""
    assert bench.measured_traffic("sc8_afm", "split_bf16") is None
    prof, srcs = bench.TRAFFIC_PROFILES["sc36_afm"]
    text = open(prof).read()
    copy = tmp_path / "profile.md"
    copy.write_text(text)
    monkeypatch.setitem(bench.TRAFFIC_PROFILES, "sc36_afm", (str(copy), srcs))
    current = bench.measured_traffic("sc36_afm", "split_bf16")
    edited = "\n".join(("kernel_source_sha256: " + "0" * 64) if ln.startswith("kernel_source_sha256:") else ln
                       for ln in text.splitlines())
    copy.write_text(edited)
    assert bench.measured_traffic("sc36_afm", "split_bf16") is None
    assert bench.measured_traffic("sc36_afm", "fp32") is None
    if current is not None:
        assert current > 0


def test_workloads_are_defined():
    for name in ("sc36_afm", "sc32_fm", "ball65k", "batch48", "sq420", "ball65k_sq", "mc_sc128"):
        assert name in bench.WORKLOADS


def test_unknown_compare_precision_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--compare", "''"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "--compare" in r.stderr
