"""Host-side logic of bench.py (no GPU): the one-GPU guard, the kernel code
hash that keys the committed counter data, and the traffic lookup."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "single MI355X" in r.stderr and r.stdout == ""


def test_kernel_code_hash_ignores_comments(tmp_path, monkeypatch):
    src = open(bench.KERNEL_SRC).read()
    base = bench.kernel_source_hash()
    edited = tmp_path / "k.hip"
    edited.write_text("// a new comment\n\n" + src.replace("\n", "\n/* block */\n", 1) + "\n// trailing\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(edited))
    assert bench.kernel_source_hash() == base
    edited.write_text(src.replace("kFan - 1", "kFan-1", 1) + "int x;\n")
    assert bench.kernel_source_hash() != base


def test_traffic_only_for_the_code_it_was_taken_on(tmp_path):
    doc = {"kernel_source_sha256_16": bench.kernel_source_hash(),
           "per_width": {"24": {"hbm_bytes_per_launch": 123}}}
    f = tmp_path / "t.json"
    f.write_text(json.dumps(doc))
    assert bench.measured_traffic(24, str(f)) == 123
    assert bench.measured_traffic(16, str(f)) is None
    doc["kernel_source_sha256_16"] = "0" * 16
    f.write_text(json.dumps(doc))
    assert bench.measured_traffic(24, str(f)) is None
    # the committed summaries match the committed kernel code
    assert bench.measured_traffic(24) is not None
    assert bench.measured_traffic(24, bench.UNEVEN_TRAFFIC_FILE) is not None
