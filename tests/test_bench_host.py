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


def test_uneven_subsets_partition_the_batch():
    """The uneven batch's per-subset rows: the disjoint groups (tail only,
    1-8, 9-16, 17-63, 64-127, >= 128 executions) cover every string once,
    1-63 is the union of its three groups, and 'all' is the whole batch."""
    import numpy as np
    from paper_2104_08865_amd import workloads as wl
    lens = wl.uneven_lengths(3)
    N = lens // wl.execution_bytes(24)
    rows = {label: (N >= lo) & (N <= hi if hi is not None else True) for label, lo, hi in bench.UNEVEN_SUBSETS}
    disjoint = ["shorter than one execution (tail only)", "1-8 executions", "9-16 executions", "17-63 executions",
                "64-127 executions", ">= 128 executions"]
    count = np.zeros(lens.size, dtype=np.int64)
    for label in disjoint:
        count += rows[label]
    assert (count == 1).all()
    assert (rows["1-63 executions"] == (rows["1-8 executions"] | rows["9-16 executions"] |
                                        rows["17-63 executions"])).all()
    assert rows["all"].all()
    assert rows["shorter than one execution (tail only)"].sum() == (lens < wl.execution_bytes(24)).sum()
