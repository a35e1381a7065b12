"""Host-side checks of bench.py (no GPU): the algorithmic byte model per site, the
single-GPU guard and the rule that committed counter traffic is used only while the
kernel sources still hash to the value recorded with the counters."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_byte_model_counts_links_once_and_vectors_per_column():
    # FP64: a folded 3x3 complex link is 144 bytes, a colour-vector complex 16 bytes;
    # 16 folded links per site; hop_eo reads P (centre), T (neighbours) and writes AP
    assert bench.model_bytes_per_site("hop_eo", 16, "fp64") == 16 * 144 + 9 * 16 * 16
    assert bench.model_bytes_per_site("hop_oe", 16, "fp64") == 16 * 144 + 6 * 16 * 16
    # 16^4 lattice, N = 16: the figure the roofline object divides by the launch time
    assert bench.model_bytes_per_site("hop_eo", 16, "fp64") * (16 ** 4 // 2) == 150994944
    # the per-RHS share of the links falls as 1/N
    per_rhs = [bench.model_bytes_per_site("hop_oe", n, "fp32") / n for n in (1, 4, 16, 64)]
    assert all(a > b for a, b in zip(per_rhs, per_rhs[1:]))
    assert bench.model_bytes_per_site("small", 16) is None


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_is_ignored_once_the_kernel_source_changes(tmp_path, monkeypatch):
    key = "unit_test_workload"
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    rec = {"kernel": "hop_eo", "workload": key, "hbm_bytes_per_launch": 123.0,
           "source_hash": bench.kernel_source_hash("hop_eo")}
    (tmp_path / f"hop_eo_{key}_pmc.json").write_text(json.dumps(rec))
    assert bench.load_traffic("hop_eo", key, 0) == 123.0
    rec["source_hash"] = "0" * 16
    (tmp_path / f"hop_eo_{key}_pmc.json").write_text(json.dumps(rec))
    assert bench.load_traffic("hop_eo", key, 0) is None
    assert bench.load_traffic("pass_a", key, 0) is None   # no record at all
