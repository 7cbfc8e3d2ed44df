"""Host logic of bench.py (no GPU): the one-GPU guard, the kernel-source hash
that keys the committed counter summaries, and the traffic lookup that must
drop a summary taken on other kernel sources."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_source_hash_is_stable_and_ignores_the_api_file(tmp_path, monkeypatch):
    h = bench.source_hash()
    assert len(h) == 16 and h == bench.source_hash()
    # a copy of the kernel sources hashes the same; an edit of a kernel file changes it,
    # an edit of the host-side API file does not
    src = os.path.join(ROOT, "paper_2206_11998_amd", "csrc")
    dst = tmp_path / "paper_2206_11998_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in os.listdir(src):
        p = os.path.join(src, f)
        if os.path.isfile(p):
            (dst / f).write_bytes(open(p, "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.source_hash() == h
    api = dst / "lp_api.hip"
    api.write_bytes(api.read_bytes() + b"\n// host-side comment\n")
    assert bench.source_hash() == h
    grid = dst / "lp_grid.hip"
    grid.write_bytes(grid.read_bytes() + b"\n// kernel-side comment\n")
    assert bench.source_hash() != h


def test_traffic_only_from_a_summary_of_the_same_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    summary = {"source_hash": "0123456789abcdef", "kernels": {"search": {"read_bytes": 3.0e8, "written_bytes": 1.0e8}}}
    (prof / "vacuum3d_2M_mixed_step_traffic.json").write_text(json.dumps(summary))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: "0123456789abcdef")
    assert bench.committed_traffic("search", "mixed") == 4.0e8
    assert bench.committed_traffic("fit+update", "mixed") is None  # kernel not in the summary
    assert bench.committed_traffic("search", "fp64") is None  # no summary for that precision
    monkeypatch.setattr(bench, "source_hash", lambda: "fedcba9876543210")
    assert bench.committed_traffic("search", "mixed") is None  # other kernel sources
