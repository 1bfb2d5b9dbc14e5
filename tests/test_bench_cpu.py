"""CPU checks of bench.py's contract that need no GPU: a run asked for more than one GPU exits with
a message (this build has no multi-GPU path), and the committed HBM-traffic record is reported only
for the raymarch sources it was taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_tied_to_the_render_sources(tmp_path, monkeypatch):
    sha = bench.source_sha(bench.RENDER_SOURCES)
    assert len(sha) == 16 and sha != bench.source_sha(bench.RENDER_SOURCES[:1])
    rec = {"render_head_1024_persp": {"source_sha": sha, "fetch_bytes_per_launch": 1.0}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic("render_head_1024_persp", sha)["fetch_bytes_per_launch"] == 1.0
    assert bench.load_traffic("render_head_1024_persp", "0" * 16) is None
    assert bench.load_traffic("other_kernel", sha) is None


def test_committed_traffic_record_names_the_timed_kernel():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)["render_head_1024_persp"]
    assert rec["views_per_launch"] == 32 and rec["fetch_bytes_per_launch"] > 0 and rec["write_bytes_per_launch"] > 0
    assert 1.9 < rec["fetch_scale"] < 2.1 and rec["write_scale"] == 1.0
