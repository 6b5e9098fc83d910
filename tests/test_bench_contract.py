"""Host-side parts of bench.py: the one-GPU guard and the DRAM-traffic figure,
which is reported only while the hot-path sources hash to the profiled ones."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    h = bench.source_hash()
    assert len(h) == 16
    prof = tmp_path / "profiles"
    prof.mkdir()
    f = prof / "k_pcg_resg4_stress8192.md"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    line = 'summary\nbench-traffic: {"source_hash": "%s", "hbm_bytes_32cube_launch": 123, ' \
           '"hbm_bytes_streamed_launches": 456}\n'
    f.write_text(line % "x")
    monkeypatch.setattr(bench, "source_hash", lambda: h)
    assert bench.traffic_from_profile(True) is None      # profiled on other sources
    f.write_text(line % h)
    assert bench.traffic_from_profile(True) == 123       # the 32^3 launch on a stream of its own
    assert bench.traffic_from_profile(False) == 456      # both streamed-weights launches on one stream
    f.unlink()
    assert bench.traffic_from_profile(True) is None      # no profile
