"""Host-side checks of bench.py's contract: it refuses more than one GPU,
and its readers of the committed rocprofv3 summaries take figures only from
summaries of the current kernel sources."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profile_readers_follow_the_sources(monkeypatch):
    digest = bench.sources_digest()
    traffic = bench.read_traffic("k_tile", "config2_batch")
    valu = bench.read_valu_insts("k_tile", "config2_batch")
    text = open(os.path.join(ROOT, "profiles", "traffic_k_tile_config2_batch.txt")).read()
    if f"sources_sha256: {digest}" in text:
        assert traffic is not None and traffic > 0
    else:
        assert traffic is None
    monkeypatch.setattr(bench, "sources_digest", lambda: "0" * 16)
    assert bench.read_traffic("k_tile", "config2_batch") is None
    assert bench.read_valu_insts("k_tile", "config2_batch") is None
    assert bench.read_traffic("k_none", "config2_batch") is None
    if valu is not None:
        assert valu > 0
