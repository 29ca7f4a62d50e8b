"""The bench's measurement plumbing on the host (no GPU): the counter
summary it reads HBM traffic from is used only while its sources and launch
knobs are the ones it was taken with, the cached launch knobs cover every
knob of the binding, and the bench refuses more than one GPU."""
import json
import os
import subprocess
import sys

import bench
from paper_1902_01010_amd import vr


def _profile(tmp_path, monkeypatch, knobs_line="launch_knobs: knn_leaf=192 xcd_chunk=256"):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    prof = tmp_path / "p.txt"
    prof.write_text("summary\nkernel: k\nsources: k.hip\n"
                    f"sources_sha256: {bench.sources_sha256(['k.hip'])}\n{knobs_line}\n"
                    "hbm_bytes_per_dispatch: 12345\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", {"knn": "p.txt"})
    return src


def test_traffic_profile_used_while_sources_and_knobs_match(tmp_path, monkeypatch):
    src = _profile(tmp_path, monkeypatch)
    assert bench.profiled_traffic("knn", {"knn_leaf": 192, "xcd_chunk": 256}) == 12345.0
    # other launch knobs than the counters were taken with
    assert bench.profiled_traffic("knn", {"knn_leaf": 128, "xcd_chunk": 256}) is None
    # a changed source
    src.write_text("kernel source, edited\n")
    assert bench.profiled_traffic("knn", {"knn_leaf": 192, "xcd_chunk": 256}) is None
    # no summary for that kernel
    assert bench.profiled_traffic("fof_link3d") is None


def test_committed_knobs_cover_the_binding():
    with open(bench.TUNE_CACHE) as fh:
        data = json.load(fh)
    assert data["arch"] == "gfx950"
    for k in vr.TUNE_KNOBS:
        assert isinstance(data[k], int), k
    assert data["unbind_wide_sweep"] and data["unbind_sweep"] and data["knn_sweep"]


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(bench.__file__), "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert "one GPU" in (r.stdout + r.stderr)
