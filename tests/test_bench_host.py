"""Host-side logic of bench.py (no GPU): the --tuning string round trip,
the guard that reports profiled HBM traffic only for the sources and tuning
it was measured on, and the one-GPU refusal."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tuning_spec_round_trip():
    spec = "r2c:y=0/16,z=2/16;c2c3:y=2/4,z=3/64"
    t = bench.parse_tuning(spec)
    assert t == {"r2c": {1: (0, 16), 2: (2, 16)}, "c2c3": {1: (2, 4), 2: (3, 64)}}
    table = {nm: {f"axis{ax}": {"variant": v, "chunk": c} for ax, (v, c) in d.items()}
             for nm, d in t.items()}
    assert bench.tuning_spec(table) == spec


def test_traffic_only_for_matching_sources_and_tuning(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (tmp_path / "paper_1508_05610_amd").mkdir()
    os.symlink(os.path.join(ROOT, "paper_1508_05610_amd", "csrc"),
               tmp_path / "paper_1508_05610_amd" / "csrc")
    rec = {"source_hash": bench.kernel_source_hash(), "tuning": "r2c:y=0/16,z=2/16",
           "records": {"k_strided<512,-1,0,1> z 512x512x512/1": {"hbm_bytes_per_launch": 123.0}}}
    (prof / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    z = "k_strided<512,-1,0,1> z 512x512x512/1"
    assert bench.measured_traffic(z, "r2c:y=0/16,z=2/16") == 123.0
    assert bench.measured_traffic(z, "r2c:y=1/16,z=2/16") is None
    # the same kernel symbol on another pass or shape is another record
    assert bench.measured_traffic("k_strided<512,-1,0,1> y 512x512x512/3", "r2c:y=0/16,z=2/16") is None
    assert bench.measured_traffic("k_x_r2c_v<256> 512x512x512/1", "r2c:y=0/16,z=2/16") is None
    rec["source_hash"] = "0" * 16
    (prof / "traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic(z, "r2c:y=0/16,z=2/16") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout == ""
