"""Host-side logic of bench.py (no GPU): the one-GPU guard, the HBM
traffic figures that are reported only for the kernel sources they were
measured on, and the choice of the HP reliable-update trigger."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_recorded_traffic_follows_the_kernel_sources():
    import bench
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as fh:
        rec = json.load(fh)
    key, k = next(iter(rec["kernels"].items()))
    name, blk = key.rsplit(" block=", 1)
    blk = int(blk)
    got = bench.recorded_traffic(name, rec["workload"], blk)
    if rec["kernel_source_sha"] == bench.kernel_source_sha():
        assert got == k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
    else:
        assert got is None
    assert bench.recorded_traffic(name, rec["workload"], blk + 1) is None
    assert bench.recorded_traffic(name, "another workload", blk) is None
    assert bench.recorded_traffic("no such kernel", rec["workload"], blk) is None


def test_source_hash_depends_on_contents(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "paper_1211_0126_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "a.hip").write_text("x")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h1 = bench.kernel_source_sha()
    (src / "a.hip").write_text("y")
    assert bench.kernel_source_sha() != h1


def test_trigger_choice_skips_stalled_candidates():
    import bench
    cands = {0.1: {"ms": 300.0, "converged": True}, 3e-3: {"ms": 260.0, "converged": True},
             1e-4: {"ms": 100.0, "converged": False}}
    assert bench.pick_delta(cands) == 3e-3
    assert bench.pick_delta({1e-4: {"ms": 1.0, "converged": False}}) == 0.1
