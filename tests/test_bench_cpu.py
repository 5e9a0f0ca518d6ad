"""The benchmark script's contract pieces that need no GPU: the one-GPU
refusal, the calibration-scaled traffic lookup and the source digests."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    for workload in ("medium", "jastrow", "density", "cusp", "det", "large", "batch96"):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--workload", workload],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2, (workload, r.stderr[-500:])
        line = json.loads(r.stdout.strip().splitlines()[-1])
        assert "error" in line and "one GPU" in line["error"] or "--gpus must be 1" in line["error"]


def test_traffic_lookup_reads_the_committed_summary():
    import bench
    # digests are stable hex strings per kernel class
    d = {c: bench.sources_digest(c) for c in ("ao", "mo", "gbar", "dcoef", "ao_adjoint")}
    assert all(len(v) == 16 for v in d.values())
    assert d["mo"] == d["gbar"] == d["dcoef"]
    # a class the summary does not hold, or another mode, has no traffic figure
    assert bench.measured_traffic("fp64", "no_such_class") is None
    assert bench.measured_traffic("no_such_mode", "mo") is None
    v = bench.measured_traffic("fp64", "ao")
    assert v is None or v > 4e9  # the AO stage writes its 4.59 GB output
