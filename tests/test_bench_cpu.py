"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message (one GPU is measured), and the traffic figure it reports is
keyed to the sources of the kernel it describes."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_summary_matches_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    d = json.load(open(os.path.join(ROOT, "profiles",
                                    "traffic_shared_rowpair_kernel_protein_search.json")))
    assert d["kernel"] == bench.KERNEL_NAME
    assert tuple(d["hashed_sources"]) == bench.TRAFFIC_SOURCES
    # reported while the sources are those the counters were taken on, else null
    if d["csrc_sha256"] == bench._csrc_sha256():
        assert bench._measured_traffic() == d["hbm_bytes_per_launch"] > 0
    else:
        assert bench._measured_traffic() is None
