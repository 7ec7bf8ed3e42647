"""bench.py's command-line contract and its committed counter summary (no GPU
needed): more than one GPU is refused with a message, and the HBM counters
that feed roofline.traffic were taken on the current kernel source."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_committed_counters_match_kernel_source():
    import bench
    p = os.path.join(ROOT, "profiles", "k_transport_water_cbct_pmc.json")
    d = json.load(open(p))
    assert d["kernel_sha"] == bench.kernel_source_hash(), \
        "re-take the transport counters after changing the kernel source"
    traffic = bench.load_traffic("water_cbct", d["histories_per_launch"])
    assert traffic is not None and traffic > 0
    # written bytes dominate: 32 B per memory-side int64 tally atomic
    assert d["write_kib_per_launch"] > 100 * d["fetch_kib_per_launch"]
