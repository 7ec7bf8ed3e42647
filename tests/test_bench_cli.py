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
    """Every committed transport counter summary was taken on the current
    kernel source with the launch configuration its workload's main leg
    times, so bench.py reports its traffic; the head's is one of them."""
    import glob

    import bench
    files = glob.glob(os.path.join(ROOT, "profiles", "k_transport_*_pmc.json"))
    names = {os.path.basename(f)[len("k_transport_"):-len("_pmc.json")] for f in files}
    assert {"head", "water_cbct"} <= names
    for name in names:
        d = json.load(open(os.path.join(ROOT, "profiles", f"k_transport_{name}_pmc.json")))
        assert d["kernel_sha"] == bench.kernel_source_hash(), \
            f"re-take the {name} transport counters after changing the kernel source"
        assert tuple(d["tuning"][k] for k in bench.TUNING_KEYS) == bench.PINNED_TUNING[name]
        assert d["commands"] == bench.counter_commands(name)
        assert bench.load_traffic(name, d["histories_per_launch"]) > 0
    w = json.load(open(os.path.join(ROOT, "profiles", "k_transport_water_cbct_pmc.json")))
    # written bytes dominate on the water cylinder: 32 B per memory-side int64 tally atomic
    assert w["write_kib_per_launch"] > 100 * w["fetch_kib_per_launch"]
