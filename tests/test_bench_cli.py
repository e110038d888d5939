"""The benchmark's command-line contract on the CPU: it measures one GPU,
so a request for more exits with status 2 and says why, before anything
touches a device; the traffic record is read only while the kernel sources
hash to the value recorded with the counters; the graph length divides the
timed steps."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single" in r.stderr
    assert r.stdout == ""


def test_traffic_record_keyed_to_sources(monkeypatch):
    sha = bench.kernel_sources_sha()
    assert len(sha) == 16 and all(c in "0123456789abcdef" for c in sha)
    rec = {}
    for line in open(os.path.join(ROOT, "profiles", "hill_tiles_walkers256_traffic.txt")):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            rec[k.strip()] = v.strip()
    # with the recorded hash the figure is read; with any other it is not
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: rec["kernel_sources_sha"])
    assert bench.measured_traffic(4096) == float(rec["traffic_bytes_per_launch.tile4096"])
    assert bench.measured_traffic(8192) is None  # no counters at that tile
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: "0" * 16)
    assert bench.measured_traffic(4096) is None


def test_graph_length_divides_the_timed_steps():
    # the timed region is whole graphs of exactly --steps steps
    for steps in (1, 7, 20, 50, 64, 97, 100, 2000):
        g = bench.graph_len(steps, 50)
        assert 1 <= g <= 50 and steps % g == 0
        assert all(steps % h for h in range(g + 1, min(50, steps) + 1))  # the largest such
    assert bench.graph_len(20, 50) == 20 and bench.graph_len(2000, 50) == 50 and bench.graph_len(97, 50) == 1


def test_tuning_cache_covers_the_benchmark_shape():
    # the benchmark's 256-walker shape (capacity = hills + 64 per walker, each
    # segment padded to 32 hills) has a recorded tiling, so the timed run
    # never searches for one; a change of the state layout shows up here
    import json

    import numpy as np

    from paper_2301_04835_amd import synth

    p = synth.WALKERS256
    d = synth.walkers_inputs(n_walkers=p["n_walkers"], seed=3)
    cap = np.asarray(d["n_hills"], dtype=np.int64) + 64
    total = int(np.sum((cap + 31) // 32 * 32))
    cache = json.load(open(os.path.join(ROOT, "paper_2301_04835_amd", "tuning_mi355x.json")))
    keys = [k for k in cache if "/D2/W%d/cap%d/fuse1" % (p["n_walkers"], total) in k]
    assert keys and all(k.startswith("gfx950") for k in keys)
