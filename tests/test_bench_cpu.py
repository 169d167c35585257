"""Host logic of bench.py (no GPU): the one-GPU contract, the algorithmic byte
counts of the dominant kernel and the matching of the committed traffic
record."""
import json
import pathlib
import subprocess
import sys

import bench

ROOT = pathlib.Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_follow_the_store_layout():
    for ndim in (2, 3):
        # SoA store: cell int32, ndim offsets, three velocities, weight (FP32)
        store = 4 + ndim * 4 + 3 * 4 + 4
        # what the method moves: read the whole store, write all but the weight
        assert bench.BYTES_PER_PARTICLE[ndim] == store + (store - 4)
    # what the gather-map sequence adds: the map entry read, the weight written
    assert bench.EXTRA_BYTES_PER_PARTICLE == {"in place": 0, "gather map": 4 + 4}
    # per cell: E and B read (6 floats), n and J written (4 floats)
    assert bench.BYTES_PER_CELL == 6 * 4 + 4 * 4


def test_at_least_ten_launches_are_timed():
    for steps, every in ((20, 10), (200, 10), (5, 10), (1000, 10), (35, 3), (10, 1)):
        k = bench.timing_stride(steps, every)
        assert 1 <= k <= every
        timed = len(range(0, steps, k))  # launches 0, k, 2k, ... are timed
        assert timed >= min(steps, bench.MIN_TIMED_LAUNCHES)


def test_traffic_record_matches_only_its_workload_and_source():
    path = ROOT / "profiles" / "traffic_gather_push_harris.json"
    rec = json.loads(path.read_text())
    n, mode = rec["n_particles"], rec["mode"]
    other = "in place" if mode == "gather map" else "gather map"
    assert bench._traffic(n + 1, mode) is None
    assert bench._traffic(n, other) is None
    got = bench._traffic(n, mode)
    if rec["source_hash"] == bench._source_hash():
        assert got == rec["bytes_per_launch"]
        assert got == rec["fetch_bytes"] + rec["write_bytes"]
    else:
        assert got is None  # the kernel changed since the counters were taken
