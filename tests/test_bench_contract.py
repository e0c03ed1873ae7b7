"""The benchmark line's accounting, on the CPU: the method's bytes per launch
(14 B per synapse generated, 28 B per synapse of calibration split over the
sort's record-moving launches), the implementation's moved bytes per kernel
of the most-significant-digit form, the committed HBM counter summaries
looked up by kernel, workload and source fingerprint, and the refusal of a
multi-GPU run."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

N = 300_000_000


def test_generation_bytes_follow_the_synapses_each_kernel_made():
    kernels = {"generate": (4, 1.5, 115_000_000), "generate_batch": (5, 2.6, 185_000_000)}
    assert bench.algorithmic_bytes("generate", N, kernels, 1) == 14.0 * 115_000_000
    assert bench.algorithmic_bytes("generate_batch", N, kernels, 1) == 14.0 * 185_000_000
    # two steps: the records are summed over both
    assert bench.algorithmic_bytes("generate_batch", N, kernels, 2) == 14.0 * 185_000_000 / 2
    # without records (one launch per call, untimed records): all synapses
    assert bench.algorithmic_bytes("generate", N, {"generate": (64, 1.4)}, 1) == 14.0 * N


def test_calibration_bytes_split_over_record_moving_launches():
    msd = {"msd_scatter_a": (1, 1.8), "msd_scatter_b": (1, 1.7), "msd_tiles_c": (1, 1.9), "msd_count_a": (1, 0.3)}
    parts = [bench.algorithmic_bytes(k, N, msd) for k in ("msd_scatter_a", "msd_scatter_b", "msd_tiles_c")]
    assert sum(parts) == pytest.approx(28.0 * N)
    assert bench.algorithmic_bytes("msd_count_a", N, msd) is None
    lsd = {"downsweep": (3, 6.5), "upsweep": (3, 0.9)}
    assert bench.algorithmic_bytes("downsweep", N, lsd) == pytest.approx(28.0 * N)


def test_moved_bytes_of_the_microcircuit_plan():
    plan = {"msd": 2, "b1": 9, "b2": 8, "b3": 5, "narrow_a": 1, "narrow_b": 1}
    per = {k: bench.moved_bytes(k, N, plan) / N for k in
           ("msd_count_a", "msd_scatter_a", "msd_count_b", "msd_scatter_b", "msd_tiles_c")}
    assert per == {"msd_count_a": 4.0, "msd_scatter_a": 22.0, "msd_count_b": 4.0, "msd_scatter_b": 16.0,
                   "msd_tiles_c": 22.0}
    wide = dict(plan, narrow_a=0, narrow_b=0)
    assert bench.moved_bytes("msd_scatter_b", N, wide) == 24.0 * N
    assert bench.moved_bytes("msd_tiles_c", N, {"msd": 0}) is None


def test_traffic_lines_match_the_committed_sources():
    # every traffic line in profiles/ that names a kernel of the current
    # sources is found; an unknown workload or kernel gives None
    found = 0
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if "traffic" not in name:
            continue
        for line in open(os.path.join(ROOT, "profiles", name)):
            line = line.strip()
            if line.startswith("{"):
                rec = json.loads(line)
                if rec["kernels_sha"] == bench.kernels_fingerprint(rec["kernel"]):
                    assert bench.measured_traffic(rec["kernel"], rec["workload"]) == rec["bytes_per_launch"]
                    found += 1
    assert found >= 1
    assert bench.measured_traffic("msd_tiles_c", "no_such_workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
