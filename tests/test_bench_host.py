"""Host-side logic of bench.py (no GPU): argument contract, kernel naming, counter lookup."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_names_follow_the_launched_instances():
    assert bench.kernel_name({"kernel": 0}) == "k_gett_small"
    assert bench.kernel_name({"kernel": 1, "tile": 1, "lds_copy": 0}) == "void k_gett_mfma<0, 2, 2>"
    assert bench.kernel_name({"kernel": 2, "tile": 3, "lds_copy": 0}) == "void k_gett_mfma<1, 1, 1>"
    assert bench.kernel_name({"kernel": 2, "tile": 0, "lds_copy": 1}) == "void k_gett_dma<1, 0>"
    assert bench.kernel_name({"kernel": 3, "tile": 0, "lds_copy": 2}) == "void k_gett_dma<2, 1>"
    assert bench.kernel_name({"kernel": 2, "tile": 0, "lds_copy": 3}) == "void k_gett_dma<1, 2>"


def test_counter_traffic_only_for_known_kernels_of_the_recorded_source_and_chunk():
    assert bench.measured_traffic("void no_such_kernel<0>", 32) is None
    t = bench.measured_traffic("void k_gett_dma<1, 0>", 32)
    # recorded for the current kernel source: a per-launch byte count of the right magnitude
    assert t is None or 1e9 < t < 1e11
    # another slice chunk runs other launches: no figure
    assert bench.measured_traffic("void k_gett_dma<1, 0>", 8) is None


def test_slice_samples_are_seeded_sorted_and_distinct():
    a = bench.sample_slices(256, 8)
    assert a == bench.sample_slices(256, 8)
    assert a == sorted(set(a)) and len(a) == 8 and all(0 <= x < 256 for x in a)
    assert bench.sample_slices(4, 8) == [0, 1, 2, 3]
