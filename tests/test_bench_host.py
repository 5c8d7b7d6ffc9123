"""Host-side pieces of the benchmark (CPU): the one-GPU guard, the
algorithmic instruction count behind the ALU roofline, and the guard that
drops a measured traffic figure once the kernel source or the launch choices
it was taken with change."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2507_10424_amd import workloads as wl  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_min_pair_instruction_counts():
    # first group of three: 2; each further group of three: 5; each leftover: 2
    assert [bench.min_pair_ops(d) for d in (1, 2, 3, 4, 5, 6, 7, 9, 16)] == [0, 2, 2, 4, 6, 7, 9, 12, 24]


def test_alu_count_of_the_36_code():
    # per row of degree 6: 6 subtractions, 7 for the min pair, 3 + 3 XORs,
    # 2 to form K, 12 for clamp and subtract = 33; per bit of degree 3: 3
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    assert bench.alu_ops_per_frame_iter(H) == 512 * 33 + 1024 * 3 == 19968


def test_alu_count_skips_rows_of_degree_below_two():
    H = np.zeros((3, 5), np.uint8)
    H[0, [0, 1, 2]] = 1  # degree 3: 3 + 2 + 2 + 2 + 6 = 15
    H[1, 3] = 0          # degree 0: nothing
    H[2, [3, 4]] = 1     # degree 2: 2 + 2 + 2 + 2 + 4 = 12
    assert bench.alu_ops_per_frame_iter(H) == 15 + 12 + int(H.sum())


def test_measured_traffic_guards():
    rec = bench.MEASURED_TRAFFIC[("qc64800", "check")]
    assert bench.measured_traffic("qc64800", "check", None) is None  # taken with chunks: needs the tuning
    other = {"path": 2, "stream_nt": 1, "stream_chunk": -1}
    assert bench.measured_traffic("qc64800", "check", other) is None
    same = dict(rec["tuning"])
    val = bench.measured_traffic("qc64800", "check", same)
    assert val in (None, rec["bytes"])  # None only once the kernel source has changed since it was measured
    assert bench.measured_traffic("regular96", "onchip", None) is None  # nothing measured
