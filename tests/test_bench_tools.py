"""CPU checks of bench.py's pure helpers (the kernel-trace concurrency summary and the survey's
per-step work model)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_trace_overlap(tmp_path):
    p = tmp_path / "kt.csv"
    rows = [("k_a", 1, 0, 10), ("k_b", 2, 5, 15), ("k_c", 1, 20, 30), ("k_d", 3, 22, 24)]
    with open(p, "w") as f:
        f.write("Kernel_Name,Queue_Id,Start_Timestamp,End_Timestamp\n")
        for n, q, a, b in rows:
            f.write(f"{n},{q},{a * 10**6},{b * 10**6}\n")
    st = bench.trace_overlap(str(p))
    assert st["kernels"] == 4 and st["queues"] == 3 and st["max_concurrent"] == 2
    assert abs(st["kernel_time_ms"] - 32) < 1e-9 and abs(st["busy_ms"] - 25) < 1e-9
    assert abs(st["share_of_busy_with_2plus"] - 7 / 25) < 1e-12


def test_survey_work_model():
    N, K, P, tiles, pw, pb = 1_000_000, 8_000_000, 2_073_600, 8160, 1.6e8, 8e7
    assert bench.survey_work("S5 sort", N, K, P, tiles, pw, pb) == (24 * K, 0.0)
    b, ops = bench.survey_work("S8 blend backward", N, K, P, tiles, pw, pb)
    assert b == 76 * K + 32 * P and ops == 20 * pw + 31 * pb
    assert abs(bench.LANE_OP_PEAK_TOPS - 39.3216) < 1e-9
    # every library stage belongs to exactly one survey step
    stages = [s for v in bench.SURVEY_STEPS.values() for s in v]
    assert len(stages) == len(set(stages)) == 9
