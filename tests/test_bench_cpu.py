"""Host-side logic of bench.py (no GPU): the algorithmic byte and MFMA counts
it reports, the guard on recorded HBM traffic, and the one-GPU contract."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_detection_bytes_per_subcarrier():
    # read H (B x U) and Y (B x S) once, write U x S x m FP32 LLRs
    assert bench.detect_bytes_per_sc(128, 16, 14, 6) == 8 * 128 * 16 + 8 * 128 * 14 + 4 * 16 * 14 * 6
    assert bench.detect_bytes_per_sc(128, 16, 14, 6) == 36096
    assert bench.detect_bytes_per_sc(128, 16, 14, 6, elem_bytes=4) == 4 * 128 * 30 + 4 * 16 * 14 * 6
    assert bench.precode_bytes_per_sc(128, 16, 14) == 8 * 128 * 16 + 8 * 16 * 14 + 8 * 128 * 14


def test_mfma_counts_match_the_instruction_counters():
    # SQ_INSTS_MFMA read 4,915,200 (detection) and 5,222,400 (precoding) per
    # launch of 19,200 subcarriers of the 128x16 workload (K = 4, S = 14)
    assert bench.mfma_count(128, 16, 14, 4, "detect") * 19200 == 4915200
    assert bench.mfma_count(128, 16, 14, 4, "precode") * 19200 == 5222400
    # U = 32: four 16x16 tiles, three in the upper triangle
    g = bench.mfma_count(256, 32, 14, 6, "gram_mf")
    assert g == 64 * (2 * 3 + 4) + 64 * 3 * 2


def test_recorded_traffic_only_for_matching_launch():
    rec = bench.recorded_traffic("detect_stream_kernel", "mixed_128x16", 19200)
    if rec is not None:                     # present while the kernel sources are unchanged
        assert rec["bytes_per_launch"] > bench.detect_bytes_per_sc(128, 16, 14, 6) * 19200 * 0.99
    assert bench.recorded_traffic("detect_stream_kernel", "mixed_128x16", 1200) is None
    assert bench.recorded_traffic("no_such_kernel", "mixed_128x16", 19200) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
