"""Host-side logic of bench.py (no GPU): the algorithmic byte and MFMA counts
it reports, the guard on recorded HBM traffic, the one-GPU contract, and the
report of sampled GPU results against the oracle."""
import os
import subprocess
import sys

import bench
import numpy as np
import pytest

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
    # U = 8: packed Gram (1 per k-step) and matched filter (2), mat-vec over
    # the 2 k-steps of real users (4 each), q = H v 3 per k-step and tile
    assert bench.mfma_count(128, 8, 14, 3, "detect") == 32 * 1 + 32 * 2 + 3 * 8
    assert bench.mfma_count(128, 8, 14, 3, "precode") == 32 * 1 + 4 * 8 + 8 * 3 * 2
    assert bench.mfma_count(128, 8, 14, 3, "gram_mf") == 32 * 3 + 32 * 3
    # U = 20: the second user tile holds one k-step of real users
    assert bench.mfma_count(64, 20, 14, 2, "detect") == 16 * 10 + 16 * 6 + 2 * 4 * 2 * 5


def test_wide_mfma_counts_match_the_instruction_counters():
    # SQ_INSTS_MFMA read 45,465,600 (detection) and 50,380,800 (precoding)
    # per launch of 19,200 subcarriers of 128x64 (K = 4, S = 14)
    assert bench.mfma_count_wide(128, 64, 14, 4, "detect") * 19200 == 45465600
    assert bench.mfma_count_wide(128, 64, 14, 4, "precode") * 19200 == 50380800
    # U = 40: role 3 has no users (no tiles, no matched filter); the
    # mat-vec runs over the 10 k-steps of real users in all four roles
    assert bench.mfma_count_wide(128, 40, 14, 4, "detect") == \
        32 * (9 + 9 + 6) + 32 * 3 * 3 + 4 * 16 * 10


def test_recorded_traffic_only_for_matching_launch():
    for persistent in (False, True):
        rec = bench.recorded_traffic("detect_stream_kernel", "mixed_128x16", 19200, persistent)
        if rec is not None:                 # present while the kernel sources are unchanged
            assert rec["bytes_per_launch"] > bench.detect_bytes_per_sc(128, 16, 14, 6) * 19200 * 0.99
    assert bench.recorded_traffic("detect_stream_kernel", "mixed_128x16", 1200) is None
    assert bench.recorded_traffic("no_such_kernel", "mixed_128x16", 19200) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_sample_index_is_sorted_and_keeps_the_last_subcarrier():
    idx = bench.sample_index(100, 24, 3)
    assert len(idx) == 24 and idx[-1] == 99 and np.all(np.diff(idx) > 0)
    assert list(bench.sample_index(5, 24, 3)) == [0, 1, 2, 3, 4]


def _detect_precode_refs(rng):
    from oracle import mimo_oracle as O
    from paper_1404_0424_amd import workload as W
    up = W.uplink_frame(rng, 6, 16, 4, 3, 4, 10.0)
    dn = W.downlink_frame(rng, 6, 16, 4, 3, 4, 10.0, H=up.H)
    return O, up, dn


def test_oracle_errors_measure_a_planted_deviation():
    """The error report against the oracle finds deviations planted in
    otherwise exact results, with the metrics' definitions."""
    O, up, dn = _detect_precode_refs(np.random.default_rng(5))
    r = O.detect_cg(up.H, up.Y, up.n0, up.es, 3, 4, "approx")
    p = O.precode_cg(up.H, dn.T, dn.beta, 3, normalize=True)
    x, L, Q = r["xhat"].copy(), r["llr"].copy(), p["Q"].copy()
    x[2, :, 1] *= 1 + 1e-3                           # one user vector, 1e-3 relative
    scale = max(1.0, float(np.abs(L[4, 1, 2]).max()))
    L[4, 1, 2, 0] += 0.5 * scale                     # one LLR, 0.5 of its symbol's scale
    Q[1, :, 0] *= 1 - 2e-4                           # one precoded vector
    samples = [{"label": "d", "op": "detect", "storage": "c32", "H": up.H, "Y": up.Y,
                "n0": up.n0, "es": up.es, "K": 3, "m": 4, "xhat": x, "llr": L},
               {"label": "p", "op": "precode", "storage": "c32", "H": up.H, "T": dn.T,
                "beta": dn.beta, "K": 3, "Q": Q}]
    e = bench.oracle_errors(samples, O)
    assert e["d"]["eps_x"] == pytest.approx(1e-3, rel=1e-6)
    assert e["d"]["eps_llr"] == pytest.approx(0.5, rel=1e-9)
    assert e["p"]["eps_q"] == pytest.approx(2e-4, rel=1e-6)
    assert e["d"]["subcarriers"] == 6


def test_oracle_errors_16bit_against_rounded_inputs():
    """For 16-bit storage the report also compares with the oracle on the
    rounded inputs: exact there for results computed from them."""
    O, up, dn = _detect_precode_refs(np.random.default_rng(6))
    rnd = lambda z: O.dequantize_bf16(O.quantize_bf16(z))          # noqa: E731
    r = O.detect_cg(rnd(up.H), rnd(up.Y), up.n0, up.es, 3, 4, "approx")
    p = O.precode_cg(rnd(up.H), dn.T, dn.beta, 3, normalize=True)
    samples = [{"label": "d", "op": "detect", "storage": "bf16", "H": up.H, "Y": up.Y,
                "n0": up.n0, "es": up.es, "K": 3, "m": 4, "xhat": r["xhat"], "llr": r["llr"]},
               {"label": "p", "op": "precode", "storage": "bf16", "H": up.H, "T": dn.T,
                "beta": dn.beta, "K": 3, "Q": p["Q"]}]
    e = bench.oracle_errors(samples, O)
    assert e["d"]["eps_x_vs_rounded_inputs"] == 0.0
    assert e["d"]["eps_llr_vs_rounded_inputs"] == 0.0
    assert e["p"]["eps_q_vs_rounded_inputs"] == 0.0
    assert 1e-4 < e["d"]["eps_x"] < 3e-2 and 1e-4 < e["p"]["eps_q"] < 3e-2


def test_cpu_all_cores_oracle_run():
    """The all-cores oracle leg: spawned worker processes (one BLAS thread
    each) run the oracle over chunks of the workload for the given time."""
    from paper_1404_0424_amd import workload as W
    wl = W.WORKLOADS["small_32x8"]
    rng = np.random.default_rng(0)
    up = W.uplink_frame(rng, 64, wl.B, wl.U, wl.S, wl.m, 10.0)
    dn = W.downlink_frame(rng, 64, wl.B, wl.U, wl.S, wl.m, 10.0, H=up.H)
    done, secs = bench.cpu_all_cores(up, dn, wl, 0.5, 2)
    assert done > 0 and done % 16 == 0 and secs >= 0.5
    assert 1 <= bench.host_workers() <= 16
    assert bench.cpu_model()
