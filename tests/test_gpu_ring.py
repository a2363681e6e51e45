"""GPU parity of the LDS-ring detection kernel (schedule variant "ring").

The ring kernel streams each subcarrier's H and Y through LDS slots in
chunks of 16 antennas and counts its outstanding memory operations itself;
it runs for complex64 storage, S <= 16, at least three chunks per
subcarrier and LLR-only calls (other calls take the stream-small kernel).
Each case runs LLR-only detection under the ring schedule and under
stream-small, checks the two bitwise equal (same MFMA k-steps in the same
order), and checks a sample of subcarriers, the last one included, against
the FP64 oracle.  The shapes cover full and partial last chunks, exactly
three chunks, the packed form (U <= 8), odd U, S = 1 and S = 16, every QAM
order, FP64 CG scalars, many subcarriers per wave (persistent grids) and
fewer subcarriers than waves.
"""
import zlib

import numpy as np
import pytest

from oracle import mimo_oracle as O
from paper_1404_0424_amd import workload as W

from _parity import TOL_L, TOL_X, dev, host, llr_err, rel_err_vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_0424_amd import _lib
    _lib.lib()


def api():
    from paper_1404_0424_amd import api as A
    return A


# (name, n_sc, B, U, S, qam_bits, K, snr_db, scalar, blocks_per_cu)
CASES = [
    ("mixed_128x16", 3000, 128, 16, 14, 6, 4, 15.0, "f32", 0),
    ("mixed_128x16_bpc2", 3000, 128, 16, 14, 6, 4, 15.0, "f32", 2),
    ("packed_128x8", 2500, 128, 8, 14, 6, 3, 10.0, "f32", 1),
    ("partial_chunk_72x12_S11", 600, 72, 12, 11, 4, 4, 12.0, "f32", 2),
    ("odd_U_40x5_S3", 500, 40, 5, 3, 6, 4, 12.0, "f32", 0),
    ("three_chunks_48x16_S16", 700, 48, 16, 16, 8, 5, 20.0, "f32", 1),
    ("qpsk_64x16_S1", 900, 64, 16, 1, 2, 2, 8.0, "f32", 3),
    ("f64_256x16", 400, 256, 16, 14, 8, 6, 25.0, "f64", 0),
    ("few_subcarriers_128x16", 7, 128, 16, 14, 6, 4, 15.0, "f32", 0),
    ("odd_B_even_U_S_49x6_S4", 300, 49, 6, 4, 4, 3, 10.0, "f32", 1),
]


def _run(H, Y, f, K, m, scalar, U, variant, bpc):
    from paper_1404_0424_amd import autotune
    saved = autotune.get_schedule("detect", U, 0)
    try:
        autotune.set_schedule("detect", U, 0, autotune.variants("detect").index(variant), bpc)
        o = api().detect_cg(H, Y, f.n0, f.es, K, m, "approx", scalar)
        torch.cuda.synchronize()
        return host(o["llr"])
    finally:
        autotune.set_schedule("detect", U, 0, *saved)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_ring_matches_stream_and_oracle(case):
    name, n, B, U, S, m, K, snr, scalar, bpc = case
    print(f"ring case {name}", flush=True)
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    f = W.uplink_frame(rng, n, B, U, S, m, snr)
    H, Y = dev(f.H), dev(f.Y)
    L_ring = _run(H, Y, f, K, m, scalar, U, "ring", bpc)
    L_ref = _run(H, Y, f, K, m, scalar, U, "stream-small", 0)
    assert np.array_equal(L_ring, L_ref), name
    idx = np.sort(np.random.default_rng(1).choice(n, min(24, n), replace=False))
    idx[-1] = n - 1
    ref = O.detect_cg(f.H[idx], f.Y[idx], f.n0, f.es, K, m, "approx")
    el = llr_err(L_ring[idx], ref["llr"])
    print(f"{name}: eps_L={el:.2e}")
    assert el <= TOL_L


# Calls the ring kernel does not take: fewer than three 16-antenna chunks,
# odd per-subcarrier arrays (B U or B S odd), S > 16, optional outputs.
FALLBACK = [
    ("two_chunks_32x8", 200, 32, 8, 14, 4, 3, 10.0, False),
    ("odd_bytes_33x5_S3", 150, 33, 5, 3, 4, 3, 10.0, False),
    ("rhs_chunks_64x8_S17", 150, 64, 8, 17, 4, 3, 10.0, False),
    ("with_xhat_128x16", 300, 128, 16, 14, 6, 4, 15.0, True),
]


@pytest.mark.parametrize("case", FALLBACK, ids=[c[0] for c in FALLBACK])
def test_ring_schedule_falls_back(case):
    from paper_1404_0424_amd import autotune
    name, n, B, U, S, m, K, snr, want_x = case
    print(f"ring fallback {name}", flush=True)
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    f = W.uplink_frame(rng, n, B, U, S, m, snr)
    H, Y = dev(f.H), dev(f.Y)
    saved = autotune.get_schedule("detect", U, 0)
    try:
        autotune.set_schedule("detect", U, 0, autotune.variants("detect").index("ring"), 0)
        o = api().detect_cg(H, Y, f.n0, f.es, K, m, xhat=want_x)
        torch.cuda.synchronize()
    finally:
        autotune.set_schedule("detect", U, 0, *saved)
    ref = O.detect_cg(f.H, f.Y, f.n0, f.es, K, m, "approx")
    assert llr_err(host(o["llr"]), ref["llr"]) <= TOL_L
    if want_x:
        assert rel_err_vec(host(o["xhat"]), ref["xhat"], axis=1) <= TOL_X
