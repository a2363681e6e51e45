"""GPU parity of the H-resident precoding kernel (schedule variant
"resident"): the channel of a subcarrier is kept in registers from the Gram
to q = H v, with capacity for 64 or 128 antennas.  Cases cover both
capacities, partial 16-antenna tiles, S = 1 .. 16, U = 1 .. 16, zero forcing,
FP32 and FP64 scalar recurrences, and persistent grids in which every
wavefront walks several subcarriers (the next subcarrier's channel is loaded
during the current one's output stage), for complex64 and FP16/BF16 channel
storage.  Each result is checked against the FP64 oracle (on the rounded
channel for 16-bit storage) and bitwise against the generic kernel, which
performs the same operations in the same order."""
import zlib

import numpy as np
import pytest

from oracle import mimo_oracle as O
from paper_1404_0424_amd import workload as W

from _parity import TOL_X, dev, host, rel_err_scalar, rel_err_vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_0424_amd import _lib
    _lib.lib()       # fail loudly if the library is missing


def api():
    from paper_1404_0424_amd import api as A
    return A


# (name, n_sc, B, U, S, K, snr_db; None = zero forcing)
CASES = [
    ("128x16_S14", 37, 128, 16, 14, 4, 15.0),
    ("100x12_S9", 29, 100, 12, 9, 4, 10.0),
    ("65x16_S16", 21, 65, 16, 16, 5, 20.0),
    ("64x8_S1", 33, 64, 8, 1, 3, 10.0),
    ("30x5_S7", 37, 30, 5, 7, 5, 5.0),
    ("6x1_S3", 9, 6, 1, 3, 1, 10.0),
    ("zf_32x8_S3", 16, 32, 8, 3, 8, None),
]


def _run(H, T, beta, K, U, normalize, scalar, schedules, code=0):
    from paper_1404_0424_amd import autotune
    saved = autotune.get_schedule("precode", U, code)
    outs = []
    try:
        for v, bpc in schedules:
            autotune.set_schedule("precode", U, code, v, bpc)
            Q, qn = api().precode_cg(H, T, beta, K, normalize, scalar)
            outs.append((host(Q), host(qn)))
    finally:
        autotune.set_schedule("precode", U, code, *saved)
    return outs


def _resident():
    from paper_1404_0424_amd import autotune
    return autotune.variants("precode").index("resident")


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("scalar", ["f32", "f64"])
@pytest.mark.parametrize("normalize", [False, True])
def test_resident_precode_parity(case, scalar, normalize):
    name, n, B, U, S, K, snr = case
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    d = W.downlink_frame(rng, n, B, U, S, 6, snr)
    r = _resident()
    outs = _run(dev(d.H), dev(d.T), d.beta, K, U, normalize, scalar,
                [(r, 0), (r, 1), (0, 0)])
    ref = O.precode_cg(d.H, d.T, d.beta, K, normalize)
    eq = rel_err_vec(outs[0][0], ref["Q"], axis=1)
    en = rel_err_scalar(outs[0][1], ref["qnorm"])
    print(f"resident {name} {scalar} norm={normalize}: eps_q={eq:.2e} eps_qnorm={en:.2e}")
    assert eq <= TOL_X and en <= TOL_X
    for q, qn in outs[1:]:
        assert np.array_equal(q, outs[0][0]) and np.array_equal(qn, outs[0][1])


@pytest.mark.parametrize("B,U,S,n", [(128, 16, 14, 2600), (50, 7, 11, 2300)])
def test_resident_persistent_grid_walks_subcarriers(B, U, S, n):
    """One block per compute unit: each wavefront handles 2-3 subcarriers,
    so the channel prefetched during an output stage is the one used next."""
    rng = np.random.default_rng(B * 1000 + U)
    d = W.downlink_frame(rng, n, B, U, S, 6, 15.0)
    r = _resident()
    outs = _run(dev(d.H), dev(d.T), d.beta, 4, U, True, "f32", [(r, 1), (r, 3), (0, 0)])
    for q, qn in outs[1:]:
        assert np.array_equal(q, outs[0][0]) and np.array_equal(qn, outs[0][1])
    idx = np.sort(np.random.default_rng(7).choice(n, 40, replace=False))
    idx[0], idx[-1] = 0, n - 1
    ref = O.precode_cg(d.H[idx], d.T[idx], d.beta, 4, True)
    assert rel_err_vec(outs[0][0][idx], ref["Q"], axis=1) <= TOL_X
    assert rel_err_scalar(outs[0][1][idx], ref["qnorm"]) <= TOL_X


def test_resident_falls_back_outside_its_shapes():
    """U > 16, S > 16 or B > 128 use the streaming / generic kernels."""
    r = _resident()
    for (n, B, U, S) in [(9, 128, 20, 5), (7, 40, 8, 17), (5, 136, 8, 4)]:
        rng = np.random.default_rng(n * B)
        d = W.downlink_frame(rng, n, B, U, S, 6, 12.0)
        outs = _run(dev(d.H), dev(d.T), d.beta, 3, U, True, "f32", [(r, 0), (0, 0)])
        assert np.array_equal(outs[0][0], outs[1][0])
        ref = O.precode_cg(d.H, d.T, d.beta, 3, True)
        assert rel_err_vec(outs[0][0], ref["Q"], axis=1) <= TOL_X


# 16-bit storage keeps B a multiple of 8; 104 and 72 antennas end in half tiles
CASES16 = [
    ("128x16_S14", 37, 128, 16, 14, 4, 15.0),
    ("104x12_S9", 29, 104, 12, 9, 4, 10.0),
    ("72x16_S16", 21, 72, 16, 16, 5, 20.0),
    ("64x8_S1", 33, 64, 8, 1, 3, 10.0),
    ("24x5_S7", 37, 24, 5, 7, 5, 5.0),
    ("8x1_S3", 9, 8, 1, 3, 1, 10.0),
]


def _quantized(H, dt):
    deq = O.dequantize_f16 if dt == "f16" else O.dequantize_bf16
    qz = O.quantize_f16 if dt == "f16" else O.quantize_bf16
    return deq(qz(H))


@pytest.mark.parametrize("case", CASES16, ids=[c[0] for c in CASES16])
@pytest.mark.parametrize("dt", ["f16", "bf16"])
@pytest.mark.parametrize("scalar", ["f32", "f64"])
def test_resident_precode_16bit_parity(case, dt, scalar):
    name, n, B, U, S, K, snr = case
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 1)
    d = W.downlink_frame(rng, n, B, U, S, 6, snr)
    Hx = api().convert(dev(d.H), dt)
    r = _resident()
    outs = _run(Hx, dev(d.T), d.beta, K, U, True, scalar, [(r, 0), (r, 1), (0, 0)],
                Hx.dtype_code)
    ref = O.precode_cg(_quantized(d.H, dt), d.T, d.beta, K, True)
    eq = rel_err_vec(outs[0][0], ref["Q"], axis=1)
    en = rel_err_scalar(outs[0][1], ref["qnorm"])
    print(f"resident {dt} {name} {scalar}: eps_q={eq:.2e} eps_qnorm={en:.2e}")
    assert eq <= TOL_X and en <= TOL_X
    for q, qn in outs[1:]:
        assert np.array_equal(q, outs[0][0]) and np.array_equal(qn, outs[0][1])


@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_resident_16bit_persistent_grid_walks_subcarriers(dt):
    n, B, U, S = 2600, 128, 16, 14
    rng = np.random.default_rng(99)
    d = W.downlink_frame(rng, n, B, U, S, 6, 15.0)
    Hx = api().convert(dev(d.H), dt)
    r = _resident()
    outs = _run(Hx, dev(d.T), d.beta, 4, U, True, "f32", [(r, 1), (r, 3), (0, 0)],
                Hx.dtype_code)
    for q, qn in outs[1:]:
        assert np.array_equal(q, outs[0][0]) and np.array_equal(qn, outs[0][1])
    idx = np.sort(np.random.default_rng(8).choice(n, 40, replace=False))
    idx[0], idx[-1] = 0, n - 1
    ref = O.precode_cg(_quantized(d.H[idx], dt), d.T[idx], d.beta, 4, True)
    assert rel_err_vec(outs[0][0][idx], ref["Q"], axis=1) <= TOL_X
