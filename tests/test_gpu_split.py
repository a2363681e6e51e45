"""GPU parity of the split kernels (schedule variant "split"): four
wavefronts per subcarrier, each accumulating the Gram (and the matched
filter) over a quarter of the antennas, wave 0 running the CG; the precoder
keeps each wave's quarter of H in registers for q = H v.

The antenna split sums the Gram in another order than the one-wavefront
kernels, so results are compared with the FP64 oracle at the usual
tolerances (and with stream-small to rounding), not bitwise.  Cases cover
the 256 x 32 Kronecker workload with FP64 CG scalars, 128 x 32, 128 x 16,
U <= 8, ragged B (uneven quarters, empty quarters at B = 8), S = 1 and 16,
zero-forcing precoding, fewer subcarriers than workgroups, persistent grids,
and the calls that fall back to the stream-small kernels.
"""
import zlib

import numpy as np
import pytest

from oracle import mimo_oracle as O
from paper_1404_0424_amd import workload as W

from _parity import TOL_L, TOL_X, dev, host, llr_err, rel_err_scalar, rel_err_vec

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


def _with(op, U, variant, bpc, fn):
    from paper_1404_0424_amd import autotune
    saved = autotune.get_schedule(op, U, 0)
    try:
        autotune.set_schedule(op, U, 0, autotune.variants(op).index(variant), bpc)
        out = fn()
        torch.cuda.synchronize()
        return out
    finally:
        autotune.set_schedule(op, U, 0, *saved)


# (name, n_sc, B, U, S, qam_bits, K, snr_db, channel, scalar, blocks_per_cu)
CASES = [
    ("corr_256x32_f64", 600, 256, 32, 14, 8, 6, 25.0, "kronecker", "f64", 0),
    ("mixed_128x32", 900, 128, 32, 14, 6, 4, 15.0, "iid", "f32", 2),
    ("mixed_128x16", 900, 128, 16, 14, 6, 4, 15.0, "iid", "f32", 0),
    ("small_U_128x8", 500, 128, 8, 14, 4, 3, 10.0, "iid", "f32", 3),
    ("ragged_30x5_S3", 400, 30, 5, 3, 6, 4, 12.0, "iid", "f32", 0),
    ("empty_quarters_8x4_S16", 300, 8, 4, 16, 2, 3, 10.0, "iid", "f32", 1),
    ("ragged_100x20_S1", 350, 100, 20, 1, 4, 5, 14.0, "iid", "f32", 0),
    ("few_subcarriers_128x32", 5, 128, 32, 14, 6, 4, 15.0, "iid", "f32", 0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_split_detection(case):
    name, n, B, U, S, m, K, snr, ch, scalar, bpc = case
    print(f"split detection {name}", flush=True)
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    f = W.uplink_frame(rng, n, B, U, S, m, snr, channel=ch, rho_bs=0.5, rho_ue=0.2)
    H, Y = dev(f.H), dev(f.Y)
    run = lambda: api().detect_cg(H, Y, f.n0, f.es, K, m, "approx", scalar, xhat=True)  # noqa: E731
    o = _with("detect", U, "split", bpc, run)
    r = _with("detect", U, "stream-small", 0, run)
    ref = O.detect_cg(f.H, f.Y, f.n0, f.es, K, m, "approx")
    ex = rel_err_vec(host(o["xhat"]), ref["xhat"], axis=1)
    el = llr_err(host(o["llr"]), ref["llr"])
    print(f"{name}: eps_x={ex:.2e} eps_L={el:.2e}")
    assert ex <= TOL_X and el <= TOL_L
    assert rel_err_vec(host(o["xhat"]), host(r["xhat"]).astype(np.complex128), axis=1) <= 1e-4


PRE_CASES = [
    ("corr_256x32_f64", 600, 256, 32, 14, 6, 25.0, "kronecker", "f64", 0, True),
    ("mixed_128x32", 900, 128, 32, 14, 4, 15.0, "iid", "f32", 2, True),
    ("mixed_128x16_unnormalized", 900, 128, 16, 14, 4, 15.0, "iid", "f32", 0, False),
    ("small_U_64x8", 500, 64, 8, 14, 3, 10.0, "iid", "f32", 3, True),
    ("ragged_30x5_S3", 400, 30, 5, 3, 4, 12.0, "iid", "f32", 0, True),
    ("empty_quarters_8x4_S16", 300, 8, 4, 16, 3, 10.0, "iid", "f32", 1, True),
    ("ragged_100x20_S1", 350, 100, 20, 1, 5, 14.0, "iid", "f32", 0, True),
    ("few_subcarriers_256x32", 3, 256, 32, 14, 6, 25.0, "iid", "f32", 0, True),
]


@pytest.mark.parametrize("case", PRE_CASES, ids=[c[0] for c in PRE_CASES])
def test_split_precoding(case):
    name, n, B, U, S, K, snr, ch, scalar, bpc, norm = case
    print(f"split precoding {name}", flush=True)
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 1)
    f = W.uplink_frame(rng, n, B, U, S, 4, snr, channel=ch, rho_bs=0.5, rho_ue=0.2)
    d = W.downlink_frame(rng, n, B, U, S, 4, snr, H=f.H)
    H, T = dev(f.H), dev(d.T)
    run = lambda: api().precode_cg(H, T, d.beta, K, norm, scalar)  # noqa: E731
    Q, qn = _with("precode", U, "split", bpc, run)
    Qr, _ = _with("precode", U, "stream-small", 0, run)
    ref = O.precode_cg(f.H, d.T, d.beta, K, norm)
    eq = rel_err_vec(host(Q), ref["Q"], axis=1)
    en = rel_err_scalar(host(qn), ref["qnorm"])
    print(f"{name}: eps_q={eq:.2e} eps_qnorm={en:.2e}")
    assert eq <= TOL_X and en <= TOL_X
    assert rel_err_vec(host(Q), host(Qr).astype(np.complex128), axis=1) <= 1e-4


def test_split_zero_forcing():
    print("split precoding zero-forcing", flush=True)
    rng = np.random.default_rng(77)
    n, B, U, S, K = 200, 64, 16, 14, 16
    f = W.uplink_frame(rng, n, B, U, S, 4, 20.0)
    d = W.downlink_frame(rng, n, B, U, S, 4, 20.0, H=f.H)
    Q, _ = _with("precode", U, "split", 0,
                 lambda: api().precode_cg(dev(f.H), dev(d.T), 0.0, K, False))
    ref = O.precode_cg(f.H, d.T, 0.0, K, False)
    assert rel_err_vec(host(Q), ref["Q"], axis=1) <= TOL_X


# calls the split kernels do not take: S > 16, 16-bit storage, B > 256 (precoding)
def test_split_schedule_falls_back():
    print("split fallbacks", flush=True)
    rng = np.random.default_rng(5)
    f = W.uplink_frame(rng, 60, 64, 8, 20, 4, 10.0)
    o = _with("detect", 8, "split", 0, lambda: api().detect_cg(dev(f.H), dev(f.Y), f.n0, f.es, 3, 4))
    assert llr_err(host(o["llr"]), O.detect_cg(f.H, f.Y, f.n0, f.es, 3, 4)["llr"]) <= TOL_L
    f2 = W.uplink_frame(rng, 40, 320, 16, 14, 4, 10.0)
    d2 = W.downlink_frame(rng, 40, 320, 16, 14, 4, 10.0, H=f2.H)
    Q, _ = _with("precode", 16, "split", 0,
                 lambda: api().precode_cg(dev(f2.H), dev(d2.T), d2.beta, 4, True))
    assert rel_err_vec(host(Q), O.precode_cg(f2.H, d2.T, d2.beta, 4, True)["Q"], axis=1) <= TOL_X
    A = api()
    Hq, Yq = A.convert(dev(f2.H), "bf16"), A.convert(dev(f2.Y), "bf16")
    from paper_1404_0424_amd import autotune
    saved = autotune.get_schedule("detect", 16, Hq.dtype_code)
    try:
        autotune.set_schedule("detect", 16, Hq.dtype_code, autotune.variants("detect").index("split"), 0)
        o = A.detect_cg(Hq, Yq, f2.n0, f2.es, 4, 4)
        torch.cuda.synchronize()
    finally:
        autotune.set_schedule("detect", 16, Hq.dtype_code, *saved)
    Hr = O.dequantize_bf16(O.quantize_bf16(f2.H))
    Yr = O.dequantize_bf16(O.quantize_bf16(f2.Y))
    assert llr_err(host(o["llr"]), O.detect_cg(Hr, Yr, f2.n0, f2.es, 4, 4)["llr"]) <= TOL_L
