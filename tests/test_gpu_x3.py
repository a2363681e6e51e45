"""GPU parity of detection with the Gram and matched filter formed from an
exact three-way bf16 split of the complex64 inputs on the 16-bit matrix
cores (schedule variant "stream-x3"; FP32 accumulation, the six leading
partial products of every product): against the FP64 oracle at the usual
tolerances and against the FP32-MFMA kernels (stream-small) to rounding.

Cases cover one and two user tiles, U <= 8 (which the FP32 form runs
packed), ragged antenna counts (partial 16-antenna groups), more than 16
right-hand sides (the generic kernel with the same blocks), FP64 CG scalars
on the correlated 256 x 32 workload, channels whose entries span many
orders of magnitude, zero receive vectors, and the 128 x 16 batch at full
size, sampled."""
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


def _run(variant, U, bpc, fn):
    from paper_1404_0424_amd import autotune
    saved = autotune.get_schedule("detect", U, 0)
    try:
        autotune.set_schedule("detect", U, 0, autotune.variants("detect").index(variant), bpc)
        out = fn()
        torch.cuda.synchronize()
        return out
    finally:
        autotune.set_schedule("detect", U, 0, *saved)


def _errors(o, ref, sel):
    return (rel_err_vec(sel(host(o["xhat"])), ref["xhat"], axis=1),
            llr_err(sel(host(o["llr"])), ref["llr"]),
            rel_err_scalar(sel(host(o["mu"])), ref["mu"]))


def _check(name, f, K, m, scalar, bpc=0, idx=None, like_fp32=False):
    """x3 against the oracle at the usual tolerances, or (like_fp32) within a
    small factor of the FP32-MFMA kernel's own error on inputs where FP32
    arithmetic itself does not reach them."""
    from paper_1404_0424_amd import api
    U = f.H.shape[2]
    H, Y = dev(f.H), dev(f.Y)
    run = lambda: api.detect_cg(H, Y, f.n0, f.es, K, m, "approx", scalar, xhat=True,  # noqa: E731
                                mu=True, sinr=True)
    o = _run("stream-x3", U, bpc, run)
    r = _run("stream-small", U, 0, run)
    sel = (lambda a: a) if idx is None else (lambda a: a[idx])
    Hs, Ys = sel(f.H), sel(f.Y)
    ref = O.detect_cg(Hs, Ys, f.n0, f.es, K, m, "approx")
    ex, el, emu = _errors(o, ref, sel)
    fx, fl, fmu = _errors(r, ref, sel)
    print(f"{name}: eps_x={ex:.2e} eps_L={el:.2e} eps_mu={emu:.2e} "
          f"(FP32 MFMA: {fx:.2e} {fl:.2e} {fmu:.2e})")
    if like_fp32:
        assert ex <= 4 * fx + 1e-6 and el <= 4 * fl + 1e-5 and emu <= 4 * fmu + 1e-6
        return
    assert ex <= TOL_X and el <= TOL_L and emu <= TOL_X
    assert rel_err_scalar(sel(host(o["sinr"])), ref["rho"]) <= 1e-5
    # to rounding of the FP32-MFMA form
    assert rel_err_vec(host(o["xhat"]), host(r["xhat"]).astype(np.complex128), axis=1) <= 2e-5


# (name, n_sc, B, U, S, qam_bits, K, snr_db, channel, scalar, blocks_per_cu)
CASES = [
    ("mixed_128x16", 400, 128, 16, 14, 6, 4, 15.0, "iid", "f32", 0),
    ("mixed_128x16_persistent", 600, 128, 16, 14, 6, 4, 15.0, "iid", "f32", 2),
    ("small_U_128x8", 300, 128, 8, 14, 6, 3, 10.0, "iid", "f32", 0),
    ("mixed_128x32", 200, 128, 32, 14, 6, 4, 15.0, "iid", "f32", 1),
    ("corr_256x32_f64", 150, 256, 32, 14, 8, 6, 25.0, "kronecker", "f64", 0),
    ("ragged_30x5_S3", 150, 30, 5, 3, 4, 4, 12.0, "iid", "f32", 0),
    ("ragged_100x20_S9", 120, 100, 20, 9, 2, 5, 14.0, "iid", "f32", 0),
    ("rhs_chunks_64x12_S23", 60, 64, 12, 23, 4, 4, 12.0, "iid", "f32", 0),
    ("square_16x16", 80, 16, 16, 16, 2, 4, 20.0, "iid", "f32", 0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_x3_detection(case):
    name, n, B, U, S, m, K, snr, ch, scalar, bpc = case
    print(f"stream-x3 {name}", flush=True)
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    f = W.uplink_frame(rng, n, B, U, S, m, snr, channel=ch, rho_bs=0.5, rho_ue=0.2)
    _check(name, f, K, m, scalar, bpc)


def test_x3_wide_dynamic_range():
    """Antenna rows scaled by gains spread over 10^-3 .. 10^3 (H and Y alike):
    each FP32 value is split relative to its own magnitude, so every product
    keeps FP32 relative accuracy whatever the scale.  The CG on these badly
    conditioned systems is itself outside the FP32 tolerances, so the split
    form is held to the FP32-MFMA kernel's own error."""
    print("stream-x3 wide dynamic range", flush=True)
    rng = np.random.default_rng(11)
    n, B, U, S, m, K = 100, 64, 8, 14, 4, 4
    f = W.uplink_frame(rng, n, B, U, S, m, 20.0)
    g = 10.0 ** rng.uniform(-3, 3, size=(n, B, 1))
    f.H[...] = f.H * g
    f.Y[...] = f.Y * g
    _check("wide_dynamic_range", f, K, m, "f64", like_fp32=True)


def test_x3_zero_receive_vectors():
    print("stream-x3 zero receive vectors", flush=True)
    rng = np.random.default_rng(12)
    f = W.uplink_frame(rng, 50, 64, 8, 6, 4, 10.0)
    f.Y[:, :, 2] = 0
    f.Y[7] = 0
    _check("zero_rhs", f, 3, 4, "f32")


def test_x3_full_size_sampled():
    print("stream-x3 full size 19200 x 128x16", flush=True)
    wl = W.WORKLOADS["mixed_128x16"]
    n = wl.n_sc * 16
    rng = np.random.default_rng(1404)
    f = W.uplink_frame(rng, n, wl.B, wl.U, wl.S, wl.m, wl.snr_db[0])
    idx = np.unique(np.concatenate([rng.choice(n, 40, replace=False), [0, n - 1]]))
    _check("full_128x16", f, wl.K, wl.m, "f32", bpc=4, idx=idx)


def _prun(variant, U, bpc, fn):
    from paper_1404_0424_amd import autotune
    saved = autotune.get_schedule("precode", U, 0)
    try:
        autotune.set_schedule("precode", U, 0, autotune.variants("precode").index(variant), bpc)
        out = fn()
        torch.cuda.synchronize()
        return out
    finally:
        autotune.set_schedule("precode", U, 0, *saved)


# (name, n_sc, B, U, S, K, snr_db, channel, scalar, blocks_per_cu, normalize)
PRE_CASES = [
    ("resident_128x16", 300, 128, 16, 14, 4, 15.0, "iid", "f32", 2, True),
    ("resident_64x8_S1", 200, 64, 8, 1, 3, 10.0, "iid", "f32", 0, True),
    ("resident_100x13_ragged", 150, 100, 13, 9, 5, 12.0, "iid", "f32", 1, False),
    ("stream_128x32", 200, 128, 32, 14, 4, 15.0, "iid", "f32", 0, True),
    ("stream_256x32_f64", 100, 256, 32, 14, 6, 25.0, "kronecker", "f64", 0, True),
    ("generic_64x12_S20", 60, 64, 12, 20, 4, 12.0, "iid", "f32", 0, True),
    ("zero_forcing_32x8", 80, 32, 8, 3, 8, None, "iid", "f32", 0, False),
]


@pytest.mark.parametrize("case", PRE_CASES, ids=[c[0] for c in PRE_CASES])
def test_x3_precoding(case):
    """Precoding with the bf16-split Gram (schedule variant "x3": the
    H-resident kernel for U <= 16, S <= 16, B <= 128, else the streaming or
    generic kernel), against the oracle and the FP32-MFMA kernels."""
    from paper_1404_0424_amd import api
    name, n, B, U, S, K, snr, ch, scalar, bpc, norm = case
    print(f"precode x3 {name}", flush=True)
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 3)
    f = W.uplink_frame(rng, n, B, U, S, 4, 10.0 if snr is None else snr, channel=ch,
                       rho_bs=0.5, rho_ue=0.2)
    d = W.downlink_frame(rng, n, B, U, S, 4, snr, H=f.H)
    H, T = dev(f.H), dev(d.T)
    run = lambda: api.precode_cg(H, T, d.beta, K, norm, scalar)  # noqa: E731
    Q, qn = _prun("x3", U, bpc, run)
    Qr, _ = _prun("stream-small", U, 0, run)
    ref = O.precode_cg(f.H, d.T, d.beta, K, norm)
    eq = rel_err_vec(host(Q), ref["Q"], axis=1)
    en = rel_err_scalar(host(qn), ref["qnorm"])
    print(f"{name}: eps_q={eq:.2e} eps_qnorm={en:.2e}")
    assert eq <= TOL_X and en <= TOL_X
    assert rel_err_vec(host(Q), host(Qr).astype(np.complex128), axis=1) <= 2e-5


@pytest.mark.parametrize("B,U,Su,Sd,bpc", [(128, 16, 14, 14, 2), (64, 8, 14, 5, 0),
                                           (100, 13, 11, 16, 1)])
def test_x3_slot(B, U, Su, Sd, bpc):
    """The fused uplink + downlink kernel with the bf16-split Gram and
    matched filter ("fused-x3"): against the oracle, and equal to the
    separate x3 detection and x3 precoding launches bit for bit (the same
    operations in the same order)."""
    from paper_1404_0424_amd import api, autotune
    print(f"slot fused-x3 {B}x{U}", flush=True)
    rng = np.random.default_rng(B * 100 + U)
    n, K = 150, 4
    f = W.uplink_frame(rng, n, B, U, Su, 6, 15.0)
    d = W.downlink_frame(rng, n, B, U, Sd, 4, 15.0, H=f.H)
    H, Y, T = dev(f.H), dev(f.Y), dev(d.T)
    saved = autotune.get_schedule("slot", U, 0)
    try:
        autotune.set_schedule("slot", U, 0, autotune.variants("slot").index("fused-x3"), bpc)
        det, Q, qn = api.detect_precode_cg(H, Y, T, f.n0, f.es, d.beta, K, K, 6, True)
        torch.cuda.synchronize()
    finally:
        autotune.set_schedule("slot", U, 0, *saved)
    o = _run("stream-x3", U, 0, lambda: api.detect_cg(H, Y, f.n0, f.es, K, 6))
    Q2, qn2 = _prun("x3", U, 0, lambda: api.precode_cg(H, T, d.beta, K, True))
    assert np.array_equal(host(det["llr"]), host(o["llr"]))
    assert np.array_equal(host(Q).view(np.uint32), host(Q2).view(np.uint32))
    assert np.array_equal(host(qn), host(qn2))
    ref = O.detect_cg(f.H, f.Y, f.n0, f.es, K, 6)
    pref = O.precode_cg(f.H, d.T, d.beta, K, True)
    assert llr_err(host(det["llr"]), ref["llr"]) <= TOL_L
    assert rel_err_vec(host(Q), pref["Q"], axis=1) <= TOL_X
