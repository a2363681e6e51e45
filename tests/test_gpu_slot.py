"""GPU parity of the uplink + downlink slot (mimo_detect_precode_cg): CG-D
detection of Y and CG-P precoding of T on one reciprocal channel, whose
Gram matrix G = H_u^H H_u = H_d H_d^H (Sec. II-B) is formed once per
subcarrier by the fused H-resident kernel.

Every result is compared bitwise with mimo_detect_cg followed by
mimo_precode_cg on the same inputs (the fused kernel performs the same
operations in the same order) and with the FP64 oracle at the usual
tolerances.  Cases cover both channel capacities (64 and 128 antennas),
partial antenna tiles, the packed form (U <= 8), different S and K in the
two directions, a precoding regularization other than N0/E_s and zero
forcing, FP64 scalar recurrences, the optional uplink outputs, every QAM
order, persistent grids in which each wavefront walks many subcarriers (the
next subcarrier's channel and receive vectors are loaded during the current
one's stages), fewer subcarriers than wavefronts, and calls the fused kernel
does not cover (they run as two launches).
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
    _lib.lib()       # fail loudly if the library is missing


def api():
    from paper_1404_0424_amd import api as A
    return A


def _slot_schedule(U, code, variant, bpc):
    from paper_1404_0424_amd import autotune
    saved = autotune.get_schedule("slot", U, code)
    autotune.set_schedule("slot", U, code, autotune.variants("slot").index(variant), bpc)
    return saved


def _restore(U, code, saved):
    from paper_1404_0424_amd import autotune
    autotune.set_schedule("slot", U, code, *saved)


def _frames(name, n, B, U, Su, Sd, m, snr, channel="iid"):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    up = W.uplink_frame(rng, n, B, U, Su, m, snr, channel=channel, rho_bs=0.5, rho_ue=0.2)
    dn = W.downlink_frame(rng, n, B, U, Sd, 4, snr, H=up.H)
    return up, dn


def _run_slot(H, Y, T, up, beta, Ku, Kd, m, normalize, scalar, aux, variant, bpc, code=0):
    U = up.H.shape[2]
    saved = _slot_schedule(U, code, variant, bpc)
    try:
        det, Q, qn = api().detect_precode_cg(H, Y, T, up.n0, up.es, beta, Ku, Kd, m, normalize,
                                             scalar, xhat=aux, mu=aux, sinr=aux)
        torch.cuda.synchronize()
    finally:
        _restore(U, code, saved)
    return {k: host(v) for k, v in det.items()}, host(Q), host(qn)


def _run_separate(H, Y, T, up, beta, Ku, Kd, m, normalize, scalar, aux):
    det = api().detect_cg(H, Y, up.n0, up.es, Ku, m, "approx", scalar, xhat=aux, mu=aux,
                          sinr=aux)
    Q, qn = api().precode_cg(H, T, beta, Kd, normalize, scalar)
    torch.cuda.synchronize()
    return {k: host(v) for k, v in det.items()}, host(Q), host(qn)


def _same(a, b):
    da, Qa, qa = a
    db, Qb, qb = b
    assert da.keys() == db.keys()
    for k in da:
        assert np.array_equal(da[k].view(np.uint32), db[k].view(np.uint32)), k
    assert np.array_equal(Qa.view(np.uint32), Qb.view(np.uint32))
    assert np.array_equal(qa.view(np.uint32), qb.view(np.uint32))


def _vs_oracle(res, up, dn_T, beta, Ku, Kd, m, normalize, aux, idx=None):
    det, Q, qn = res
    H = up.H if idx is None else up.H[idx]
    Y = up.Y if idx is None else up.Y[idx]
    T = dn_T if idx is None else dn_T[idx]
    sel = (lambda a: a) if idx is None else (lambda a: a[idx])
    ref = O.detect_cg(H, Y, up.n0, up.es, Ku, m, "approx")
    el = llr_err(sel(det["llr"]), ref["llr"])
    assert el <= TOL_L, el
    if aux:
        assert rel_err_vec(sel(det["xhat"]), ref["xhat"], axis=1) <= TOL_X
        assert rel_err_scalar(sel(det["mu"]), ref["mu"]) <= TOL_X
        assert rel_err_scalar(sel(det["sinr"]), ref["rho"]) <= TOL_X
    pref = O.precode_cg(H, T, beta, Kd, normalize)
    eq = rel_err_vec(sel(Q), pref["Q"], axis=1)
    en = rel_err_scalar(sel(qn), pref["qnorm"])
    assert eq <= TOL_X and en <= TOL_X, (eq, en)
    return el, eq


# (name, n_sc, B, U, S_ul, S_dl, K_ul, K_dl, qam_bits, snr_db, beta factor (x N0/E_s,
#  0 = zero forcing), normalize, scalar, optional outputs, blocks_per_cu)
CASES = [
    ("128x16_S14", 61, 128, 16, 14, 14, 4, 4, 6, 15.0, 1.0, True, "f32", False, 0),
    ("128x16_persistent", 301, 128, 16, 14, 14, 4, 4, 6, 15.0, 1.0, True, "f32", False, 1),
    ("64x8_packed", 97, 64, 8, 14, 9, 3, 5, 4, 10.0, 1.0, False, "f32", False, 2),
    ("100x13_ragged_f64", 45, 100, 13, 11, 16, 5, 2, 8, 20.0, 2.5, True, "f64", False, 0),
    ("30x5_S1_S3", 77, 30, 5, 1, 3, 2, 6, 2, 5.0, 1.0, True, "f32", False, 3),
    ("16x16_square", 40, 16, 16, 16, 16, 4, 4, 6, 25.0, 1.0, True, "f32", False, 0),
    ("65x16_zf_downlink", 33, 65, 16, 7, 12, 4, 8, 6, 20.0, 0.0, False, "f32", False, 1),
    ("128x12_aux", 50, 128, 12, 14, 14, 4, 4, 6, 15.0, 1.0, True, "f32", True, 0),
    ("128x16_one_subcarrier", 1, 128, 16, 14, 14, 4, 4, 6, 15.0, 1.0, True, "f32", True, 4),
    ("96x16_f64_persistent_aux", 203, 96, 16, 14, 10, 6, 3, 6, 12.0, 0.5, True, "f64", True, 1),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_slot_matches_separate_and_oracle(case):
    name, n, B, U, Su, Sd, Ku, Kd, m, snr, bf, norm, scalar, aux, bpc = case
    print(f"slot {name}", flush=True)
    up, dn = _frames(name, n, B, U, Su, Sd, m, snr)
    beta = bf * up.n0 / up.es
    H, Y, T = dev(up.H), dev(up.Y), dev(dn.T)
    fused = _run_slot(H, Y, T, up, beta, Ku, Kd, m, norm, scalar, aux, "fused", bpc)
    sep = _run_separate(H, Y, T, up, beta, Ku, Kd, m, norm, scalar, aux)
    _same(fused, sep)
    el, eq = _vs_oracle(fused, up, dn.T, beta, Ku, Kd, m, norm, aux)
    print(f"{name}: eps_L={el:.2e} eps_q={eq:.2e}")


# calls the fused kernel does not cover run as two launches: U > 16, S > 16,
# B > 128; the "separate" variant always does
FALLBACK = [
    ("128x20_two_tiles", 30, 128, 20, 14, 14, 4, 4, 6, 15.0),
    ("64x8_S20_ul", 25, 64, 8, 20, 5, 3, 3, 4, 10.0),
    ("256x16_B", 12, 256, 16, 14, 14, 4, 4, 6, 15.0),
]


@pytest.mark.parametrize("case", FALLBACK, ids=[c[0] for c in FALLBACK])
def test_slot_outside_the_fused_kernel(case):
    name, n, B, U, Su, Sd, Ku, Kd, m, snr = case
    print(f"slot fallback {name}", flush=True)
    up, dn = _frames(name, n, B, U, Su, Sd, m, snr)
    beta = up.n0 / up.es
    H, Y, T = dev(up.H), dev(up.Y), dev(dn.T)
    fused = _run_slot(H, Y, T, up, beta, Ku, Kd, m, True, "f32", False, "fused", 0)
    sep = _run_separate(H, Y, T, up, beta, Ku, Kd, m, True, "f32", False)
    _same(fused, sep)
    _vs_oracle(fused, up, dn.T, beta, Ku, Kd, m, True, False)


def test_slot_separate_variant_and_16bit_storage():
    print("slot separate variant, bf16 storage", flush=True)
    n, B, U, S, K, m = 40, 128, 16, 14, 4, 6
    up, dn = _frames("bf16", n, B, U, S, S, m, 15.0)
    beta = up.n0 / up.es
    A = api()
    H, Y, T = dev(up.H), dev(up.Y), dev(dn.T)
    a = _run_slot(H, Y, T, up, beta, K, K, m, True, "f32", False, "separate", 0)
    b = _run_slot(H, Y, T, up, beta, K, K, m, True, "f32", False, "fused", 0)
    _same(a, b)
    Hq, Yq = A.convert(H, "bf16"), A.convert(Y, "bf16")
    c = _run_slot(Hq, Yq, T, up, beta, K, K, m, True, "f32", False, "fused", 0, Hq.dtype_code)
    d = _run_separate(Hq, Yq, T, up, beta, K, K, m, True, "f32", False)
    _same(c, d)
    Hr = O.dequantize_bf16(O.quantize_bf16(up.H))
    Yr = O.dequantize_bf16(O.quantize_bf16(up.Y))
    assert llr_err(c[0]["llr"], O.detect_cg(Hr, Yr, up.n0, up.es, K, m)["llr"]) <= TOL_L
    assert rel_err_vec(c[1], O.precode_cg(Hr, dn.T, beta, K, True)["Q"], axis=1) <= TOL_X


# 16-bit channel storage in the fused kernel: (name, n_sc, B, U, S_ul, S_dl, K_ul, K_dl,
# qam_bits, storage, scalar, optional outputs, blocks_per_cu)
CASES16 = [
    ("128x16_bf16", 37, 128, 16, 14, 14, 4, 4, 6, "bf16", "f32", True, 0),
    ("128x16_f16_persistent", 211, 128, 16, 14, 9, 4, 5, 6, "f16", "f32", False, 3),
    ("64x12_f16_B64", 29, 64, 12, 5, 16, 3, 4, 4, "f16", "f32", True, 0),
    ("96x8_bf16_f64", 23, 96, 8, 16, 1, 5, 3, 8, "bf16", "f64", True, 2),
    ("120x5_f16_ragged", 17, 120, 5, 3, 7, 2, 6, 2, "f16", "f32", False, 0),
]


@pytest.mark.parametrize("case", CASES16, ids=[c[0] for c in CASES16])
def test_slot_16bit_fused(case):
    """The fused kernel with FP16/BF16 channel and receive-vector storage:
    bitwise the two separate 16-bit calls, and the oracle on the same rounded
    inputs."""
    name, n, B, U, Su, Sd, Ku, Kd, m, dt, scalar, aux, bpc = case
    print(f"slot 16-bit {name}", flush=True)
    up, dn = _frames(name, n, B, U, Su, Sd, m, 15.0)
    beta = up.n0 / up.es
    A = api()
    Hq, Yq, T = A.convert(dev(up.H), dt), A.convert(dev(up.Y), dt), dev(dn.T)
    fused = _run_slot(Hq, Yq, T, up, beta, Ku, Kd, m, True, scalar, aux, "fused", bpc,
                      Hq.dtype_code)
    sep = _run_separate(Hq, Yq, T, up, beta, Ku, Kd, m, True, scalar, aux)
    _same(fused, sep)
    deq = O.dequantize_f16 if dt == "f16" else O.dequantize_bf16
    qz = O.quantize_f16 if dt == "f16" else O.quantize_bf16
    Hr, Yr = deq(qz(up.H)), deq(qz(up.Y))
    assert llr_err(fused[0]["llr"], O.detect_cg(Hr, Yr, up.n0, up.es, Ku, m)["llr"]) <= TOL_L
    assert rel_err_vec(fused[1], O.precode_cg(Hr, dn.T, beta, Kd, True)["Q"], axis=1) <= TOL_X


def test_slot_full_size_sampled():
    """The 16-frame 128x16 batch (19,200 subcarriers) in the launch shape the
    benchmark times: bitwise against the two separate launches everywhere,
    and against the oracle on sampled subcarriers (the last one included)."""
    print("slot full size 19200 x 128x16", flush=True)
    wl = W.WORKLOADS["mixed_128x16"]
    n = wl.n_sc * 16
    rng = np.random.default_rng(1404)
    up = W.uplink_frame(rng, n, wl.B, wl.U, wl.S, wl.m, wl.snr_db[0])
    dn = W.downlink_frame(rng, n, wl.B, wl.U, wl.S, wl.m, wl.snr_db[0], H=up.H)
    H, Y, T = dev(up.H), dev(up.Y), dev(dn.T)
    for bpc in (0, 3):
        fused = _run_slot(H, Y, T, up, dn.beta, wl.K, wl.K, wl.m, True, "f32", False, "fused",
                          bpc)
        sep = _run_separate(H, Y, T, up, dn.beta, wl.K, wl.K, wl.m, True, "f32", False)
        _same(fused, sep)
    idx = np.unique(np.concatenate([rng.choice(n, 40, replace=False), [0, n - 1]]))
    _vs_oracle(fused, up, dn.T, dn.beta, wl.K, wl.K, wl.m, True, False, idx)
