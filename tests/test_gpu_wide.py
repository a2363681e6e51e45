"""GPU parity of CG-D detection, CG-P precoding and the standalone Gram and
matched filter for 32 < U <= 64 (the
four-wavefront kernels: one workgroup per subcarrier, one 16-user tile per
wavefront, the CG inner products summed over the wavefronts through LDS).

Against the FP64 oracle at the usual tolerances: detection with the
approximate SINR of eqs. (13)-(15) and max-log LLRs of eq. (4), precoding by
eq. (16) with q = H_u v (Algorithm 1 output).  Cases cover partial user tiles
(U = 33, 40, 57), the full 64, ragged antenna counts, one and several chunks
of 16 right-hand sides (S = 1, 5, 16, 17, 40), every QAM order, FP32 and FP64
scalar recurrences, the optional outputs, zero forcing and the unnormalized
precoder, a square system (B = U), a zero receive vector (every right-hand
side freezes at once), a Kronecker-correlated channel, and the uplink +
downlink slot call (two launches of these kernels, bitwise equal to the
separate calls).  A 1,200-subcarrier batch at 128x64 is checked on sampled
subcarriers.  Calls these kernels do not cover are rejected by validation
(tests/test_abi.py).
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


def _rng(name):
    return np.random.default_rng(zlib.crc32(name.encode()))


# (name, n_sc, B, U, S, K, qam_bits, snr_db, scalar, optional outputs, channel)
DETECT = [
    ("128x33_S14", 37, 128, 33, 14, 4, 6, 15.0, "f32", True, "iid"),
    ("128x40_S5_f64", 29, 128, 40, 5, 5, 4, 12.0, "f64", True, "iid"),
    ("100x48_S17", 21, 100, 48, 17, 4, 8, 25.0, "f32", False, "iid"),
    ("256x64_S16", 19, 256, 64, 16, 6, 6, 20.0, "f32", True, "iid"),
    ("70x57_S1", 43, 70, 57, 1, 8, 2, 10.0, "f64", True, "iid"),
    ("200x64_S40_kron", 9, 200, 64, 40, 6, 8, 25.0, "f64", False, "kronecker"),
    ("64x64_square", 15, 64, 64, 14, 16, 4, 20.0, "f64", True, "iid"),
]


@pytest.mark.parametrize("case", DETECT, ids=[c[0] for c in DETECT])
def test_wide_detection_matches_oracle(case):
    name, n, B, U, S, K, m, snr, scalar, aux, ch = case
    print(f"wide detect {name}", flush=True)
    f = W.uplink_frame(_rng(name), n, B, U, S, m, snr, channel=ch, rho_bs=0.5, rho_ue=0.2)
    o = api().detect_cg(dev(f.H), dev(f.Y), f.n0, f.es, K, m, "approx", scalar, xhat=aux,
                        mu=aux, sinr=aux)
    torch.cuda.synchronize()
    ref = O.detect_cg(f.H, f.Y, f.n0, f.es, K, m, "approx")
    el = llr_err(host(o["llr"]), ref["llr"])
    assert el <= TOL_L, el
    if aux:
        ex = rel_err_vec(host(o["xhat"]), ref["xhat"], axis=1)
        assert ex <= TOL_X, ex
        assert rel_err_scalar(host(o["mu"]), ref["mu"]) <= TOL_X
        assert rel_err_scalar(host(o["sinr"]), ref["rho"]) <= TOL_X
    print(f"{name}: eps_L={el:.2e}")


# (name, n_sc, B, U, S, K, beta factor (x N0/E_s, 0 = zero forcing), normalize, scalar)
PRECODE = [
    ("128x33_S14", 37, 128, 33, 14, 4, 1.0, True, "f32"),
    ("128x48_S16_zf", 25, 128, 48, 16, 8, 0.0, True, "f32"),
    ("96x64_S17_f64", 17, 96, 64, 17, 6, 2.0, False, "f64"),
    ("256x64_S1", 31, 256, 64, 1, 4, 1.0, True, "f32"),
    ("65x40_S40_unnormalized", 11, 65, 40, 40, 5, 0.5, False, "f32"),
]


@pytest.mark.parametrize("case", PRECODE, ids=[c[0] for c in PRECODE])
def test_wide_precoding_matches_oracle(case):
    name, n, B, U, S, K, bf, norm, scalar = case
    print(f"wide precode {name}", flush=True)
    rng = _rng(name)
    up = W.uplink_frame(rng, n, B, U, 1, 4, 15.0)
    d = W.downlink_frame(rng, n, B, U, S, 4, 15.0, H=up.H)
    beta = bf * d.beta
    Q, qn = api().precode_cg(dev(d.H), dev(d.T), beta, K, norm, scalar)
    torch.cuda.synchronize()
    ref = O.precode_cg(d.H, d.T, beta, K, norm)
    eq = rel_err_vec(host(Q), ref["Q"], axis=1)
    en = rel_err_scalar(host(qn), ref["qnorm"])
    print(f"{name}: eps_q={eq:.2e} eps_norm={en:.2e}")
    assert eq <= TOL_X and en <= TOL_X, (eq, en)


@pytest.mark.parametrize("B,U,S,n", [(128, 33, 14, 23), (100, 48, 17, 9), (256, 64, 40, 5),
                                     (64, 64, 1, 7)])
def test_wide_gram_mf_matches_oracle(B, U, S, n):
    """mimo_gram_mf for 32 < U <= 64: A = H^H H + reg I (exactly Hermitian,
    real diagonal) and b = H^H y against the oracle, with and without Y."""
    print(f"wide gram_mf {B}x{U} S={S}", flush=True)
    f = W.uplink_frame(_rng(f"gram{B}x{U}"), n, B, U, S, 4, 10.0)
    A, b = api().gram_mf(dev(f.H), dev(f.Y), reg=0.37)
    torch.cuda.synchronize()
    A0 = O.regularized_gram(f.H, 0.37)
    Ag = host(A)
    eA = np.max(np.linalg.norm(Ag - A0, axis=(1, 2)) / np.linalg.norm(A0, axis=(1, 2)))
    eb = rel_err_vec(host(b), O.matched_filter(f.H, f.Y), axis=1)
    assert eA <= 2e-6 and eb <= 2e-6, (eA, eb)
    assert np.array_equal(Ag, np.conj(np.swapaxes(Ag, 1, 2)))
    A2, b2 = api().gram_mf(dev(f.H), None, reg=0.0)
    assert b2 is None
    assert np.max(np.abs(host(A2) - O.gram(f.H))) <= 2e-6 * np.max(np.abs(A0))


def test_wide_zero_receive_vectors():
    """y = 0 on some subcarriers and right-hand sides: b = 0, every CG step
    freezes at once, xhat = 0, mu = 0 and z = 0 (the degenerate-case rule of
    Algorithm 1's recursion); the others are unaffected."""
    print("wide zero receive vectors", flush=True)
    n, B, U, S, K, m = 13, 96, 44, 6, 4, 4
    f = W.uplink_frame(_rng("zero_y"), n, B, U, S, m, 15.0)
    Y = f.Y.copy()
    Y[3] = 0
    Y[7, :, 2] = 0
    o = api().detect_cg(dev(f.H), dev(Y), f.n0, f.es, K, m, "approx", "f32", xhat=True, mu=True)
    torch.cuda.synchronize()
    ref = O.detect_cg(f.H, Y, f.n0, f.es, K, m, "approx")
    assert np.all(host(o["xhat"])[3] == 0) and np.all(host(o["mu"])[3] == 0)
    assert np.all(host(o["xhat"])[7, :, 2] == 0)
    assert llr_err(host(o["llr"]), ref["llr"]) <= TOL_L
    assert rel_err_vec(host(o["xhat"]), ref["xhat"], axis=1) <= TOL_X


def test_wide_slot_matches_separate_calls():
    """mimo_detect_precode_cg at U = 48 runs the two four-wavefront kernels:
    bitwise the separate calls, and the oracle's results."""
    print("wide slot 128x48", flush=True)
    n, B, U, Su, Sd, Ku, Kd, m = 27, 128, 48, 14, 9, 4, 5, 6
    rng = _rng("slot48")
    up = W.uplink_frame(rng, n, B, U, Su, m, 15.0)
    dn = W.downlink_frame(rng, n, B, U, Sd, 4, 15.0, H=up.H)
    A = api()
    H, Y, T = dev(up.H), dev(up.Y), dev(dn.T)
    det, Q, qn = A.detect_precode_cg(H, Y, T, up.n0, up.es, dn.beta, Ku, Kd, m, True, "f32",
                                     xhat=True, mu=True, sinr=True)
    det2 = A.detect_cg(H, Y, up.n0, up.es, Ku, m, "approx", "f32", xhat=True, mu=True, sinr=True)
    Q2, qn2 = A.precode_cg(H, T, dn.beta, Kd, True, "f32")
    torch.cuda.synchronize()
    for k in det:
        assert np.array_equal(host(det[k]).view(np.uint32), host(det2[k]).view(np.uint32)), k
    assert np.array_equal(host(Q).view(np.uint32), host(Q2).view(np.uint32))
    assert np.array_equal(host(qn).view(np.uint32), host(qn2).view(np.uint32))
    ref = O.detect_cg(up.H, up.Y, up.n0, up.es, Ku, m, "approx")
    assert llr_err(host(det["llr"]), ref["llr"]) <= TOL_L
    pref = O.precode_cg(up.H, dn.T, dn.beta, Kd, True)
    assert rel_err_vec(host(Q), pref["Q"], axis=1) <= TOL_X


def test_wide_full_batch_sampled():
    """1,200 subcarriers x 14 symbols at B = 128, U = 64 (64-QAM, 15 dB,
    K = 4): detection and precoding against the oracle on sampled
    subcarriers, the first and last included."""
    print("wide 1200 x 128x64", flush=True)
    n, B, U, S, K, m = 1200, 128, 64, 14, 4, 6
    rng = np.random.default_rng(6464)
    up = W.uplink_frame(rng, n, B, U, S, m, 15.0)
    dn = W.downlink_frame(rng, n, B, U, S, m, 15.0, H=up.H)
    A = api()
    H = dev(up.H)
    o = A.detect_cg(H, dev(up.Y), up.n0, up.es, K, m, "approx", "f32", xhat=True)
    Q, qn = A.precode_cg(H, dev(dn.T), dn.beta, K, True, "f32")
    torch.cuda.synchronize()
    idx = np.unique(np.concatenate([rng.choice(n, 30, replace=False), [0, n - 1]]))
    ref = O.detect_cg(up.H[idx], up.Y[idx], up.n0, up.es, K, m, "approx")
    assert llr_err(host(o["llr"])[idx], ref["llr"]) <= TOL_L
    assert rel_err_vec(host(o["xhat"])[idx], ref["xhat"], axis=1) <= TOL_X
    pref = O.precode_cg(up.H[idx], dn.T[idx], dn.beta, K, True)
    assert rel_err_vec(host(Q)[idx], pref["Q"], axis=1) <= TOL_X
    assert rel_err_scalar(host(qn)[idx], pref["qnorm"]) <= TOL_X
