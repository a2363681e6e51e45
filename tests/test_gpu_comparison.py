"""GPU parity for the comparison methods (Sec. III-F): the Cholesky-based
exact soft-output MMSE detector / MMSE and ZF precoder and the truncated
Neumann series, through the C ABI against the FP64 oracle on the same seeded
inputs (tile-spanning, ragged and degenerate shapes)."""
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


# (name, n_sc, B, U, S, m, K, snr_db, channel); K = Neumann terms
CASES = [
    ("small_32x8", 64, 32, 8, 1, 4, 3, 10.0, "iid"),
    ("plain_128x8_10dB", 48, 128, 8, 14, 6, 3, 10.0, "iid"),
    ("mixed_128x16", 64, 128, 16, 14, 6, 3, 15.0, "iid"),
    ("mixed_128x32", 40, 128, 32, 14, 6, 3, 15.0, "iid"),
    ("corr_256x32", 24, 256, 32, 14, 8, 4, 25.0, "kronecker"),
    ("ragged_30x5_S17", 37, 30, 5, 17, 2, 2, 5.0, "iid"),
    ("ragged_80x20", 13, 80, 20, 3, 4, 5, 12.0, "iid"),
    ("single_user", 9, 6, 1, 2, 8, 1, 10.0, "iid"),
    ("square_16x16", 11, 16, 16, 5, 4, 2, 15.0, "iid"),
    # U S m = 90, not a multiple of 4: the staged LLR tile is written in 8-byte pieces
    ("odd_tile_40x5_S3", 29, 40, 5, 3, 6, 3, 12.0, "iid"),
]


def _uplink(case, seed=0):
    name, n, B, U, S, m, K, snr, ch = case
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 100 + seed)
    return W.uplink_frame(rng, n, B, U, S, m, snr, channel=ch, rho_bs=0.5, rho_ue=0.2)


def _check_detect(name, out, ref, tol_rho=1e-3):
    ex = rel_err_vec(host(out["xhat"]), ref["xhat"], axis=1)
    el = llr_err(host(out["llr"]), ref["llr"])
    emu = rel_err_scalar(host(out["mu"]), ref["mu"])
    erho = rel_err_scalar(host(out["sinr"]), ref["rho"])
    print(f"{name}: eps_x={ex:.2e} eps_L={el:.2e} eps_mu={emu:.2e} eps_rho={erho:.2e}")
    assert ex <= TOL_X and el <= TOL_L and emu <= TOL_X and erho <= tol_rho


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_detect_cholesky_parity(case):
    name, n, B, U, S, m, K, snr, ch = case
    f = _uplink(case)
    out = api().detect_cholesky(dev(f.H), dev(f.Y), f.n0, f.es, m, xhat=True, mu=True, sinr=True)
    torch.cuda.synchronize()
    _check_detect("cholesky " + name, out, O.detect_cholesky(f.H, f.Y, f.n0, f.es, m))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_detect_neumann_parity(case):
    name, n, B, U, S, m, K, snr, ch = case
    f = _uplink(case, 1)
    out = api().detect_neumann(dev(f.H), dev(f.Y), f.n0, f.es, K, m, xhat=True, mu=True,
                               sinr=True)
    torch.cuda.synchronize()
    _check_detect(f"neumann K={K} " + name, out, O.detect_neumann(f.H, f.Y, f.n0, f.es, K, m))


@pytest.mark.parametrize("K", [1, 2, 6])
def test_detect_neumann_terms(K):
    f = W.uplink_frame(np.random.default_rng(31), 20, 128, 16, 14, 6, 15.0)
    out = api().detect_neumann(dev(f.H), dev(f.Y), f.n0, f.es, K, 6, xhat=True, mu=True,
                               sinr=True)
    _check_detect(f"neumann K={K}", out, O.detect_neumann(f.H, f.Y, f.n0, f.es, K, 6))


def test_cholesky_detector_equals_cg_exact_at_K_equals_U_on_gpu():
    f = W.uplink_frame(np.random.default_rng(32), 16, 64, 8, 6, 4, 12.0)
    A = api()
    ch = A.detect_cholesky(dev(f.H), dev(f.Y), f.n0, f.es, 4, xhat=True, mu=True, sinr=True)
    cg = A.detect_cg(dev(f.H), dev(f.Y), f.n0, f.es, 8, 4, "exact", "f64", xhat=True, mu=True,
                     sinr=True)
    assert rel_err_vec(host(ch["xhat"]), host(cg["xhat"]).astype(np.complex128), axis=1) <= 2 * TOL_X
    assert llr_err(host(ch["llr"]), host(cg["llr"]).astype(np.float64)) <= 2 * TOL_L


@pytest.mark.parametrize("method", ["cholesky", "neumann"])
def test_zero_receive_vector_and_zero_channel_column(method):
    f = W.uplink_frame(np.random.default_rng(33), 12, 32, 8, 6, 4, 10.0)
    H, Y = f.H.copy(), f.Y.copy()
    Y[3] = 0                        # whole subcarrier silent
    Y[7, :, 2] = 0                  # one right-hand side silent
    H[5, :, 4] = 0                  # user 4 absent on subcarrier 5 (mu = 0 rule)
    Y[5] = H[5] @ f.X[5]
    A = api()
    if method == "cholesky":
        out = A.detect_cholesky(dev(H), dev(Y), f.n0, f.es, 4, xhat=True, mu=True, sinr=True)
        ref = O.detect_cholesky(H, Y, f.n0, f.es, 4)
    else:
        out = A.detect_neumann(dev(H), dev(Y), f.n0, f.es, 3, 4, xhat=True, mu=True, sinr=True)
        ref = O.detect_neumann(H, Y, f.n0, f.es, 3, 4)
    llr = host(out["llr"])
    assert np.all(np.isfinite(llr))
    assert np.all(host(out["xhat"])[3] == 0) and np.all(host(out["xhat"])[7, :, 2] == 0)
    assert np.all(host(out["xhat"])[5, 4] == 0)
    assert np.max(np.abs(llr[5, 4])) <= 1e-3 * max(1.0, np.max(np.abs(ref["llr"][5])))
    keep = np.ones(12, bool)
    keep[5] = False
    assert rel_err_vec(host(out["xhat"])[keep], ref["xhat"][keep], axis=1) <= TOL_X
    assert llr_err(llr[keep], ref["llr"][keep]) <= TOL_L


@pytest.mark.parametrize("dt", ["f16", "bf16"])
@pytest.mark.parametrize("method", ["cholesky", "neumann"])
def test_16bit_storage_matches_oracle_on_quantized_inputs(dt, method):
    f = W.uplink_frame(np.random.default_rng(34), 24, 128, 16, 14, 6, 15.0)
    A = api()
    H16, Y16 = A.convert(dev(f.H), dt), A.convert(dev(f.Y), dt)
    deq = O.dequantize_f16 if dt == "f16" else O.dequantize_bf16
    qz = O.quantize_f16 if dt == "f16" else O.quantize_bf16
    Hq, Yq = deq(qz(f.H)), deq(qz(f.Y))
    if method == "cholesky":
        out = A.detect_cholesky(H16, Y16, f.n0, f.es, 6, xhat=True)
        ref = O.detect_cholesky(Hq, Yq, f.n0, f.es, 6)
    else:
        out = A.detect_neumann(H16, Y16, f.n0, f.es, 3, 6, xhat=True)
        ref = O.detect_neumann(Hq, Yq, f.n0, f.es, 3, 6)
    assert rel_err_vec(host(out["xhat"]), ref["xhat"], axis=1) <= TOL_X
    assert llr_err(host(out["llr"]), ref["llr"]) <= TOL_L
    rng = np.random.default_rng(35)
    d = W.downlink_frame(rng, 24, 128, 16, 14, 6, 15.0)
    fn = A.precode_cholesky if method == "cholesky" else A.precode_neumann
    args = () if method == "cholesky" else (3,)
    Q, qn = fn(A.convert(dev(d.H), dt), dev(d.T), d.beta, *args, normalize=True)
    oref = (O.precode_cholesky(deq(qz(d.H)), d.T, d.beta, True) if method == "cholesky"
            else O.precode_neumann(deq(qz(d.H)), d.T, d.beta, 3, True))
    assert rel_err_vec(host(Q), oref["Q"], axis=1) <= TOL_X
    assert rel_err_scalar(host(qn), oref["qnorm"]) <= TOL_X


# (name, n_sc, B, U, S, K, snr_db or None for zero forcing)
PRECODE_CASES = [
    ("small_32x8", 64, 32, 8, 1, 3, 10.0),
    ("plain_128x8", 48, 128, 8, 14, 3, 10.0),
    ("mixed_128x16", 48, 128, 16, 14, 3, 15.0),
    ("mixed_128x32", 24, 128, 32, 14, 3, 15.0),
    ("corr_256x32", 16, 256, 32, 14, 4, 25.0),
    ("ragged_30x5_S17", 37, 30, 5, 17, 2, 5.0),
    ("zf_32x8", 16, 32, 8, 3, 4, None),
]


@pytest.mark.parametrize("case", PRECODE_CASES, ids=[c[0] for c in PRECODE_CASES])
@pytest.mark.parametrize("method", ["cholesky", "neumann"])
@pytest.mark.parametrize("normalize", [False, True])
def test_precode_parity(case, method, normalize):
    name, n, B, U, S, K, snr = case
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 200)
    ch = "kronecker" if "corr" in name else "iid"
    d = W.downlink_frame(rng, n, B, U, S, 6, snr, channel=ch, rho_bs=0.5, rho_ue=0.2)
    A = api()
    if method == "cholesky":
        Q, qn = A.precode_cholesky(dev(d.H), dev(d.T), d.beta, normalize)
        ref = O.precode_cholesky(d.H, d.T, d.beta, normalize)
    else:
        Q, qn = A.precode_neumann(dev(d.H), dev(d.T), d.beta, K, normalize)
        ref = O.precode_neumann(d.H, d.T, d.beta, K, normalize)
    eq = rel_err_vec(host(Q), ref["Q"], axis=1)
    en = rel_err_scalar(host(qn), ref["qnorm"])
    print(f"{method} {name} norm={normalize}: eps_q={eq:.2e} eps_qnorm={en:.2e}")
    assert eq <= TOL_X and en <= TOL_X
    if snr is None and method == "cholesky":    # zero forcing: H_d q = t
        HdQ = np.conj(np.swapaxes(d.H, 1, 2)) @ host(Q).astype(np.complex128)
        if normalize:
            HdQ = HdQ * ref["qnorm"][:, None, :]
        assert rel_err_vec(HdQ, d.T, axis=1) <= 1e-3


@pytest.mark.parametrize("method", ["cholesky", "neumann"])
def test_full_size_sampled(method):
    # bench's batch of the 128x16 workload (16 frames, 19,200 subcarriers) in
    # one launch: the streaming kernels' persistent grid makes every wave walk
    # several subcarriers; 150 sampled subcarriers (the last one included)
    # checked against the oracle
    wl = W.WORKLOADS["mixed_128x16"]
    n = 16 * wl.n_sc
    rng = np.random.default_rng(36)
    f = W.uplink_frame(rng, n, wl.B, wl.U, wl.S, wl.m, wl.snr_db[0])
    d = W.downlink_frame(rng, n, wl.B, wl.U, wl.S, wl.m, wl.snr_db[0], H=f.H)
    A = api()
    idx = np.sort(np.random.default_rng(37).choice(n, 150, replace=False))
    idx[-1] = n - 1
    if method == "cholesky":
        out = A.detect_cholesky(dev(f.H), dev(f.Y), f.n0, f.es, wl.m, xhat=True)
        Q, _ = A.precode_cholesky(dev(f.H), dev(d.T), d.beta, True)
        ref = O.detect_cholesky(f.H[idx], f.Y[idx], f.n0, f.es, wl.m)
        pref = O.precode_cholesky(f.H[idx], d.T[idx], d.beta, True)
    else:
        out = A.detect_neumann(dev(f.H), dev(f.Y), f.n0, f.es, 3, wl.m, xhat=True)
        Q, _ = A.precode_neumann(dev(f.H), dev(d.T), d.beta, 3, True)
        ref = O.detect_neumann(f.H[idx], f.Y[idx], f.n0, f.es, 3, wl.m)
        pref = O.precode_neumann(f.H[idx], d.T[idx], d.beta, 3, True)
    assert rel_err_vec(host(out["xhat"])[idx], ref["xhat"], axis=1) <= TOL_X
    assert llr_err(host(out["llr"])[idx], ref["llr"]) <= TOL_L
    assert rel_err_vec(host(Q)[idx], pref["Q"], axis=1) <= TOL_X
