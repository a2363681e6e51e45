"""GPU parity of the precoders at the edges of their input range, against the
FP64 oracle: low SNR (large beta, where ||q||^2 must not be formed as
v^H A v - beta ||v||^2), zero symbol vectors with power normalization
(||q|| = 0 gives s = 0, Sec. II-B), and square and rank-deficient channels
(eq. (6) with B = U, and with two equal user columns).  Every precoding
kernel variant is run: the resident one (U <= 16), the streaming ones and
the generic one, and the Cholesky / Neumann precoders that share the output
stage."""
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
    _lib.lib()


def api():
    from paper_1404_0424_amd import api as A
    return A


VARIANTS = ["resident", "stream", "stream-small", "generic"]


def _with_variant(U, variant, fn):
    from paper_1404_0424_amd import autotune
    saved = autotune.get_schedule("precode", U, 0)
    try:
        autotune.set_schedule("precode", U, 0, autotune.variants("precode").index(variant),
                              8 if variant == "resident" else 0)
        return fn()
    finally:
        autotune.set_schedule("precode", U, 0, *saved)


def _check(Q, qn, ref, label):
    eq = rel_err_vec(host(Q), ref["Q"], axis=1)
    en = rel_err_scalar(host(qn), ref["qnorm"])
    print(f"{label}: eps_q={eq:.2e} eps_qnorm={en:.2e}")
    assert eq <= TOL_X and en <= TOL_X
    assert np.all(np.isfinite(host(Q)))


# (name, n_sc, B, U, S, K, snr_db)
LOW_SNR = [
    ("mixed_128x16_0dB", 40, 128, 16, 14, 4, 0.0),
    ("mixed_128x16_m10dB", 40, 128, 16, 14, 4, -10.0),
    ("mixed_128x16_m20dB", 40, 128, 16, 14, 4, -20.0),
    ("mixed_128x32_m20dB", 24, 128, 32, 14, 4, -20.0),
    ("plain_128x8_m20dB", 40, 128, 8, 14, 3, -20.0),
]


@pytest.mark.parametrize("case", LOW_SNR, ids=[c[0] for c in LOW_SNR])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("normalize", [False, True])
def test_low_snr(case, variant, normalize):
    name, n, B, U, S, K, snr = case
    d = W.downlink_frame(np.random.default_rng(zlib.crc32(name.encode())), n, B, U, S, 6, snr)
    Q, qn = _with_variant(U, variant, lambda: api().precode_cg(dev(d.H), dev(d.T), d.beta, K,
                                                                normalize))
    _check(Q, qn, O.precode_cg(d.H, d.T, d.beta, K, normalize),
           f"{name} {variant} beta={d.beta:.3g} norm={normalize}")


@pytest.mark.parametrize("method", ["cholesky", "neumann"])
@pytest.mark.parametrize("snr", [0.0, -20.0])
def test_low_snr_comparison_precoders(method, snr):
    d = W.downlink_frame(np.random.default_rng(int(-snr) + 17), 40, 128, 16, 14, 6, snr)
    A = api()
    if method == "cholesky":
        Q, qn = A.precode_cholesky(dev(d.H), dev(d.T), d.beta, True)
        ref = O.precode_cholesky(d.H, d.T, d.beta, True)
    else:
        Q, qn = A.precode_neumann(dev(d.H), dev(d.T), d.beta, 3, True)
        ref = O.precode_neumann(d.H, d.T, d.beta, 3, True)
    _check(Q, qn, ref, f"{method} {snr:g} dB")


ZERO_SHAPES = [(128, 16, 14, 4), (128, 8, 14, 3), (128, 32, 14, 4), (30, 5, 17, 3)]


@pytest.mark.parametrize("B,U,S,K", ZERO_SHAPES, ids=[f"{b}x{u}_S{s}" for b, u, s, _ in ZERO_SHAPES])
@pytest.mark.parametrize("variant", VARIANTS)
def test_zero_symbol_vectors_normalized(B, U, S, K, variant):
    """t = 0 freezes the CG at v = 0 (its residual norm is zero), so q = 0,
    ||q|| = 0 and the normalized output s is 0; the other vectors of the same
    subcarrier and the other subcarriers are unaffected."""
    d = W.downlink_frame(np.random.default_rng(B + U + S), 12, B, U, S, 4, 15.0)
    T = d.T.copy()
    T[2] = 0                       # a whole subcarrier
    T[5, :, 1] = 0                 # one vector
    T[5, :, S - 1] = 0             # the last vector
    T[9, :, 0] = 0
    Q, qn = _with_variant(U, variant, lambda: api().precode_cg(dev(d.H), dev(T), d.beta, K, True))
    ref = O.precode_cg(d.H, T, d.beta, K, True)
    Qh, qh = host(Q), host(qn)
    for (i, s) in [(2, slice(None)), (5, 1), (5, S - 1), (9, 0)]:
        assert np.all(Qh[i][:, s] == 0) and np.all(qh[i][s] == 0)
    _check(Q, qn, ref, f"zero t {B}x{U} {variant}")


SQUARE = [("square_16x16_15dB", 16, 16, 15.0, 4), ("square_16x16_0dB", 16, 16, 0.0, 4),
          ("square_32x32_15dB", 32, 32, 15.0, 6), ("square_16x16_zf_K3", 16, 16, None, 3),
          ("square_8x8_zf_K2", 8, 8, None, 2)]


@pytest.mark.parametrize("case", SQUARE, ids=[c[0] for c in SQUARE])
@pytest.mark.parametrize("variant", VARIANTS)
def test_square_channel(case, variant):
    """B = U: G is a full square Gram, the hardest conditioning of the
    paper's model (kappa(G) up to ~1e4 here).  With beta > 0, kappa(A) stays
    small and any K is checked; zero forcing (beta = 0) is checked at small K:
    at K = U on kappa ~ 1e3..1e4 the FP32 iterates of Algorithm 1 leave the
    FP64 ones in any FP32 implementation (a numpy float32 CG is off by
    1e-1..1 there, by 7e-7 at K = 3)."""
    name, B, U, snr, K = case
    d = W.downlink_frame(np.random.default_rng(zlib.crc32(name.encode())), 24, B, U, 5, 4, snr)
    Q, qn = _with_variant(U, variant, lambda: api().precode_cg(dev(d.H), dev(d.T), d.beta, K,
                                                                True))
    _check(Q, qn, O.precode_cg(d.H, d.T, d.beta, K, True), f"{name} {variant}")


def test_rank_deficient_channel_mmse():
    """Two equal user columns (rank U - 1): G is singular, A = G + beta I is
    not; MMSE precoding stays finite and matches the oracle."""
    d = W.downlink_frame(np.random.default_rng(3), 24, 64, 8, 14, 6, 10.0)
    H = d.H.copy()
    H[:, :, 3] = H[:, :, 5]
    Q, qn = api().precode_cg(dev(H), dev(d.T), d.beta, 6, True)
    _check(Q, qn, O.precode_cg(H, d.T, d.beta, 6, True), "rank-deficient 64x8")
