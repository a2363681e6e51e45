"""Seeded random configurations through the C ABI against the FP64 oracle.

Each case draws its own shape and parameters (seed = case index): U from 1
to 64 (the four-wavefront kernels above 32), B from U to 256, S from 1 to
40 (one to three chunks of 16 right-hand sides), K from 1 to min(8, U), every QAM
order, SNR 0-25 dB, FP32 or FP64 CG scalars, complex64 or 16-bit storage
(U <= 32, B a multiple of 8), i.i.d. or Kronecker-correlated channels.  Per
case: detection with the approximate SINR (LLRs, xhat, mu, rho), the exact
SINR where the case draws it (U <= 32), precoding (MMSE or zero forcing,
normalized or not), the uplink + downlink slot (bitwise the two separate
calls), and detection and precoding from a cached Gram matrix (bitwise the
direct calls for U > 8, against the oracle at U <= 8).  16-bit storage is
checked against the oracle on the same rounded inputs.  Tolerances as the
other parity tests (Sec. III, Algorithm 1; eqs. (4), (12)-(16)).
"""
import numpy as np
import pytest

from oracle import mimo_oracle as O
from paper_1404_0424_amd import workload as W

from _parity import TOL_L, TOL_X, dev, host, llr_err, rel_err_scalar, rel_err_vec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_CASES = 80
U_CHOICES = [1, 2, 3, 5, 7, 8, 9, 12, 16, 17, 23, 24, 31, 32, 33, 40, 48, 57, 64]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_0424_amd import _lib
    _lib.lib()       # fail loudly if the library is missing


def api():
    from paper_1404_0424_amd import api as A
    return A


def draw(i):
    rng = np.random.default_rng(7000 + i)
    U = int(rng.choice(U_CHOICES))
    storage = "c32" if U > 32 or rng.random() < 0.7 else str(rng.choice(["f16", "bf16"]))
    B = int(rng.integers(U, 257))
    if storage != "c32":
        B = max(8, -(-B // 8) * 8)
    c = dict(U=U, B=B, storage=storage,
             n=int(rng.integers(2, 8)), S=int(rng.integers(1, 41)),
             K=min(U, int(rng.integers(1, 9))),     # K <= U: CG is exact at K = U
             m=int(rng.choice([2, 4, 6, 8])), snr=float(rng.uniform(0.0, 25.0)),
             scalar=str(rng.choice(["f32", "f64"])),
             channel="kronecker" if rng.random() < 0.25 else "iid",
             exact=bool(U <= 32 and storage == "c32" and rng.random() < 0.35),
             zf=bool(B >= 2 * U and rng.random() < 0.25),
             normalize=bool(rng.random() < 0.7),
             Sd=int(rng.integers(1, 41)))
    return c


CASES = [draw(i) for i in range(N_CASES)]


def _name(c):
    return (f"{c['B']}x{c['U']}_S{c['S']}_K{c['K']}_m{c['m']}_{c['storage']}_{c['scalar']}"
            f"{'_exact' if c['exact'] else ''}{'_zf' if c['zf'] else ''}")


def _quantized(x, dt):
    if dt == "c32":
        return x
    if dt == "f16":
        return O.dequantize_f16(O.quantize_f16(x))
    return O.dequantize_bf16(O.quantize_bf16(x))


@pytest.mark.parametrize("i", range(N_CASES), ids=[f"{i}-{_name(c)}" for i, c in enumerate(CASES)])
def test_random_configuration(i):
    c = CASES[i]
    print(f"random case {i}: {c}", flush=True)
    rng = np.random.default_rng(9000 + i)
    n, B, U, S, K, m, dt = c["n"], c["B"], c["U"], c["S"], c["K"], c["m"], c["storage"]
    up = W.uplink_frame(rng, n, B, U, S, m, c["snr"], channel=c["channel"], rho_bs=0.5,
                        rho_ue=0.2)
    dn = W.downlink_frame(rng, n, B, U, c["Sd"], m, c["snr"], H=up.H)
    beta = 0.0 if c["zf"] else dn.beta
    A = api()
    H, Y, T = dev(up.H), dev(up.Y), dev(dn.T)
    if dt != "c32":
        H, Y = A.convert(H, dt), A.convert(Y, dt)
    Hq, Yq = _quantized(up.H, dt), _quantized(up.Y, dt)

    # detection, approximate SINR (eqs. (13)-(15)), max-log LLRs (eq. (4))
    o = A.detect_cg(H, Y, up.n0, up.es, K, m, "approx", c["scalar"], xhat=True, mu=True,
                    sinr=True)
    Q, qn = A.precode_cg(H, T, beta, K, c["normalize"], c["scalar"])
    torch.cuda.synchronize()
    ref = O.detect_cg(Hq, Yq, up.n0, up.es, K, m, "approx")
    el = llr_err(host(o["llr"]), ref["llr"])
    ex = rel_err_vec(host(o["xhat"]), ref["xhat"], axis=1)
    assert el <= TOL_L and ex <= TOL_X, (el, ex)
    assert rel_err_scalar(host(o["mu"]), ref["mu"]) <= TOL_X
    assert rel_err_scalar(host(o["sinr"]), ref["rho"]) <= TOL_X

    # precoding (eq. (16), q = H_u v, optional s = q / ||q||, Sec. II-B)
    pref = O.precode_cg(Hq, dn.T, beta, K, c["normalize"])
    eq = rel_err_vec(host(Q), pref["Q"], axis=1)
    assert eq <= TOL_X, eq
    assert rel_err_scalar(host(qn), pref["qnorm"]) <= TOL_X

    # exact in-loop SINR (Sec. III-C-1, eq. (12))
    if c["exact"]:
        oe = A.detect_cg(H, Y, up.n0, up.es, K, m, "exact", c["scalar"], mu=True)
        torch.cuda.synchronize()
        refe = O.detect_cg(Hq, Yq, up.n0, up.es, K, m, "exact")
        assert llr_err(host(oe["llr"]), refe["llr"]) <= TOL_L
        assert rel_err_scalar(host(oe["mu"]), refe["mu"]) <= TOL_X

    # uplink + downlink slot on the same channel: bitwise the separate calls
    det, Qs, qns = A.detect_precode_cg(H, Y, T, up.n0, up.es, beta, K, K, m, c["normalize"],
                                      c["scalar"], xhat=True)
    torch.cuda.synchronize()
    assert np.array_equal(host(det["llr"]).view(np.uint32), host(o["llr"]).view(np.uint32))
    assert np.array_equal(host(det["xhat"]).view(np.uint32), host(o["xhat"]).view(np.uint32))
    assert np.array_equal(host(Qs).view(np.uint32), host(Q).view(np.uint32))
    assert np.array_equal(host(qns).view(np.uint32), host(qn).view(np.uint32))

    # from a cached Gram matrix (U <= 32)
    if U <= 32:
        G, _ = A.gram_mf(H, None, reg=0.0)
        og = A.detect_cg_gram(G, H, Y, up.n0, up.es, K, m, c["scalar"], xhat=True)
        Qg, qng = A.precode_cg_gram(G, H, T, beta, K, c["normalize"], c["scalar"])
        torch.cuda.synchronize()
        if U > 8:
            assert np.array_equal(host(og["llr"]).view(np.uint32), host(o["llr"]).view(np.uint32))
            assert np.array_equal(host(Qg).view(np.uint32), host(Q).view(np.uint32))
            assert np.array_equal(host(qng).view(np.uint32), host(qn).view(np.uint32))
        else:
            assert llr_err(host(og["llr"]), ref["llr"]) <= TOL_L
            assert rel_err_vec(host(og["xhat"]), ref["xhat"], axis=1) <= TOL_X
            assert rel_err_vec(host(Qg), pref["Q"], axis=1) <= TOL_X
    print(f"case {i}: eps_L={el:.2e} eps_x={ex:.2e} eps_q={eq:.2e}", flush=True)


N_BATCHES = 16


def draw_batch(i):
    """A batch of 2-8 frames of one kernel class (users 1-16 or 17-32, one
    storage type, QAM order and scalar precision), each with its own shape,
    K and SNR; about half carry their cached Gram matrix."""
    rng = np.random.default_rng(8000 + i)
    wide = bool(rng.random() < 0.5)
    storage = "c32" if rng.random() < 0.7 else str(rng.choice(["f16", "bf16"]))
    b = dict(storage=storage, m=int(rng.choice([2, 4, 6, 8])),
             scalar=str(rng.choice(["f32", "f64"])), frames=[])
    for _ in range(int(rng.integers(2, 9))):
        U = int(rng.integers(17, 33) if wide else rng.integers(1, 17))
        B = int(rng.integers(U, 257))
        if storage != "c32":
            B = max(8, -(-B // 8) * 8)
        b["frames"].append(dict(U=U, B=B, n=int(rng.integers(1, 6)), S=int(rng.integers(1, 41)),
                                K=min(U, int(rng.integers(1, 7))),
                                snr=float(rng.uniform(0.0, 25.0)),
                                gram=bool(rng.random() < 0.5),
                                normalize=bool(rng.random() < 0.7)))
    return b


BATCHES = [draw_batch(i) for i in range(N_BATCHES)]


@pytest.mark.parametrize("i", range(N_BATCHES),
                         ids=[f"{i}-{len(b['frames'])}frames_{b['storage']}_{b['scalar']}_m{b['m']}"
                              for i, b in enumerate(BATCHES)])
def test_random_batch_equals_single_calls(i):
    """mimo_detect_cg_batch / mimo_precode_cg_batch over a random mix of
    frames: each frame bitwise its single call (detect_cg or detect_cg_gram,
    precode_cg or precode_cg_gram as the frame carries G)."""
    b = BATCHES[i]
    print(f"random batch {i}: {b}", flush=True)
    rng = np.random.default_rng(10000 + i)
    A = api()
    dt, m, scalar = b["storage"], b["m"], b["scalar"]
    ups, dfr, pfr = [], [], []
    for f in b["frames"]:
        up = W.uplink_frame(rng, f["n"], f["B"], f["U"], f["S"], m, f["snr"])
        dn = W.downlink_frame(rng, f["n"], f["B"], f["U"], f["S"], 4, f["snr"], H=up.H)
        H, Y, T = dev(up.H), dev(up.Y), dev(dn.T)
        if dt != "c32":
            H, Y = A.convert(H, dt), A.convert(Y, dt)
        G = A.gram_mf(H, None, 0.0)[0] if f["gram"] else None
        ups.append((H, Y, T, G, up, dn))
        dfr.append((H, Y, up.n0, up.es, G))
        pfr.append((H, T, dn.beta, f["normalize"], G))
    Ks = [f["K"] for f in b["frames"]]
    dets = A.detect_cg_batch(dfr, Ks, m, scalar)
    pres = A.precode_cg_batch(pfr, Ks, scalar, qnorm=True)
    torch.cuda.synchronize()
    for j, (f, (H, Y, T, G, up, dn)) in enumerate(zip(b["frames"], ups)):
        if G is not None:
            d1 = A.detect_cg_gram(G, H, Y, up.n0, up.es, f["K"], m, scalar)
            Q1, q1 = A.precode_cg_gram(G, H, T, dn.beta, f["K"], f["normalize"], scalar)
        else:
            d1 = A.detect_cg(H, Y, up.n0, up.es, f["K"], m, "approx", scalar)
            Q1, q1 = A.precode_cg(H, T, dn.beta, f["K"], f["normalize"], scalar)
        torch.cuda.synchronize()
        assert np.array_equal(host(dets[j]["llr"]).view(np.uint32),
                              host(d1["llr"]).view(np.uint32)), j
        assert np.array_equal(host(pres[j][0]).view(np.uint32), host(Q1).view(np.uint32)), j
        assert np.array_equal(host(pres[j][1]).view(np.uint32), host(q1).view(np.uint32)), j
    # and the oracle on the first frame
    f, (H, Y, T, G, up, dn) = b["frames"][0], ups[0]
    Hq, Yq = _quantized(up.H, dt), _quantized(up.Y, dt)
    assert llr_err(host(dets[0]["llr"]), O.detect_cg(Hq, Yq, up.n0, up.es, f["K"], m,
                                                     "approx")["llr"]) <= TOL_L
    assert rel_err_vec(host(pres[0][0]), O.precode_cg(Hq, dn.T, dn.beta, f["K"],
                                                      f["normalize"])["Q"], axis=1) <= TOL_X
