"""GPU tests of detection and precoding from a cached Gram matrix
(mimo_detect_cg_gram, mimo_precode_cg_gram, batched frames with a gram
pointer).  G = H^H H of a channel (Sec. II-A; H_d H_d^H by reciprocity,
Sec. II-B) is written once by mimo_gram_mf with reg = 0; the calls add
N0/E_s or beta to its diagonal and read H only for the matched filter or
q = H_u v.

With G from the same H and storage type, the outputs are bitwise those of
mimo_detect_cg / mimo_precode_cg for U > 8 (the A operand, its diagonal and
the matched filter are the same values); at U <= 8 those calls form the
Gram in a packed form that rounds differently, and the cached form is checked
against the FP64 oracle instead.
"""
import ctypes
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


def _bits(x):
    return host(x).view(np.uint32)


def _frames(name, n, B, U, S, m, snr):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    up = W.uplink_frame(rng, n, B, U, S, m, snr)
    dn = W.downlink_frame(rng, n, B, U, S, 4, snr, H=up.H)
    return up, dn


# (name, n_sc, B, U, S, K, qam_bits, scalar, storage)
BITWISE = [
    ("128x16_S14", 53, 128, 16, 14, 4, 6, "f32", "c32"),
    ("128x32_S14", 29, 128, 32, 14, 4, 6, "f32", "c32"),
    ("64x12_S20_f64", 21, 64, 12, 20, 3, 4, "f64", "c32"),
    ("100x20_S5", 33, 100, 20, 5, 5, 8, "f32", "c32"),
    ("256x32_S14_f64", 11, 256, 32, 14, 6, 8, "f64", "c32"),
    ("128x16_bf16", 41, 128, 16, 14, 4, 6, "f32", "bf16"),
    ("64x24_f16", 17, 64, 24, 9, 4, 4, "f32", "f16"),
]


@pytest.mark.parametrize("case", BITWISE, ids=[c[0] for c in BITWISE])
def test_cached_gram_is_bitwise_the_direct_call(case):
    name, n, B, U, S, K, m, scalar, storage = case
    print(f"cached gram {name}", flush=True)
    up, dn = _frames(name, n, B, U, S, m, 15.0)
    A = api()
    H, Y, T = dev(up.H), dev(up.Y), dev(dn.T)
    if storage != "c32":
        H, Y = A.convert(H, storage), A.convert(Y, storage)
    G, _ = A.gram_mf(H, None, reg=0.0)
    d0 = A.detect_cg(H, Y, up.n0, up.es, K, m, "approx", scalar, xhat=True, mu=True, sinr=True)
    d1 = A.detect_cg_gram(G, H, Y, up.n0, up.es, K, m, scalar, xhat=True, mu=True, sinr=True)
    Q0, q0 = A.precode_cg(H, T, dn.beta, K, True, scalar)
    Q1, q1 = A.precode_cg_gram(G, H, T, dn.beta, K, True, scalar)
    torch.cuda.synchronize()
    for k in d0:
        assert np.array_equal(_bits(d0[k]), _bits(d1[k])), k
    assert np.array_equal(_bits(Q0), _bits(Q1))
    assert np.array_equal(_bits(q0), _bits(q1))
    if storage == "c32":
        ref = O.detect_cg(up.H, up.Y, up.n0, up.es, K, m, "approx")
        assert llr_err(host(d1["llr"]), ref["llr"]) <= TOL_L
        assert rel_err_vec(host(Q1), O.precode_cg(up.H, dn.T, dn.beta, K, True)["Q"],
                           axis=1) <= TOL_X


@pytest.mark.parametrize("B,U,S,K,m", [(32, 8, 1, 3, 4), (64, 5, 14, 3, 2), (128, 8, 14, 3, 6)])
def test_cached_gram_small_u_matches_oracle(B, U, S, K, m):
    print(f"cached gram {B}x{U}", flush=True)
    up, dn = _frames(f"small{B}x{U}", 37, B, U, S, m, 10.0)
    A = api()
    H, Y, T = dev(up.H), dev(up.Y), dev(dn.T)
    G, _ = A.gram_mf(H, None, reg=0.0)
    d = A.detect_cg_gram(G, H, Y, up.n0, up.es, K, m, "f32", xhat=True, mu=True)
    Q, qn = A.precode_cg_gram(G, H, T, dn.beta, K, True, "f32")
    torch.cuda.synchronize()
    ref = O.detect_cg(up.H, up.Y, up.n0, up.es, K, m, "approx")
    assert llr_err(host(d["llr"]), ref["llr"]) <= TOL_L
    assert rel_err_vec(host(d["xhat"]), ref["xhat"], axis=1) <= TOL_X
    assert rel_err_scalar(host(d["mu"]), ref["mu"]) <= TOL_X
    pref = O.precode_cg(up.H, dn.T, dn.beta, K, True)
    assert rel_err_vec(host(Q), pref["Q"], axis=1) <= TOL_X
    assert rel_err_scalar(host(qn), pref["qnorm"]) <= TOL_X


def test_batched_frames_with_and_without_gram():
    """A batch mixing frames with a cached Gram and frames without: each
    frame bitwise as its single call."""
    print("batched frames with cached gram", flush=True)
    from paper_1404_0424_amd import _lib as L
    A = api()
    shapes = [(24, 128, 16, 14, 6), (17, 64, 20, 14, 6), (9, 128, 16, 14, 6), (12, 96, 32, 14, 6)]
    ups, dns, Hs, Ys, Ts, Gs = [], [], [], [], [], []
    for i, (n, B, U, S, m) in enumerate(shapes):
        up, dn = _frames(f"batch{i}", n, B, U, S, m, 15.0)
        ups.append(up)
        dns.append(dn)
        Hs.append(dev(up.H))
        Ys.append(dev(up.Y))
        Ts.append(dev(dn.T))
        Gs.append(A.gram_mf(Hs[-1], None, reg=0.0)[0] if i % 2 == 0 else None)
    K, m = 4, 6
    llrs = [torch.empty((n, U, S, m), dtype=torch.float32, device="cuda")
            for (n, B, U, S, _) in shapes]
    Qs = [torch.empty((n, B, S), dtype=torch.complex64, device="cuda")
          for (n, B, U, S, _) in shapes]
    fr = (L.MimoFrame * len(shapes))()
    fp = (L.MimoFrame * len(shapes))()
    for i, (n, B, U, S, _) in enumerate(shapes):
        g = Gs[i].data_ptr() if Gs[i] is not None else None
        fr[i] = L.MimoFrame(n, B, U, S, K, Hs[i].data_ptr(), Ys[i].data_ptr(), llrs[i].data_ptr(),
                            None, ups[i].n0, ups[i].es, 0.0, 0, g)
        fp[i] = L.MimoFrame(n, B, U, S, K, Hs[i].data_ptr(), Ts[i].data_ptr(), Qs[i].data_ptr(),
                            None, 0.0, 0.0, dns[i].beta, 1, g)
    L.check(L.lib().mimo_detect_cg_batch(ctypes.addressof(fr), len(shapes), 0, m, 0, None))
    L.check(L.lib().mimo_precode_cg_batch(ctypes.addressof(fp), len(shapes), 0, 0, None))
    torch.cuda.synchronize()
    for i in range(len(shapes)):
        if Gs[i] is not None:
            d = A.detect_cg_gram(Gs[i], Hs[i], Ys[i], ups[i].n0, ups[i].es, K, m)
            Q, _ = A.precode_cg_gram(Gs[i], Hs[i], Ts[i], dns[i].beta, K, True)
        else:
            d = A.detect_cg(Hs[i], Ys[i], ups[i].n0, ups[i].es, K, m)
            Q, _ = A.precode_cg(Hs[i], Ts[i], dns[i].beta, K, True)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(llrs[i]), _bits(d["llr"])), i
        assert np.array_equal(_bits(Qs[i]), _bits(Q)), i


@pytest.mark.parametrize("B,U,S,dt", [(128, 16, 14, "c32"), (96, 12, 9, "c32"), (128, 32, 14, "c32"),
                                      (64, 16, 14, "bf16"), (100, 5, 14, "c32")])
def test_cached_gram_every_schedule(B, U, S, dt):
    """The cached-Gram calls under every schedule form that takes G (generic,
    stream, stream-small; for precoding also the H-resident kernel), each
    bitwise the direct call under the same schedule for U > 8 and within the
    oracle's tolerance at U <= 8; the other forms fall back to one of these."""
    print(f"cached gram schedules {B}x{U} {dt}", flush=True)
    from paper_1404_0424_amd import autotune as T
    up, dn = _frames(f"sched{B}x{U}{dt}", 23, B, U, S, 6, 12.0)
    A = api()
    H, Y, T_ = dev(up.H), dev(up.Y), dev(dn.T)
    code = 0
    if dt != "c32":
        H, Y = A.convert(H, dt), A.convert(Y, dt)
        code = {"f16": 1, "bf16": 2}[dt]
    G, _ = A.gram_mf(H, None, reg=0.0)
    saved = {op: T.get_schedule(op, U, code) for op in ("detect", "precode")}
    ref = O.detect_cg(up.H, up.Y, up.n0, up.es, 4, 6, "approx") if dt == "c32" else None
    try:
        for op, names in (("detect", T.variants("detect")), ("precode", T.variants("precode"))):
            for v, name in enumerate(names):
                for bpc in (0, 4):
                    T.set_schedule(op, U, code, v, bpc)
                    if op == "detect":
                        a = host(A.detect_cg(H, Y, up.n0, up.es, 4, 6)["llr"])
                        b = host(A.detect_cg_gram(G, H, Y, up.n0, up.es, 4, 6)["llr"])
                    else:
                        a = host(A.precode_cg(H, T_, dn.beta, 4, True)[0])
                        b = host(A.precode_cg_gram(G, H, T_, dn.beta, 4, True)[0])
                    torch.cuda.synchronize()
                    if U > 8 and name in ("generic", "stream", "stream-small", "resident"):
                        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (op, name, bpc)
                    elif op == "detect" and ref is not None:
                        assert llr_err(b, ref["llr"]) <= TOL_L, (op, name, bpc)
                    elif ref is not None:
                        pref = O.precode_cg(up.H, dn.T, dn.beta, 4, True)
                        assert rel_err_vec(b, pref["Q"], axis=1) <= TOL_X, (op, name, bpc)
    finally:
        for op, (v, b) in saved.items():
            T.set_schedule(op, U, code, v, b)
