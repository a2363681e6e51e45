"""Every kernel instantiation the schedules can reach: storage type (complex64,
FP16, BF16) x user width (U <= 16, U = 32) x CG scalar precision (FP32,
FP64) x each detection and precoding variant, on a small ragged shape,
against the FP64 oracle on the inputs the GPU read (RNE-rounded for 16-bit
storage), and bitwise equal across variants."""
import itertools
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


def _rounded(x, dt):
    if dt == "c32":
        return x
    qz, deq = ((O.quantize_f16, O.dequantize_f16) if dt == "f16"
               else (O.quantize_bf16, O.dequantize_bf16))
    return deq(qz(x))


COMBOS = list(itertools.product(["c32", "f16", "bf16"], [12, 32], ["f32", "f64"]))


@pytest.mark.parametrize("dt,U,scalar", COMBOS, ids=[f"{d}-U{u}-{s}" for d, u, s in COMBOS])
def test_every_variant_of_every_instantiation(dt, U, scalar):
    from paper_1404_0424_amd import autotune
    n, B, S, m, K = 21, 72, 11, 4, 4       # B: 4.5 antenna tiles, S: ragged rhs chunk
    rng = np.random.default_rng(zlib.crc32(f"{dt}{U}{scalar}".encode()))
    f = W.uplink_frame(rng, n, B, U, S, m, 12.0)
    d = W.downlink_frame(rng, n, B, U, S, m, 12.0, H=f.H)
    A = api()
    H, Y, T = dev(f.H), dev(f.Y), dev(d.T)
    code = 0
    if dt != "c32":
        H, Y = A.convert(H, dt), A.convert(Y, dt)
        code = H.dtype_code
    dets, pres = {}, {}
    saved = [autotune.get_schedule(op, U, code) for op in ("detect", "precode")]
    try:
        for v, name in enumerate(autotune.variants("detect")):
            if name in autotune.BASELINE_VARIANTS | autotune.ROUNDING_VARIANTS:
                continue
            autotune.set_schedule("detect", U, code, v, 0)
            o = A.detect_cg(H, Y, f.n0, f.es, K, m, "approx", scalar, xhat=True)
            dets[name] = (host(o["llr"]), host(o["xhat"]))
        for v, name in enumerate(autotune.variants("precode")):
            if name in autotune.ROUNDING_VARIANTS:
                continue
            autotune.set_schedule("precode", U, code, v, 2)
            q, qn = A.precode_cg(H, T, d.beta, K, True, scalar)
            pres[name] = (host(q), host(qn))
    finally:
        for op, (v, b) in zip(("detect", "precode"), saved):
            autotune.set_schedule(op, U, code, v, b)
    Hr, Yr = _rounded(f.H, dt), _rounded(f.Y, dt)
    ref = O.detect_cg(Hr, Yr, f.n0, f.es, K, m, "approx")
    refp = O.precode_cg(Hr, d.T, d.beta, K, True)
    first = next(iter(dets.values()))
    assert rel_err_vec(first[1], ref["xhat"], axis=1) <= TOL_X
    assert llr_err(first[0], ref["llr"]) <= TOL_L
    for name, o in dets.items():
        assert np.array_equal(o[0], first[0]) and np.array_equal(o[1], first[1]), name
    firstp = next(iter(pres.values()))
    assert rel_err_vec(firstp[0], refp["Q"], axis=1) <= TOL_X
    assert rel_err_scalar(firstp[1], refp["qnorm"]) <= TOL_X
    for name, o in pres.items():
        assert np.array_equal(o[0], firstp[0]) and np.array_equal(o[1], firstp[1]), name
