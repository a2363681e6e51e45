"""GPU parity of detection with the CG mat-vec on VALU FMAs (schedule variant
"stream-valu", the measured alternative to the MFMA mat-vec): against the
FP64 oracle at the usual tolerances and against stream-small to rounding
(the VALU form sums each product in another order)."""
import zlib

import numpy as np
import pytest

from oracle import mimo_oracle as O
from paper_1404_0424_amd import workload as W

from _parity import TOL_L, TOL_X, dev, host, llr_err, rel_err_vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_0424_amd import _lib
    _lib.lib()


def _run(variant, U, fn):
    from paper_1404_0424_amd import autotune
    saved = autotune.get_schedule("detect", U, 0)
    try:
        autotune.set_schedule("detect", U, 0, autotune.variants("detect").index(variant), 0)
        out = fn()
        torch.cuda.synchronize()
        return out
    finally:
        autotune.set_schedule("detect", U, 0, *saved)


CASES = [
    ("mixed_128x16", 400, 128, 16, 14, 6, 4, 15.0, "iid", "f32"),
    ("packed_128x8", 400, 128, 8, 14, 6, 3, 10.0, "iid", "f32"),
    ("corr_256x32_f64", 200, 256, 32, 14, 8, 6, 25.0, "kronecker", "f64"),
    ("ragged_30x5_S3", 150, 30, 5, 3, 4, 4, 12.0, "iid", "f32"),
    ("ragged_100x20_S9", 120, 100, 20, 9, 2, 5, 14.0, "iid", "f32"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_valu_matvec_detection(case):
    from paper_1404_0424_amd import api
    name, n, B, U, S, m, K, snr, ch, scalar = case
    print(f"stream-valu {name}", flush=True)
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    f = W.uplink_frame(rng, n, B, U, S, m, snr, channel=ch, rho_bs=0.5, rho_ue=0.2)
    H, Y = dev(f.H), dev(f.Y)
    run = lambda: api.detect_cg(H, Y, f.n0, f.es, K, m, "approx", scalar, xhat=True)  # noqa: E731
    o = _run("stream-valu", U, run)
    r = _run("stream-small", U, run)
    ref = O.detect_cg(f.H, f.Y, f.n0, f.es, K, m, "approx")
    assert rel_err_vec(host(o["xhat"]), ref["xhat"], axis=1) <= TOL_X
    assert llr_err(host(o["llr"]), ref["llr"]) <= TOL_L
    assert rel_err_vec(host(o["xhat"]), host(r["xhat"]).astype(np.complex128), axis=1) <= 1e-4
