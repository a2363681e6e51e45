"""Native serving runtime (include/mimo_serve.h) on the GPU: each result is
the same alone and in a mix of concurrent mixed-shape requests (bitwise, and
bitwise equal to a single mimo_detect_cg / mimo_precode_cg call), matches
the FP64 oracle, a small HBM budget makes requests wait without the pool
ever holding more than the budget, and outputs return to the pool when the
caller drops them."""
import collections
import gc

import numpy as np
import pytest

from oracle import mimo_oracle as O
from paper_1404_0424_amd import workload as W

from _parity import TOL_L, TOL_X, dev, host, llr_err, rel_err_vec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(64, 8, 48), (128, 16, 64), (256, 32, 24), (128, 8, 80), (64, 16, 40), (256, 16, 32)]


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_0424_amd import native_serving as NS
    from paper_1404_0424_amd import serving as SV
    rng = np.random.default_rng(4048)
    chans = {i: W.iid_channel(rng, n, B, U) for i, (B, U, n) in enumerate(SHAPES)}
    return NS, SV, rng, chans


def _uplink(SV, rng, H, ch, m=6, snr=12.0, S=14, **kw):
    n, B, U = H.shape
    bits = W.random_bits(rng, (n, U, S), m)
    n0 = W.n0_from_snr_db(snr, U, B)
    Y = H @ W.qam_map(bits, m) + W.awgn(rng, (n, B, S), n0)
    return SV.UplinkRequest(ch, dev(Y), n0, 1.0, m, 3, **kw), Y


def _downlink(SV, rng, H, ch, S=14):
    n, B, U = H.shape
    T = W.qam_map(W.random_bits(rng, (n, U, S), 4), 4)
    return SV.DownlinkRequest(ch, dev(T), 0.3, 3, True), T


def test_alone_vs_mix_single_call_and_oracle(setup):
    NS, SV, rng, chans = setup
    from paper_1404_0424_amd import api
    print("native serving: alone vs mix", flush=True)
    srv = NS.NativeServer(hbm_budget=4 << 30, n_slots=4)
    for i, H in chans.items():
        srv.register_channel(i, H, "c32")
    up, Y = _uplink(SV, rng, chans[1], 1)
    dn, T = _downlink(SV, rng, chans[2], 2)
    alone_up = host(srv.submit(up).result(timeout=60).outputs["llr"])
    alone_dn = host(srv.submit(dn).result(timeout=60).outputs["Q"])
    futs = []
    for k in range(40):
        ch = int(rng.integers(len(chans)))
        r = _uplink(SV, rng, chans[ch], ch)[0] if k % 2 else _downlink(SV, rng, chans[ch], ch)[0]
        futs.append(srv.submit(r))
        if k == 9:
            f_up = srv.submit(up)
        if k == 25:
            f_dn = srv.submit(dn)
    mix_up = host(f_up.result(timeout=60).outputs["llr"])
    mix_dn = host(f_dn.result(timeout=60).outputs["Q"])
    for f in futs:
        res = f.result(timeout=60)
        for v in res.outputs.values():
            if v is not None:
                assert torch.isfinite(v).all()
    del res, futs
    st = srv.stats()
    srv.close()
    assert np.array_equal(alone_up, mix_up)
    assert np.array_equal(alone_dn, mix_dn)
    H1, H2 = dev(chans[1]), dev(chans[2])
    single_up = host(api.detect_cg(H1, up.Y, up.n0, 1.0, 3, 6)["llr"])
    single_dn = host(api.precode_cg(H2, dn.T, 0.3, 3, True)[0])
    assert np.array_equal(alone_up, single_up)
    assert np.array_equal(alone_dn, single_dn)
    ref = O.detect_cg(chans[1], Y, up.n0, 1.0, 3, 6)
    assert llr_err(alone_up, ref["llr"]) <= TOL_L
    pref = O.precode_cg(chans[2], T, 0.3, 3, normalize=True)
    assert rel_err_vec(alone_dn, pref["Q"], axis=1) <= TOL_X
    assert st["frames"] == 44 and st["p99_ms"] >= st["p50_ms"] > 0
    assert st["mean_batch"] >= 1.0


def test_exact_sinr_and_xhat_requests(setup):
    NS, SV, rng, chans = setup
    from paper_1404_0424_amd import api
    print("native serving: exact SINR and xhat", flush=True)
    srv = NS.NativeServer(hbm_budget=1 << 30, n_slots=2)
    srv.register_channel("a", chans[4], "c32")
    ex, _ = _uplink(SV, rng, chans[4], "a", sinr_mode="exact")
    xr, Yx = _uplink(SV, rng, chans[4], "a", want_xhat=True)
    r_ex = srv.submit(ex).result(timeout=60)
    r_x = srv.submit(xr).result(timeout=60)
    L_ex, L_x, X = host(r_ex.outputs["llr"]), host(r_x.outputs["llr"]), host(r_x.outputs["xhat"])
    del r_ex, r_x
    srv.close()
    H = dev(chans[4])
    assert np.array_equal(L_ex, host(api.detect_cg(H, ex.Y, ex.n0, 1.0, 3, 6, "exact")["llr"]))
    o = api.detect_cg(H, xr.Y, xr.n0, 1.0, 3, 6, xhat=True)
    assert np.array_equal(L_x, host(o["llr"])) and np.array_equal(X, host(o["xhat"]))
    ref = O.detect_cg(chans[4], Yx, xr.n0, 1.0, 3, 6)
    assert rel_err_vec(X, ref["xhat"], axis=1) <= TOL_X


def test_registered_gram_is_bitwise_the_direct_calls(setup):
    """Channels registered with their Gram matrix (mimo_server_register_channel_gram):
    batched uplink and downlink frames of U > 8 read G instead of forming it,
    exact-SINR frames and U <= 8 ignore it; every result is bitwise the
    single direct call's, also after the channel is registered again with
    another H (and its G), and the channel bytes count G."""
    NS, SV, rng, chans = setup
    from paper_1404_0424_amd import api
    print("native serving: registered Gram", flush=True)
    srv = NS.NativeServer(hbm_budget=4 << 30, n_slots=3)
    base = srv.cache_bytes
    for i, H in chans.items():
        srv.register_channel(i, H, "c32", gram=True)
    n_h = sum(H.shape[0] * H.shape[1] * H.shape[2] * 8 for H in chans.values())
    n_g = sum(H.shape[0] * H.shape[2] ** 2 * 8 for H in chans.values() if H.shape[2] > 8)
    assert srv.cache_bytes - base == n_h + n_g
    srv.register_channel("h16", chans[5], "bf16", gram=True)
    jobs = []
    for i in chans:
        jobs.append((i, "c32") + _uplink(SV, rng, chans[i], i))
        jobs.append((i, "c32") + _downlink(SV, rng, chans[i], i))
    jobs.append((4, "c32") + _uplink(SV, rng, chans[4], 4, sinr_mode="exact"))
    jobs.append(("h16", "bf16") + _uplink(SV, rng, chans[5], "h16"))
    jobs.append(("h16", "bf16") + _downlink(SV, rng, chans[5], "h16"))
    futs = [srv.submit(j[2]) for j in jobs]
    outs = []
    for f in futs:
        o = f.result(timeout=60).outputs
        outs.append(host(o["llr"] if "llr" in o else o["Q"]))
    # the same channel id registered again with another H: its new G is used
    H2 = W.iid_channel(rng, *chans[1].shape)
    srv.register_channel(1, H2, "c32", gram=True)
    up2, _ = _uplink(SV, rng, H2, 1)
    dn2, _ = _downlink(SV, rng, H2, 1)
    o_up2 = host(srv.submit(up2).result(timeout=60).outputs["llr"])
    o_dn2 = host(srv.submit(dn2).result(timeout=60).outputs["Q"])
    srv.close()
    for (ch, dt, req, _), out in zip(jobs, outs):
        H = dev(chans[5] if ch == "h16" else chans[ch])
        if dt != "c32":
            H = api.convert(H, dt)
        if isinstance(req, SV.UplinkRequest):
            Yin = req.Y if dt == "c32" else api.convert(req.Y, dt)
            ref = api.detect_cg(H, Yin, req.n0, 1.0, 3, 6, req.sinr_mode)["llr"]
        else:
            ref = api.precode_cg(H, req.T, 0.3, 3, True)[0]
        assert np.array_equal(out.view(np.uint32), host(ref).view(np.uint32)), (ch, type(req))
    Hd2 = dev(H2)
    assert np.array_equal(o_up2, host(api.detect_cg(Hd2, up2.Y, up2.n0, 1.0, 3, 6)["llr"]))
    assert np.array_equal(o_dn2, host(api.precode_cg(Hd2, dn2.T, 0.3, 3, True)[0]))


def test_channel_replaced_while_requests_are_queued(setup):
    """A request runs on the channel arrays registered when it was submitted:
    the binding keeps them alive after the channel id is registered again,
    even when their memory would otherwise be handed out and overwritten."""
    NS, SV, rng, chans = setup
    from paper_1404_0424_amd import api
    print("native serving: channel replaced while queued", flush=True)
    H_old = chans[2]
    srv = NS.NativeServer(hbm_budget=1 << 30, n_slots=2)
    srv.register_channel("r", H_old, "c32", gram=True)
    srv.pause()
    up, _ = _uplink(SV, rng, H_old, "r")
    fut = srv.submit(up)
    srv.register_channel("r", W.iid_channel(rng, *H_old.shape), "c32", gram=True)
    gc.collect()
    n, B, U = H_old.shape
    # same-size blocks: the caching allocator hands out freed ones first
    junk = [torch.full((n, B, U), 7.0 + 7.0j, dtype=torch.complex64, device="cuda"),
            torch.full((n, U, U), 7.0 + 7.0j, dtype=torch.complex64, device="cuda")]
    torch.cuda.synchronize()
    srv.resume()
    out = host(fut.result(timeout=60).outputs["llr"])
    srv.close()
    del junk
    ref = api.detect_cg(dev(H_old), up.Y, up.n0, 1.0, 3, 6)["llr"]
    assert np.array_equal(out, host(ref))


def test_small_budget_16bit_channel_and_pool_release(setup):
    NS, SV, rng, chans = setup
    print("native serving: small budget, 16-bit channel", flush=True)
    H = chans[1]
    n, B, U = H.shape
    req, Y = _uplink(SV, rng, H, "h16")
    S, m = 14, 6
    # output (LLRs) + scratch (Y in 16-bit storage), each rounded to 256 B
    need = -(-n * U * S * m * 4 // 256) * 256 + -(-n * B * S * 4 // 256) * 256
    cache = n * B * U * 4
    budget = cache + 2 * need                      # two requests at a time
    srv = NS.NativeServer(hbm_budget=budget, n_slots=4)
    srv.register_channel("h16", H, "f16")
    assert srv.cache_bytes == cache
    # outputs a caller holds stay in the pool (and count against the budget):
    # read each result in order and drop it, so later requests can be admitted
    futs = collections.deque(srv.submit(_uplink(SV, rng, H, "h16")[0]) for _ in range(10))
    f0 = srv.submit(req)
    while futs:
        f = futs.popleft()
        f.result(timeout=60)
        del f
    gc.collect()
    out = host(f0.result(timeout=60).outputs["llr"])
    del f0
    gc.collect()
    srv.drain(timeout=60)
    peak, waits, pool_left = srv.peak_bytes, srv.budget_waits, srv.pool_bytes
    too_big = srv.submit(_uplink(SV, rng, H, "h16", S=64)[0])
    with pytest.raises(Exception):
        too_big.result(timeout=60)
    srv.close()
    assert peak <= budget
    assert waits >= 1
    assert pool_left == 0
    deq = O.dequantize_f16(O.quantize_f16(H))
    Yq = O.dequantize_f16(O.quantize_f16(Y))
    ref = O.detect_cg(deq, Yq, req.n0, 1.0, 3, 6)
    assert llr_err(out, ref["llr"]) <= TOL_L


def test_paused_backlog_is_batched(setup):
    NS, SV, rng, chans = setup
    print("native serving: paused backlog", flush=True)
    srv = NS.NativeServer(hbm_budget=2 << 30, n_slots=2, start_paused=True, keep_outputs=False)
    srv.register_channel(0, chans[0], "c32")
    srv.register_channel(3, chans[3], "c32")
    futs = [srv.submit(_uplink(SV, rng, chans[k % 2 * 3], k % 2 * 3)[0]) for k in range(64)]
    srv.resume()
    for f in futs:
        assert f.result(timeout=60).outputs == {}
    st = srv.stats()
    srv.close()
    assert st["frames"] == 64
    assert st["mean_batch"] > 4            # same-class frames share launches
