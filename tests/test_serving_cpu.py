"""The serving scheduler on the CPU with a fake executor: arrival-order
admission, the HBM budget (channel cache included) is never exceeded,
oversize requests are rejected, waiting requests are admitted as memory and
slots free up, and stats are reported."""
import threading
import time

import numpy as np
import pytest

from paper_1404_0424_amd import serving as SV


class FakeExecutor:
    """Completes each launch after `delay` seconds; records concurrency."""

    def __init__(self, delay=0.002, batching=False):
        self.delay = delay
        self.batching = batching
        self.channels = {}
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0

    def now(self):
        return time.perf_counter()

    def channel_bytes(self, H, dtype):
        return int(np.prod(H.shape)) * (8 if dtype == "c32" else 4)

    def register_channel(self, ch_id, H, dtype):
        self.channels[ch_id] = H

    def unregister_channel(self, ch_id):
        self.channels.pop(ch_id, None)

    def request_bytes(self, req):
        n, B, U = self.channels[req.ch_id].shape
        if isinstance(req, SV.UplinkRequest):
            return 4 * n * U * req.Y.shape[2] * req.qam_bits
        return 8 * n * B * req.T.shape[2]

    def batch_key(self, req):
        return (type(req).__name__, req.ch_id) if self.batching else id(req)

    def launch(self, reqs, slot, readies=()):
        with self.lock:
            self.running += len(reqs)
            self.max_running = max(self.max_running, self.running)
        return {"t_end": time.perf_counter() + self.delay, "reqs": reqs, "closed": False}

    def done(self, h):
        if not h["closed"] and time.perf_counter() >= h["t_end"]:
            with self.lock:
                self.running -= len(h["reqs"])
            h["closed"] = True
        return h["closed"]

    def finish(self, h):
        return [({"echo": r}, time.perf_counter(), 14, 0) for r in h["reqs"]]


def _up(ch, n=10, S=14, m=4):
    return SV.UplinkRequest(ch, np.zeros((n, 8, S)), 0.1, 1.0, m, 3)


def test_fifo_and_concurrency():
    ex = FakeExecutor(0.003)
    srv = SV.Server(ex, hbm_budget=1 << 30, n_slots=3)
    srv.register_channel("a", np.zeros((10, 8, 4)))
    reqs = [_up("a") for _ in range(12)]
    futs = [srv.submit(r) for r in reqs]
    res = [f.result(timeout=10) for f in futs]
    srv.close()
    assert [id(r) for r in reqs] == srv.admit_order           # arrival order
    assert 1 < ex.max_running <= 3                            # overlap, within slots
    assert all(r.outputs["echo"] is q for r, q in zip(res, reqs))
    st = srv.stats()
    assert st["frames"] == 12 and st["p99_ms"] >= st["p50_ms"] > 0


def test_budget_is_never_exceeded_and_waiters_are_admitted():
    ex = FakeExecutor(0.002)
    per_req = 4 * 10 * 4 * 14 * 4                             # request_bytes of _up
    cache = 10 * 8 * 4 * 8
    budget = cache + 2 * per_req + 100                        # room for two at a time
    srv = SV.Server(ex, hbm_budget=budget, n_slots=8)
    srv.register_channel("a", np.zeros((10, 8, 4)))
    futs = [srv.submit(_up("a")) for _ in range(10)]
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert srv.peak_bytes <= budget
    assert ex.max_running == 2                                # memory, not slots, limited it
    assert srv.budget_waits >= 1 and srv.cache_bytes == cache


def test_stats_skip_leaves_out_the_first_requests():
    ex = FakeExecutor(0.001)
    srv = SV.Server(ex, hbm_budget=1 << 30, n_slots=2)
    srv.register_channel("a", np.zeros((10, 8, 4)))
    futs = [srv.submit(_up("a")) for _ in range(10)]
    res = [f.result(timeout=10) for f in futs]
    srv.close()
    assert srv.budget_waits == 0
    full, tail = srv.stats(), srv.stats(skip=4)
    assert full["frames"] == 10 and tail["frames"] == 6
    lat = sorted(r.latency for r in sorted(res, key=lambda r: r.t_submit)[4:])
    assert tail["p50_ms"] == pytest.approx(float(np.percentile(lat, 50)) * 1e3)
    assert srv.stats(skip=10) == {"frames": 0}


def test_rejections():
    ex = FakeExecutor()
    srv = SV.Server(ex, hbm_budget=10_000, n_slots=2)
    with pytest.raises(SV.AdmissionError):
        srv.register_channel("big", np.zeros((100, 8, 4)))   # 25,600 B > budget
    srv.register_channel("a", np.zeros((2, 8, 4)))
    with pytest.raises(SV.AdmissionError):
        srv.submit(_up("a", n=2, S=200, m=8)).result(timeout=5)
    with pytest.raises(KeyError):
        srv.submit(_up("nope")).result(timeout=5)
    ok = srv.submit(_up("a", n=2, S=2))
    assert ok.result(timeout=5).outputs
    srv.close()


def test_downlink_and_unregister():
    ex = FakeExecutor(0.001)
    srv = SV.Server(ex, hbm_budget=1 << 20, n_slots=2)
    srv.register_channel("c", np.zeros((4, 16, 2)))
    r = srv.submit(SV.DownlinkRequest("c", np.zeros((4, 2, 3)), 0.1, 2)).result(timeout=5)
    assert r.latency >= 0
    srv.unregister_channel("c")
    with pytest.raises(KeyError):
        srv.submit(SV.DownlinkRequest("c", np.zeros((4, 2, 3)), 0.1, 2)).result(timeout=5)
    srv.close()


def test_batching_groups_same_class_and_keeps_head_first():
    ex = FakeExecutor(0.004, batching=True)
    srv = SV.Server(ex, hbm_budget=1 << 30, n_slots=1, max_batch=4)
    srv.register_channel("a", np.zeros((10, 8, 4)))
    srv.register_channel("b", np.zeros((10, 8, 4)))
    # the slot is busy with the first request while the rest queue up
    reqs = [_up("a")] + [_up("a" if k % 2 else "b") for k in range(9)]
    futs = [srv.submit(r) for r in reqs]
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert max(srv.batch_sizes) > 1 and max(srv.batch_sizes) <= 4
    assert sum(srv.batch_sizes) == 10
    # every launch starts with the oldest request still waiting
    arrival = {id(r): k for k, r in enumerate(reqs)}
    admitted = set()
    for grp in srv.admit_groups:
        waiting = [k for k in range(len(reqs)) if k not in admitted]
        assert arrival[grp[0]] == min(waiting)
        admitted.update(arrival[i] for i in grp)


def test_paused_start_queues_then_releases_the_backlog():
    ex = FakeExecutor(0.001, batching=True)
    srv = SV.Server(ex, hbm_budget=1 << 30, n_slots=2, start_paused=True, max_batch=8)
    srv.register_channel("a", np.zeros((10, 8, 4)))
    futs = [srv.submit(_up("a")) for _ in range(20)]
    time.sleep(0.05)
    assert not any(f.done() for f in futs) and srv.admit_order == []
    t_rel = time.perf_counter()
    srv.resume()
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert max(srv.batch_sizes) > 1                       # the backlog was batched
    st = srv.stats()
    assert st["frames"] == 20
    # latency counts from the release, not from the earlier submissions
    assert st["p99_ms"] < (time.perf_counter() - t_rel) * 1e3 + 1.0
