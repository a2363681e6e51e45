"""Continuous-batching serving loop for uplink detection / downlink precoding.

Requests (one OFDM frame each: all subcarriers x S symbols of one channel)
arrive at any time through :meth:`Server.submit`.  A scheduler thread admits
them in arrival order whenever a stream slot is free and the HBM budget has
room for the request's buffers, and launches each admitted request on its
own HIP stream, so requests that arrive while others are running overlap on
the device.  Channel state (H, and its 16-bit copy when requested) stays on
the device across frames, keyed by channel id; uplink and downlink share it
by reciprocity (the precoder uses H_d = H_u^H).

Latency is arrival to completion of the request's last kernel: completion
times come from HIP events measured against a reference event whose host
time was taken when the server started.

The HBM budget covers the channel cache and the device buffers of admitted
requests until their kernels complete.  Outputs handed back to the caller
(through the request's future) are the caller's from then on and sit outside
the budget: the server keeps no reference to them, only the timing and work
counts of completed requests for :meth:`Server.stats`.

The scheduling logic is independent of the GPU: an *executor* object does
the device work (``GpuExecutor`` here), so the admission and ordering rules
can be exercised with any executor that implements the same methods.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import itertools
import threading
import time

import numpy as np


@dataclasses.dataclass
class UplinkRequest:
    ch_id: object
    Y: object                 # device complex64 tensor (n_sc, B, S) or numpy array
    n0: float
    es: float
    qam_bits: int
    K: int
    sinr_mode: str = "approx"
    scalar_prec: str = "f32"
    want_xhat: bool = False


@dataclasses.dataclass
class DownlinkRequest:
    ch_id: object
    T: object                 # device complex64 tensor (n_sc, U, S) or numpy array
    beta: float
    K: int
    normalize: bool = True
    scalar_prec: str = "f32"


@dataclasses.dataclass
class Result:
    outputs: dict             # device tensors (llr / xhat or Q / qnorm)
    t_submit: float
    t_admit: float
    t_done: float
    solves: int
    llr_bits: int

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


@dataclasses.dataclass
class _Done:
    """What the server keeps of a completed request (no device buffers)."""
    t_submit: float
    t_done: float
    solves: int
    llr_bits: int


class AdmissionError(RuntimeError):
    """A request can never fit the HBM budget."""


@dataclasses.dataclass(eq=False)          # queue entries compare by identity
class _Pending:
    req: object
    fut: cf.Future
    t_submit: float
    need: int
    ready: object = None
    key: object = None        # executor batch key, computed once at submission


class Server:
    """FIFO continuous batching over ``n_slots`` concurrent streams within
    ``hbm_budget`` bytes (channel cache included)."""

    def __init__(self, executor, hbm_budget: int = 16 << 30, n_slots: int = 4,
                 poll_interval: float = 20e-6, max_batch: int = 32, lookahead: int = 128,
                 start_paused: bool = False):
        self.ex = executor
        self.max_batch = max_batch
        self.lookahead = lookahead
        self.batch_sizes: list = []        # frames per launch
        self.admit_groups: list = []       # request ids of each launch
        self.budget = int(hbm_budget)
        self.n_slots = n_slots
        self.poll_interval = poll_interval
        self._lock = threading.Condition()
        self._queue: collections.deque[_Pending] = collections.deque()
        self._inflight: list = []          # (group, bytes, handle, slot, t_admit)
        self._free_slots = list(range(n_slots))
        self._reserved = 0                 # bytes of admitted requests
        self._channels: dict = {}          # ch_id -> bytes
        self._done: list[_Done] = []
        self._running = True
        self._paused = bool(start_paused)  # queue requests without admitting them
        self._t_resume = None              # when a paused server was released
        self._t_first = None
        self.peak_bytes = 0                # largest reserved + cached bytes seen
        self.budget_waits = 0              # queue heads that waited for HBM budget
        self._blocked = None               # the head currently waiting for budget
        self.admit_order: list = []        # ids of requests in admission order
        self._thread = threading.Thread(target=self._loop, name="mimo-serving", daemon=True)
        self._thread.start()

    # ------------------------------------------------------------ channels
    def register_channel(self, ch_id, H, dtype: str = "c32") -> None:
        """Keep H (n_sc, B, U) on the device for later requests."""
        with self._lock:
            need = self.ex.channel_bytes(H, dtype)
            old = self._channels.get(ch_id, 0)
            if self._cache_bytes() - old + need + self._reserved > self.budget:
                raise AdmissionError(f"channel {ch_id!r} ({need} B) exceeds the HBM budget")
            self.ex.register_channel(ch_id, H, dtype)
            self._channels[ch_id] = need

    def unregister_channel(self, ch_id) -> None:
        with self._lock:
            self.ex.unregister_channel(ch_id)
            self._channels.pop(ch_id, None)
            self._lock.notify_all()

    def _cache_bytes(self) -> int:
        return sum(self._channels.values())

    @property
    def cache_bytes(self) -> int:
        """Device bytes held by registered channels (part of the budget)."""
        with self._lock:
            return self._cache_bytes()

    # ------------------------------------------------------------ requests
    def submit(self, req) -> cf.Future:
        fut: cf.Future = cf.Future()
        t = self.ex.now()
        with self._lock:
            if req.ch_id not in self._channels:
                fut.set_exception(KeyError(f"channel {req.ch_id!r} is not registered"))
                return fut
            need = self.ex.request_bytes(req)
            if need + self._cache_bytes() > self.budget:
                fut.set_exception(AdmissionError(
                    f"request needs {need} B, budget {self.budget} B minus cache "
                    f"{self._cache_bytes()} B"))
                return fut
            if self._t_first is None:
                self._t_first = t
            ready = self.ex.on_submit(req) if hasattr(self.ex, "on_submit") else None
            self._queue.append(_Pending(req, fut, t, need, ready, self.ex.batch_key(req)))
            self._lock.notify_all()
        return fut

    def pause(self) -> None:
        """Stop admitting new requests (those in flight complete); submissions
        queue until :meth:`resume`."""
        with self._lock:
            self._paused = True
            self._t_resume = None

    def resume(self) -> None:
        """Start admitting (a server created with start_paused=True queues
        submissions until then, so a backlog can be released at once)."""
        with self._lock:
            if self._paused:
                self._paused = False
                self._t_resume = self.ex.now()
                self._lock.notify_all()

    def drain(self, timeout: float | None = None) -> None:
        """Wait until every submitted request has completed."""
        deadline = None if timeout is None else time.perf_counter() + timeout
        with self._lock:
            while self._queue or self._inflight:
                left = None if deadline is None else deadline - time.perf_counter()
                if left is not None and left <= 0:
                    raise TimeoutError("serving queue did not drain")
                self._lock.wait(timeout=0.001 if left is None else min(left, 0.001))

    def close(self) -> None:
        self.drain()
        with self._lock:
            self._running = False
            self._lock.notify_all()
        self._thread.join()

    # ------------------------------------------------------------ stats
    def stats(self, reset: bool = False, skip: int = 0) -> dict:
        """Latency and throughput of the completed requests; ``skip`` leaves
        out the first requests by submission time (a warm-up).  For a server
        started paused, time counts from its release (requests submitted
        before it arrive then)."""
        with self._lock:
            done = list(self._done)
            t_rel = self._t_resume
            if reset:
                self._done.clear()
                self._t_first = None
        done = sorted(done, key=lambda r: r.t_submit)[skip:]
        if not done:
            return {"frames": 0}
        arrive = (lambda r: r.t_submit) if t_rel is None else (lambda r: max(r.t_submit, t_rel))
        lat = np.array([r.t_done - arrive(r) for r in done])
        t0 = min(arrive(r) for r in done)
        t1 = max(r.t_done for r in done)
        span = max(t1 - t0, 1e-12)
        return {"frames": len(done),
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3),
                "frames_per_s": len(done) / span,
                "solves_per_s": sum(r.solves for r in done) / span,
                "llr_gbit_s": sum(r.llr_bits for r in done) / span / 1e9}

    # ------------------------------------------------------------ scheduler
    def _loop(self) -> None:
        while True:
            with self._lock:
                if not self._running:
                    return
                if self._paused:
                    self._lock.wait(timeout=0.01)
                    continue
                self._admit_locked()
                busy = bool(self._inflight)
                if not busy and not self._queue:
                    self._lock.wait(timeout=0.01)
                    continue
            self._poll()
            time.sleep(self.poll_interval)

    def _admit_locked(self) -> None:
        """Admit the queue head when it fits, together with later queued
        requests of the same kernel class (one batched launch, up to
        max_batch frames, within the budget).  The head never waits behind a
        later request."""
        while self._queue and self._free_slots:
            head = self._queue[0]
            cache = self._cache_bytes()
            if self._reserved + head.need + cache > self.budget:
                if self._blocked is not head:
                    self._blocked = head
                    self.budget_waits += 1
                return
            key = head.key
            group, total = [head], head.need
            for p in itertools.islice(self._queue, 1, self.lookahead):
                if len(group) >= self.max_batch:
                    break
                if (p.key == key
                        and self._reserved + total + p.need + cache <= self.budget):
                    group.append(p)
                    total += p.need
            for p in group:
                self._queue.remove(p)
            slot = self._free_slots.pop(0)
            self._reserved += total
            self.peak_bytes = max(self.peak_bytes, self._reserved + cache)
            self.admit_order.extend(id(p.req) for p in group)
            self.admit_groups.append([id(p.req) for p in group])
            self.batch_sizes.append(len(group))
            t_admit = self.ex.now()
            try:
                handle = self.ex.launch([p.req for p in group], slot, [p.ready for p in group])
            except Exception as e:          # noqa: BLE001 - reported through the futures
                self._reserved -= total
                self._free_slots.append(slot)
                for p in group:
                    p.fut.set_exception(e)
                continue
            self._inflight.append((group, total, handle, slot, t_admit))

    def _poll(self) -> None:
        finished = []
        with self._lock:
            for item in list(self._inflight):
                group, total, handle, slot, t_admit = item
                if self.ex.done(handle):
                    self._inflight.remove(item)
                    self._reserved -= total
                    self._free_slots.append(slot)
                    finished.append(item)
            if finished:
                self._lock.notify_all()
        for group, total, handle, slot, t_admit in finished:
            try:
                per = self.ex.finish(handle)
                results = [Result(o, p.t_submit, t_admit, t_done, solves, bits)
                           for p, (o, t_done, solves, bits) in zip(group, per)]
                with self._lock:
                    self._done.extend(_Done(r.t_submit, r.t_done, r.solves, r.llr_bits)
                                      for r in results)
                for p, r in zip(group, results):
                    p.fut.set_result(r)
            except Exception as e:          # noqa: BLE001
                for p in group:
                    p.fut.set_exception(e)


class GpuExecutor:
    """Device work for :class:`Server` through the C ABI, one HIP stream per
    slot (all at default priority).  With ``input_events`` (default) each
    submission records an event on the caller's current stream that the slot
    stream waits for, so inputs written there just before submitting are
    complete; a caller whose inputs are already synchronized can turn it off
    and save that per-request cost."""

    def __init__(self, n_slots: int = 4, device: int = 0, input_events: bool = True):
        import torch

        from . import api
        self.torch = torch
        self.api = api
        self.dev = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(n_slots)]
        self.input_events = input_events
        self.channels: dict = {}
        # host/device clock alignment: a reference event whose host time is
        # bracketed as tightly as possible (best of several round trips)
        best = None
        for _ in range(20):
            ev = torch.cuda.Event(enable_timing=True)
            ta = time.perf_counter()
            ev.record()
            ev.synchronize()
            tb = time.perf_counter()
            if best is None or tb - ta < best[2] - best[1]:
                best = (ev, ta, tb)
        self._ref, ta, tb = best
        self._t_ref = 0.5 * (ta + tb)

    def now(self) -> float:
        return time.perf_counter()

    def _dev_c64(self, x):
        t = self.torch
        if isinstance(x, np.ndarray):
            return t.from_numpy(np.ascontiguousarray(x.astype(np.complex64))).to(self.dev)
        return x

    def channel_bytes(self, H, dtype: str) -> int:
        n = int(np.prod(H.shape))
        return n * (8 if dtype == "c32" else 4)

    def register_channel(self, ch_id, H, dtype: str) -> None:
        Hd = self._dev_c64(H)
        if dtype == "c32":
            self.channels[ch_id] = (Hd, dtype)
        else:
            self.channels[ch_id] = (self.api.convert(Hd, dtype), dtype)
        self.torch.cuda.synchronize(self.dev)

    def unregister_channel(self, ch_id) -> None:
        self.channels.pop(ch_id, None)

    def _shape(self, ch_id):
        H, dtype = self.channels[ch_id]
        if dtype == "c32":
            return tuple(H.shape), dtype
        return (H.n, H.R, H.C), dtype

    def request_bytes(self, req) -> int:
        (n, B, U), dtype = self._shape(req.ch_id)
        if isinstance(req, UplinkRequest):
            S = req.Y.shape[2]
            b = 4 * n * U * S * req.qam_bits + (8 * n * U * S if req.want_xhat else 0)
            if isinstance(req.Y, np.ndarray):
                b += 8 * n * B * S
            if dtype != "c32":
                b += 4 * n * B * S
            return b
        S = req.T.shape[2]
        b = 8 * n * B * S + 4 * n * S
        if isinstance(req.T, np.ndarray):
            b += 8 * n * U * S
        return b

    def on_submit(self, req):
        """Called at submission: device inputs written on the caller's stream
        must be complete before the slot stream reads them."""
        if not self.input_events:
            return None
        ev = self.torch.cuda.Event()
        ev.record()
        return ev

    def batch_key(self, req):
        """Requests with equal keys can share one batched launch."""
        (n, B, U), dtype = self._shape(req.ch_id)
        if isinstance(req, UplinkRequest):
            if req.sinr_mode != "approx":
                return ("up-exact", id(req))          # never batched
            return ("up", U <= 16, dtype, req.qam_bits, req.scalar_prec, req.want_xhat)
        return ("dn", U <= 16, dtype, req.scalar_prec)

    def launch(self, reqs, slot: int, readies=()):
        t = self.torch
        st = self.streams[slot]
        for ev in readies:
            if ev is not None:
                st.wait_event(ev)
        outs, work = [], []
        with t.cuda.stream(st):
            first = reqs[0]
            if isinstance(first, UplinkRequest) and first.sinr_mode != "approx":
                H, dtype = self.channels[first.ch_id]
                Y = self._dev_c64(first.Y)
                if dtype != "c32":
                    Y = self.api.convert(Y, dtype, stream=st)
                o = self.api.detect_cg(H, Y, first.n0, first.es, first.K, first.qam_bits,
                                       first.sinr_mode, first.scalar_prec, xhat=first.want_xhat,
                                       stream=st)
                outs.append(o)
            elif isinstance(first, UplinkRequest):
                frames = []
                for r in reqs:
                    H, dtype = self.channels[r.ch_id]
                    Y = self._dev_c64(r.Y)
                    if dtype != "c32":
                        Y = self.api.convert(Y, dtype, stream=st)
                    frames.append((H, Y, r.n0, r.es))
                outs = self.api.detect_cg_batch(frames, [r.K for r in reqs], first.qam_bits,
                                                first.scalar_prec, xhat=first.want_xhat,
                                                stream=st)
            else:
                frames = [(self.channels[r.ch_id][0], self._dev_c64(r.T), r.beta, r.normalize)
                          for r in reqs]
                res = self.api.precode_cg_batch(frames, [r.K for r in reqs], first.scalar_prec,
                                                qnorm=True, stream=st)
                outs = [{"Q": q, "qnorm": qn} for q, qn in res]
            for r, o in zip(reqs, outs):
                if isinstance(r, UplinkRequest):
                    n, U, S, m = o["llr"].shape
                    work.append((n * S, n * S * U * m))
                else:
                    work.append((r.T.shape[0] * r.T.shape[2], 0))
            ev = t.cuda.Event(enable_timing=True)
            ev.record(st)
        return (ev, outs, work, reqs)         # requests kept alive until completion

    def done(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle):
        ev, outs, work, _ = handle
        t_done = self._t_ref + self._ref.elapsed_time(ev) / 1e3
        return [(o, t_done, w[0], w[1]) for o, w in zip(outs, work)]
