"""Python front end of the native serving runtime (include/mimo_serve.h).

The scheduler -- request queue, HBM-budget admission, batching of
same-class frames into one launch, HIP streams, completion tracking -- runs
in a C++ thread inside libmimocg.so; this module only marshals requests in
and completions out.  It takes the request types of :mod:`serving`
(``UplinkRequest``, ``DownlinkRequest``) and returns the same ``Result``
objects through futures, so the two servers are interchangeable for a
caller.

Memory: the native server allocates one device pool of ``hbm_budget``
bytes at creation.  Outputs of a completed request live in that pool and
are handed over as torch tensors (DLPack, no copy); their memory returns to
the pool when the last of them is deleted, so outputs the caller keeps count
against the budget, and device memory the server holds never exceeds it.
Channels are registered as device tensors that this object keeps alive;
inputs (Y, T) must be complex64 device tensors (numpy inputs are copied to
the device at submission and kept until completion).
"""
from __future__ import annotations

import concurrent.futures as cf
import ctypes
import threading

import numpy as np

from . import _lib as L
from .serving import DownlinkRequest, Result, UplinkRequest

_PyCapsule_New = ctypes.pythonapi.PyCapsule_New
_PyCapsule_New.restype = ctypes.py_object
_PyCapsule_New.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p]

_DTYPES = {"c32": L.MIMO_C32, "f16": L.MIMO_C16, "bf16": L.MIMO_CBF16}


class Prepared:
    """A request marshalled for :meth:`NativeServer.submit`."""
    __slots__ = ("req", "c", "ref", "keep", "fn")

    def __init__(self, req, c, keep, fn):
        self.req, self.c, self.keep, self.fn = req, c, keep, fn
        self.ref = ctypes.byref(c)


class NativeServer:
    """Continuous batching in the native runtime over ``n_slots`` HIP
    streams within ``hbm_budget`` bytes (registered channels included)."""

    def __init__(self, hbm_budget: int = 16 << 30, n_slots: int = 4, max_batch: int = 32,
                 lookahead: int = 128, start_paused: bool = False, device: int = 0,
                 input_events: bool = True, keep_outputs: bool = True):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.input_events = input_events
        self.keep_outputs = keep_outputs
        self.budget = int(hbm_budget)
        self._lib = L.lib()
        cfg = L.MimoServerConfig(int(hbm_budget), int(n_slots), int(max_batch), int(lookahead),
                                 int(bool(start_paused)), int(bool(keep_outputs)))
        h = ctypes.c_void_p()
        L.check(self._lib.mimo_server_create(ctypes.byref(cfg), int(device), ctypes.byref(h)))
        self._h = h
        self._lock = threading.Lock()
        self._pending: dict = {}          # req_id -> (future, request, inputs kept alive)
        self._channels: dict = {}         # ch_id -> (int id, device tensor, dtype, shape)
        self._next_ch = 1
        self._closing = False
        self._thread = threading.Thread(target=self._completions, name="mimo-native-completions",
                                        daemon=True)
        self._thread.start()

    # ------------------------------------------------------------ channels
    def register_channel(self, ch_id, H, dtype: str = "c32", gram: bool = False) -> None:
        """Keep H (n_sc, B, U) on the device (in ``dtype`` storage) for later
        requests.  ``gram``: also form its Gram matrix G = H^H H once
        (mimo_gram_mf, reg = 0) and register it, so that the frames of this
        channel skip the Gram's products (mimo_server_register_channel_gram)."""
        from . import api
        t = self.torch
        Hd = H if isinstance(H, t.Tensor) else t.from_numpy(
            np.ascontiguousarray(np.asarray(H).astype(np.complex64))).to(self.dev)
        n, B, U = (int(x) for x in Hd.shape)
        if dtype == "c32":
            store = Hd.contiguous()
            ptr = store.data_ptr()
        else:
            store = api.convert(Hd, dtype)
            ptr = store.data.data_ptr()
        # (channels of up to 8 users form a packed Gram per frame and ignore G)
        G = api.gram_mf(store, None, 0.0)[0] if gram and U > 8 else None
        t.cuda.synchronize(self.dev)
        with self._lock:
            cid = self._channels[ch_id][0] if ch_id in self._channels else self._next_ch
            if ch_id not in self._channels:
                self._next_ch += 1
            L.check(self._lib.mimo_server_register_channel_gram(
                self._h, cid, ptr, G.data_ptr() if G is not None else None, _DTYPES[dtype], n, B,
                U))
            self._channels[ch_id] = (cid, store, dtype, (n, B, U), G)

    def unregister_channel(self, ch_id) -> None:
        with self._lock:
            cid = self._channels.pop(ch_id)[0]
            L.check(self._lib.mimo_server_unregister_channel(self._h, cid))

    @property
    def cache_bytes(self) -> int:
        c, p = ctypes.c_int64(), ctypes.c_int64()
        L.check(self._lib.mimo_server_memory(self._h, ctypes.byref(c), ctypes.byref(p)))
        return c.value

    @property
    def pool_bytes(self) -> int:
        c, p = ctypes.c_int64(), ctypes.c_int64()
        L.check(self._lib.mimo_server_memory(self._h, ctypes.byref(c), ctypes.byref(p)))
        return p.value

    # ------------------------------------------------------------ requests
    def _device_c64(self, x):
        t = self.torch
        if isinstance(x, t.Tensor):
            if x.dtype != t.complex64 or not x.is_cuda or not x.is_contiguous():
                raise ValueError("inputs must be contiguous complex64 device tensors")
            return x
        return t.from_numpy(np.ascontiguousarray(np.asarray(x).astype(np.complex64))).to(self.dev)

    def prepare(self, req) -> "Prepared":
        """Marshal a request once (device inputs, C struct), so that
        submitting it costs only the queue insertion; a prepared request can
        be submitted any number of times."""
        ch = self._channels.get(req.ch_id)
        if ch is None:
            raise KeyError(f"channel {req.ch_id!r} is not registered")
        cid = ch[0]
        if isinstance(req, UplinkRequest):
            Y = self._device_c64(req.Y)
            c = L.MimoUplinkReq(cid, Y.data_ptr(), int(Y.shape[2]), int(req.qam_bits), int(req.K),
                                L.MIMO_SINR_APPROX if req.sinr_mode == "approx" else L.MIMO_SINR_EXACT,
                                L.MIMO_SCALAR_F64 if req.scalar_prec == "f64" else L.MIMO_SCALAR_F32,
                                int(bool(req.want_xhat)), float(req.n0), float(req.es))
            return Prepared(req, c, Y, self._lib.mimo_server_submit_uplink)
        if isinstance(req, DownlinkRequest):
            T = self._device_c64(req.T)
            c = L.MimoDownlinkReq(cid, T.data_ptr(), int(T.shape[2]), int(req.K),
                                  int(bool(req.normalize)),
                                  L.MIMO_SCALAR_F64 if req.scalar_prec == "f64" else L.MIMO_SCALAR_F32,
                                  float(req.beta))
            return Prepared(req, c, T, self._lib.mimo_server_submit_downlink)
        raise TypeError(f"unknown request type {type(req).__name__}")

    def submit(self, req, future: bool = True):
        """Queue a request (or a prepared one).  Returns a Future of its
        Result, or None with ``future=False`` (fire and forget: the request
        still counts in :meth:`stats`)."""
        fut = cf.Future() if future else None
        try:
            p = req if isinstance(req, Prepared) else self.prepare(req)
        except (KeyError, ValueError) as e:
            if fut is None:
                raise
            fut.set_exception(e)
            return fut
        stream = self.torch.cuda.current_stream(self.dev).cuda_stream if self.input_events else None
        rid = ctypes.c_int64()
        with self._lock:
            st = p.fn(self._h, p.ref, stream, ctypes.byref(rid))
            if st == L.MIMO_OK:
                # the request runs on the channel arrays registered now: keep
                # them alive until it completes, even if the channel is
                # registered again or dropped meanwhile
                self._pending[rid.value] = (fut, p.req, (p.keep, self._channels.get(p.req.ch_id)))
        if st != L.MIMO_OK:
            try:
                L.check(st)
            except L.MimoError as e:
                if fut is None:
                    raise
                fut.set_exception(e)
        return fut

    def _tensor(self, rid: int, which: int):
        p = ctypes.c_void_p()
        L.check(self._lib.mimo_server_dlpack(self._h, rid, which, ctypes.byref(p)))
        return self.torch.utils.dlpack.from_dlpack(_PyCapsule_New(p, b"dltensor", None))

    def _completions(self) -> None:
        buf = (L.MimoCompletion * 64)()
        while True:
            n = self._lib.mimo_server_poll(self._h, buf, 64, 20000)
            if n < 0:
                return
            for c in buf[:n]:
                with self._lock:
                    fut, req, _keep = self._pending.pop(c.req_id)
                if fut is None:                   # submitted without a future
                    if self.keep_outputs:
                        self._lib.mimo_server_release(self._h, c.req_id)
                    fut = req = _keep = None
                    continue
                outs = None
                try:
                    if c.status != L.MIMO_OK:
                        raise L.MimoError(c.status, f"request {c.req_id} failed at launch")
                    outs = {}
                    if self.keep_outputs:
                        if c.kind == 0:
                            outs["llr"] = self._tensor(c.req_id, 0)
                            outs["xhat"] = self._tensor(c.req_id, 1) if c.out2 else None
                        else:
                            outs["Q"] = self._tensor(c.req_id, 0)
                            outs["qnorm"] = self._tensor(c.req_id, 1)
                    res = Result(outs, c.t_submit, c.t_admit, c.t_done, int(c.solves),
                                 int(c.llr_bits))
                except Exception as e:            # noqa: BLE001 - reported through the future
                    res = e
                finally:
                    # the caller's hold; tensors handed out keep the buffers
                    if self.keep_outputs:
                        self._lib.mimo_server_release(self._h, c.req_id)
                if isinstance(res, Exception):
                    fut.set_exception(res)
                else:
                    fut.set_result(res)
                # hold no reference to the outputs here: dropped results
                # return their memory to the pool at once
                fut = req = _keep = res = outs = None
            if n == 0 and self._closing:
                with self._lock:
                    if not self._pending:
                        return

    # ------------------------------------------------------------ control
    def pause(self) -> None:
        L.check(self._lib.mimo_server_pause(self._h))

    def resume(self) -> None:
        L.check(self._lib.mimo_server_resume(self._h))

    def drain(self, timeout: float | None = None) -> None:
        us = -1 if timeout is None else int(timeout * 1e6)
        st = self._lib.mimo_server_drain(self._h, us)
        if st != L.MIMO_OK:
            raise TimeoutError("serving queue did not drain")

    def close(self) -> None:
        """Wait for every request, resolve the futures, free the pool.
        Output tensors still held become invalid: copy what you keep."""
        if self._h is None:
            return
        self.drain()
        self._closing = True
        self._thread.join()
        L.check(self._lib.mimo_server_destroy(self._h))
        self._h = None

    def stats(self, reset: bool = False, skip: int = 0) -> dict:
        s = L.MimoServerStats()
        L.check(self._lib.mimo_server_stats_get(self._h, int(skip), int(bool(reset)),
                                                ctypes.byref(s)))
        if s.frames == 0:
            return {"frames": 0}
        return {"frames": int(s.frames), "p50_ms": s.p50_ms, "p99_ms": s.p99_ms,
                "mean_ms": s.mean_ms, "frames_per_s": s.frames_per_s,
                "solves_per_s": s.solves_per_s, "llr_gbit_s": s.llr_gbit_s,
                "launches": int(s.launches), "mean_batch": s.mean_batch}

    @property
    def peak_bytes(self) -> int:
        s = L.MimoServerStats()
        L.check(self._lib.mimo_server_stats_get(self._h, 0, 0, ctypes.byref(s)))
        return int(s.peak_bytes)

    @property
    def budget_waits(self) -> int:
        s = L.MimoServerStats()
        L.check(self._lib.mimo_server_stats_get(self._h, 0, 0, ctypes.byref(s)))
        return int(s.budget_waits)
