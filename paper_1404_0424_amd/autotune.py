"""Autotuner for kernel schedules (kernel variant x persistent grid size).

The library keeps a process-wide table of schedules indexed by operation,
user class (U <= 16, U <= 32) and storage type (include/mimo_cg.h,
mimo_tune_set).  This module times every candidate schedule on the caller's
own inputs with HIP events on the current stream, installs the fastest, and
can persist the table as JSON and load it back:

    python -m paper_1404_0424_amd.autotune --workload mixed_128x16 --out tuning.json

Every schedule runs the same per-system arithmetic in the same order, so the
choice changes speed only (a GPU test checks the outputs are bitwise equal).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

from . import _lib as L

BLOCKS_PER_CU = (0, 1, 2, 3, 4, 5, 6, 8)
BASELINE_VARIANTS = {"plain"}      # reference mappings, never chosen
# variants that sum in another order (the Gram over antenna quarters; the CG
# mat-vec on VALU FMAs; the Gram and matched filter from bf16 splits): equal to
# the others to rounding, not bit for bit
ROUNDING_VARIANTS = {"split", "stream-valu", "stream-x3", "x3", "fused-x3"}
# variants that form the Gram and matched filter from bf16 splits of the FP32
# inputs (FP32-accurate, on the 16-bit matrix cores); a caller that wants FP32
# products throughout excludes them
X3_VARIANTS = {"stream-x3", "x3", "fused-x3"}
# variants whose launches take their grids from other table entries
GRID_FREE = {("slot", "separate")}
OPS = {"detect": L.MIMO_OP_DETECT, "precode": L.MIMO_OP_PRECODE,
       "gram_mf": L.MIMO_OP_GRAM_MF, "slot": L.MIMO_OP_SLOT}


def variants(op: str) -> list[str]:
    lib = L.lib()
    code = OPS[op]
    return [lib.mimo_tune_variant_name(code, v).decode()
            for v in range(lib.mimo_tune_variant_count(code))]


def user_class(U: int) -> int:
    return 0 if U <= 16 else 1


def set_schedule(op: str, U: int, dtype_code: int, variant: int, blocks_per_cu: int) -> None:
    L.check(L.lib().mimo_tune_set(OPS[op], user_class(U), dtype_code, variant, blocks_per_cu))


def get_schedule(op: str, U: int, dtype_code: int) -> tuple[int, int]:
    v, b = ctypes.c_int(), ctypes.c_int()
    L.check(L.lib().mimo_tune_get(OPS[op], user_class(U), dtype_code, ctypes.byref(v),
                                  ctypes.byref(b)))
    return v.value, b.value


def time_call(fn, reps: int = 5, warmup: int = 2) -> float:
    """Mean seconds per call of back-to-back launches (HIP events)."""
    import torch
    for _ in range(warmup):
        fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def _warm(fn, seconds: float) -> None:
    """Run ``fn`` for ``seconds`` of wall time (synchronized every few calls)
    so that the first candidate is not timed while the device clocks are
    still coming up from an idle spell."""
    import time

    import torch
    t0 = time.perf_counter()
    i = 0
    while True:
        fn()
        i += 1
        if i % 8 == 0:
            torch.cuda.synchronize()
            if time.perf_counter() - t0 >= seconds:
                break


def tune(op: str, U: int, dtype_code: int, fn, reps: int = 5, log=None, exclude=()) -> dict:
    """Time ``fn`` (which launches ``op`` on fixed inputs) under every
    candidate schedule (variants named in ``exclude`` left out), install the
    fastest, return the measurements."""
    _warm(fn, 0.1)
    results = []
    for v, name in enumerate(variants(op)):
        if name in BASELINE_VARIANTS or name in exclude:
            continue
        for b in BLOCKS_PER_CU:
            if (op, name) in GRID_FREE and b != 0:
                continue
            set_schedule(op, U, dtype_code, v, b)
            t = time_call(fn, reps)
            results.append({"variant": v, "blocks_per_cu": b, "seconds": t})
            if log:
                log(f"tune {op} U={U} dtype={dtype_code}: variant={variants(op)[v]} "
                    f"blocks/CU={b}: {t * 1e6:.1f} us")
    best = min(results, key=lambda r: r["seconds"])
    set_schedule(op, U, dtype_code, best["variant"], best["blocks_per_cu"])
    return {"op": op, "user_class": user_class(U), "dtype": dtype_code, "best": best,
            "candidates": results}


def save(entries: list[dict], path: str) -> None:
    table = [{"op": e["op"], "user_class": e["user_class"], "dtype": e["dtype"],
              "variant": e["best"]["variant"], "blocks_per_cu": e["best"]["blocks_per_cu"],
              "seconds": e["best"]["seconds"]} for e in entries]
    with open(path, "w") as f:
        json.dump({"arch": "gfx950", "schedules": table}, f, indent=1)


def load(path: str) -> int:
    """Install the schedules of a JSON table written by :func:`save`."""
    with open(path) as f:
        table = json.load(f)["schedules"]
    for e in table:
        L.check(L.lib().mimo_tune_set(OPS[e["op"]], int(e["user_class"]), int(e["dtype"]),
                                      int(e["variant"]), int(e["blocks_per_cu"])))
    return len(table)


def tune_workload(name: str, frames: int = 16, dtypes=("c32", "f16", "bf16"), log=None):
    """Tune detection and precoding for a named workload on synthetic frames."""
    import numpy as np
    import torch

    from . import api
    from . import workload as W

    wl = W.WORKLOADS[name]
    n = wl.n_sc * frames
    rng = W.rng_for(77, 0)
    up = W.uplink_frame(rng, n, wl.B, wl.U, wl.S, wl.m, wl.snr_db[0], channel=wl.channel,
                        rho_bs=wl.rho_bs, rho_ue=wl.rho_ue)
    dn = W.downlink_frame(rng, n, wl.B, wl.U, wl.S, wl.m, wl.snr_db[0], H=up.H)
    dev = torch.device("cuda")
    H = torch.from_numpy(up.H.astype(np.complex64)).to(dev)
    Y = torch.from_numpy(up.Y.astype(np.complex64)).to(dev)
    T = torch.from_numpy(dn.T.astype(np.complex64)).to(dev)
    llr = torch.empty((n, wl.U, wl.S, wl.m), dtype=torch.float32, device=dev)
    Q = torch.empty((n, wl.B, wl.S), dtype=torch.complex64, device=dev)
    sc = "f64" if wl.scalar_f64 else "f32"
    entries = []
    for dt in dtypes:
        if dt == "c32":
            Hx, Yx, code = H, Y, L.MIMO_C32
        else:
            Hx, Yx = api.convert(H, dt), api.convert(Y, dt)
            code = Hx.dtype_code
        entries.append(tune("detect", wl.U, code, lambda: api.detect_cg(
            Hx, Yx, up.n0, up.es, wl.K, wl.m, "approx", sc, out={"llr": llr}), log=log))
        entries.append(tune("precode", wl.U, code, lambda: api.precode_cg(
            Hx, T, dn.beta, wl.K, True, sc, qnorm=False, out=Q), log=log))
        # the uplink + downlink slot, after its separate form's schedules
        entries.append(tune("slot", wl.U, code, lambda: api.detect_precode_cg(
            Hx, Yx, T, up.n0, up.es, dn.beta, wl.K, wl.K, wl.m, True, sc, qnorm=False,
            out={"llr": llr, "Q": Q}), log=log))
    return entries


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="mixed_128x16")
    ap.add_argument("--frames", type=int, default=16)
    ap.add_argument("--out", default="tuning.json")
    args = ap.parse_args(argv)
    entries = tune_workload(args.workload, args.frames,
                            log=lambda m: print(m, file=sys.stderr, flush=True))
    save(entries, args.out)
    for e in entries:
        b = e["best"]
        print(f"{e['op']} user_class={e['user_class']} dtype={e['dtype']}: "
              f"{variants(e['op'])[b['variant']]} blocks/CU={b['blocks_per_cu']} "
              f"{b['seconds'] * 1e6:.1f} us")
    print(f"wrote {os.path.abspath(args.out)}")


if __name__ == "__main__":
    main()
