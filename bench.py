#!/usr/bin/env python3
"""Benchmark of the CG detection + precoding hot path on one MI355X.

One step = one TDD slot over a batch of F frames of the named workload:
uplink soft-output detection (Gram + matched filter, K CG iterations with
in-loop SINR, max-log LLRs) followed by downlink CG precoding with power
normalization on the same (reciprocal) channels.  Inputs are seeded
synthetic frames already resident in HBM; the batch (default 16 frames,
~0.7 GB) is larger than the 256 MB Infinity Cache, so HBM is what is timed.

Prints progress to stderr and ONE JSON line to stdout.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload mixed_128x16]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP32_VECTOR_TFLOPS = 157.3      # MI355X FP32 vector peak
METRIC = "MMSE-CG subcarrier-solves/s + LLR Gbit/s at B=128,U=16; p50/p99 frame latency"
CFG_INDEX = {"small_32x8": 1, "plain_128x8": 2, "mixed_128x16": 3, "mixed_128x32": 3,
             "corr_256x32": 5}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# kernel symbol that each detection schedule variant launches
DETECT_KERNEL = {"generic": "detect_approx_kernel", "stream": "detect_stream_kernel",
                 "stream-small": "detect_stream_kernel", "plain": "detect_plain_kernel",
                 "ring": "detect_ring_kernel", "split": "detect_split_kernel",
                 "stream-valu": "detect_stream_kernel", "stream-x3": "detect_stream_kernel"}
# translation units the complex64 approximate-SINR detection kernels are built from
DETECT_SOURCES = ["detect.hip", "detect_core.hpp", "detect_ring.hip", "split.hip", "cg_core.hpp",
                  "gram_phase.hpp", "llr.hpp", "kernels.hpp", "common.hpp"]
# ... and the fused uplink + downlink slot kernel
SLOT_KERNEL = "slot_resident_kernel"
SLOT_SOURCES = ["slot.hip", "resident.hpp", "precode_out.hpp", "detect_core.hpp", "cg_core.hpp",
                "gram_phase.hpp", "llr.hpp", "kernels.hpp", "common.hpp"]
PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")


def recorded_traffic(kernel, workload, n_sc, persistent=False, sources=None):
    """HBM bytes per launch of ``kernel`` from the committed counter summary
    profiles/<kernel>_<workload>_c32.md (FETCH_SIZE + WRITE_SIZE passes,
    scaled by a plain copy of known size), for a grid of one wavefront per
    subcarrier or, with ``persistent``, a capped (persistent) grid.  The
    summary records the source digest of the kernel's files and the
    subcarriers per launch; a figure taken from other sources or another
    launch size is not reported."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_c32.md")
    if not os.path.exists(path):
        return None
    from paper_1404_0424_amd.build import source_digest
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- `") and "` = " in line:
                k, v = line[3:].split("` = ", 1)
                rec[k] = v.strip().strip("`")
    try:
        if (rec.get("source_digest") != source_digest(sources or DETECT_SOURCES)
                or int(rec["subcarriers_per_launch"]) != n_sc):
            return None
        key = "hbm_bytes_per_launch_persistent" if persistent else "hbm_bytes_per_launch"
        return {"bytes_per_launch": float(rec[key]),
                "file": os.path.relpath(path, os.path.dirname(PROFILES))}
    except (KeyError, ValueError):
        return None


def detect_bytes_per_sc(B, U, S, m, elem_bytes=8):
    """Algorithmic HBM bytes of detection per subcarrier: read H and Y once,
    write the LLRs (FP32)."""
    return elem_bytes * B * U + elem_bytes * B * S + 4 * U * S * m


def precode_bytes_per_sc(B, U, S, elem_bytes=8):
    """Read H and T, write Q (complex64)."""
    return elem_bytes * B * U + 8 * U * S + 8 * B * S


def slot_bytes_per_sc(B, U, S, m, elem_bytes=8):
    """Uplink + downlink slot on one channel: read H once, Y and T, write the
    LLRs and Q."""
    return (elem_bytes * B * U + elem_bytes * B * S + 8 * U * S + 4 * U * S * m
            + 8 * B * S)


def slot_fused_covers(B, U, S, storage="c32"):
    """Whether mimo_detect_precode_cg runs the fused kernel for this shape."""
    return storage == "c32" and U <= 16 and S <= 16 and B <= 128


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mixed_128x16")
    ap.add_argument("--frames", type=int, default=16, help="frames per step (batch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true", help="keep the library's default schedules")
    ap.add_argument("--schedules", help="load a schedule table saved by --save-schedules "
                    "(or the autotuner) instead of tuning")
    ap.add_argument("--save-schedules", help="write the tuned schedule table to this file")
    ap.add_argument("--detect-schedule", metavar="VARIANT:BLOCKS_PER_CU",
                    help="run detection under this schedule instead of tuning (e.g. stream-valu:0)")
    ap.add_argument("--precode-schedule", metavar="VARIANT:BLOCKS_PER_CU",
                    help="run precoding under this schedule instead of tuning (e.g. split:2)")
    ap.add_argument("--slot-schedule", metavar="VARIANT:BLOCKS_PER_CU",
                    help="run the uplink + downlink step under this schedule instead of tuning "
                         "(fused:4, or separate:0 for the two launches)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream leg")
    ap.add_argument("--serving-frames", type=int, default=2000)
    ap.add_argument("--serving-skip", type=int, default=200,
                    help="serving frames left out of the statistics (warm-up)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-configuration leg (32x8, 128x8 SNR sweep, 128x32, "
                         "256x32 correlated, Gram-stage MFMA utilisation)")
    ap.add_argument("--no-wide", action="store_true",
                    help="skip the more-than-32-users leg (128x48, 128x64)")
    ap.add_argument("--no-comparison", action="store_true",
                    help="skip the comparison-methods leg (Cholesky, Neumann, CGLS, CG-D vs K)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy 3x (reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU (use --gpus 1): subcarriers are independent "
              "systems, so the path shards by subcarrier with no cross-GPU exchange and "
              "the whole-job rate is the per-GPU rate times the GPU count.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_1404_0424_amd import api
    from paper_1404_0424_amd import workload as W

    wl = W.WORKLOADS[args.workload]
    F = args.frames
    n = wl.n_sc * F
    snr = wl.snr_db[0] if len(wl.snr_db) == 1 else 10.0
    t = time.perf_counter()
    rng = W.rng_for(CFG_INDEX.get(wl.name, 9), 0)
    up = W.uplink_frame(rng, n, wl.B, wl.U, wl.S, wl.m, snr, channel=wl.channel,
                        rho_bs=wl.rho_bs, rho_ue=wl.rho_ue)
    dn = W.downlink_frame(rng, n, wl.B, wl.U, wl.S, wl.m, snr, H=up.H)
    log(f"generated {F} frames of {wl.name} in {time.perf_counter() - t:.1f}s")

    dev = torch.device("cuda:0")
    H = torch.from_numpy(up.H.astype(np.complex64)).to(dev)
    Y = torch.from_numpy(up.Y.astype(np.complex64)).to(dev)
    T = torch.from_numpy(dn.T.astype(np.complex64)).to(dev)
    llr = torch.empty((n, wl.U, wl.S, wl.m), dtype=torch.float32, device=dev)
    Q = torch.empty((n, wl.B, wl.S), dtype=torch.complex64, device=dev)
    scalar = "f64" if wl.scalar_f64 else "f32"
    n0, es, beta, K, m = up.n0, up.es, dn.beta, wl.K, wl.m

    def run_separate(Hx, Yx, steps):
        """The step as two launches with events between them (per-kernel
        times of detection and precoding)."""
        evs = []
        for _ in range(steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event(enable_timing=True)
            e0.record()
            api.detect_cg(Hx, Yx, n0, es, K, m, "approx", scalar, out={"llr": llr})
            e1.record()
            api.precode_cg(Hx, T, beta, K, normalize=True, scalar_prec=scalar, qnorm=False, out=Q)
            e2.record()
            evs.append((e0, e1, e2))
        return evs

    def slot_call(Hx, Yx):
        api.detect_precode_cg(Hx, Yx, T, n0, es, beta, K, K, m, True, scalar, qnorm=False,
                              out={"llr": llr, "Q": Q})

    def run_slot(Hx, Yx, steps):
        """The step as one mimo_detect_precode_cg call (its tuned schedule:
        the fused kernel, or the two launches)."""
        evs = []
        for _ in range(steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            slot_call(Hx, Yx)
            e1.record()
            evs.append((e0, e1))
        return evs

    def timed(Hx, Yx, label, separate=False):
        run = run_separate if separate else run_slot
        gpu_warm([lambda: run(Hx, Yx, 1)], 0.1)
        run(Hx, Yx, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs = run(Hx, Yx, args.steps)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        if separate:
            det = float(np.mean([a.elapsed_time(b) for a, b, _ in evs])) / 1e3
            pre = float(np.mean([b.elapsed_time(c) for _, b, c in evs])) / 1e3
            log(f"{label}: {wall * 1e3:.3f} ms/step (detect {det * 1e3:.3f} ms, "
                f"precode {pre * 1e3:.3f} ms)")
            return wall, det, pre
        ker = float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3
        log(f"{label}: {wall * 1e3:.3f} ms/step ({ker * 1e3:.3f} ms between the step's events)")
        return wall, ker

    def kernel_time(fn, reps=20, batches=3):
        """Average duration of back-to-back launches between two events on
        the stream the kernels run on (torch's current stream); the median
        over ``batches`` such groups of ``reps`` launches, so that one host
        stall while the queue runs dry does not set the figure.  The device
        first runs ``fn`` for a while (gpu_warm)."""
        gpu_warm([fn], 0.03)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(batches):
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / reps / 1e3)
        return sorted(ts)[len(ts) // 2]

    from paper_1404_0424_amd import autotune
    tuned = {}
    ops = ("detect", "precode", "slot")
    if args.schedules:
        autotune.load(args.schedules)
        for op in ops:
            v, b = autotune.get_schedule(op, wl.U, 0)
            tuned[op] = {"variant": autotune.variants(op)[v], "blocks_per_cu": b,
                         "from": os.path.basename(args.schedules)}
        log(f"loaded schedules: {tuned}")
    elif args.detect_schedule or args.precode_schedule or args.slot_schedule:
        for op, spec in zip(ops, (args.detect_schedule, args.precode_schedule,
                                  args.slot_schedule)):
            if spec:
                name, bpc = spec.split(":")
                autotune.set_schedule(op, wl.U, 0, autotune.variants(op).index(name), int(bpc))
            v, b = autotune.get_schedule(op, wl.U, 0)
            tuned[op] = {"variant": autotune.variants(op)[v], "blocks_per_cu": b, "from": "command line"}
        log(f"schedules: {tuned}")
    elif not args.no_tune:
        # schedules picked by the autotuner on these inputs (not timed); the
        # slot's "separate" form runs the two tuned schedules
        # (FP32 products throughout: the bf16-split forms are timed apart)
        x3 = autotune.X3_VARIANTS
        e1 = autotune.tune("detect", wl.U, 0, lambda: api.detect_cg(
            H, Y, n0, es, K, m, "approx", scalar, out={"llr": llr}), exclude=x3)
        e2 = autotune.tune("precode", wl.U, 0, lambda: api.precode_cg(
            H, T, beta, K, normalize=True, scalar_prec=scalar, qnorm=False, out=Q), exclude=x3)
        e3 = autotune.tune("slot", wl.U, 0, lambda: slot_call(H, Y), exclude=x3)
        if args.save_schedules:
            autotune.save([e1, e2, e3], args.save_schedules)
        for e in (e1, e2, e3):
            b = e["best"]
            tuned[e["op"]] = {"variant": autotune.variants(e["op"])[b["variant"]],
                              "blocks_per_cu": b["blocks_per_cu"],
                              "us": round(b["seconds"] * 1e6, 1)}
        log(f"autotuned schedules: {tuned}")

    # the step: one mimo_detect_precode_cg call; slot_s = average time
    # between the events around it in the timed steps (the roofline uses it)
    wall, slot_s = timed(H, Y, "complex64 slot")
    wall_eager = wall
    # context: the same step as two launches (detection, then precoding)
    wall_sep, det_s, pre_s = timed(H, Y, "complex64 separate launches", separate=True)
    det_b2b = kernel_time(lambda: api.detect_cg(H, Y, n0, es, K, m, "approx", scalar,
                                                out={"llr": llr}))
    pre_b2b = kernel_time(lambda: api.precode_cg(H, T, beta, K, normalize=True,
                                                 scalar_prec=scalar, qnorm=False, out=Q))
    slot_b2b = kernel_time(lambda: slot_call(H, Y))
    log(f"back-to-back: detect {det_b2b * 1e3:.3f} ms, precode {pre_b2b * 1e3:.3f} ms, "
        f"slot {slot_b2b * 1e3:.3f} ms per launch")
    # context: the same launches with the Gram and matched filter formed from
    # bf16 splits of the FP32 inputs (FP32-accurate), each at its best grid
    saved = {op: autotune.get_schedule(op, wl.U, 0) for op in ("detect", "precode", "slot")}
    x3t = {}
    for op, name, fn in (("detect", "stream-x3", lambda: api.detect_cg(
                              H, Y, n0, es, K, m, "approx", scalar, out={"llr": llr})),
                         ("precode", "x3", lambda: api.precode_cg(
                              H, T, beta, K, normalize=True, scalar_prec=scalar, qnorm=False,
                              out=Q)),
                         ("slot", "fused-x3", lambda: slot_call(H, Y))):
        best = None
        for bpc in (0, 2, 4, 6, 8):
            autotune.set_schedule(op, wl.U, 0, autotune.variants(op).index(name), bpc)
            tt = kernel_time(fn)
            best = tt if best is None else min(best, tt)
        x3t[op] = best
    for op, (v, b) in saved.items():
        autotune.set_schedule(op, wl.U, 0, v, b)
    split_x3 = {"detect_ms": x3t["detect"] * 1e3, "precode_ms": x3t["precode"] * 1e3,
                "slot_ms": x3t["slot"] * 1e3, "slot_solves_per_s": 2 * n * wl.S / x3t["slot"],
                "what": "back-to-back launches with the Gram and matched filter from an exact "
                        "three-way bf16 split of the FP32 inputs on the 16-bit matrix cores "
                        "(FP32 accumulation); not used for value"}
    log(f"bf16-split Gram: detect {x3t['detect'] * 1e3:.3f} ms, precode "
        f"{x3t['precode'] * 1e3:.3f} ms, slot {x3t['slot'] * 1e3:.3f} ms")
    # context: detection and precoding from the channel's Gram matrix formed
    # once beforehand (mimo_gram_mf, reg = 0), as for a channel held over
    # several frames; not the step, which forms the Gram in every call
    Gc, _ = api.gram_mf(H, None, 0.0)
    tdg = kernel_time(lambda: api.detect_cg_gram(Gc, H, Y, n0, es, K, m, scalar,
                                                 out={"llr": llr}))
    tpg = kernel_time(lambda: api.precode_cg_gram(Gc, H, T, beta, K, True, scalar, qnorm=False,
                                                  out=Q))
    del Gc
    cached_gram = {"detect_ms": tdg * 1e3, "precode_ms": tpg * 1e3,
                   "direct_detect_ms": det_b2b * 1e3, "direct_precode_ms": pre_b2b * 1e3,
                   "what": "mimo_detect_cg_gram / mimo_precode_cg_gram back to back with G "
                           "formed beforehand (the tuned schedules' cached-Gram forms); the "
                           "direct calls' back-to-back times beside them"}
    log(f"cached Gram: detect {tdg * 1e3:.3f} ms, precode {tpg * 1e3:.3f} ms")

    # the same step captured once as a hipGraph and replayed
    from paper_1404_0424_amd.graphs import StepGraph
    g = StepGraph(lambda: slot_call(H, Y))
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    wall_graph = (time.perf_counter() - t0) / args.steps
    log(f"hipGraph replay: {wall_graph * 1e3:.3f} ms/step")
    launch = "eager"
    if wall_graph < wall:
        wall, launch = wall_graph, "hipGraph replay"

    # baseline: the plain FP32 per-system mapping (VALU Gram/CG, one rhs at a time)
    plain = None
    if not args.no_variants and not wl.scalar_f64:
        v_saved = autotune.get_schedule("detect", wl.U, 0)
        autotune.set_schedule("detect", wl.U, 0, autotune.variants("detect").index("plain"), 0)
        plain_s = kernel_time(lambda: api.detect_cg(H, Y, n0, es, K, m, "approx", scalar,
                                                    out={"llr": llr}), reps=3)
        autotune.set_schedule("detect", wl.U, 0, *v_saved)
        plain = {"uplink_solves_per_s": n * wl.S / plain_s, "detect_kernel_ms": plain_s * 1e3,
                 "what": "plain FP32 per-system detection: VALU Gram/matched filter/CG, "
                         "one right-hand side at a time, complex64 storage"}
        log(f"plain FP32 per-system detection: {plain_s * 1e3:.3f} ms")
    # a solve is one (subcarrier, OFDM symbol) system; a step solves each of
    # the batch's n x S systems twice, once by uplink detection and once by
    # downlink precoding, and `value` counts both (uplink.solves_per_s is the
    # detection-only rate over the separate detection kernel's time)
    solves = 2 * n * wl.S
    llr_bits = n * wl.S * wl.U * wl.m
    det_bytes = detect_bytes_per_sc(wl.B, wl.U, wl.S, wl.m) * n
    pre_bytes = precode_bytes_per_sc(wl.B, wl.U, wl.S) * n
    slot_v, slot_bpc = autotune.get_schedule("slot", wl.U, 0)
    fused = (autotune.variants("slot")[slot_v] in ("fused", "fused-x3")
             and slot_fused_covers(wl.B, wl.U, wl.S))
    det_v, det_bpc = autotune.get_schedule("detect", wl.U, 0)
    if fused:
        # dominant (only) kernel of the step: the fused slot kernel
        dom_kernel, dom_bps = SLOT_KERNEL, slot_bytes_per_sc(wl.B, wl.U, wl.S, wl.m)
        dom_s, dom_bpc, dom_src = slot_s, slot_bpc, SLOT_SOURCES
        dom_mfma = mfma_count(wl.B, wl.U, wl.S, wl.K, "slot")
    else:
        dom_kernel = DETECT_KERNEL[autotune.variants("detect")[det_v]]
        dom_bps = detect_bytes_per_sc(wl.B, wl.U, wl.S, wl.m)
        dom_s, dom_bpc, dom_src = det_s, det_bpc, DETECT_SOURCES
        dom_mfma = mfma_count(wl.B, wl.U, wl.S, wl.K, "detect")
    dom_bytes = dom_bps * n
    achieved = dom_bytes / dom_s / 1e9
    traffic = recorded_traffic(dom_kernel, wl.name, n, persistent=dom_bpc > 0, sources=dom_src)
    # reference: a plain device copy moving the same number of bytes (half
    # read, half written), timed the same way
    src = torch.empty(dom_bytes // 8, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    copy_s = kernel_time(lambda: dst.copy_(src), reps=10)
    copy_gbs = 2 * src.numel() * 4 / copy_s / 1e9
    del src, dst
    log(f"device copy of the same byte count: {copy_gbs:.0f} GB/s; {dom_kernel} "
        f"{achieved:.0f} GB/s")

    result = {
        "metric": METRIC,
        "value": solves / wall,
        "unit": "subcarrier-solves/s (uplink detections + downlink precodings)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if scalar == "f32" else "f32 (f64 CG scalars)",
        "data": "synthetic",
        "config": {"workload": wl.name, "B": wl.B, "U": wl.U, "subcarriers_per_frame": wl.n_sc,
                   "S": wl.S, "qam_bits": wl.m, "K": wl.K, "snr_db": snr, "channel": wl.channel,
                   "frames_per_step": F,
                   "step": "uplink detection + downlink precoding on the same (reciprocal) "
                           "channels, one mimo_detect_precode_cg call",
                   "storage": "complex64"},
        "llr_gbit_s": llr_bits / wall / 1e9,
        "schedules": tuned,
        "launch": launch,
        "eager_ms_per_step": wall_eager * 1e3,
        "graph_ms_per_step": wall_graph * 1e3,
        "slot_kernel_ms": slot_s * 1e3,
        "slot_kernel_ms_back_to_back": slot_b2b * 1e3,
        "separate_launches": {"ms_per_step": wall_sep * 1e3,
                              "solves_per_s": solves / wall_sep,
                              "what": "the same step as mimo_detect_cg then mimo_precode_cg "
                                      "(H read and the Gram formed once per direction)"},
        "plain_fp32_per_system": plain,
        "bf16_split_gram": split_x3,
        "cached_gram": cached_gram,
        "uplink": {"solves_per_s": n * wl.S / det_s, "llr_gbit_s": llr_bits / det_s / 1e9,
                   "kernel_ms": det_s * 1e3, "hbm_gbs": det_bytes / det_s / 1e9,
                   "hbm_frac": det_bytes / det_s / 1e9 / HBM_PEAK_GBS,
                   "kernel_ms_back_to_back": det_b2b * 1e3},
        "downlink": {"solves_per_s": n * wl.S / pre_s, "kernel_ms": pre_s * 1e3,
                     "hbm_gbs": pre_bytes / pre_s / 1e9,
                     "kernel_ms_back_to_back": pre_b2b * 1e3},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "traffic_source": traffic["file"] if traffic else None,
                     "kernel": dom_kernel,
                     "copy_reference_gbs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs,
                     "bytes_per_subcarrier": dom_bps,
                     "subcarriers_per_launch": n,
                     "mfma_issued_tflops": dom_mfma * n * MFMA_FLOPS / dom_s / 1e12,
                     "mfma_frac": dom_mfma * n * MFMA_FLOPS / dom_s / MFMA_PEAK_FP32},
    }

    samples = []          # GPU results checked against the oracle in the baseline leg
    if not args.no_variants:
        variants = {}
        for dt in ("f16", "bf16"):
            H16, Y16 = api.convert(H, dt), api.convert(Y, dt)
            torch.cuda.synchronize()
            if not args.no_tune:
                autotune.tune("detect", wl.U, H16.dtype_code, lambda: api.detect_cg(
                    H16, Y16, n0, es, K, m, "approx", scalar, out={"llr": llr}))
                autotune.tune("precode", wl.U, H16.dtype_code, lambda: api.precode_cg(
                    H16, T, beta, K, normalize=True, scalar_prec=scalar, qnorm=False, out=Q))
                autotune.tune("slot", wl.U, H16.dtype_code, lambda: slot_call(H16, Y16),
                              exclude=autotune.X3_VARIANTS)
            w2, d2, p2 = timed(H16, Y16, dt, separate=True)
            w3, s3 = timed(H16, Y16, f"{dt} slot")
            o = api.detect_cg(H16, Y16, n0, es, K, m, "approx", scalar, xhat=True,
                              out={"llr": llr})
            api.precode_cg(H16, T, beta, K, normalize=True, scalar_prec=scalar, qnorm=False,
                           out=Q)
            idx = sample_index(n, 24, 2)
            samples += [detect_sample(f"{wl.name}/{dt}/detect", idx, up.H, up.Y, n0, es, K, m,
                                      o, dt),
                        precode_sample(f"{wl.name}/{dt}/precode", idx, up.H, dn.T, beta, K, Q,
                                       dt)]
            del o
            b16 = detect_bytes_per_sc(wl.B, wl.U, wl.S, wl.m, elem_bytes=4) * n
            variants[dt] = {"solves_per_s": solves / w2, "ms_per_step": w2 * 1e3,
                            "uplink_solves_per_s": n * wl.S / d2,
                            "llr_gbit_s": llr_bits / w2 / 1e9,
                            "detect_kernel_ms": d2 * 1e3, "detect_hbm_gbs": b16 / d2 / 1e9,
                            "precode_kernel_ms": p2 * 1e3,
                            "slot_ms_per_step": w3 * 1e3, "slot_solves_per_s": solves / w3,
                            "slot_kernel_ms": s3 * 1e3,
                            "storage": f"{dt} H and Y, FP32 accumulate and CG"}
            del H16, Y16
        # exact in-loop SINR (parity mode, Sec. III-C-1): one U x U x U complex
        # product per iteration and right-hand side plus B = L_K G, on MFMA for
        # U <= 16 (FP32 matrix peak) and VALU for two user tiles (vector peak)
        ex_s = kernel_time(lambda: api.detect_cg(H, Y, n0, es, K, m, "exact", scalar), reps=3)
        ex_flops = 8.0 * wl.U ** 3 * (K + 1) * wl.S * n
        ex_peak = MFMA_PEAK_FP32 / 1e12 if wl.U <= 16 else FP32_VECTOR_TFLOPS
        variants["exact_sinr"] = {
            "subcarriers": n, "detect_kernel_ms": ex_s * 1e3,
            "uplink_solves_per_s": n * wl.S / ex_s,
            "roofline": {"bound": "mfma" if wl.U <= 16 else "alu",
                         "achieved": ex_flops / ex_s / 1e12, "peak": ex_peak, "unit": "TFLOP/s",
                         "frac": ex_flops / ex_s / 1e12 / ex_peak},
            "what": "exact SINR tracker: E = A P each iteration, then B = L_K G (and the "
                    "diagonal of B L_K^H), 8 U^3 flops per product and right-hand side"}
        log(f"exact-SINR detection ({n} subcarriers): {ex_s * 1e3:.3f} ms, "
            f"{ex_flops / ex_s / 1e12:.1f} TFLOP/s of the tracker's products")
        result["variants"] = variants

    if not args.no_latency:
        # one frame (wl.n_sc subcarriers) on an idle GPU: UL detect + DL precode
        H1, Y1, T1 = H[:wl.n_sc], Y[:wl.n_sc], T[:wl.n_sc]
        l1 = torch.empty((wl.n_sc, wl.U, wl.S, wl.m), dtype=torch.float32, device=dev)
        Q1 = torch.empty((wl.n_sc, wl.B, wl.S), dtype=torch.complex64, device=dev)
        lat = []
        for i in range(60):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            api.detect_precode_cg(H1, Y1, T1, n0, es, beta, K, K, m, True, scalar, qnorm=False,
                                  out={"llr": l1, "Q": Q1})
            e1.record()
            torch.cuda.synchronize()
            if i >= 10:
                lat.append(e0.elapsed_time(e1))
        result["frame_latency_ms"] = {"p50": float(np.percentile(lat, 50)),
                                      "p99": float(np.percentile(lat, 99)),
                                      "what": "one frame, UL detect + DL precode, idle GPU"}

    if not args.no_configs:
        result["configs"] = configs_leg(api, autotune, kernel_time, dev, samples)
    if not args.no_wide:
        result["users_over_32"] = wide_leg(api, kernel_time, dev, samples)

    if not args.no_comparison:
        result["comparison"] = comparison_leg(api, autotune, H, Y, T, llr, Q, up, dn, wl, n,
                                              kernel_time)

    if not args.no_serving:
        result["serving"] = serving_leg(args.serving_frames, args.serving_skip)
        nat = serving_leg(args.serving_frames, args.serving_skip, native=True)
        nat["saturation_vs_batched_step"] = nat["saturation"]["solves_per_s"] / result["value"]
        result["serving"]["native"] = nat

    if args.copy_calibration:
        nbytes = 512 << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = nbytes
        del src, dst

    if not args.no_cpu_baseline:
        # the complex64 outputs (the variants above reused the buffers)
        o = api.detect_cg(H, Y, n0, es, K, m, "approx", scalar, xhat=True, out={"llr": llr})
        api.precode_cg(H, T, beta, K, normalize=True, scalar_prec=scalar, qnorm=False, out=Q)
        torch.cuda.synchronize()
        idx = sample_index(n, 24, 1)
        samples[:0] = [detect_sample(f"{wl.name}/c32/detect", idx, up.H, up.Y, n0, es, K, m, o),
                       precode_sample(f"{wl.name}/c32/precode", idx, up.H, dn.T, beta, K, Q)]
        del o
        result["cpu_baseline"] = cpu_baseline(up, dn, wl, llr, Q, args.cpu_seconds, samples)

    print(json.dumps(result), flush=True)


MFMA_PEAK_FP32 = 157.3e12        # MI355X dense FP32 MFMA, FLOP/s
MFMA_FLOPS = 2 * 16 * 16 * 4     # one v_mfma_f32_16x16x4_f32


def sample_index(n, k, seed):
    """k sorted subcarrier indices of a batch of n, the last one included."""
    idx = np.sort(np.random.default_rng(seed).choice(n, min(k, n), replace=False))
    idx[-1] = n - 1
    return idx


def detect_sample(label, idx, H, Y, n0, es, K, m, out, storage="c32"):
    """Sampled detection outputs copied to the host, with the FP64 inputs
    they came from, for the oracle check in the CPU-baseline leg."""
    import torch
    it = torch.from_numpy(idx).to(out["llr"].device)
    return {"label": label, "op": "detect", "storage": storage, "H": H[idx], "Y": Y[idx],
            "n0": n0, "es": es, "K": K, "m": m,
            "xhat": out["xhat"][it].cpu().numpy(), "llr": out["llr"][it].cpu().numpy()}


def precode_sample(label, idx, H, T, beta, K, Q, storage="c32"):
    """Sampled (normalized) precoder outputs, as detect_sample."""
    import torch
    it = torch.from_numpy(idx).to(Q.device)
    return {"label": label, "op": "precode", "storage": storage, "H": H[idx], "T": T[idx],
            "beta": beta, "K": K, "Q": Q[it].cpu().numpy()}


def rel_err_vec(x, ref, axis):
    """max over vectors of the relative 2-norm error along ``axis``."""
    num = np.linalg.norm(np.asarray(x, dtype=np.complex128) - ref, axis=axis)
    den = np.linalg.norm(ref, axis=axis)
    return float(np.max(np.where(den > 0, num / np.where(den > 0, den, 1.0), num)))


def llr_err(L, ref):
    """max over symbols of max_b |L - L_ref| / max(1, max_b |L_ref|)."""
    d = np.max(np.abs(np.asarray(L, dtype=np.float64) - ref), axis=-1)
    return float(np.max(d / np.maximum(1.0, np.max(np.abs(ref), axis=-1))))


def oracle_errors(samples, O):
    """Error of each sampled GPU result against the FP64 oracle on the same
    inputs; for 16-bit storage also against the oracle on the RNE-rounded
    inputs the GPU actually read."""
    out = {}
    for smp in samples:
        st = smp["storage"]
        rnd = None
        if st != "c32":
            qz, deq = ((O.quantize_f16, O.dequantize_f16) if st == "f16"
                       else (O.quantize_bf16, O.dequantize_bf16))
            rnd = lambda x: deq(qz(x))                       # noqa: E731
        if smp["op"] == "detect":
            args = (smp["n0"], smp["es"], smp["K"], smp["m"], "approx")
            r = O.detect_cg(smp["H"], smp["Y"], *args)
            rec = {"eps_x": rel_err_vec(smp["xhat"], r["xhat"], axis=1),
                   "eps_llr": llr_err(smp["llr"], r["llr"])}
            if rnd is not None:
                r = O.detect_cg(rnd(smp["H"]), rnd(smp["Y"]), *args)
                rec["eps_x_vs_rounded_inputs"] = rel_err_vec(smp["xhat"], r["xhat"], axis=1)
                rec["eps_llr_vs_rounded_inputs"] = llr_err(smp["llr"], r["llr"])
        else:
            p = O.precode_cg(smp["H"], smp["T"], smp["beta"], smp["K"], normalize=True)
            rec = {"eps_q": rel_err_vec(smp["Q"], p["Q"], axis=1)}
            if rnd is not None:
                p = O.precode_cg(rnd(smp["H"]), smp["T"], smp["beta"], smp["K"], normalize=True)
                rec["eps_q_vs_rounded_inputs"] = rel_err_vec(smp["Q"], p["Q"], axis=1)
        rec["subcarriers"] = int(smp["H"].shape[0])
        out[smp["label"]] = rec
    return out


def gpu_warm(fns, seconds):
    """Keep the device busy with ``fns`` (round robin, synchronized every few
    calls so that the queue stays short) for ``seconds`` of wall time.  After
    an idle spell (inputs drawn on the host) launches run 10-20% slower for
    the first few tens of milliseconds of work, until the clocks are back up;
    untimed."""
    import torch
    t0 = time.perf_counter()
    i = 0
    while True:
        fns[i % len(fns)]()
        i += 1
        if i % 8 == 0:
            torch.cuda.synchronize()
            if time.perf_counter() - t0 >= seconds:
                break


def mfma_count(B, U, S, K, op):
    """v_mfma_f32_16x16x4_f32 instructions per subcarrier issued by the
    complex64 kernels: Gram tiles (3 per k-step on a diagonal tile, 4 off
    it), the three-product matched filter, 4 W per k-step of 4 users in a
    CG mat-vec and 3 per k-step in q = H v (k-steps past the last user are
    skipped); k-steps of 4 antennas for the Gram and matched filter.  The
    detectors and precoders run the packed form at U <= 8 (one product per
    k-step for the Gram, two for the matched filter); the standalone Gram
    kernel does not."""
    W = 1 if U <= 16 else 2
    ksteps = -(-B // 4)
    chunks = -(-S // 16)
    nk = min(4 * W, -(-U // 4))
    if op == "gram_mf":
        return ksteps * (3 * W + 4 * (W * (W - 1) // 2)) + chunks * ksteps * 3 * W
    packed = U <= 8
    gram = ksteps * (1 if packed else 3 * W + 4 * (W * (W - 1) // 2))
    mf = ksteps * (2 if packed else 3 * W)
    matvec = 4 * W * nk
    if op == "detect":
        return gram + chunks * (mf + K * matvec)
    if op == "slot":
        # one Gram; uplink matched filter and K mat-vecs; downlink K + 1
        # mat-vecs and q = H v
        return gram + chunks * (mf + K * matvec + (K + 1) * matvec + (-(-B // 16)) * 3 * nk)
    # precode: Gram, K mat-vecs + one for ||q||^2, q = H v per 16-antenna tile
    return gram + chunks * ((K + 1) * matvec + (-(-B // 16)) * 3 * nk)


def mfma_count_wide(B, U, S, K, op):
    """v_mfma_f32_16x16x4_f32 instructions per subcarrier of the four-wavefront
    kernels (32 < U <= 64): Gram tiles in three products (roles 0 and 1 three
    tiles, roles 2 and 3 two; a role without users skips its tiles and
    matched filter), the three-product matched filter of each role, the
    CG mat-vec of every role (4 per k-step of 4 users) and, for precoding,
    ||q||^2 and q = H v (3 per k-step per 16-antenna tile)."""
    ksteps = -(-B // 4)
    chunks = -(-S // 16)
    nk = -(-U // 4)
    roles = [r for r in range(4) if 16 * r < U]
    gram = ksteps * sum(9 if r < 2 else 6 for r in roles)
    mf = ksteps * 3 * len(roles)
    matvec = 4 * 4 * nk
    if op == "detect":
        return gram + chunks * (mf + K * matvec)
    return gram + chunks * ((K + 1) * matvec + (-(-B // 16)) * 3 * nk)


def wide_leg(api, kernel_time, dev, samples):
    """Detection and precoding with more than 32 users (the four-wavefront
    kernels) on 4,800 subcarriers x 14 symbols of 128x48 and 128x64 (64-QAM,
    15 dB, K = 4, i.i.d. channel): time, HBM rate, issued-MFMA rate, and
    sampled subcarriers against the oracle."""
    import torch
    from paper_1404_0424_amd import workload as W
    out = {}
    n, B, S, K, m, snr = 4800, 128, 14, 4, 6, 15.0
    for U in (48, 64):
        rng = W.rng_for(9, U)
        up = W.uplink_frame(rng, n, B, U, S, m, snr)
        dn = W.downlink_frame(rng, n, B, U, S, m, snr, H=up.H)
        H = torch.from_numpy(up.H.astype(np.complex64)).to(dev)
        Y = torch.from_numpy(up.Y.astype(np.complex64)).to(dev)
        T = torch.from_numpy(dn.T.astype(np.complex64)).to(dev)
        llr = torch.empty((n, U, S, m), dtype=torch.float32, device=dev)
        Q = torch.empty((n, B, S), dtype=torch.complex64, device=dev)
        fd = lambda: api.detect_cg(H, Y, up.n0, up.es, K, m, "approx", "f32", out={"llr": llr})
        fp = lambda: api.precode_cg(H, T, dn.beta, K, True, "f32", qnorm=False, out=Q)
        td, tp = kernel_time(fd, reps=10), kernel_time(fp, reps=10)
        o = api.detect_cg(H, Y, up.n0, up.es, K, m, "approx", "f32", xhat=True,
                          out={"llr": llr})
        idx = sample_index(n, 12, 5)
        samples += [detect_sample(f"wide_128x{U}/detect", idx, up.H, up.Y, up.n0, up.es, K, m, o),
                    precode_sample(f"wide_128x{U}/precode", idx, up.H, dn.T, dn.beta, K, Q)]
        del o
        db = detect_bytes_per_sc(B, U, S, m) * n
        pb = precode_bytes_per_sc(B, U, S) * n
        fd_fl = mfma_count_wide(B, U, S, K, "detect") * n * MFMA_FLOPS
        fp_fl = mfma_count_wide(B, U, S, K, "precode") * n * MFMA_FLOPS
        out[f"128x{U}"] = {
            "subcarriers": n, "S": S, "K": K, "qam_bits": m,
            "detect_ms": td * 1e3, "precode_ms": tp * 1e3,
            "uplink_solves_per_s": n * S / td, "downlink_solves_per_s": n * S / tp,
            "detect_hbm_gbs": db / td / 1e9, "precode_hbm_gbs": pb / tp / 1e9,
            "detect_mfma_frac": fd_fl / td / MFMA_PEAK_FP32,
            "precode_mfma_frac": fp_fl / tp / MFMA_PEAK_FP32}
        log(f"U = {U} (128x{U}, {n} subcarriers): detect {td * 1e3:.3f} ms "
            f"({fd_fl / td / MFMA_PEAK_FP32:.2f} of FP32 MFMA peak issued), precode "
            f"{tp * 1e3:.3f} ms ({fp_fl / tp / MFMA_PEAK_FP32:.2f})")
        del H, Y, T, llr, Q
        torch.cuda.empty_cache()
    return out


def configs_leg(api, autotune, kernel_time, dev, samples):
    """Each workload configuration on its own batch (autotuned schedule,
    back-to-back launches): detection and precoding rates, the detection
    kernel's HBM rate and issued-MFMA rate, and the standalone Gram +
    matched-filter kernel's MFMA utilisation (the Gram stage) at U = 32."""
    import torch
    from paper_1404_0424_amd import workload as W
    plan = [("small_32x8", 1024, (10.0,)),
            ("plain_128x8", 16, tuple(float(x) for x in range(0, 21, 2))),
            ("mixed_128x32", 8, (15.0,)), ("corr_256x32", 1, (25.0,))]
    out = {}
    for name, F, snrs in plan:
        wl = W.WORKLOADS[name]
        n = wl.n_sc * F
        scalar = "f64" if wl.scalar_f64 else "f32"
        rows = {}
        for snr in snrs:
            rng = W.rng_for(CFG_INDEX[name], 1)
            up = W.uplink_frame(rng, n, wl.B, wl.U, wl.S, wl.m, snr, channel=wl.channel,
                                rho_bs=wl.rho_bs, rho_ue=wl.rho_ue)
            dn = W.downlink_frame(rng, n, wl.B, wl.U, wl.S, wl.m, snr, H=up.H)
            H = torch.from_numpy(up.H.astype(np.complex64)).to(dev)
            Y = torch.from_numpy(up.Y.astype(np.complex64)).to(dev)
            T = torch.from_numpy(dn.T.astype(np.complex64)).to(dev)
            llr = torch.empty((n, wl.U, wl.S, wl.m), dtype=torch.float32, device=dev)
            Q = torch.empty((n, wl.B, wl.S), dtype=torch.complex64, device=dev)
            fd = lambda: api.detect_cg(H, Y, up.n0, up.es, wl.K, wl.m, "approx", scalar,
                                       out={"llr": llr})
            fp = lambda: api.precode_cg(H, T, dn.beta, wl.K, True, scalar, qnorm=False, out=Q)
            fs = lambda: api.detect_precode_cg(H, Y, T, up.n0, up.es, dn.beta, wl.K, wl.K,
                                               wl.m, True, scalar, qnorm=False,
                                               out={"llr": llr, "Q": Q})
            if snr == snrs[0]:
                x3 = autotune.X3_VARIANTS
                autotune.tune("detect", wl.U, 0, fd, exclude=x3)
                autotune.tune("precode", wl.U, 0, fp, exclude=x3)
                autotune.tune("slot", wl.U, 0, fs, exclude=x3)
            gpu_warm([fd, fp, fs], 0.15)   # the device idled while the inputs were drawn
            td, tp, ts = kernel_time(fd, reps=10), kernel_time(fp, reps=10), kernel_time(fs, reps=10)
            sv, sb = autotune.get_schedule("slot", wl.U, 0)
            dsaved, psaved = autotune.get_schedule("detect", wl.U, 0), autotune.get_schedule(
                "precode", wl.U, 0)
            autotune.set_schedule("detect", wl.U, 0, autotune.variants("detect").index("stream-x3"),
                                  dsaved[1])
            autotune.set_schedule("precode", wl.U, 0, autotune.variants("precode").index("x3"),
                                  psaved[1])
            tdx, tpx = kernel_time(fd, reps=10), kernel_time(fp, reps=10)
            autotune.set_schedule("detect", wl.U, 0, *dsaved)
            autotune.set_schedule("precode", wl.U, 0, *psaved)
            o = api.detect_cg(H, Y, up.n0, up.es, wl.K, wl.m, "approx", scalar, xhat=True,
                              out={"llr": llr})
            idx = sample_index(n, 24, 3)
            samples += [detect_sample(f"{name}/{snr:g}dB/detect", idx, up.H, up.Y, up.n0, up.es,
                                      wl.K, wl.m, o),
                        precode_sample(f"{name}/{snr:g}dB/precode", idx, up.H, dn.T, dn.beta,
                                       wl.K, Q)]
            del o
            det_b = detect_bytes_per_sc(wl.B, wl.U, wl.S, wl.m) * n
            mf = mfma_count(wl.B, wl.U, wl.S, wl.K, "detect") * n * MFMA_FLOPS
            rows[f"{snr:g}dB"] = {
                "detect_ms": td * 1e3, "precode_ms": tp * 1e3,
                "uplink_solves_per_s": n * wl.S / td, "downlink_solves_per_s": n * wl.S / tp,
                "llr_gbit_s": n * wl.S * wl.U * wl.m / td / 1e9,
                "detect_hbm_gbs": det_b / td / 1e9, "detect_frac": det_b / td / 1e9 / HBM_PEAK_GBS,
                "detect_mfma_tflops": mf / td / 1e12,
                "detect_mfma_frac": mf / td / MFMA_PEAK_FP32,
                "slot_ms": ts * 1e3, "slot_solves_per_s": 2 * n * wl.S / ts,
                "bf16_split_gram": {"detect_ms": tdx * 1e3, "precode_ms": tpx * 1e3},
                "slot_schedule": {"variant": autotune.variants("slot")[sv], "blocks_per_cu": sb,
                                  "fused_kernel": slot_fused_covers(wl.B, wl.U, wl.S)}}
            if name in ("mixed_128x32", "corr_256x32") and snr == snrs[0]:
                fg = lambda: api.gram_mf(H, Y, up.n0 / up.es)
                eg = autotune.tune("gram_mf", wl.U, 0, fg)
                tg = kernel_time(fg, reps=10)
                gf = mfma_count(wl.B, wl.U, wl.S, wl.K, "gram_mf") * n * MFMA_FLOPS
                gb = (8 * wl.B * wl.U + 8 * wl.B * wl.S + 8 * wl.U * wl.U + 8 * wl.U * wl.S) * n
                rows[f"{snr:g}dB"]["gram_stage"] = {
                    "kernel_ms": tg * 1e3, "mfma_tflops": gf / tg / 1e12,
                    "mfma_frac": gf / tg / MFMA_PEAK_FP32, "hbm_gbs": gb / tg / 1e9,
                    "schedule": {"variant": autotune.variants("gram_mf")[eg["best"]["variant"]],
                                 "blocks_per_cu": eg["best"]["blocks_per_cu"]},
                    "what": "standalone mimo_gram_mf (A = H^H H + reg I and b = H^H Y)"}
            log(f"config {name} ({F} frames) {snr:g} dB: detect {td * 1e3:.3f} ms "
                f"({det_b / td / 1e9:.0f} GB/s, MFMA {mf / td / 1e12:.1f} TF), "
                f"precode {tp * 1e3:.3f} ms, slot {ts * 1e3:.3f} ms"
                + (f"; Gram stage {rows[f'{snr:g}dB']['gram_stage']['mfma_frac']:.2f} of FP32 "
                   f"MFMA peak" if "gram_stage" in rows[f"{snr:g}dB"] else ""))
            del H, Y, T, llr, Q
        out[name] = {"frames": F, "subcarriers": n, "K": wl.K, "scalar_prec": scalar,
                     "by_snr": rows}
        torch.cuda.empty_cache()
    return out


def comparison_leg(api, autotune, H, Y, T, llr, Q, up, dn, wl, n, kernel_time):
    """The comparison methods on the same batch: average launch time (HIP
    events, back-to-back launches) and algorithmic HBM rate of CG-D for
    K = 1..16, the Cholesky detector, the Neumann series and CGLS, and the
    matching precoders.  Gives the K up to which CG-D is faster than the
    exact Cholesky detector on this GPU, beside the crossover of the
    real-multiplication count (Sec. IV-A)."""
    from paper_1404_0424_amd import complexity
    n0, es, beta, m = up.n0, up.es, dn.beta, wl.m
    det_b = detect_bytes_per_sc(wl.B, wl.U, wl.S, m) * n
    pre_b = precode_bytes_per_sc(wl.B, wl.U, wl.S) * n

    def rec(sec, nbytes):
        gbs = nbytes / sec / 1e9
        return {"ms": sec * 1e3, "hbm_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}

    det = {"cg": {}, "neumann": {}, "cgls": {}}
    for K in range(1, 17):
        det["cg"][K] = rec(kernel_time(lambda: api.detect_cg(
            H, Y, n0, es, K, m, "approx", out={"llr": llr}), reps=5), det_b)
    det["cholesky"] = rec(kernel_time(lambda: api.detect_cholesky(
        H, Y, n0, es, m, out={"llr": llr}), reps=5), det_b)
    for K in (1, 2, 3):
        det["neumann"][K] = rec(kernel_time(lambda: api.detect_neumann(
            H, Y, n0, es, K, m, out={"llr": llr}), reps=5), det_b)
    for K in (1, 2, 3, 4):
        det["cgls"][K] = rec(kernel_time(lambda: api.detect_cgls(
            H, Y, n0, es, K, m, out={"llr": llr}), reps=5), det_b)
    ch = det["cholesky"]["ms"]
    gpu_x = max([K for K, r in det["cg"].items() if r["ms"] <= ch], default=0)
    # CG stage: least-squares slope of the launch time over K = 1..16 (the
    # Gram, matched filter and LLR work does not depend on K)
    ks = np.array(sorted(det["cg"]))
    ts = np.array([det["cg"][K]["ms"] for K in ks]) * 1e-3
    slope = float(np.polyfit(ks, ts, 1)[0])
    # one CG iteration's MFMA work per subcarrier: the mat-vec E = A P of all
    # right-hand sides (4 W products per k-step of 4 users); its floor is that
    # work at the FP32 MFMA peak.  The CG moves no HBM bytes (A, P and the
    # vectors stay in LDS and registers), so it has no HBM roofline: what it
    # costs is the launch time it adds per iteration.
    W_ = 1 if wl.U <= 16 else 2
    it_flops = 4 * W_ * min(4 * W_, -(-wl.U // 4)) * MFMA_FLOPS * -(-wl.S // 16) * n
    floor_s = it_flops / MFMA_PEAK_FP32
    at_k = det["cg"][wl.K]["ms"] * 1e-3
    cg_stage = {"ms_per_iteration": slope * 1e3,
                "mfma_floor_ms_per_iteration": floor_s * 1e3,
                "slope_over_floor": slope / floor_s,
                "stage_ms_at_K": slope * wl.K * 1e3,
                "stage_share_of_launch_at_K": slope * wl.K / at_k,
                "what": "least-squares slope of the detection launch time over K = 1..16 "
                        "(the Gram, matched-filter and LLR work does not depend on K); the "
                        "floor is one iteration's mat-vec MFMAs at the FP32 MFMA peak; the "
                        "CG stage reads and writes no HBM"}
    pre = {
        "cg_K%d" % wl.K: rec(kernel_time(lambda: api.precode_cg(
            H, T, beta, wl.K, True, qnorm=False, out=Q), reps=5), pre_b),
        "cholesky": rec(kernel_time(lambda: api.precode_cholesky(
            H, T, beta, True, qnorm=False, out=Q), reps=5), pre_b),
        "neumann_K3": rec(kernel_time(lambda: api.precode_neumann(
            H, T, beta, 3, True, qnorm=False, out=Q), reps=5), pre_b),
        "cgls_K%d" % wl.K: rec(kernel_time(lambda: api.precode_cgls(
            H, T, beta, wl.K, True, qnorm=False, out=Q), reps=5), pre_b),
    }
    log("comparison detect ms: cg " + " ".join(f"K{K}={r['ms']:.3f}" for K, r in det["cg"].items())
        + f"; cholesky {ch:.3f}; neumann "
        + " ".join(f"K{K}={r['ms']:.3f}" for K, r in det["neumann"].items()) + "; cgls "
        + " ".join(f"K{K}={r['ms']:.3f}" for K, r in det["cgls"].items()))
    log("comparison precode ms: " + " ".join(f"{k}={r['ms']:.3f}" for k, r in pre.items()))
    log(f"CG-D faster than Cholesky up to K={gpu_x} on this GPU; "
        f"real-multiplication crossover K={complexity.crossover(wl.B, wl.U)}")
    return {"workload": wl.name, "subcarriers_per_launch": n, "detect": det, "precode": pre,
            "cg_faster_than_cholesky_up_to_K": gpu_x, "cg_stage": cg_stage,
            "multiplication_count_crossover_K": complexity.crossover(wl.B, wl.U),
            "what": "average launch time of back-to-back launches; hbm_gbs = algorithmic "
                    "bytes (H, Y in, LLR out / H, T in, Q out) per launch time"}


def serving_leg(n_frames, skip, native=False):
    """Mixed-shape uplink/downlink frames through the continuous-batching
    server: saturation throughput (all frames queued, then released at once), then Poisson
    arrivals at 50%, 80% and 95% of it, and 80% under a small HBM budget that
    makes requests wait for memory; p50/p99 arrival-to-completion latency
    over all but the first ``skip`` frames of each run.  ``native``: the C++
    scheduler of include/mimo_serve.h (NativeServer) instead of the Python
    one (Server)."""
    import torch

    from paper_1404_0424_amd import native_serving as NS
    from paper_1404_0424_amd import serving as SV
    from paper_1404_0424_amd import workload as W

    tag = "native " if native else ""

    rng = W.rng_for(4, 0)
    chans, _ = W.serving_stream(rng, 16, 0, 0.0)
    ex = SV.GpuExecutor(n_slots=4, input_events=False)    # inputs synchronized below
    dev = torch.device("cuda")
    data = {}
    for ch in chans:
        Y = (ch.H @ W.qam_map(W.random_bits(rng, (ch.n_sc, ch.U, 14), 6), 6)
             + W.awgn(rng, (ch.n_sc, ch.B, 14), W.n0_from_snr_db(15.0, ch.U, ch.B)))
        T = W.qam_map(W.random_bits(rng, (ch.n_sc, ch.U, 14), 6), 6)
        data[ch.ch_id] = (torch.from_numpy(Y.astype(np.complex64)).to(dev),
                          torch.from_numpy(T.astype(np.complex64)).to(dev))
    torch.cuda.synchronize()
    by_id = {c.ch_id: c for c in chans}

    def request(f):
        c = by_id[f.ch_id]
        n0 = W.n0_from_snr_db(f.snr_db, c.U, c.B)
        if f.uplink:
            return SV.UplinkRequest(f.ch_id, data[f.ch_id][0], n0, 1.0, f.m, 3)
        return SV.DownlinkRequest(f.ch_id, data[f.ch_id][1], n0, 3, True)

    def run(rate, frames_n, dtype="c32", budget=16 << 30, gram=False):
        frames = W.serving_frames(W.rng_for(4, 1 + int(rate)), 16, frames_n, rate)
        # the native server's consumer reads no outputs (they return to the
        # pool at completion) and submits pre-marshalled requests without
        # futures; statistics come from the server's completion records
        srv = (NS.NativeServer(hbm_budget=budget, n_slots=4, input_events=False,
                               keep_outputs=False) if native
               else SV.Server(ex, hbm_budget=budget, n_slots=4))
        for c in chans:
            if gram:
                srv.register_channel(c.ch_id, c.H, dtype, gram=True)
            else:
                srv.register_channel(c.ch_id, c.H, dtype)
        reqs = [srv.prepare(request(f)) if native else request(f) for f in frames]
        submit = (lambda r: srv.submit(r, future=False)) if native else srv.submit
        # warm up every shape class once
        for f in {(by_id[f.ch_id].B, by_id[f.ch_id].U, f.uplink, f.m): f for f in frames}.values():
            srv.submit(request(f)).result(timeout=60)
        srv.drain(timeout=60)
        if rate <= 0:
            srv.pause()          # saturation: queue every frame, then release them at once
        srv.stats(reset=True)
        t0 = time.perf_counter()
        for f, r in zip(frames, reqs):
            target = t0 + f.t_arrival
            while True:                      # wait for the arrival time, yielding the GIL
                d = target - time.perf_counter()
                if d <= 0:
                    break
                time.sleep(d - 1e-4 if d > 2e-4 else 0)
            submit(r)
        srv.resume()
        srv.drain(timeout=120)
        st = srv.stats(skip=min(skip, len(frames) // 2))
        if not native:
            st["mean_batch"] = (float(np.mean(srv.batch_sizes[-len(frames):]))
                                if srv.batch_sizes else 0)
        st["budget_bytes"] = budget
        st["budget_waits"] = srv.budget_waits
        srv.close()
        return st

    def device_rate(frames_n):
        """Solves/s of the same stream's frames in ideal batches: grouped by
        kernel class, 32 frames per batched launch, back to back on one
        stream, no scheduler (the device rate a server can approach)."""
        frames = W.serving_frames(W.rng_for(4, 1), 16, frames_n, 0.0)
        groups = {}
        for f in frames:
            c = by_id[f.ch_id]
            groups.setdefault((f.uplink, c.U <= 16, f.m if f.uplink else 0), []).append(f)
        Hd = {c.ch_id: torch.from_numpy(c.H.astype(np.complex64)).to(dev) for c in chans}
        launches = []
        for (up, _, m), fs in groups.items():
            for i in range(0, len(fs), 32):
                chunk = fs[i:i + 32]
                if up:
                    fr = [(Hd[f.ch_id], data[f.ch_id][0],
                           W.n0_from_snr_db(f.snr_db, by_id[f.ch_id].U, by_id[f.ch_id].B), 1.0)
                          for f in chunk]
                    launches.append(lambda fr=fr, m=m: api.detect_cg_batch(fr, 3, m))
                else:
                    fr = [(Hd[f.ch_id], data[f.ch_id][1],
                           W.n0_from_snr_db(f.snr_db, by_id[f.ch_id].U, by_id[f.ch_id].B), True)
                          for f in chunk]
                    launches.append(lambda fr=fr: api.precode_cg_batch(fr, 3))
        solves = sum(by_id[f.ch_id].n_sc * 14 for f in frames)
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for fn in launches:
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        return {"solves_per_s": solves / (best * 1e-3), "frames_per_s": frames_n / (best * 1e-3),
                "launches": len(launches), "ms": best}

    from paper_1404_0424_amd import api
    ideal = device_rate(n_frames)
    log(f"serving stream in ideal batches (no scheduler): {ideal['frames_per_s']:.0f} frames/s, "
        f"{ideal['solves_per_s']:.3g} solves/s")

    old_switch = sys.getswitchinterval()
    sys.setswitchinterval(2e-5)              # submitter and scheduler threads share the GIL

    sat = run(0.0, n_frames)
    sat["vs_ideal_batches"] = sat["solves_per_s"] / ideal["solves_per_s"]
    log(f"{tag}serving saturation: {sat['frames_per_s']:.0f} frames/s, "
        f"{sat['solves_per_s']:.3g} solves/s, p50 {sat['p50_ms']:.3f} ms, p99 {sat['p99_ms']:.3f} ms")
    out = {"workload": "Poisson uplink/downlink frames, B in {64,128,256}, U in {8,16,32}, "
                       "300-1200 subcarriers x 14 symbols, 16/64/256-QAM, 5-25 dB, K=3, "
                       "16 device-resident channels, 4 stream slots, 16 GiB budget",
           "scheduler": ("C++ scheduler thread (include/mimo_serve.h), device pool of the budget"
                         if native else "Python scheduler thread (serving.Server)"),
           "frames_per_run": n_frames, "frames_left_out": min(skip, n_frames // 2),
           "ideal_batches": ideal, "saturation": sat}
    for load in (0.5, 0.8, 0.95):
        st = run(load * sat["frames_per_s"], n_frames)
        log(f"{tag}serving load {load}: offered {load * sat['frames_per_s']:.0f}/s, achieved "
            f"{st['frames_per_s']:.0f}/s, p50 {st['p50_ms']:.3f} ms, p99 {st['p99_ms']:.3f} ms")
        out[f"load_{load}"] = st
    # small budget: the channel cache plus room for two of the largest
    # requests, so that admission waits for memory
    # (uplink: LLRs of 256-QAM; downlink: Q and the norms; complex64 channels)
    need = max(max(4 * c.n_sc * c.U * 14 * 8, 8 * c.n_sc * c.B * 14 + 4 * c.n_sc * 14)
               for c in chans)
    cache = sum(8 * c.n_sc * c.B * c.U for c in chans)
    small = cache + 2 * need + 4096          # + pool rounding of the native server
    st = run(0.8 * sat["frames_per_s"], n_frames, budget=small)
    log(f"{tag}serving load 0.8, budget {small / 2**20:.0f} MiB: achieved "
        f"{st['frames_per_s']:.0f}/s, p50 {st['p50_ms']:.3f} ms, p99 {st['p99_ms']:.3f} ms, "
        f"{st['budget_waits']} budget waits")
    out["load_0.8_small_budget"] = st
    # mixed precision: channels kept on the device in BF16 (Gram / matched
    # filter on 16-bit MFMA, FP32 accumulate and CG); uplink Y is rounded to
    # BF16 on the slot stream per frame
    sat16 = run(0.0, n_frames, "bf16")
    log(f"{tag}serving saturation, BF16 channel storage: {sat16['frames_per_s']:.0f} frames/s, "
        f"{sat16['solves_per_s']:.3g} solves/s")
    out["saturation_bf16"] = sat16
    if native:
        # each channel registered with its Gram matrix, formed once: the
        # frames of channels with U > 8 skip the Gram's products (outputs
        # bitwise unchanged)
        satg = run(0.0, n_frames, gram=True)
        satg["vs_ideal_batches"] = satg["solves_per_s"] / ideal["solves_per_s"]
        log(f"{tag}serving saturation, cached Gram per channel: {satg['frames_per_s']:.0f} "
            f"frames/s, {satg['solves_per_s']:.3g} solves/s, p50 {satg['p50_ms']:.3f} ms")
        out["saturation_cached_gram"] = satg
    sys.setswitchinterval(old_switch)
    return out


def _oracle_chunk(args):
    """One chunk of the CPU baseline in a worker process: the FP64 oracle's
    detection and precoding of a few subcarriers, one BLAS thread."""
    H, Y, T, n0, es, beta, K, m = args
    from threadpoolctl import threadpool_limits

    from oracle import mimo_oracle as O
    with threadpool_limits(1):
        O.detect_cg(H, Y, n0, es, K, m, "approx")
        O.precode_cg(H, T, beta, K, normalize=True)
    return H.shape[0]


def _worker_init(root):
    sys.path.insert(0, root)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def host_workers():
    """Worker processes for the all-cores oracle run: the CPUs this process
    may run on, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_all_cores(up, dn, wl, seconds, workers):
    """The oracle over random chunks of the same batch on `workers` processes
    (spawned children, one BLAS thread each), for about `seconds` of wall
    time after the pool has started.  Returns (subcarriers, seconds)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    root = os.path.dirname(os.path.abspath(__file__))
    chunk = 16
    rng = np.random.default_rng(1)

    def task():
        idx = np.sort(rng.choice(up.H.shape[0], chunk, replace=False))
        return (up.H[idx], up.Y[idx], dn.T[idx], up.n0, up.es, dn.beta, wl.K, wl.m)

    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"),
                                initializer=_worker_init, initargs=(root,)) as pool:
        list(pool.map(_oracle_chunk, [task() for _ in range(workers)]))    # start every worker
        done = 0
        t0 = time.perf_counter()
        pending = {pool.submit(_oracle_chunk, task()) for _ in range(2 * workers)}
        while pending:
            fin, pending = cf.wait(pending, return_when=cf.FIRST_COMPLETED)
            for f in fin:
                done += f.result()
                if time.perf_counter() - t0 < seconds:
                    pending.add(pool.submit(_oracle_chunk, task()))
        return done, time.perf_counter() - t0


def cpu_baseline(up, dn, wl, llr_gpu, Q_gpu, seconds, samples=()):
    """The FP64 oracle on the host on a bounded sample of the same workload:
    single-threaded, and on all the host cores this run may use (worker
    processes over subcarriers); also reports the GPU's error against it on
    that sample and on the sampled results of every other leg (storage
    types, configurations)."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from oracle import mimo_oracle as O
    from threadpoolctl import threadpool_limits
    chunk = 32
    rng = np.random.default_rng(0)
    done = 0
    el = eq = None
    with threadpool_limits(1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            idx = np.sort(rng.choice(up.H.shape[0], chunk, replace=False))
            r = O.detect_cg(up.H[idx], up.Y[idx], up.n0, up.es, wl.K, wl.m, "approx")
            p = O.precode_cg(up.H[idx], dn.T[idx], dn.beta, wl.K, normalize=True)
            done += chunk
            if el is None:
                llr_h = llr_gpu[idx].cpu().numpy().astype(np.float64)
                Q_h = Q_gpu[idx].cpu().numpy().astype(np.complex128)
                d = np.max(np.abs(llr_h - r["llr"]), axis=-1) / np.maximum(
                    1.0, np.max(np.abs(r["llr"]), axis=-1))
                el = float(d.max())
                eq = float(np.max(np.linalg.norm(Q_h - p["Q"], axis=1)
                                  / np.linalg.norm(p["Q"], axis=1)))
        el_s = time.perf_counter() - t0
    one = 2 * done * wl.S / el_s
    log(f"cpu oracle, 1 thread: {done} subcarriers in {el_s:.1f}s")
    workers = host_workers()
    done_all, el_all = cpu_all_cores(up, dn, wl, seconds, workers)
    allc = 2 * done_all * wl.S / el_all
    log(f"cpu oracle, {workers} processes: {done_all} subcarriers in {el_all:.1f}s")
    errors = oracle_errors(samples, O)
    for k, v in errors.items():
        log(f"error vs oracle {k}: " + ", ".join(f"{a}={b:.2e}" for a, b in v.items()
                                                if a != "subcarriers"))
    return {"value": allc, "unit": "subcarrier-solves/s (uplink detections + downlink "
                                   "precodings)", "cores": workers, "kind": "oracle",
            "sample": f"{done_all} random subcarriers of the timed batch ({wl.S} symbols each), "
                      f"uplink detection + downlink precoding, numpy FP64, {workers} worker "
                      f"processes of one thread each, {el_all:.1f} s",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "single_thread": {"value": one, "cores": 1,
                              "sample": f"{done} random subcarriers, {el_s:.1f} s"},
            "gpu_error_vs_oracle_on_sample": {"eps_llr": el, "eps_q": eq},
            "gpu_error_vs_oracle_by_result": errors}


if __name__ == "__main__":
    main()
