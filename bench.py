"""Benchmark of the stacking hot path on one MI355X.

A step is one whole pass of the hot path over one synthetic workload already resident
in HBM: create a stack, add every target (host planning), finalize (binning, LDS
accumulation with the Eq. 2 rotation and Eq. 3-4 rebinning, every output cell written).

Default workload: 50 targets x 43 antennas (903 baselines) x 120 integrations x 4 spws x
240 channels x 2 polarisations, z ~ U(1.5, 3.5), onto a 512 x 512 x 960 grid.

Prints one JSON line: throughput in stacked vis*chan*pol samples/s, the accumulation
kernel against the HBM roofline (algorithmic bytes / its hipEvent-timed duration), the
device's measured copy bandwidth, the FP64 CPU oracle timed on a bounded sample of the
same workload on the host cores, and two more legs: many small stacks stacked one per
launch against one batched graph launch (plain and compensated), and a stack streamed
from pinned host memory in waves (its end-to-end rate includes the host-to-device copies).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stacked vis·chan·pol/s + HBM GB/s vs peak; batched/compensated vs plain speedup"
PEAK_HBM_GBS = 8000.0   # MI355X HBM3E, AMD public specification
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "accum_c2_counters.json")
PROFILE_REBIN = os.path.join(ROOT, "profiles", "rebin_c2_counters.json")
REBIN_SRC = os.path.join(ROOT, "paper_2609_01897_amd", "csrc", "vista_rebin.hip")
KERNEL_SRC = os.path.join(ROOT, "paper_2609_01897_amd", "csrc", "vista_accum.hip")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(targets, grid, kahan=False):
    """Bytes the method must move: 8 B vis + 1 B flag per sample, uvw (24 B) and weights
    (4 B per pol) per row, and one write of the grid state (16 B per cell)."""
    nb = 0
    ns = 0
    for t in targets:
        nrow, nch, npol = int(t.vis.shape[0]), int(t.vis.shape[1]), int(t.vis.shape[2])
        s = nrow * nch * npol
        ns += s
        nb += s * (8 + (1 if t.flag is not None else 0))
        nb += nrow * (24 + 4 * npol) if not t.weight_per_chan else nrow * 24 + s * 4
    ncell = int(grid["nu"]) * int(grid["nv"]) * int(grid["nchan"])
    nb += ncell * 16
    return nb, ns


def counter_traffic(config_name, shape):
    """Counter-measured HBM bytes of one accumulation launch, if the committed summary was
    taken on the current kernel source, on this workload and in this launch shape."""
    try:
        d = json.load(open(PROFILE_COUNTERS))
        h = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        want = {k: int(shape[k]) for k in ("tile_u", "tile_v", "jblock", "waves")} if shape else None
        if d.get("kernel_sha256") == h and d.get("config") == config_name and d.get("launch_shape") == want:
            return d.get("hbm_bytes_per_launch")
    except Exception:
        pass
    return None


def rebin_counter_traffic(config_name, nout):
    """Counter-measured HBM bytes of one rebinning launch, if the committed summary was
    taken on the current kernel source, on this workload and window width."""
    try:
        d = json.load(open(PROFILE_REBIN))
        h = hashlib.sha256(open(REBIN_SRC, "rb").read()).hexdigest()
        if d.get("kernel_sha256") == h and d.get("config") == config_name and d.get("nout") == nout:
            return d.get("hbm_bytes_per_launch")
    except Exception:
        pass
    return None


def cpu_baseline(targets_dev, grid, n_targets):
    """The FP64 oracle on the first n_targets targets (all rows and channels)."""
    import oracle
    hosts = [t.to("cpu") for t in targets_dev[:n_targets]]
    ns = sum(int(t.vis.numel()) for t in hosts)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    oracle.lib()
    t0 = time.perf_counter()
    oracle.stack(grid, hosts, stats=False, threads=threads, want=("S", "W", "N"))
    dt = time.perf_counter() - t0
    return dict(value=ns / dt, unit="vis·chan·pol/s", cores=threads, kind="oracle",
                sample="%d of %d targets of the workload (all rows, channels, pols; %d samples), %.1f s"
                % (n_targets, len(targets_dev), ns, dt))


def copy_probe(nbytes, steps):
    """Time the plain copy kernel; its counter readings scale those of the stacking kernel."""
    import torch
    from paper_2609_01897_amd import vista
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    vista.debug_copy(dst, src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        vista.debug_copy(dst, src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": steps + 1,
                      "ms_per_launch": ms, "GB/s": 2 * nbytes / (ms / 1e3) / 1e9}), flush=True)


def hbm_copy_rate(nbytes=4 << 30, reps=5):
    """Measured copy bandwidth of the device (the library's plain 16-byte-vector copy kernel,
    read + written bytes over hipEvent time), reported beside the specification peak."""
    import torch
    from paper_2609_01897_amd import vista
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    vista.debug_copy(dst, src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        vista.debug_copy(dst, src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms / 1e3) / 1e9


STREAM_TARGETS = 8
STREAM_WAVE_TARGETS = 3


def streamed_leg():
    """The streamed recipe, reduced to a bounded sample: one stack of 8 targets of the
    full-scale shape (903 baselines x 60 integrations x 3840 channels x 2 pols; grid
    1024 x 1024 x 1920 with Kahan compensation) whose visibilities, flags, uvw and weights
    sit in pinned host memory.  The batch copies them to the device in waves of 3 targets on
    its copy stream, double-buffered against compute, and carries the compensated grid state
    across the waves.  The end-to-end rate includes every host-to-device byte."""
    import dataclasses
    import torch
    import synth
    from paper_2609_01897_amd import vista
    cfg = synth.config("c5")
    grid = synth.make_grid(cfg)
    t0 = time.perf_counter()
    pin = lambda x: None if x is None else torch.empty(x.shape, dtype=x.dtype, pin_memory=True).copy_(x)
    hs = []
    for i in range(STREAM_TARGETS):
        d = synth.make_target(cfg, i, device="cuda")
        hs.append(dataclasses.replace(d, uvw=pin(d.uvw), vis=pin(d.vis), weight=pin(d.weight), flag=pin(d.flag)))
        del d
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    nsamp = sum(int(t.vis.numel()) for t in hs)
    staged = [sum(((int(x.numel()) * x.element_size() + 255) // 256) * 256 for x in (t.uvw, t.vis, t.weight, t.flag))
              for t in hs]
    in_bytes = sum(int(x.numel()) * x.element_size() for t in hs for x in (t.uvw, t.vis, t.weight, t.flag))
    log("streamed recipe: %d targets, %.3g samples, %.1f GB in pinned host memory, prepared in %.1f s"
        % (len(hs), nsamp, in_bytes / 1e9, time.perf_counter() - t0))
    out = vista.alloc_outputs(grid)

    phases = {}

    def run():
        c = [time.perf_counter()]
        b = vista.Batch([dict(grid, flags=vista.F_KAHAN)])
        b.set_stream_budget(STREAM_WAVE_TARGETS * max(staged))
        for t in hs:
            b.add(0, t)
        b.set_output(0, out)
        c.append(time.perf_counter())
        b.run()
        c.append(time.perf_counter())
        st = b.finalize(0)
        tim = b.timings()
        b.close()
        c.append(time.perf_counter())
        phases.update(setup_ms=(c[1] - c[0]) * 1e3, run_ms=(c[2] - c[1]) * 1e3, finalize_ms=(c[3] - c[2]) * 1e3)
        return st, tim

    run()                                       # warm-up (pools, code objects)
    torch.cuda.synchronize()
    t = time.perf_counter()
    st, tim = run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3
    assert st["n_samples"] == nsamp, (st, nsamp)
    compute_ms = tim["bin_ms"] + tim["accum_ms"]
    log("streamed recipe: %.1f ms end to end over %d waves (host-to-device copies %.1f ms, device compute %.1f ms)"
        % (ms, tim["n_waves"], tim["h2d_ms"], compute_ms))
    del out, hs
    torch.cuda.empty_cache()
    return {
        "workload": "streamed recipe reduced: 1 stack of %d targets x 903 baselines x 60 integrations x 3840 chan x "
                    "2 pol from pinned host memory, waves of %d targets, grid 1024x1024x1920, Kahan"
                    % (STREAM_TARGETS, STREAM_WAVE_TARGETS),
        "samples": nsamp,
        "input_bytes": in_bytes,
        "waves": tim["n_waves"],
        "end_to_end_ms": ms,
        "samples_per_s_end_to_end": nsamp / (ms / 1e3),
        "input_GBps_end_to_end": in_bytes / (ms / 1e3) / 1e9,
        "h2d_copy_ms": tim["h2d_ms"],
        "h2d_GBps": in_bytes / (tim["h2d_ms"] / 1e3) / 1e9 if tim["h2d_ms"] > 0 else None,
        "device_compute_ms": compute_ms,
        "samples_per_s_device": nsamp / (compute_ms / 1e3),
        "host_phases_ms": phases,
    }


def rotated_leg(targets, grid, flags, tuning, out, steps=3):
    """The same step with Eq. 1's rotation switched on for every target (uv cells from the
    rotated baseline): whole-step time and the accumulation kernel's hipEvent time."""
    import dataclasses
    import torch
    from paper_2609_01897_amd import vista
    rot = [dataclasses.replace(t, rotate_uvw=True) for t in targets]

    def step():
        s = vista.Stack(grid, flags=flags, tuning=tuning)
        for t in rot:
            s.add(t)
        st = s.finalize(out)
        tim = s.timings()
        s.close()
        return st, tim

    step()
    torch.cuda.synchronize()
    acc = []
    t0 = time.perf_counter()
    for _ in range(steps):
        st, tim = step()
        acc.append(tim["accum_ms"])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    log("rotated: step %.2f ms, accumulate %.2f ms, %d outside uv" % (ms, sum(acc) / len(acc), st["n_outside_uv"]))
    return {"ms_per_step": ms, "accumulate_ms": sum(acc) / len(acc), "records": tim["n_records"],
            "n_outside_uv": st["n_outside_uv"]}


def imaged_leg(grid, out, reps=3):
    """Dirty image cube of the stacked grid the timed steps produced: every rest channel
    inverted by the library's 2-D FFT.  Algorithmic bytes: the grid read once (8 B sum plus
    4 B weight per cell) and the image written once (4 B per cell)."""
    import torch
    from paper_2609_01897_amd import vista
    img, _, tim = vista.image(grid, out["sum_wvis"], out["sum_w"])       # warm-up
    ks = []
    for _ in range(reps):
        _, _, tim = vista.image(grid, out["sum_wvis"], out["sum_w"], out=img)
        ks.append(tim["accum_ms"])
    torch.cuda.synchronize()
    kms = sorted(ks)[len(ks) // 2]
    ncell = int(grid["nu"]) * int(grid["nv"]) * int(grid["nchan"])
    nbytes = ncell * 16
    achieved = nbytes / (kms / 1e3) / 1e9
    log("imaged: %d x %d x %d cube in %.2f ms (%.0f GB/s algorithmic)"
        % (grid["nchan"], grid["nv"], grid["nu"], kms, achieved))
    del img
    return {"workload": "dirty image of every rest channel of the stacked %dx%dx%d grid"
                        % (grid["nu"], grid["nv"], grid["nchan"]),
            "cells": ncell, "algorithmic_bytes": nbytes, "kernel_ms": kms,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": achieved / PEAK_HBM_GBS, "traffic": None}}


REBIN_NOUT = 480


def rebinned_leg(targets, cfg, grid, reps=3):
    """The paper's per-row product on the same resident targets: every row of every target
    rebinned onto its own window of REBIN_NOUT channels of the common rest width around the
    line (visibilities, flags, normalisers and rest-frame baselines written).  Algorithmic
    bytes: the input channels the windows reach (8 B vis + 1 B flag per sample) and each
    row's uvw, plus every output (8 + 1 + 4 B per output sample, 24 B per row)."""
    import numpy as np
    import torch
    from paper_2609_01897_amd import vista
    dfreq, central = float(grid["dfreq"]), float(cfg.line_rest)
    outs, los, tim = vista.rebin_rows(targets, REBIN_NOUT, dfreq, central)      # warm-up, allocates
    torch.cuda.synchronize()
    nbytes = 0
    nin = 0
    nout_samples = 0
    for t, lo in zip(targets, los):
        f = np.asarray(t.chan_freq, np.float64)
        w = np.abs(np.gradient(f)) if t.chan_width is None else np.asarray(t.chan_width, np.float64)
        opz = 1.0 + float(t.z)
        reach = ((f + 0.5 * w) * opz > lo) & ((f - 0.5 * w) * opz < lo + REBIN_NOUT * dfreq)
        nrow, npol = int(t.vis.shape[0]), int(t.vis.shape[2])
        nin += nrow * int(reach.sum()) * npol
        nout_samples += nrow * REBIN_NOUT * npol
        nbytes += nrow * int(reach.sum()) * npol * 9 + nrow * 24 + nrow * REBIN_NOUT * npol * 13 + nrow * 24
    kernel_ms, call_ms = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        _, _, tim = vista.rebin_rows(targets, REBIN_NOUT, dfreq, central, outs=outs)
        call_ms.append((time.perf_counter() - t0) * 1e3)
        kernel_ms.append(tim["accum_ms"])
    kms = sorted(kernel_ms)[len(kernel_ms) // 2]
    cms = sorted(call_ms)[len(call_ms) // 2]
    achieved = nbytes / (kms / 1e3) / 1e9
    log("rebinned rows: kernel %.2f ms, call %.2f ms; %.3g input samples, %.0f GB/s algorithmic"
        % (kms, cms, nin, achieved))
    del outs
    torch.cuda.empty_cache()
    return {
        "workload": "per-row rebinned product: the %d targets above, each row onto its own window of %d "
                    "channels of the common rest width around the line" % (len(targets), REBIN_NOUT),
        "input_samples": nin,
        "output_samples": nout_samples,
        "algorithmic_bytes": nbytes,
        "kernel_ms": kms,
        "call_ms": cms,
        "samples_per_s": nin / (cms / 1e3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": rebin_counter_traffic(cfg.name, REBIN_NOUT)},
    }


BATCH_STACKS = 64
BATCH_MU = math.log(4.0)     # targets per stack ~ clip(round(lognormal(log 4, 1)), 1, 64)
BATCH_N_INT = 10


def batched_leg(reps: int):
    """The batched recipe, reduced to fit a one-minute bench: 64 stacks with lognormal
    target counts and mixed channel layouts, stacked (a) one stack per launch sequence,
    (b) as one batch (one captured graph), (c) as one batch with Kahan compensation.
    Every form writes every stack's output grid (the batch writes them in place)."""
    import torch
    import synth
    from paper_2609_01897_amd import vista
    sizes = synth.batch_stack_sizes(BATCH_STACKS, seed=20260904, lo=1, hi=64, mu=BATCH_MU)
    base = synth.config("c4", n_int=BATCH_N_INT)
    t0 = time.perf_counter()
    stacks = []
    for s, n in enumerate(sizes):
        cfg = synth.config("c4", n_int=BATCH_N_INT, seed=base.seed + 1000 * (s + 1))
        stacks.append([synth.make_target(cfg, i, device="cuda") for i in range(n)])
    grid = synth.make_grid(base)
    torch.cuda.synchronize()
    nsamp = sum(int(t.vis.numel()) for ts in stacks for t in ts)
    log("batched recipe: %d stacks, %d targets, %.3g samples, generated in %.1f s"
        % (len(stacks), sum(sizes), nsamp, time.perf_counter() - t0))
    outs = [vista.alloc_outputs(grid) for _ in stacks]

    def plain():
        for s, ts in enumerate(stacks):
            vista.stack(grid, ts, out=outs[s])

    def batched(flags):
        g = dict(grid, flags=flags)
        b = vista.Batch([g] * len(stacks))
        for s, ts in enumerate(stacks):
            for t in ts:
                b.add(s, t)
            b.set_output(s, outs[s])            # written in place by the run
        b.run()
        for s in range(len(stacks)):
            b.finalize(s)
        tim = b.timings()
        b.close()
        return tim

    def timed(fn, *a):
        fn(*a)                                  # warm-up (code objects, pools, graph path)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn(*a)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3

    ms_plain = timed(plain)
    ms_batch = timed(batched, 0)
    ms_kahan = timed(batched, vista.F_KAHAN)
    log("batched recipe: plain %.1f ms, batched %.1f ms, batched+Kahan %.1f ms" % (ms_plain, ms_batch, ms_kahan))
    del stacks, outs
    torch.cuda.empty_cache()
    return {
        "workload": "batched recipe reduced: %d stacks, targets per stack lognormal(log 4, 1) in [1, 64] "
                    "(%d total), 12-50 antennas, %d integrations, channels from {128, 480, 960, 3840}, "
                    "grid 256x256x256 per stack" % (len(sizes), sum(sizes), BATCH_N_INT),
        "samples": nsamp,
        "plain_one_stack_per_launch_ms": ms_plain,
        "batched_graph_ms": ms_batch,
        "batched_kahan_ms": ms_kahan,
        "speedup_batched_vs_plain": ms_plain / ms_batch,
        "speedup_batched_kahan_vs_plain": ms_plain / ms_kahan,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--targets", type=int, default=0, help="use only this many targets (0 = all)")
    ap.add_argument("--flags", default="", help="comma list: kahan,deterministic,phase_fp32,plain_fp32")
    ap.add_argument("--cpu-targets", type=int, default=12, help="targets in the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--no-streamed", action="store_true", help="skip the pinned-host streamed leg")
    ap.add_argument("--no-rebinned", action="store_true", help="skip the per-row rebinned leg")
    ap.add_argument("--no-rotated", action="store_true", help="skip the step with Eq. 1's rotation on")
    ap.add_argument("--no-imaged", action="store_true", help="skip the dirty-image leg")
    ap.add_argument("--no-autotune", action="store_true", help="time the default launch shape")
    ap.add_argument("--tuning", default="", help="tile_u,tile_v,jblock,waves")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run the library's plain copy kernel on MIB MiB, --steps times (calibrates "
                         "hardware byte counters), and print its bytes and time")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the design notes "
              "describe how the work would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2609_01897_amd import vista

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    vista.lib()
    if args.copy_probe:
        copy_probe(args.copy_probe << 20, args.steps)
        return
    copy_gbps = hbm_copy_rate()
    log("measured copy bandwidth %.0f GB/s (specification peak %.0f GB/s)" % (copy_gbps, PEAK_HBM_GBS))
    cfg = synth.config(args.config)
    ntg = args.targets or cfg.n_targets
    grid = synth.make_grid(cfg)
    flags = 0
    for f in filter(None, args.flags.split(",")):
        flags |= {"kahan": vista.F_KAHAN, "deterministic": vista.F_DETERMINISTIC,
                  "phase_fp32": vista.F_PHASE_FP32, "plain_fp32": vista.F_PLAIN_FP32}[f]
    tuning = None
    if args.tuning:
        a = [int(x) for x in args.tuning.split(",")]
        tuning = dict(tile_u=a[0], tile_v=a[1], jblock=a[2], waves=a[3])

    t0 = time.perf_counter()
    targets = []
    for i in range(ntg):
        targets.append(synth.make_target(cfg, i, device="cuda"))
    torch.cuda.synchronize()
    log("generated %d targets on the GPU in %.1f s" % (ntg, time.perf_counter() - t0))
    nbytes, nsamp = algorithmic_bytes(targets, grid)
    out = vista.alloc_outputs(grid)

    tuned = None
    if tuning is None and not args.no_autotune:
        t0 = time.perf_counter()
        s = vista.Stack(grid, flags=flags)
        for t in targets:
            s.add(t)
        tuned = s.autotune()
        s.close()
        tuning = tuned
        log("autotuned launch shape %s in %.1f s" % (tuned, time.perf_counter() - t0))

    def step():
        s = vista.Stack(grid, flags=flags, tuning=tuning)
        for t in targets:
            s.add(t)
        st = s.finalize(out)
        tim = s.timings()
        s.close()
        return st, tim

    for i in range(args.warmup):
        st, tim = step()
        log("warmup %d: total %.2f ms (bin %.2f, accum %.2f), %d records" % (
            i, tim["total_ms"], tim["bin_ms"], tim["accum_ms"], tim["n_records"]))
    torch.cuda.synchronize()
    accum = []
    binms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        st, tim = step()
        accum.append(tim["accum_ms"])
        binms.append(tim["bin_ms"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / args.steps * 1e3
    value = nsamp / (ms / 1e3)
    acc_ms = sum(accum) / len(accum)
    achieved = nbytes / (acc_ms / 1e3) / 1e9
    log("step %.2f ms, accumulate %.2f ms, binning %.2f ms; %.3e samples/s; %.0f GB/s algorithmic" % (
        ms, acc_ms, sum(binms) / len(binms), value, achieved))
    assert st["n_samples"] == nsamp, (st, nsamp)
    traffic = counter_traffic(cfg.name, tuning)

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "vis·chan·pol/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "%s: %d targets x %d baselines x %d integrations x %d chan x %d pol, grid %dx%dx%d"
                        % (cfg.name, ntg, cfg.n_ant[0] * (cfg.n_ant[0] - 1) // 2, cfg.n_int, cfg.nchan[0],
                           cfg.npol, grid["nu"], grid["nv"], grid["nchan"]),
            "samples": nsamp,
            "algorithmic_bytes": nbytes,
            "flags": args.flags or "plain",
            "phase_argument": "f64" if not (flags & vista.F_PHASE_FP32) else "f32",
            "accumulate_ms": acc_ms,
            "binning_ms": sum(binms) / len(binms),
            "records": tim["n_records"],
            "units": tim["n_units"],
            "launch_shape": dict(tuning or {}, source="autotuned" if tuned else ("given" if tuning else "default")),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
        },
        "hbm_copy_GBps": copy_gbps,
    }
    if not args.no_cpu:
        log("timing the FP64 oracle on %d targets" % args.cpu_targets)
        res["cpu_baseline"] = cpu_baseline(targets, grid, args.cpu_targets)
    if not args.no_imaged:
        res["imaged"] = imaged_leg(grid, out)
    if not args.no_rotated:
        res["rotated"] = rotated_leg(targets, grid, flags, tuning, out)
    del out
    torch.cuda.empty_cache()
    if not args.no_rebinned:
        res["rebinned"] = rebinned_leg(targets, cfg, grid)
    del targets                               # the other legs bring their own inputs
    torch.cuda.empty_cache()
    if not args.no_batched:
        res["batched"] = batched_leg(reps=2)
    if not args.no_streamed:
        res["streamed"] = streamed_leg()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
