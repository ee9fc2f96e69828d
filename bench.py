"""Benchmark of the stacking hot path on one MI355X.

A step is one whole pass of the hot path over one synthetic workload already resident
in HBM: create a stack, add every target (host planning), finalize (binning, LDS
accumulation with the Eq. 2 rotation and Eq. 3-4 rebinning, every output cell written).

Default workload: 50 targets x 43 antennas (903 baselines) x 120 integrations x 4 spws x
240 channels x 2 polarisations, z ~ U(1.5, 3.5), onto a 512 x 512 x 960 grid.

Prints one JSON line: throughput in stacked vis*chan*pol samples/s, the accumulation
kernel against the HBM roofline (algorithmic bytes / its hipEvent-timed duration), the
device's measured copy bandwidth, the FP64 CPU oracle timed on a bounded sample of the
same workload on the host cores (all of them and one), and further legs, each with its
own roofline and, where forms are compared, every form's error against the oracle:
  forms      -- the same workload in the plain FP32 form (FP32 per-tile sums) and the
                deterministic form, with the compensated form's accuracy beside them;
  precision  -- the precision recipe in {FP32, FP64 phase argument} x {plain FP32,
                compensated} accumulation;
  batched    -- the batched recipe at its own shape (64 stacks, 3871 targets, 3.4e11
                samples, drawing on a device-resident pool of distinct datasets): plain
                FP32 one stack per launch against one batched, compensated launch;
  streamed   -- one full stack of the streamed recipe (200 targets, 750 GB) from pinned
                host memory in waves, compensated and plain carried state;
  imaged, rotated, rebinned -- the dirty image cube, Eq. 1's rotation, the per-row product.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stacked vis·chan·pol/s + HBM GB/s vs peak; batched/compensated vs plain speedup"
PEAK_HBM_GBS = 8000.0   # MI355X HBM3E, AMD public specification
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "accum_c2_counters.json")
PROFILE_ORDERED = os.path.join(ROOT, "profiles", "ordered_c2_counters.json")
PROFILE_REBIN = os.path.join(ROOT, "profiles", "rebin_c2_counters.json")
PROFILE_BATCHED = os.path.join(ROOT, "profiles", "batched_c4_counters.json")
PROFILE_IMAGE = os.path.join(ROOT, "profiles", "image_c2_counters.json")
IMAGE_SRC = os.path.join(ROOT, "paper_2609_01897_amd", "csrc", "vista_image.hip")
REBIN_SRC = os.path.join(ROOT, "paper_2609_01897_amd", "csrc", "vista_rebin.hip")
KERNEL_SRC = os.path.join(ROOT, "paper_2609_01897_amd", "csrc", "vista_accum.hip")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(targets, grid, ngrids=1):
    """Bytes the method must move: 8 B vis + 1 B flag per sample, uvw (24 B) and weights
    (4 B per pol) per row, and one write of the grid state (16 B per cell) per grid."""
    nb = 0
    ns = 0
    for t in targets:
        nrow, nch, npol = int(t.vis.shape[0]), int(t.vis.shape[1]), int(t.vis.shape[2])
        s = nrow * nch * npol
        ns += s
        nb += s * (8 + (1 if t.flag is not None else 0))
        nb += nrow * (24 + 4 * npol) if not t.weight_per_chan else nrow * 24 + s * 4
    ncell = int(grid["nu"]) * int(grid["nv"]) * int(grid["nchan"])
    nb += ncell * 16 * ngrids
    return nb, ns


def roofline(nbytes, ms, traffic=None):
    achieved = nbytes / (ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic}


def counter_traffic(config_name, shape, path=None):
    """Counter-measured HBM bytes of one accumulation launch, if the committed summary (the
    packed kernel's unless `path` names another) was taken on the current kernel source, on
    this workload and in this launch shape."""
    try:
        d = json.load(open(path or PROFILE_COUNTERS))
        h = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        want = {k: int(shape[k]) for k in ("tile_u", "tile_v", "jblock", "waves")} if shape else None
        if d.get("kernel_sha256") == h and d.get("config") == config_name and d.get("launch_shape") == want:
            return d.get("hbm_bytes_per_launch")
    except Exception:
        pass
    return None


def parse_tuning(text):
    """A launch shape from "tile_u,tile_v,jblock,waves" ("" -> None)."""
    if not text:
        return None
    a = [int(x) for x in text.split(",")]
    return dict(tile_u=a[0], tile_v=a[1], jblock=a[2], waves=a[3])


def batched_counter_traffic(shape):
    """Counter-measured HBM bytes of the batched recipe's accumulation launch, if the
    committed summary was taken on the current kernel source and in this launch shape."""
    try:
        d = json.load(open(PROFILE_BATCHED))
        h = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        want = {k: int(shape[k]) for k in ("tile_u", "tile_v", "jblock", "waves")} if shape else None
        if d.get("kernel_sha256") == h and d.get("config") == "c4" and d.get("launch_shape") == want:
            return d.get("hbm_bytes_per_launch")
    except Exception:
        pass
    return None


def image_counter_traffic(config_name):
    """Counter-measured HBM bytes of one imaging call (every pass), if the committed summary
    was taken on the current kernel source and workload."""
    try:
        d = json.load(open(PROFILE_IMAGE))
        h = hashlib.sha256(open(IMAGE_SRC, "rb").read()).hexdigest()
        if d.get("kernel_sha256") == h and d.get("config") == config_name:
            return d.get("hbm_bytes_per_call")
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


def host_threads():
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


# ----------------------------------------------------------------------------------------
# The cpu_baseline leg: the FP64 oracle on the host's cores.  It is timed on a bounded
# sample of the workload (all cores, and one core), and it computes, untimed, the reference
# slabs that the accuracy figures of the other legs compare against.  Nothing else in this
# file touches the oracle.

def cpu_baseline(targets_dev, grid, n_targets):
    """The oracle on the first n_targets targets (all rows, channels and rest channels).
    Returns the baseline record and the oracle's grid (the reference of the c2 forms)."""
    import oracle
    hosts = [t.to("cpu") for t in targets_dev[:n_targets]]
    ns = sum(int(t.vis.numel()) for t in hosts)
    threads = host_threads()
    oracle.lib()
    t0 = time.perf_counter()
    ref = oracle.stack(grid, hosts, stats=False, threads=threads, want=("S", "W", "N", "A"))
    dt = time.perf_counter() - t0
    rec = dict(value=ns / dt, unit="vis·chan·pol/s", cores=threads, kind="oracle",
               sample="%d of %d targets of the workload (all rows, channels, pols; %d samples), %.1f s"
               % (n_targets, len(targets_dev), ns, dt))
    return rec, ref


def cpu_baseline_single_core(target_dev, grid, rows):
    """The oracle on one core over the first `rows` rows of one target."""
    import oracle
    h = target_dev.to("cpu")
    h = dataclasses.replace(h, uvw=h.uvw[:rows].contiguous(), vis=h.vis[:rows].contiguous(),
                            weight=h.weight[:rows].contiguous(),
                            flag=None if h.flag is None else h.flag[:rows].contiguous())
    ns = int(h.vis.numel())
    t0 = time.perf_counter()
    oracle.stack(grid, [h], stats=False, threads=1, want=("S", "W", "N", "A"))
    dt = time.perf_counter() - t0
    return dict(value=ns / dt, unit="vis·chan·pol/s", cores=1,
                sample="the first %d rows of one target (%d samples), %.1f s" % (rows, ns, dt))


def cpu_baseline_reference(grid, views, jlo, jhi):
    """Untimed reference: the oracle over rest channels [jlo, jhi) from target views
    (dicts of host arrays, channel ranges and parameters)."""
    import oracle
    t0 = time.perf_counter()
    ref = oracle.stack(grid, views, jlo=jlo, jhi=jhi, stats=False, threads=host_threads())
    return ref, time.perf_counter() - t0


def slab_views(grid, targets, bulk_of, jlo, jhi):
    """Oracle inputs for rest channels [jlo, jhi): each target's channel range [k0, k1) that
    can reach them (a superset: one channel width and two rest channels to spare each side,
    and the oracle adds only what overlaps; the channel-to-rest map is monotonic, so the
    range is contiguous).  bulk_of(t, k0, k1) returns the host arrays holding that range
    and the first channel and channel count of their rows."""
    import numpy as np
    views = []
    e0 = grid["freq_lo"] + (jlo - 2) * grid["dfreq"]
    e1 = grid["freq_lo"] + (jhi + 2) * grid["dfreq"]
    for t in targets:
        opz = 1.0 + float(t.z)
        f = np.asarray(t.chan_freq, np.float64)
        w = np.asarray(t.chan_width, np.float64) if t.chan_width is not None else np.abs(np.gradient(f))
        lo, hi = (f - w) * opz, (f + w) * opz
        ks = np.nonzero((hi > e0) & (lo < e1))[0]
        if ks.size == 0:
            continue
        k0, k1 = int(ks.min()), int(ks.max()) + 1
        bulk, kdata, kstride = bulk_of(t, k0, k1)
        views.append(dict(bulk, chan_freq=t.chan_freq, chan_width=t.chan_width, l=t.l, m=t.m, z=t.z,
                          kbeg=k0, kend=k1, kdata=kdata, kstride=kstride))
    return views


def copied_range(t, k0, k1):
    """Host copies of channels [k0, k1) of a device-resident target."""
    cp = lambda x: None if x is None else x[:, k0:k1].contiguous().cpu().numpy()
    w = cp(t.weight) if t.weight_per_chan else t.weight.cpu().numpy()
    return (dict(uvw=t.uvw.cpu().numpy(), vis=cp(t.vis), weight=w, flag=cp(t.flag),
                 weight_per_chan=bool(t.weight_per_chan)), k0, k1 - k0)


def in_place(t, k0, k1):
    """Host views (no copy) of a target whose arrays are in pinned host memory."""
    np_ = lambda x: None if x is None else x.numpy()
    return (dict(uvw=np_(t.uvw), vis=np_(t.vis), weight=np_(t.weight), flag=np_(t.flag),
                 weight_per_chan=bool(t.weight_per_chan)), 0, int(t.nchan))


# ----------------------------------------------------------------------------------------
# Accuracy of a GPU result against a reference slab (NumPy only).

def errors(ref, out, jlo, jhi):
    """Per-cell errors on rest channels [jlo, jhi): |dS|/A and |dW|/W over cells with
    contributions, |dS|/|S| over signal-dominated cells (|S| >= 0.1 A), counts equal."""
    import numpy as np
    N = out["count"][jlo:jhi].cpu().numpy().astype(np.int64)
    S = out["sum_wvis"][jlo:jhi].cpu().numpy().astype(np.complex128)
    W = out["sum_w"][jlo:jhi].cpu().numpy().astype(np.float64)
    nz = ref["N"] > 0
    A = ref["A"][nz]
    dS = np.abs(S[nz] - ref["S"][nz])
    es = dS / A
    ew = np.abs(W[nz] - ref["W"][nz]) / ref["W"][nz]
    sig = np.abs(ref["S"][nz]) >= 0.1 * A
    er = dS[sig] / np.abs(ref["S"][nz][sig]) if sig.any() else np.zeros(1)
    return {"counts_equal": bool(np.array_equal(N, ref["N"].astype(np.int64))),
            "max_dS_over_A": float(es.max()), "median_dS_over_A": float(np.median(es)),
            "max_dW_over_W": float(ew.max()), "median_dW_over_W": float(np.median(ew)),
            "max_dS_over_S_signal": float(er.max()), "median_dS_over_S_signal": float(np.median(er)),
            "cells": int(nz.sum()), "signal_cells": int(sig.sum()), "rest_channels": [jlo, jhi]}


# ----------------------------------------------------------------------------------------

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
    """Measured copy bandwidth of the device, read + written bytes over hipEvent time: the
    library's plain 16-byte-vector copy kernel, and the runtime's own device-to-device copy
    (hipMemcpyAsync, through torch's copy_) as a check that the first is the device's rate
    and not the kernel's.  Returns (kernel GB/s, runtime copy GB/s)."""
    import torch
    from paper_2609_01897_amd import vista
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    rates = []
    for copy in (lambda: vista.debug_copy(dst, src), lambda: dst.copy_(src)):
        copy()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            copy()
        e1.record()
        torch.cuda.synchronize()
        rates.append(2 * nbytes / (e0.elapsed_time(e1) / reps / 1e3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return rates[0], rates[1]


def timed_steps(step, steps):
    """Run step() once untimed, then `steps` times; returns (ms per step, mean accumulate ms,
    the last step's (stats, timings))."""
    import torch
    step()
    torch.cuda.synchronize()
    acc = []
    t0 = time.perf_counter()
    for _ in range(steps):
        st, tim = step()
        acc.append(tim["accum_ms"])
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3, sum(acc) / len(acc), (st, tim)


def stack_step(grid, targets, flags, tuning, out):
    from paper_2609_01897_amd import vista

    def step():
        s = vista.Stack(grid, flags=flags, tuning=tuning)
        for t in targets:
            s.add(t)
        st = s.finalize(out)
        tim = s.timings()
        s.close()
        return st, tim
    return step


# ------------------------------------------------------------------------- c2 forms

FORMS_SLAB = (432, 528)     # 96 rest channels around the line, reached by every target


def forms_leg(targets, grid, nbytes, ref, ref_targets, compensated_tuning, steps=3, autotune=True, config_name="c2"):
    """The c2 workload in the plain FP32 form (FP32 per-tile sums) and the deterministic
    form (fixed-order compensated FP32 per-tile sums), timed on all targets, each in the
    launch shape the autotuner picks for it (as the main step's compensated form is); the
    accuracy of each form, and of the compensated form the main step runs, on the
    cpu_baseline sample against its oracle grid."""
    import torch
    from paper_2609_01897_amd import vista
    out = vista.alloc_outputs(grid)
    res = {}
    forms = [("compensated", 0, compensated_tuning), ("plain_fp32", vista.F_PLAIN_FP32, None),
             ("deterministic", vista.F_DETERMINISTIC | vista.F_KAHAN, None)]
    for name, flags, tuning in forms:
        rec = {}
        if name != "compensated":
            if autotune:
                t0 = time.perf_counter()
                s = vista.Stack(grid, flags=flags)
                for t in targets:
                    s.add(t)
                tuning = s.autotune()
                s.close()
                log("form %s: autotuned launch shape %s in %.1f s" % (name, tuning, time.perf_counter() - t0))
            ms, acc_ms, (st, tim) = timed_steps(stack_step(grid, targets, flags, tuning, out), steps)
            traffic = counter_traffic(config_name, tuning, PROFILE_ORDERED) if name == "deterministic" else None
            rec.update(ms_per_step=ms, accumulate_ms=acc_ms, samples_per_s=st["n_samples"] / (ms / 1e3),
                       roofline=roofline(nbytes, acc_ms, traffic=traffic),
                       launch_shape=dict(tuning or {}, source="autotuned" if autotune else "default"))
            log("form %s: step %.2f ms, accumulate %.2f ms" % (name, ms, acc_ms))
        if ref is not None:
            s = vista.Stack(grid, flags=flags, tuning=tuning)
            for t in ref_targets:
                s.add(t)
            s.finalize(out)
            s.close()
            torch.cuda.synchronize()
            sl = {k: v[FORMS_SLAB[0]:FORMS_SLAB[1]] for k, v in ref.items()}
            rec["accuracy"] = errors(sl, out, *FORMS_SLAB)
            log("form %s: max |dS|/A %.2e, max |dW|/W %.2e" % (name, rec["accuracy"]["max_dS_over_A"],
                                                                rec["accuracy"]["max_dW_over_W"]))
        res[name] = rec
    del out
    torch.cuda.empty_cache()
    res["accuracy_sample"] = "the cpu_baseline sample's targets stacked alone, rest channels %d-%d" % FORMS_SLAB
    return res


# ---------------------------------------------------------------------- c3 precision

PREC_SLAB = (936, 984)      # 48 rest channels on the [CII] line


def precision_leg(steps=3, with_reference=True):
    """The precision recipe (20 targets, 16 km baselines, offsets to 60", 1920 channels,
    grid 512 x 512 x 1920) in four forms: phase argument in FP32 or FP64, per-tile sums plain
    FP32 or compensated (FP64).  Each timed; each compared with the oracle on 48 rest
    channels around the line (where signal dominates)."""
    import torch
    import synth
    from paper_2609_01897_amd import vista
    cfg = synth.config("c3")
    grid = synth.make_grid(cfg)
    t0 = time.perf_counter()
    targets = [synth.make_target(cfg, i, device="cuda") for i in range(cfg.n_targets)]
    torch.cuda.synchronize()
    nbytes, nsamp = algorithmic_bytes(targets, grid)
    log("precision recipe: %d targets, %.3g samples, generated in %.1f s" % (len(targets), nsamp,
                                                                          time.perf_counter() - t0))
    ref = None
    ref_s = None
    if with_reference:
        views = slab_views(grid, targets, copied_range, *PREC_SLAB)
        ref, ref_s = cpu_baseline_reference(grid, views, *PREC_SLAB)
        del views
    out = vista.alloc_outputs(grid)
    res = {"workload": "precision recipe: %d targets x 903 baselines (<= 16 km) x 60 integrations x 1920 chan x "
                       "2 pol, [CII] at z ~ U(4.4, 4.8), offsets up to 60 arcsec, grid 512x512x1920" % len(targets),
           "samples": nsamp, "algorithmic_bytes": nbytes, "forms": {}}
    for arg in ("fp32", "fp64"):
        for acc in ("plain_fp32", "compensated"):
            flags = (vista.F_PHASE_FP32 if arg == "fp32" else 0) | (vista.F_PLAIN_FP32 if acc == "plain_fp32" else 0)
            ms, acc_ms, (st, tim) = timed_steps(stack_step(grid, targets, flags, None, out), steps)
            rec = {"ms_per_step": ms, "accumulate_ms": acc_ms, "samples_per_s": nsamp / (ms / 1e3),
                   "roofline": roofline(nbytes, acc_ms)}
            if ref is not None:
                rec["accuracy"] = errors(ref, out, *PREC_SLAB)
            res["forms"]["phase_%s_%s" % (arg, acc)] = rec
            log("precision %s argument, %s: step %.2f ms, accumulate %.2f ms%s" % (
                arg, acc, ms, acc_ms, "" if ref is None else ", max |dS|/A %.2e, max |dS|/|S| (signal) %.2e" % (
                    rec["accuracy"]["max_dS_over_A"], rec["accuracy"]["max_dS_over_S_signal"])))
    if ref_s is not None:
        res["oracle_reference_s"] = ref_s
    del out, targets
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------------------ c4 batched

BATCH_STACKS = 64
BATCH_SIZES_SEED = 20260904
BATCH_POOL_BYTES = 120e9      # device-resident pool of distinct datasets
BATCH_CHECK = (3, (124, 132))  # stack checked against the oracle, and its rest channels


def batched_leg(reps=1, with_reference=True, forms=None, autotune=True, batched_tuning=None):
    """The batched recipe at its own shape: 64 stacks of clip(round(lognormal(ln 40, 1)),
    5, 500) targets (3871 in all), 12-50 antennas, 60 integrations, channels from {128, 480,
    960, 3840}, z ~ U(0.5, 4), grids of 256 x 256 x 256.  Its 3.1 TB of input exceed HBM, so
    targets draw on a device-resident pool of distinct datasets (each target with its own
    z, offset and channel axis); every target's bytes are read in full.  Forms: (a) plain
    FP32, one stack per launch; (b) compensated, one stack per launch; (c) every stack in
    one batched, compensated launch (one captured graph).  Each form runs the launch shape
    the autotuner picks for it: the batched form on the whole batch, the per-launch forms
    on the stack of median size (one shape for all 64 launches); with autotune=False every
    form takes the library default.  batched_tuning, if given, is the batched form's shape
    (no autotuning for it)."""
    import torch
    import synth
    from paper_2609_01897_amd import vista
    cfg = synth.config("c4")
    grid = synth.make_grid(cfg)
    sizes = synth.batch_stack_sizes(BATCH_STACKS, seed=BATCH_SIZES_SEED)
    t0 = time.perf_counter()
    pool = []
    pool_bytes = 0
    while pool_bytes < BATCH_POOL_BYTES:
        e = len(pool)
        t = synth.make_target(cfg, e, device="cuda", nchan=int(cfg.nchan[e % len(cfg.nchan)]))
        pool.append(t)
        pool_bytes += sum(int(x.numel()) * x.element_size() for x in (t.uvw, t.vis, t.weight, t.flag))
    stacks = [synth.pool_targets(cfg, pool, n, seed=BATCH_SIZES_SEED * 100 + s) for s, n in enumerate(sizes)]
    torch.cuda.synchronize()
    all_t = [t for ts in stacks for t in ts]
    nbytes, nsamp = algorithmic_bytes(all_t, grid, ngrids=len(stacks))
    log("batched recipe: %d stacks, %d targets over a pool of %d datasets (%.0f GB), %.3g samples, %.2f TB "
        "algorithmic, prepared in %.1f s" % (len(stacks), len(all_t), len(pool), pool_bytes / 1e9, nsamp,
                                              nbytes / 1e12, time.perf_counter() - t0))
    outs = [vista.alloc_outputs(grid) for _ in stacks]

    def per_launch(flags, tuning):
        def run():
            acc = 0.0
            for s, ts in enumerate(stacks):
                _, st, tim = vista.stack(grid, ts, flags=flags, out=outs[s], tuning=tuning, with_timings=True)
                acc += tim["accum_ms"]
            return acc
        return run

    def batched(flags, tuning):
        def run():
            g = dict(grid, flags=flags)
            b = vista.Batch([g] * len(stacks), tuning=tuning)
            for s, ts in enumerate(stacks):
                for t in ts:
                    b.add(s, t)
                b.set_output(s, outs[s])            # written in place by the run
            b.run()
            for s in range(len(stacks)):
                b.finalize(s)
            tim = b.timings()
            b.close()
            return tim["accum_ms"]
        return run

    def timed(fn):
        fn()                                     # warm-up (code objects, pools, graph path)
        torch.cuda.synchronize()
        t = time.perf_counter()
        acc = 0.0
        for _ in range(reps):
            acc += fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3, acc / reps

    si, slab = BATCH_CHECK
    ref = None
    ref_s = None
    if with_reference:
        views = slab_views(grid, stacks[si], copied_range, *slab)
        ref, ref_s = cpu_baseline_reference(grid, views, *slab)
        del views
    res = {"workload": "batched recipe: %d stacks, clip(round(lognormal(ln 40, 1)), 5, 500) targets per stack (%d "
                       "total), 12-50 antennas, 60 integrations, channels from {128, 480, 960, 3840}, z ~ U(0.5, 4), "
                       "grid 256x256x256 per stack; targets draw on a device-resident pool of %d distinct datasets "
                       "(%.0f GB)" % (len(stacks), len(all_t), len(pool), pool_bytes / 1e9),
           "samples": nsamp, "algorithmic_bytes": nbytes}
    median = sorted(range(len(stacks)), key=lambda i: (len(stacks[i]), i))[len(stacks) // 2]

    def shape_for(name, flags):
        """The form's launch shape and where it came from."""
        if name == "batched_compensated" and batched_tuning:
            return batched_tuning, "given"
        if not autotune:
            return None, "default"
        t0 = time.perf_counter()
        if name == "batched_compensated":
            b = vista.Batch([dict(grid, flags=flags)] * len(stacks))
            for s, ts in enumerate(stacks):
                for t in ts:
                    b.add(s, t)
            tu = b.autotune()
            b.close()
            src = "autotuned on the whole batch"
        else:
            st = vista.Stack(grid, flags=flags)
            for t in stacks[median]:
                st.add(t)
            tu = st.autotune()
            st.close()
            src = "autotuned on the stack of median size (%d targets)" % len(stacks[median])
        log("batched recipe, %s: %s launch shape %s in %.1f s" % (name, src, tu, time.perf_counter() - t0))
        return tu, src

    all_forms = [("plain_fp32_one_stack_per_launch", vista.F_PLAIN_FP32, per_launch),
                 ("compensated_one_stack_per_launch", 0, per_launch),
                 ("batched_compensated", 0, batched)]
    for name, flags, make in all_forms:
        if forms and name not in forms:
            continue
        tuning, src = shape_for(name, flags)
        ms, acc_ms = timed(make(flags, tuning))
        rec = {"ms": ms, "accumulate_ms": acc_ms, "samples_per_s": nsamp / (ms / 1e3),
               "launch_shape": dict(tuning or {}, source=src),
               "roofline": roofline(nbytes, acc_ms,
                                    batched_counter_traffic(tuning) if name == "batched_compensated" else None)}
        if ref is not None:
            rec["accuracy"] = errors(ref, outs[si], *slab)
            rec["accuracy"]["stack"] = si
        res[name] = rec
        log("batched recipe, %s: %.1f ms (accumulate %.1f ms, %.0f GB/s)%s" % (
            name, ms, acc_ms, rec["roofline"]["achieved"],
            "" if ref is None else ", max |dS|/A %.2e" % rec["accuracy"]["max_dS_over_A"]))
    if not forms:
        res["speedup_batched_compensated_vs_plain_fp32_per_launch"] = (
            res["plain_fp32_one_stack_per_launch"]["ms"] / res["batched_compensated"]["ms"])
        res["speedup_batched_vs_per_launch_same_precision"] = (
            res["compensated_one_stack_per_launch"]["ms"] / res["batched_compensated"]["ms"])
    if ref_s is not None:
        res["oracle_reference_s"] = ref_s
    del outs, stacks, pool, all_t
    torch.cuda.empty_cache()
    return res


# ----------------------------------------------------------------------- c5 streamed

STREAM_TARGETS = 200
STREAM_POOL = 8
STREAM_BUDGET = 48 << 30      # bytes per staging buffer (two of them)
STREAM_SLAB = (952, 968)


def streamed_leg(with_reference=True):
    """One full stack of the streamed recipe: 200 targets x 903 baselines x 60 integrations
    x 3840 channels x 2 pols, streamed from pinned host memory in waves through two staging
    buffers on a copy stream, the grid state (1024 x 1024 x 1920) carried across the waves
    with compensated merges (VISTA_F_KAHAN) and, for comparison, plain FP32 merges.  The
    pinned memory holds a pool of 8 distinct datasets; each target has its own z, offset
    and channel axis, and every target's bytes cross the host link.  The end-to-end rate
    includes every host-to-device byte; the kernels' HBM fraction is reported apart."""
    import torch
    import synth
    from paper_2609_01897_amd import vista
    cfg = synth.config("c5")
    t0 = time.perf_counter()
    pin = lambda x: None if x is None else torch.empty(x.shape, dtype=x.dtype, pin_memory=True).copy_(x)
    pool = []
    for e in range(STREAM_POOL):
        d = synth.make_target(cfg, e, device="cuda")
        pool.append(dataclasses.replace(d, uvw=pin(d.uvw), vis=pin(d.vis), weight=pin(d.weight), flag=pin(d.flag)))
        del d
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    targets = synth.pool_targets(cfg, pool, STREAM_TARGETS, seed=cfg.seed * 100 + 7)
    nsamp = sum(int(t.vis.numel()) for t in targets)
    in_bytes = sum(int(x.numel()) * x.element_size() for t in targets for x in (t.uvw, t.vis, t.weight, t.flag))
    log("streamed recipe: %d targets, %.3g samples, %.0f GB through a pinned pool of %d datasets, prepared in %.1f s"
        % (len(targets), nsamp, in_bytes / 1e9, len(pool), time.perf_counter() - t0))
    ref = None
    ref_s = None
    if with_reference:
        base = synth.make_grid(cfg)
        views = slab_views(base, targets, in_place, *STREAM_SLAB)      # pinned: read in place
        ref, ref_s = cpu_baseline_reference(base, views, *STREAM_SLAB)
        del views
    res = {"workload": "streamed recipe, one full stack: %d targets x 903 baselines x 60 integrations x 3840 chan x "
                       "2 pol from pinned host memory (a pool of %d distinct datasets), grid 1024x1024x1920"
                       % (len(targets), len(pool)),
           "samples": nsamp, "input_bytes": in_bytes}
    for name, flags in (("compensated", vista.F_KAHAN), ("plain_carried_state", 0)):
        grid = synth.make_grid(cfg, flags)
        out = vista.alloc_outputs(grid)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        b = vista.Batch([grid])
        b.set_stream_budget(STREAM_BUDGET)
        for t in targets:
            b.add(0, t)
        b.set_output(0, out)
        tc = time.perf_counter()                 # end to end: the run (copies, compute) and finalize
        b.run()
        st = b.finalize(0)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - tc) * 1e3
        setup_ms = (tc - ts) * 1e3
        tim = b.timings()
        b.close()
        assert st["n_samples"] == nsamp, (st, nsamp)
        ncell = int(grid["nu"]) * int(grid["nv"]) * int(grid["nchan"])
        waves = tim["n_waves"]
        # kernel bytes: the samples and rows, the carried state read and written by every
        # wave (28 B per cell each way: three FP32 sums, three compensations, a count; 16 B
        # each way without compensation), the outputs once
        state = 28 if flags & vista.F_KAHAN else 16
        kbytes, _ = algorithmic_bytes(targets, grid)
        kbytes += ncell * 2 * state * waves
        rec = {"end_to_end_ms": ms, "setup_ms": setup_ms, "waves": waves, "samples_per_s_end_to_end": nsamp / (ms / 1e3),
               "input_GBps_end_to_end": in_bytes / (ms / 1e3) / 1e9, "h2d_copy_ms": tim["h2d_ms"],
               "h2d_GBps": in_bytes / (tim["h2d_ms"] / 1e3) / 1e9 if tim["h2d_ms"] > 0 else None,
               "device_bin_ms": tim["bin_ms"], "device_accumulate_ms": tim["accum_ms"],
               "kernel_bytes": kbytes, "kernel_roofline": roofline(kbytes, tim["accum_ms"])}
        if ref is not None:
            rec["accuracy"] = errors(ref, out, *STREAM_SLAB)
        res[name] = rec
        log("streamed %s: %.0f ms end to end over %d waves (copies %.0f ms, accumulate %.0f ms)%s" % (
            name, ms, waves, tim["h2d_ms"], tim["accum_ms"],
            "" if ref is None else ", max |dS|/A %.2e, max |dW|/W %.2e" % (rec["accuracy"]["max_dS_over_A"],
                                                                           rec["accuracy"]["max_dW_over_W"])))
        del out
        torch.cuda.empty_cache()
    if ref_s is not None:
        res["oracle_reference_s"] = ref_s
    del targets, pool
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------------------- other legs

def rotated_leg(targets, grid, flags, tuning, out, steps=3):
    """The same step with Eq. 1's rotation switched on for every target (uv cells from the
    rotated baseline): whole-step time and the accumulation kernel's hipEvent time."""
    rot = [dataclasses.replace(t, rotate_uvw=True) for t in targets]
    ms, acc_ms, (st, tim) = timed_steps(stack_step(grid, rot, flags, tuning, out), steps)
    log("rotated: step %.2f ms, accumulate %.2f ms, %d outside uv" % (ms, acc_ms, st["n_outside_uv"]))
    return {"ms_per_step": ms, "accumulate_ms": acc_ms, "records": tim["n_records"],
            "n_outside_uv": st["n_outside_uv"]}


def imaged_leg(grid, out, config_name, reps=3):
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
    rl = roofline(nbytes, kms, image_counter_traffic(config_name))
    log("imaged: %d x %d x %d cube in %.2f ms (%.0f GB/s algorithmic)"
        % (grid["nchan"], grid["nv"], grid["nu"], kms, rl["achieved"]))
    del img
    return {"workload": "dirty image of every rest channel of the stacked %dx%dx%d grid"
                        % (grid["nu"], grid["nv"], grid["nchan"]),
            "cells": ncell, "algorithmic_bytes": nbytes, "kernel_ms": kms, "roofline": rl}


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
    rl = roofline(nbytes, kms, rebin_counter_traffic(cfg.name, REBIN_NOUT))
    log("rebinned rows: kernel %.2f ms, call %.2f ms; %.3g input samples, %.0f GB/s algorithmic"
        % (kms, cms, nin, rl["achieved"]))
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
        "roofline": rl,
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
    ap.add_argument("--cpu-1core-rows", type=int, default=21672, help="rows of the oracle's one-core sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (timing and every accuracy figure)")
    ap.add_argument("--no-forms", action="store_true", help="skip the plain FP32 and deterministic forms")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision recipe")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched recipe")
    ap.add_argument("--batched-forms", default="", help="comma list of the batched recipe's forms to run "
                    "(plain_fp32_one_stack_per_launch, compensated_one_stack_per_launch, batched_compensated); "
                    "default all")
    ap.add_argument("--batched-tuning", default="", help="tile_u,tile_v,jblock,waves of the batched recipe's "
                    "batched form (default: autotuned on the batch)")
    ap.add_argument("--no-streamed", action="store_true", help="skip the pinned-host streamed recipe")
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
    copy_gbps, memcpy_gbps = hbm_copy_rate()
    log("measured copy bandwidth %.0f GB/s (the runtime's device-to-device copy: %.0f GB/s; specification "
        "peak %.0f GB/s)" % (copy_gbps, memcpy_gbps, PEAK_HBM_GBS))
    cfg = synth.config(args.config)
    ntg = args.targets or cfg.n_targets
    grid = synth.make_grid(cfg)
    flags = 0
    for f in filter(None, args.flags.split(",")):
        flags |= {"kahan": vista.F_KAHAN, "deterministic": vista.F_DETERMINISTIC,
                  "phase_fp32": vista.F_PHASE_FP32, "plain_fp32": vista.F_PLAIN_FP32}[f]
    tuning = parse_tuning(args.tuning)

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

    step = stack_step(grid, targets, flags, tuning, out)
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
    rl = roofline(nbytes, acc_ms, counter_traffic(cfg.name, tuning))
    log("step %.2f ms, accumulate %.2f ms, binning %.2f ms; %.3e samples/s; %.0f GB/s algorithmic" % (
        ms, acc_ms, sum(binms) / len(binms), value, rl["achieved"]))
    assert st["n_samples"] == nsamp, (st, nsamp)
    del step                                  # it holds the workload and the grid

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
            "flags": args.flags or "compensated (FP64 per-tile sums)",
            "phase_argument": "f64" if not (flags & vista.F_PHASE_FP32) else "f32",
            "accumulate_ms": acc_ms,
            "binning_ms": sum(binms) / len(binms),
            "records": tim["n_records"],
            "units": tim["n_units"],
            "launch_shape": dict(tuning or {}, source="autotuned" if tuned else ("given" if tuning else "default")),
        },
        "roofline": rl,
        "hbm_copy_GBps": copy_gbps,
        "hbm_copy_GBps_runtime_memcpy": memcpy_gbps,
    }
    ref = None
    if not args.no_cpu:
        log("timing the FP64 oracle on %d targets (all cores), then on %d rows of one target (one core)"
            % (args.cpu_targets, args.cpu_1core_rows))
        res["cpu_baseline"], ref = cpu_baseline(targets, grid, args.cpu_targets)
        res["cpu_baseline"]["single_core"] = cpu_baseline_single_core(targets[0], grid, args.cpu_1core_rows)
        log("oracle: %.3g samples/s on %d cores, %.3g on one" % (
            res["cpu_baseline"]["value"], res["cpu_baseline"]["cores"], res["cpu_baseline"]["single_core"]["value"]))
    if not args.no_imaged:
        res["imaged"] = imaged_leg(grid, out, cfg.name)
    if not args.no_rotated:
        res["rotated"] = rotated_leg(targets, grid, flags, tuning, out)
    del out
    torch.cuda.empty_cache()
    if not args.no_forms and flags == 0:
        res["forms"] = forms_leg(targets, grid, nbytes, ref, targets[:args.cpu_targets], tuning,
                                 autotune=not args.no_autotune, config_name=cfg.name)
    ref = None
    if not args.no_rebinned:
        res["rebinned"] = rebinned_leg(targets, cfg, grid)
    del targets                               # the other legs bring their own inputs
    torch.cuda.empty_cache()
    for name, skip, leg in (("precision", args.no_precision, precision_leg), ("batched", args.no_batched, batched_leg),
                            ("streamed", args.no_streamed, streamed_leg)):
        if skip:
            continue
        try:
            kw = {}
            if name == "batched":
                kw = {"forms": [f for f in args.batched_forms.split(",") if f], "autotune": not args.no_autotune,
                      "batched_tuning": parse_tuning(args.batched_tuning)}
            res[name] = leg(with_reference=not args.no_cpu, **kw)
        except Exception as e:                  # the main line is printed whatever a leg does
            log("%s leg failed: %r" % (name, e))
            res[name] = {"error": repr(e)}
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
