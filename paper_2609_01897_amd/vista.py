"""ctypes binding of libvista.so (include/vista.h).  Argument marshalling only.

Tensors are passed by ``data_ptr()``; the HIP stream is torch's current stream unless one
is given.  Every computation runs in the library's gfx950 kernels.  Loading fails loudly
when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# VISTA_LIB selects another build of the library (e.g. a host-sanitized one).
LIB_PATH = os.environ.get("VISTA_LIB") or os.path.join(HERE, "_build", "libvista.so")

VISTA_OK, VISTA_E_ARG, VISTA_E_STATE, VISTA_E_NOMEM, VISTA_E_HIP, VISTA_E_RANGE = 0, -1, -2, -3, -4, -5
MEM_HOST, MEM_HOST_PINNED, MEM_DEVICE = 0, 1, 2
F_KAHAN, F_DETERMINISTIC, F_SPECTRAL_NEAREST, F_PHASE_FP32, F_PLAIN_FP32 = 1, 2, 4, 8, 16
STAT_NAMES = ("n_samples", "n_flagged", "n_bad_weight", "n_outside_uv", "n_outside_band", "n_used",
              "n_contrib")
_ERR = {VISTA_E_ARG: "VISTA_E_ARG", VISTA_E_STATE: "VISTA_E_STATE", VISTA_E_NOMEM: "VISTA_E_NOMEM",
        VISTA_E_HIP: "VISTA_E_HIP", VISTA_E_RANGE: "VISTA_E_RANGE"}


class VistaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_ERR.get(code, code), msg))
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("nu", C.c_int32), ("nv", C.c_int32), ("du", C.c_double), ("dv", C.c_double),
                ("nchan", C.c_int32), ("freq_lo", C.c_double), ("dfreq", C.c_double),
                ("flags", C.c_uint32)]


class TargetDesc(C.Structure):
    _fields_ = [("nrow", C.c_int64), ("nchan", C.c_int32), ("npol", C.c_int32), ("uvw", C.c_void_p),
                ("vis", C.c_void_p), ("weight", C.c_void_p), ("flag", C.c_void_p),
                ("chan_freq", C.c_void_p), ("chan_width", C.c_void_p), ("l", C.c_double),
                ("m", C.c_double), ("z", C.c_double), ("weight_per_chan", C.c_int32), ("mem", C.c_int32),
                ("rotate_uvw", C.c_int32), ("ra0", C.c_double), ("dec0", C.c_double), ("ra1", C.c_double),
                ("dec1", C.c_double)]


class Output(C.Structure):
    _fields_ = [("sum_wvis", C.c_void_p), ("sum_w", C.c_void_p), ("count", C.c_void_p),
                ("sum_wvis64", C.c_void_p), ("sum_w64", C.c_void_p), ("mem", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in STAT_NAMES]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n in STAT_NAMES}


class RebinDesc(C.Structure):
    _fields_ = [("nout", C.c_int32), ("dfreq", C.c_double), ("central_freq", C.c_double)]


class RebinOutput(C.Structure):
    _fields_ = [("vis", C.c_void_p), ("flag", C.c_void_p), ("wsum", C.c_void_p), ("uvw", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("tile_u", C.c_int32), ("tile_v", C.c_int32), ("jblock", C.c_int32), ("waves", C.c_int32),
                ("wg_per_cu", C.c_int32)]


class Timings(C.Structure):
    _fields_ = [("bin_ms", C.c_double), ("accum_ms", C.c_double), ("finalize_ms", C.c_double),
                ("total_ms", C.c_double), ("h2d_ms", C.c_double), ("n_records", C.c_int64),
                ("n_units", C.c_int64), ("n_accum_launches", C.c_int32), ("n_waves", C.c_int32)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


SYMBOLS = {
    "vista_stack_create": ([C.POINTER(GridDesc), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "vista_stack_add_target": ([C.c_void_p, C.POINTER(TargetDesc)], C.c_int),
    "vista_stack_set_tuning": ([C.c_void_p, C.POINTER(Tuning)], C.c_int),
    "vista_stack_finalize": ([C.c_void_p, C.POINTER(Output), C.POINTER(Stats)], C.c_int),
    "vista_stack_timings": ([C.c_void_p, C.POINTER(Timings)], C.c_int),
    "vista_stack_destroy": ([C.c_void_p], C.c_int),
    "vista_stack_autotune": ([C.c_void_p, C.POINTER(Tuning)], C.c_int),
    "vista_batch_autotune": ([C.c_void_p, C.POINTER(Tuning)], C.c_int),
    "vista_batch_create": ([C.c_int32, C.POINTER(GridDesc), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "vista_batch_add_target": ([C.c_void_p, C.c_int32, C.POINTER(TargetDesc)], C.c_int),
    "vista_batch_set_tuning": ([C.c_void_p, C.POINTER(Tuning)], C.c_int),
    "vista_batch_set_stream_budget": ([C.c_void_p, C.c_int64], C.c_int),
    "vista_batch_run": ([C.c_void_p], C.c_int),
    "vista_batch_finalize": ([C.c_void_p, C.c_int32, C.POINTER(Output), C.POINTER(Stats)], C.c_int),
    "vista_batch_timings": ([C.c_void_p, C.POINTER(Timings)], C.c_int),
    "vista_batch_destroy": ([C.c_void_p], C.c_int),
    "vista_plan_spectral_grid": ([C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                  C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "vista_debug_indices": ([C.POINTER(GridDesc), C.POINTER(TargetDesc), C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p], C.c_int),
    "vista_debug_rotate": ([C.POINTER(GridDesc), C.POINTER(TargetDesc), C.c_void_p, C.c_void_p], C.c_int),
    "vista_debug_copy": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "vista_batch_set_output": ([C.c_void_p, C.c_int32, C.POINTER(Output)], C.c_int),
    "vista_image": ([C.POINTER(GridDesc), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                     C.POINTER(Timings)], C.c_int),
    "vista_image_noalloc": ([C.POINTER(GridDesc), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
                            C.c_int),
    "vista_rebin_window": ([C.POINTER(RebinDesc), C.POINTER(TargetDesc), C.POINTER(C.c_double)], C.c_int),
    "vista_rebin_rows": ([C.POINTER(RebinDesc), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                          C.POINTER(Timings)], C.c_int),
    "vista_release_workspace": ([], C.c_int),
    "vista_last_error": ([], C.c_char_p),
    "vista_version": ([], C.c_char_p),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvista.so is not built (run __graft_entry__.build() or "
                               "python paper_2609_01897_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SYMBOLS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int):
    if rc != VISTA_OK:
        raise VistaError(rc, lib().vista_last_error().decode())


def grid_desc(g: dict, flags: int | None = None) -> GridDesc:
    return GridDesc(int(g["nu"]), int(g["nv"]), float(g["du"]), float(g["dv"]), int(g["nchan"]),
                    float(g["freq_lo"]), float(g["dfreq"]), int(g.get("flags", 0) if flags is None else flags))


def _ptr(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr() or None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError("unsupported array type %r" % type(x))


def _mem_of(x) -> int:
    if hasattr(x, "is_cuda") and x.is_cuda:
        return MEM_DEVICE
    if hasattr(x, "is_pinned") and x.is_pinned():
        return MEM_HOST_PINNED
    return MEM_HOST


def target_desc(t, keep: list) -> TargetDesc:
    """Describe a target object (attributes uvw, vis, weight, flag, chan_freq, chan_width,
    l, m, z, weight_per_chan) without copying its data.  Host arrays that must outlive the
    call are appended to ``keep``."""
    freq = np.ascontiguousarray(t.chan_freq, dtype=np.float64)
    width = None if t.chan_width is None else np.ascontiguousarray(t.chan_width, dtype=np.float64)
    keep.extend([freq, width])
    nrow = int(t.uvw.shape[0])
    return TargetDesc(nrow, int(freq.shape[0]), int(t.vis.shape[2]), _ptr(t.uvw), _ptr(t.vis), _ptr(t.weight),
                      _ptr(t.flag), freq.ctypes.data, None if width is None else width.ctypes.data,
                      float(t.l), float(t.m), float(t.z), int(bool(t.weight_per_chan)), _mem_of(t.vis),
                      int(bool(getattr(t, "rotate_uvw", False))), float(getattr(t, "ra0", 0.0)),
                      float(getattr(t, "dec0", 0.0)), float(getattr(t, "ra1", 0.0)), float(getattr(t, "dec1", 0.0)))


def current_stream():
    """torch's current HIP stream (the null stream when no GPU is visible)."""
    import torch
    if not torch.cuda.is_available():
        return None
    return torch.cuda.current_stream().cuda_stream


class Stack:
    """One stack: create, add targets, finalize into output tensors."""

    def __init__(self, grid: dict, flags: int | None = None, stream=None, tuning: dict | None = None):
        self.grid = dict(grid)
        self.desc = grid_desc(grid, flags)
        self.stream = current_stream() if stream is None else stream
        h = C.c_void_p()
        _check(lib().vista_stack_create(C.byref(self.desc), self.stream, C.byref(h)))
        self.h = h
        self._keep = []
        if tuning:
            self.set_tuning(**tuning)

    def set_tuning(self, tile_u=0, tile_v=0, jblock=0, waves=0, wg_per_cu=0):
        tu = Tuning(tile_u, tile_v, jblock, waves, wg_per_cu)
        _check(lib().vista_stack_set_tuning(self.h, C.byref(tu)))

    def add(self, t):
        d = target_desc(t, self._keep)
        self._keep.append(t)
        _check(lib().vista_stack_add_target(self.h, C.byref(d)))

    def finalize(self, out: dict) -> dict:
        """``out`` maps sum_wvis/sum_w/count/sum_wvis64/sum_w64 to tensors (or None)."""
        o = Output(_ptr(out.get("sum_wvis")), _ptr(out.get("sum_w")), _ptr(out.get("count")),
                   _ptr(out.get("sum_wvis64")), _ptr(out.get("sum_w64")),
                   _mem_of(next(v for v in out.values() if v is not None)))
        st = Stats()
        _check(lib().vista_stack_finalize(self.h, C.byref(o), C.byref(st)))
        return st.as_dict()

    def autotune(self) -> dict:
        """Time the built launch shapes on this stack's targets and keep the fastest."""
        tu = Tuning()
        _check(lib().vista_stack_autotune(self.h, C.byref(tu)))
        return dict(tile_u=tu.tile_u, tile_v=tu.tile_v, jblock=tu.jblock, waves=tu.waves)

    def timings(self) -> dict:
        t = Timings()
        _check(lib().vista_stack_timings(self.h, C.byref(t)))
        return t.as_dict()

    def close(self):
        if self.h:
            lib().vista_stack_destroy(self.h)
            self.h = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def alloc_outputs(grid: dict, device="cuda", fp64: bool = False) -> dict:
    import torch
    shape = (int(grid["nchan"]), int(grid["nv"]), int(grid["nu"]))
    out = dict(sum_wvis=torch.empty(shape, dtype=torch.complex64, device=device),
               sum_w=torch.empty(shape, dtype=torch.float32, device=device),
               count=torch.empty(shape, dtype=torch.int32, device=device))
    if fp64:
        out["sum_wvis64"] = torch.empty(shape, dtype=torch.complex128, device=device)
        out["sum_w64"] = torch.empty(shape, dtype=torch.float64, device=device)
    return out


def stack(grid: dict, targets, flags: int | None = None, fp64: bool = False, tuning: dict | None = None,
          out: dict | None = None, with_timings: bool = False):
    """Stack ``targets`` (device tensors) into freshly allocated device outputs."""
    s = Stack(grid, flags, tuning=tuning)
    try:
        for t in targets:
            s.add(t)
        out = alloc_outputs(grid, fp64=fp64) if out is None else out
        st = s.finalize(out)
        tim = s.timings()
    finally:
        s.close()
    return (out, st, tim) if with_timings else (out, st)


class Batch:
    """Several independent stacks in one launch sequence."""

    def __init__(self, grids: list, stream=None, tuning: dict | None = None):
        self.grids = [dict(g) for g in grids]
        arr = (GridDesc * len(grids))(*[grid_desc(g) for g in grids])
        self.stream = current_stream() if stream is None else stream
        h = C.c_void_p()
        _check(lib().vista_batch_create(len(grids), arr, self.stream, C.byref(h)))
        self.h = h
        self._keep = []
        if tuning:
            tu = Tuning(tuning.get("tile_u", 0), tuning.get("tile_v", 0), tuning.get("jblock", 0),
                        tuning.get("waves", 0), tuning.get("wg_per_cu", 0))
            _check(lib().vista_batch_set_tuning(self.h, C.byref(tu)))

    def add(self, stack_index: int, t):
        d = target_desc(t, self._keep)
        self._keep.append(t)
        _check(lib().vista_batch_add_target(self.h, int(stack_index), C.byref(d)))

    def set_stream_budget(self, nbytes: int):
        _check(lib().vista_batch_set_stream_budget(self.h, int(nbytes)))

    def set_output(self, stack_index: int, out: dict):
        """Register a stack's outputs before run(); device outputs are written in place."""
        o = _output(out)
        self._keep.append(out)
        _check(lib().vista_batch_set_output(self.h, int(stack_index), C.byref(o)))

    def run(self):
        _check(lib().vista_batch_run(self.h))

    def finalize(self, stack_index: int, out: dict | None = None) -> dict:
        st = Stats()
        o = C.byref(_output(out)) if out is not None else None
        _check(lib().vista_batch_finalize(self.h, int(stack_index), o, C.byref(st)))
        return st.as_dict()

    def autotune(self) -> dict:
        """Time the built launch shapes on this batch's targets and keep the fastest."""
        tu = Tuning()
        _check(lib().vista_batch_autotune(self.h, C.byref(tu)))
        return dict(tile_u=tu.tile_u, tile_v=tu.tile_v, jblock=tu.jblock, waves=tu.waves)

    def timings(self) -> dict:
        t = Timings()
        _check(lib().vista_batch_timings(self.h, C.byref(t)))
        return t.as_dict()

    def close(self):
        if self.h:
            lib().vista_batch_destroy(self.h)
            self.h = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _output(out: dict) -> Output:
    return Output(_ptr(out.get("sum_wvis")), _ptr(out.get("sum_w")), _ptr(out.get("count")),
                  _ptr(out.get("sum_wvis64")), _ptr(out.get("sum_w64")),
                  _mem_of(next(v for v in out.values() if v is not None)))


def debug_indices(grid: dict, t, stream=None) -> dict:
    keep = []
    d = target_desc(t, keep)
    g = grid_desc(grid)
    n = int(t.uvw.shape[0]) * int(len(t.chan_freq))
    shape = (int(t.uvw.shape[0]), int(len(t.chan_freq)))
    iu = np.empty(shape, np.int32); iv = np.empty(shape, np.int32)
    j0 = np.empty(shape, np.int32); nj = np.empty(shape, np.int32)
    s = current_stream() if stream is None else stream
    _check(lib().vista_debug_indices(C.byref(g), C.byref(d), s, iu.ctypes.data, iv.ctypes.data, j0.ctypes.data,
                                     nj.ctypes.data))
    del n
    return dict(iu=iu, iv=iv, j0=j0, nj=nj)


def debug_rotate(grid: dict, t, flags: int | None = None, stream=None):
    import torch
    keep = []
    d = target_desc(t, keep)
    g = grid_desc(grid, flags)
    out = torch.empty_like(t.vis)
    s = current_stream() if stream is None else stream
    _check(lib().vista_debug_rotate(C.byref(g), C.byref(d), s, _ptr(out)))
    return out


def debug_copy(dst, src, stream=None):
    """dst <- src (same byte size) by the library's plain copy kernel."""
    n = dst.numel() * dst.element_size()
    if n != src.numel() * src.element_size():
        raise ValueError("sizes differ")
    s = current_stream() if stream is None else stream
    _check(lib().vista_debug_copy(_ptr(dst), _ptr(src), n, s))


def plan_spectral_grid(chan_freqs, chan_widths, zs, central_freq: float, nchan_out: int):
    n = len(chan_freqs)
    fs = [np.ascontiguousarray(f, np.float64) for f in chan_freqs]
    ws = [None if w is None else np.ascontiguousarray(w, np.float64) for w in chan_widths]
    fp = (C.c_void_p * n)(*[f.ctypes.data for f in fs])
    wp = (C.c_void_p * n)(*[None if w is None else w.ctypes.data for w in ws])
    nc = np.asarray([f.shape[0] for f in fs], np.int32)
    zz = np.asarray(zs, np.float64)
    lo = C.c_double(0)
    df = C.c_double(0)
    _check(lib().vista_plan_spectral_grid(n, C.cast(fp, C.c_void_p), C.cast(wp, C.c_void_p), nc.ctypes.data,
                                          zz.ctypes.data, float(central_freq), int(nchan_out), C.byref(lo),
                                          C.byref(df)))
    return lo.value, df.value


def version() -> str:
    return lib().vista_version().decode()


def rebin_window(t, nout: int, dfreq: float, central_freq: float) -> float:
    """Lower edge [Hz] of target t's own output window (``vista_rebin_window``)."""
    keep = []
    d = RebinDesc(int(nout), float(dfreq), float(central_freq))
    td = target_desc(t, keep)
    lo = C.c_double(0.0)
    _check(lib().vista_rebin_window(C.byref(d), C.byref(td), C.byref(lo)))
    return lo.value


def rebin_rows(targets, nout: int, dfreq: float, central_freq: float, outs=None, want=("vis", "flag", "wsum", "uvw"),
               stream=None):
    """Per-row rebinned product of device-resident targets (``vista_rebin_rows``).

    ``outs`` (one dict per target with vis/flag/wsum/uvw tensors, any of the last three may
    be None) is allocated on the targets' device when not given, with the fields in
    ``want``.  Returns (outs, freq_lo list, timings dict)."""
    import torch
    targets = list(targets)
    if outs is None:
        outs = []
        for t in targets:
            nrow, npol = int(t.vis.shape[0]), int(t.vis.shape[2])
            dev = t.vis.device
            o = dict(vis=torch.empty((nrow, int(nout), npol), dtype=torch.complex64, device=dev))
            o["flag"] = torch.empty((nrow, int(nout), npol), dtype=torch.uint8, device=dev) if "flag" in want else None
            o["wsum"] = torch.empty((nrow, int(nout), npol), dtype=torch.float32, device=dev) if "wsum" in want else None
            o["uvw"] = torch.empty((nrow, 3), dtype=torch.float64, device=dev) if "uvw" in want else None
            outs.append(o)
    keep = []
    n = len(targets)
    tds = (TargetDesc * max(1, n))(*[target_desc(t, keep) for t in targets])
    ods = (RebinOutput * max(1, n))(*[RebinOutput(_ptr(o.get("vis")), _ptr(o.get("flag")), _ptr(o.get("wsum")),
                                                  _ptr(o.get("uvw"))) for o in outs])
    lo = (C.c_double * max(1, n))()
    tim = Timings()
    d = RebinDesc(int(nout), float(dfreq), float(central_freq))
    s = current_stream() if stream is None else stream
    _check(lib().vista_rebin_rows(C.byref(d), n, C.cast(tds, C.c_void_p), C.cast(ods, C.c_void_p), s,
                                  C.cast(lo, C.c_void_p), C.byref(tim)))
    return outs, [lo[i] for i in range(n)], tim.as_dict()


def image(grid: dict, sum_wvis, sum_w, beam: bool = False, out=None, stream=None):
    """Dirty image of every rest channel of a stacked grid (``vista_image``): device tensors
    sum_wvis complex64 and sum_w float32 [nchan, nv, nu]; returns (image, beam or None,
    timings dict)."""
    import torch
    img = torch.empty(sum_w.shape, dtype=torch.float32, device=sum_w.device) if out is None else out
    bm = torch.empty_like(img) if beam else None
    tim = Timings()
    s = current_stream() if stream is None else stream
    _check(lib().vista_image(C.byref(grid_desc(grid)), _ptr(sum_wvis), _ptr(sum_w), _ptr(img), _ptr(bm), s,
                             C.byref(tim)))
    return img, bm, tim.as_dict()


def release_workspace():
    """Free the calling thread's cached launch workspace (``vista_release_workspace``)."""
    _check(lib().vista_release_workspace())


def image_noalloc(grid: dict, sum_wvis, sum_w, image, beam=None, stream=None):
    """``vista_image_noalloc``: the dirty images written into the given device tensors with
    no device allocation; only enqueued on the stream (torch's current one by default)."""
    s = current_stream() if stream is None else stream
    _check(lib().vista_image_noalloc(C.byref(grid_desc(grid)), _ptr(sum_wvis), _ptr(sum_w), _ptr(image),
                                     _ptr(beam), s))
