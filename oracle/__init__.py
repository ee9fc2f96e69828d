"""FP64 CPU oracle for the ViSta stacking hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  The GPU library never does, and nothing here touches it.

``stack()`` wraps the C reference in ``vista_oracle.c`` (plain FP64 loops, see that
file's header for the definition and the paper passages it follows); ``brute`` holds a
second, pure-Python implementation of the same definition for tiny inputs.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

STAT_NAMES = ("n_samples", "n_flagged", "n_bad_weight", "n_outside_uv", "n_outside_band", "n_used",
              "n_contrib")
F_SPECTRAL_NEAREST = 4


class _Grid(C.Structure):
    _fields_ = [("nu", C.c_int32), ("nv", C.c_int32), ("nchan", C.c_int32), ("du", C.c_double),
                ("dv", C.c_double), ("freq_lo", C.c_double), ("dfreq", C.c_double),
                ("flags", C.c_uint32)]


class _Target(C.Structure):
    _fields_ = [("nrow", C.c_int64), ("nchan", C.c_int32), ("npol", C.c_int32),
                ("uvw", C.c_void_p), ("vis", C.c_void_p), ("weight", C.c_void_p),
                ("flag", C.c_void_p), ("chan_freq", C.c_void_p), ("chan_width", C.c_void_p),
                ("l", C.c_double), ("m", C.c_double), ("z", C.c_double),
                ("weight_per_chan", C.c_int32), ("kbeg", C.c_int32), ("kend", C.c_int32),
                ("rotate", C.c_int32), ("ra0", C.c_double), ("dec0", C.c_double), ("ra1", C.c_double),
                ("dec1", C.c_double), ("kdata", C.c_int32), ("kstride", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = C.CDLL(_build.LIB)
        p, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        _lib.ora_stack.argtypes = [C.POINTER(_Grid), i32, C.POINTER(_Target), i32, i32, p, p, p, p, p,
                                   C.c_int]
        _lib.ora_indices.argtypes = [C.POINTER(_Grid), C.POINTER(_Target), p, p, p, p]
        _lib.ora_rotate.argtypes = [C.POINTER(_Target), p]
        _lib.ora_channel_table.argtypes = [C.POINTER(_Grid), C.POINTER(_Target), p, p, p, p, p, p, p,
                                           C.POINTER(i32)]
        _lib.ora_plan_spectral_grid.argtypes = [i32, p, p, p, p, C.c_double, i32, C.POINTER(C.c_double),
                                                C.POINTER(C.c_double)]
        _lib.ora_check.argtypes = [C.POINTER(_Grid), i32, C.POINTER(_Target)]
        _lib.ora_frame_matrix.argtypes = [C.POINTER(_Target), p, p]
        _lib.ora_image.argtypes = [i32, i32, i32, p, p, p, p]
        _lib.ora_image_pixels.argtypes = [i32, i32, p, p, i32, p, p, p]
        _lib.ora_rebin_window.argtypes = [C.POINTER(_Target), C.c_double, C.c_double, i32, C.POINTER(C.c_double)]
        _lib.ora_rebin_rows.argtypes = [C.POINTER(_Target), C.c_double, C.c_double, i32, p, p, p, p]
    return _lib


def _grid(g: dict) -> _Grid:
    return _Grid(int(g["nu"]), int(g["nv"]), int(g["nchan"]), float(g["du"]), float(g["dv"]),
                 float(g["freq_lo"]), float(g["dfreq"]), int(g.get("flags", 0)))


def _host(t) -> dict:
    """Accept a synth.Target or a dict of arrays; return contiguous NumPy arrays."""
    d = t.numpy() if hasattr(t, "numpy") and not isinstance(t, dict) else dict(t)
    out = dict(d)
    out["uvw"] = np.ascontiguousarray(d["uvw"], dtype=np.float64)
    vis = np.asarray(d["vis"])
    if np.iscomplexobj(vis):
        vis = np.ascontiguousarray(vis.astype(np.complex64, copy=False)).view(np.float32)
    out["vis"] = np.ascontiguousarray(vis, dtype=np.float32)
    out["weight"] = np.ascontiguousarray(d["weight"], dtype=np.float32)
    out["flag"] = None if d.get("flag") is None else np.ascontiguousarray(d["flag"], dtype=np.uint8)
    out["chan_freq"] = np.ascontiguousarray(d["chan_freq"], dtype=np.float64)
    cw = d.get("chan_width")
    out["chan_width"] = None if cw is None else np.ascontiguousarray(cw, dtype=np.float64)
    out["kbeg"] = int(d.get("kbeg", 0))
    out["kend"] = int(d.get("kend", out["chan_freq"].shape[0]))
    # the data arrays may hold more channels than [kbeg, kend): [kdata, kdata + kstride)
    out["kdata"] = int(d.get("kdata", out["kbeg"]))
    out["kstride"] = int(d.get("kstride", 0))
    return out


def _target(h: dict) -> _Target:
    ptr = lambda a: None if a is None else a.ctypes.data
    nrow = int(h["uvw"].shape[0])
    nchan = int(h["chan_freq"].shape[0])
    npol = int(h["weight"].shape[-1])
    return _Target(nrow, nchan, npol, ptr(h["uvw"]), ptr(h["vis"]), ptr(h["weight"]), ptr(h["flag"]),
                   ptr(h["chan_freq"]), ptr(h["chan_width"]), float(h["l"]), float(h["m"]),
                   float(h["z"]), int(bool(h.get("weight_per_chan", False))), h["kbeg"], h["kend"],
                   int(bool(h.get("rotate_uvw", False))), float(h.get("ra0", 0.0)), float(h.get("dec0", 0.0)),
                   float(h.get("ra1", 0.0)), float(h.get("dec1", 0.0)), h["kdata"], h["kstride"])


def stack(grid: dict, targets, jlo: int = 0, jhi: int | None = None, stats: bool = True,
          threads: int = 0, want=("S", "W", "A", "N")) -> dict:
    """FP64 stack of ``targets`` over rest channels [jlo, jhi).

    Returns S (complex128), W, A (float64) and N (uint64) shaped [jhi-jlo, nv, nu], and
    the sample classification as a dict when ``stats``.
    """
    L = lib()
    jhi = int(grid["nchan"]) if jhi is None else int(jhi)
    hs = [_host(t) for t in targets]
    arr = (_Target * max(1, len(hs)))(*[_target(h) for h in hs])
    shape = (jhi - jlo, int(grid["nv"]), int(grid["nu"]))
    S = np.zeros(shape + (2,), np.float64) if "S" in want else None
    W = np.zeros(shape, np.float64) if "W" in want else None
    A = np.zeros(shape, np.float64) if "A" in want else None
    N = np.zeros(shape, np.uint64) if "N" in want else None
    st = np.zeros(7, np.uint64) if stats else None
    ptr = lambda a: None if a is None else a.ctypes.data
    g = _grid(grid)
    rc = L.ora_stack(C.byref(g), len(hs), arr, int(jlo), jhi, ptr(S), ptr(W), ptr(A), ptr(N), ptr(st),
                     int(threads))
    if rc:
        raise ValueError("oracle rejected the inputs (code %d)" % rc)
    out = dict(S=None if S is None else S.view(np.complex128)[..., 0], W=W, A=A, N=N)
    if stats:
        out["stats"] = {k: int(v) for k, v in zip(STAT_NAMES, st)}
    return out


def check(grid: dict, targets) -> bool:
    hs = [_host(t) for t in targets]
    arr = (_Target * max(1, len(hs)))(*[_target(h) for h in hs])
    g = _grid(grid)
    return lib().ora_check(C.byref(g), len(hs), arr) == 0


def indices(grid: dict, target) -> dict:
    """Per (row, channel) uv cell before the bounds test, first rest channel and |J_k|."""
    h = _host(target)
    t = _target(h)
    nk = h["kend"] - h["kbeg"]
    shape = (int(h["uvw"].shape[0]), nk)
    iu = np.zeros(shape, np.int64); iv = np.zeros(shape, np.int64)
    j0 = np.zeros(shape, np.int32); nj = np.zeros(shape, np.int32)
    g = _grid(grid)
    rc = lib().ora_indices(C.byref(g), C.byref(t), iu.ctypes.data, iv.ctypes.data, j0.ctypes.data,
                           nj.ctypes.data)
    if rc:
        raise ValueError("oracle rejected the inputs (code %d)" % rc)
    return dict(iu=iu, iv=iv, j0=j0, nj=nj)


def rotate(target) -> np.ndarray:
    """V' = V exp(+2 pi i t) for every sample, complex128 [nrow, nchan, npol]."""
    h = _host(target)
    t = _target(h)
    nk = h["kend"] - h["kbeg"]
    out = np.zeros((int(h["uvw"].shape[0]), nk, int(h["weight"].shape[-1]), 2), np.float64)
    if lib().ora_rotate(C.byref(t), out.ctypes.data):
        raise ValueError("oracle rejected the target")
    return out.view(np.complex128)[..., 0]


def channel_table(grid: dict, target) -> dict:
    """a_k, W_k, rest edges and J_k (CSR start/j/f) of one target."""
    h = _host(target)
    t = _target(h)
    g = _grid(grid)
    n = int(h["chan_freq"].shape[0])
    npairs = C.c_int32(0)
    L = lib()
    if L.ora_channel_table(C.byref(g), C.byref(t), None, None, None, None, None, None, None,
                           C.byref(npairs)):
        raise ValueError("oracle rejected the inputs")
    a = np.zeros(n); width = np.zeros(n); lo = np.zeros(n); hi = np.zeros(n)
    start = np.zeros(n + 1, np.int32)
    j = np.zeros(max(1, npairs.value), np.int32); f = np.zeros(max(1, npairs.value))
    L.ora_channel_table(C.byref(g), C.byref(t), a.ctypes.data, width.ctypes.data, lo.ctypes.data,
                        hi.ctypes.data, start.ctypes.data, j.ctypes.data, f.ctypes.data, C.byref(npairs))
    return dict(a=a, width=width, lo=lo, hi=hi, start=start, j=j[:npairs.value], f=f[:npairs.value])


def plan_spectral_grid(chan_freqs, chan_widths, zs, central_freq: float, nchan_out: int):
    """(freq_lo, dfreq) of the paper's common rest grid: widest rest channel, centred."""
    n = len(chan_freqs)
    fs = [np.ascontiguousarray(f, np.float64) for f in chan_freqs]
    ws = [None if w is None else np.ascontiguousarray(w, np.float64) for w in chan_widths]
    fp = (C.c_void_p * n)(*[f.ctypes.data for f in fs])
    wp = (C.c_void_p * n)(*[None if w is None else w.ctypes.data for w in ws])
    nc = np.asarray([f.shape[0] for f in fs], np.int32)
    zz = np.asarray(zs, np.float64)
    lo = C.c_double(0); df = C.c_double(0)
    rc = lib().ora_plan_spectral_grid(n, C.cast(fp, C.c_void_p), C.cast(wp, C.c_void_p),
                                      nc.ctypes.data, zz.ctypes.data, float(central_freq),
                                      int(nchan_out), C.byref(lo), C.byref(df))
    if rc:
        raise ValueError("oracle rejected the inputs")
    return lo.value, df.value


def rebin_window(target, central_freq: float, dfreq: float, nout: int) -> float:
    """Lower edge of the target's own output window of nout channels of width dfreq:
    centred on central_freq, moved to the nearest edge of its rest-frame band when it does
    not fit (``ora_rebin_window``)."""
    h = _host(target)
    t = _target(h)
    lo = C.c_double(0.0)
    if lib().ora_rebin_window(C.byref(t), float(central_freq), float(dfreq), int(nout), C.byref(lo)):
        raise ValueError("oracle rejected the inputs")
    return lo.value


def rebin_rows(target, freq_lo: float, dfreq: float, nout: int) -> dict:
    """The target's rows rebinned onto [freq_lo + j dfreq, freq_lo + (j+1) dfreq), j < nout
    (``ora_rebin_rows``): vis complex128 [nrow, nout, npol] (Eq. 3 per row, flagged inputs
    left out), flag uint8 (1 where nothing unflagged overlaps), wsum float64 (the Eq. 3
    normaliser), uvw float64 [nrow, 3] (divided by 1 + z)."""
    h = _host(target)
    t = _target(h)
    nrow, npol = int(h["uvw"].shape[0]), int(h["weight"].shape[-1])
    out = np.zeros((nrow, int(nout), npol, 2), np.float64)
    flag = np.zeros((nrow, int(nout), npol), np.uint8)
    wsum = np.zeros((nrow, int(nout), npol), np.float64)
    uvw = np.zeros((nrow, 3), np.float64)
    rc = lib().ora_rebin_rows(C.byref(t), float(freq_lo), float(dfreq), int(nout), out.ctypes.data,
                              flag.ctypes.data, wsum.ctypes.data, uvw.ctypes.data)
    if rc:
        raise ValueError("oracle rejected the inputs (code %d)" % rc)
    return dict(vis=out.view(np.complex128)[..., 0], flag=flag, wsum=wsum, uvw=uvw)


def rotation(target) -> tuple:
    """Eq. 1's rotation of the target as the oracle applies it: (R [3, 3], l, m, n - 1)."""
    h = _host(target)
    t = _target(h)
    R = np.zeros(9, np.float64)
    lm = np.zeros(3, np.float64)
    if lib().ora_frame_matrix(C.byref(t), R.ctypes.data, lm.ctypes.data):
        raise ValueError("oracle rejected the target")
    return R.reshape(3, 3), float(lm[0]), float(lm[1]), float(lm[2])


def image(S, W, beam: bool = False):
    """Dirty image of every channel of a stacked grid by direct Fourier inversion
    (``ora_image``): S complex [nchan, nv, nu], W [nchan, nv, nu] -> image float64
    [nchan, nv, nu] (and the dirty beam)."""
    S = np.ascontiguousarray(np.asarray(S, np.complex128))
    W = np.ascontiguousarray(np.asarray(W, np.float64))
    nchan, nv, nu = W.shape
    img = np.zeros(W.shape, np.float64)
    bm = np.zeros(W.shape, np.float64) if beam else None
    if lib().ora_image(nu, nv, nchan, S.ctypes.data, W.ctypes.data, img.ctypes.data,
                       None if bm is None else bm.ctypes.data):
        raise ValueError("oracle rejected the inputs")
    return (img, bm) if beam else img


def image_pixels(S, W, q, p):
    """Selected pixels (q[i], p[i]) of one channel's dirty image (``ora_image_pixels``)."""
    S = np.ascontiguousarray(np.asarray(S, np.complex128))
    W = np.ascontiguousarray(np.asarray(W, np.float64))
    q = np.ascontiguousarray(q, np.int32)
    p = np.ascontiguousarray(p, np.int32)
    nv, nu = W.shape
    out = np.zeros(q.shape[0], np.float64)
    if lib().ora_image_pixels(nu, nv, S.ctypes.data, W.ctypes.data, int(q.shape[0]), q.ctypes.data,
                              p.ctypes.data, out.ctypes.data):
        raise ValueError("oracle rejected the inputs")
    return out
