"""Host-side checks of the C ABI that need no GPU: every declared symbol is exported,
argument validation rejects bad inputs before any device work, and handle states."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from paper_2609_01897_amd import vista

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vista.h")).read()
    return sorted(set(re.findall(r"\b(vista_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = vista.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(vista.SYMBOLS), set(names) ^ set(vista.SYMBOLS)


def test_version():
    assert "gfx950" in vista.version()


def _grid(**kw):
    g = synth.make_grid("tiny")
    g.update(kw)
    return g


def _create(g):
    d = vista.grid_desc(g)
    h = C.c_void_p()
    return vista.lib().vista_stack_create(C.byref(d), None, C.byref(h)), h


@pytest.mark.parametrize("bad", [dict(nu=0), dict(nv=-3), dict(du=0.0), dict(dv=float("nan")), dict(nchan=0),
                                 dict(dfreq=-1.0), dict(freq_lo=float("inf")), dict(flags=1 << 9)])
def test_bad_grid_rejected(bad):
    rc, h = _create(_grid(**bad))
    assert rc == vista.VISTA_E_ARG
    assert vista.lib().vista_last_error()


def _target_variants():
    t = synth.make_target("tiny", 0)
    yield "z", dict(z=-1.0)
    yield "z_nan", dict(z=float("nan"))
    yield "lm", dict(l=0.8, m=0.6)
    f = t.chan_freq.copy(); f[3] = f[2]
    yield "nonmonotonic", dict(chan_freq=f)
    f = t.chan_freq.copy(); f[1] = -f[1]
    yield "negative_freq", dict(chan_freq=f)
    yield "single_no_width", dict(chan_freq=t.chan_freq[:1])
    yield "bad_width", dict(chan_width=np.full(t.nchan, -1.0))


@pytest.mark.parametrize("name,change", list(_target_variants()), ids=[n for n, _ in _target_variants()])
def test_bad_target_rejected(name, change):
    rc, h = _create(_grid())
    assert rc == 0
    t = synth.make_target("tiny", 0)
    for k, v in change.items():
        setattr(t, k, v)
    if name == "single_no_width":
        t.vis = t.vis[:, :1].contiguous(); t.flag = t.flag[:, :1].contiguous(); t.chan_width = None
    keep = []
    d = vista.target_desc(t, keep)
    assert vista.lib().vista_stack_add_target(h, C.byref(d)) == vista.VISTA_E_ARG
    # a rejected target changes nothing: the handle stays open
    good = synth.make_target("tiny", 1)
    d2 = vista.target_desc(good, keep)
    assert vista.lib().vista_stack_add_target(h, C.byref(d2)) == vista.VISTA_OK
    vista.lib().vista_stack_destroy(h)


def test_null_and_misaligned_arguments():
    L = vista.lib()
    g = vista.grid_desc(_grid())
    assert L.vista_stack_create(None, None, None) == vista.VISTA_E_ARG
    assert L.vista_stack_add_target(None, None) == vista.VISTA_E_ARG
    rc, h = _create(_grid())
    assert L.vista_stack_add_target(h, None) == vista.VISTA_E_ARG
    t = synth.make_target("tiny", 0)
    keep = []
    d = vista.target_desc(t, keep)
    d.vis = d.vis + 4            # complex64 pairs are read 16 bytes at a time
    assert L.vista_stack_add_target(h, C.byref(d)) == vista.VISTA_E_ARG
    d = vista.target_desc(t, keep)
    d.npol = 3
    assert L.vista_stack_add_target(h, C.byref(d)) == vista.VISTA_E_ARG
    d = vista.target_desc(t, keep)
    d.mem = 7
    assert L.vista_stack_add_target(h, C.byref(d)) == vista.VISTA_E_ARG
    tu = vista.Tuning(3, 3, 7, 4, 0)
    assert L.vista_stack_set_tuning(h, C.byref(tu)) == vista.VISTA_E_ARG
    assert L.vista_stack_destroy(h) == vista.VISTA_OK
    assert L.vista_stack_destroy(None) == vista.VISTA_E_ARG
    del g


def test_plan_spectral_grid_matches_paper_rule():
    f1 = 30e9 + np.arange(64) * 15.625e6
    f2 = (40e9 + np.arange(200) * 7.8125e6)[::-1].copy()
    lo, df = vista.plan_spectral_grid([f1, f2], [None, None], [2.5, 3.0], 115.2712018e9, 64)
    assert df == 15.625e6 * 3.5
    assert lo == 115.2712018e9 - 32 * df
    with pytest.raises(vista.VistaError):
        vista.plan_spectral_grid([f1[:1]], [None], [1.0], 1e9, 4)


def test_batch_validation():
    L = vista.lib()
    g1 = _grid()
    g2 = _grid(flags=vista.F_KAHAN)
    arr = (vista.GridDesc * 2)(vista.grid_desc(g1), vista.grid_desc(g2))
    h = C.c_void_p()
    assert L.vista_batch_create(2, arr, None, C.byref(h)) == vista.VISTA_E_ARG
    arr = (vista.GridDesc * 2)(vista.grid_desc(g1), vista.grid_desc(g1))
    assert L.vista_batch_create(2, arr, None, C.byref(h)) == vista.VISTA_OK
    t = synth.make_target("tiny", 0)
    keep = []
    d = vista.target_desc(t, keep)
    assert L.vista_batch_add_target(h, 5, C.byref(d)) == vista.VISTA_E_ARG
    assert L.vista_batch_add_target(h, 1, C.byref(d)) == vista.VISTA_OK
    out = vista.Output()
    assert L.vista_batch_finalize(h, 0, C.byref(out), None) == vista.VISTA_E_STATE
    assert L.vista_batch_destroy(h) == vista.VISTA_OK


def test_failure_paths_forced_from_host(monkeypatch):
    """Without a device (or with the injected faults) finalize fails cleanly, poisons the
    handle, and destroy still succeeds."""
    for env in ({"VISTA_FAULT_INJECT": "alloc"}, {"VISTA_DEVICE_MEM_LIMIT": "16"}):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        s = vista.Stack(_grid(), stream=None)
        s.add(synth.make_target("tiny", 0))
        with pytest.raises(vista.VistaError) as e:
            s.finalize(vista.alloc_outputs(_grid(), device="cpu"))
        assert e.value.code == vista.VISTA_E_NOMEM
        with pytest.raises(vista.VistaError) as e:
            s.add(synth.make_target("tiny", 1))
        assert e.value.code == vista.VISTA_E_STATE
        s.close()
        for k in env:
            monkeypatch.delenv(k)



def test_autotune_needs_device_targets():
    """Host-memory targets cannot be timed in place: the autotuner refuses them before any
    device work."""
    cfg = synth.config("tiny")
    g = synth.make_grid(cfg)
    s = vista.Stack(g)
    s.add(synth.make_target(cfg, 0))
    with pytest.raises(vista.VistaError) as e:
        s.autotune()
    assert e.value.code == vista.VISTA_E_ARG
    s.close()


@pytest.mark.parametrize("variant", ["plain", "descending", "jitter_width", "single_channel"])
def test_rebin_window_matches_oracle_bit_for_bit(variant):
    """The library's window edge (host FP64) equals the oracle's for windows that fit,
    overhang either end of the rest band, or are wider than it."""
    import oracle
    cfg = synth.config("small")
    kw = {"plain": {}, "descending": dict(descending=True), "jitter_width": dict(chan_jitter=0.4, with_width=True),
          "single_channel": dict(nchan=1, with_width=True)}[variant]
    g = synth.make_grid(cfg)
    for i in range(3):
        t = synth.make_target(cfg, i, **kw)
        opz = 1.0 + t.z
        for central, nout in ((cfg.line_rest, 40), (float(t.chan_freq.min()) * opz, 12),
                              (float(t.chan_freq.max()) * opz, 12), (cfg.line_rest, 5000)):
            lo = vista.rebin_window(t, nout, g["dfreq"], central)
            assert lo == oracle.rebin_window(t, central, g["dfreq"], nout)


def test_rebin_validation():
    """Bad descriptors, host-memory data and missing outputs are refused before any device
    work."""
    cfg = synth.config("tiny")
    g = synth.make_grid(cfg)
    t = synth.make_target(cfg, 0)
    for nout, dfreq, central in ((0, g["dfreq"], 1e11), (4, 0.0, 1e11), (4, -1.0, 1e11), (4, g["dfreq"], float("inf")),
                                 ((1 << 20) + 1, g["dfreq"], 1e11)):
        with pytest.raises(vista.VistaError) as e:
            vista.rebin_window(t, nout, dfreq, central)
        assert e.value.code == vista.VISTA_E_ARG
    with pytest.raises(vista.VistaError) as e:                 # host data
        vista.rebin_rows([t], 8, g["dfreq"], cfg.line_rest)
    assert e.value.code == vista.VISTA_E_ARG and "device" in str(e.value)
    d = vista.RebinDesc(8, g["dfreq"], cfg.line_rest)
    rc = vista.lib().vista_rebin_rows(C.byref(d), -1, None, None, None, None, None)
    assert rc == vista.VISTA_E_ARG
    rc = vista.lib().vista_rebin_rows(C.byref(d), 1, None, None, None, None, None)
    assert rc == vista.VISTA_E_ARG
    rc = vista.lib().vista_rebin_rows(C.byref(d), 0, None, None, None, None, None)   # nothing to do
    assert rc == vista.VISTA_OK


def test_rotation_fields_validated():
    """rotate_uvw must be 0 or 1; with it, the angles must be finite and the stacking
    position in the phase centre's front hemisphere (checked before any device work)."""
    import dataclasses
    import math
    cfg = synth.config("tiny")
    g = synth.make_grid(cfg)
    t = synth.make_target(cfg, 0)
    ok = dataclasses.replace(t, rotate_uvw=True)
    vista.rebin_window(ok, 8, g["dfreq"], cfg.line_rest)
    for bad in (dataclasses.replace(t, rotate_uvw=True, dec1=float("nan")),
                dataclasses.replace(t, rotate_uvw=True, ra1=t.ra0 + math.pi, dec1=-t.dec0)):
        with pytest.raises(vista.VistaError) as e:
            vista.rebin_window(bad, 8, g["dfreq"], cfg.line_rest)
        assert e.value.code == vista.VISTA_E_ARG
    d = vista.target_desc(t, [])
    d.rotate_uvw = 2
    lo = C.c_double()
    rd = vista.RebinDesc(8, g["dfreq"], cfg.line_rest)
    assert vista.lib().vista_rebin_window(C.byref(rd), C.byref(d), C.byref(lo)) == vista.VISTA_E_ARG


def test_image_validation():
    """Sizes that are not powers of two in 2..4096, missing arrays and host memory are
    refused before any device work."""
    g = dict(nu=64, nv=64, du=1.0, dv=1.0, nchan=2, freq_lo=1e9, dfreq=1e6)
    S = np.zeros((2, 64, 64), np.complex64)
    W = np.zeros((2, 64, 64), np.float32)
    img = np.zeros((2, 64, 64), np.float32)
    L = vista.lib()
    for bad in (dict(g, nu=48), dict(g, nv=1), dict(g, nu=8192), dict(g, nchan=0)):
        rc = L.vista_image(C.byref(vista.grid_desc(bad)), S.ctypes.data, W.ctypes.data, img.ctypes.data, None,
                           None, None)
        assert rc == vista.VISTA_E_ARG
    rc = L.vista_image(C.byref(vista.grid_desc(g)), None, W.ctypes.data, img.ctypes.data, None, None, None)
    assert rc == vista.VISTA_E_ARG
    rc = L.vista_image(C.byref(vista.grid_desc(g)), S.ctypes.data, W.ctypes.data, img.ctypes.data, None, None,
                       None)
    assert rc == vista.VISTA_E_ARG and "device" in vista.lib().vista_last_error().decode()


def test_too_fine_rest_grid_refused_at_add():
    """A rest grid so fine that an input channel would overlap more than 255 rest channels
    is refused when the target is added (planning of ordinary targets waits for the
    launch)."""
    cfg = synth.config("small")
    t = synth.make_target(cfg, 0)
    g = dict(synth.make_grid(cfg))
    g["dfreq"] = g["dfreq"] / 2000
    g["nchan"] = 200000
    g["freq_lo"] = cfg.line_rest - 0.5 * g["nchan"] * g["dfreq"]
    s = vista.Stack(g, stream=None)
    with pytest.raises(vista.VistaError) as e:
        s.add(t)
    assert e.value.code == vista.VISTA_E_ARG and "255" in str(e.value)
    s.close()



def _stack_and_drop(g, targets):
    s = vista.Stack(g)
    try:
        for t in targets:
            s.add(t)
    finally:
        s.close()


def test_background_planning_survives_drop_and_fork():
    """Targets are planned on library threads from add time on.  Dropping a stack right
    after its adds waits for that planning; a forked child, which has none of the parent's
    threads, plans on a pool of its own.  (The inputs are drawn before the fork: the child
    runs only the library.)"""
    import os
    import signal
    import time
    cfg = synth.config("small")
    g = synth.make_grid(cfg)
    targets = [synth.make_target(cfg, i) for i in range(6)]
    for _ in range(3):
        _stack_and_drop(g, targets)
    pid = os.fork()
    if pid == 0:
        code = 1
        try:
            _stack_and_drop(g, targets)
            code = 0
        finally:
            os._exit(code)
    deadline = time.time() + 60
    while True:
        done, status = os.waitpid(pid, os.WNOHANG)
        if done:
            break
        if time.time() > deadline:
            os.kill(pid, signal.SIGKILL)
            os.waitpid(pid, 0)
            pytest.fail("the forked child did not finish its adds")
        time.sleep(0.05)
    assert os.WIFEXITED(status) and os.WEXITSTATUS(status) == 0


def test_injected_launch_failure_is_raised_before_the_launch(monkeypatch):
    """VISTA_FAULT_INJECT=launch fails the next kernel launch from the host, before the
    kernel is enqueued: the call returns VISTA_E_HIP with the injected message."""
    monkeypatch.setenv("VISTA_FAULT_INJECT", "launch")
    src = np.zeros(64, np.uint8)
    dst = np.zeros(64, np.uint8)
    L = vista.lib()
    rc = L.vista_debug_copy(dst.ctypes.data, src.ctypes.data, 64, None)
    assert rc == vista.VISTA_E_HIP
    assert "injected launch failure" in L.vista_last_error().decode()
    monkeypatch.delenv("VISTA_FAULT_INJECT")
