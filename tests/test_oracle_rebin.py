"""Pins of the oracle's per-row rebinned product (CPU only).

The paper's per-row kernel (Sec. 3.2) rebins each row of each target onto the target's own
output window (Sec. 3.1) with Eq. 3 and the Eq. 4 weights, after the Eq. 2 shift.  The C
oracle (``oracle.rebin_rows``, ``oracle.rebin_window``) is checked here against a second,
pure-Python implementation on tiny inputs and against closed forms that do not go through
either: aligned channels give back the input, half-shifted channels average neighbours, a
constant spectrum stays constant whatever the channel layout and flags, a point source at
the shifted position stays real, and the window placement of hand-computed bands.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import brute


def _dict_target(freq, width, z, nrow=5, npol=2, seed=0, l=0.0, m=0.0, vis=None, flag=None):
    rng = np.random.default_rng(seed)
    freq = np.asarray(freq, np.float64)
    n = freq.shape[0]
    if vis is None:
        vis = (rng.normal(size=(nrow, n, npol)) + 1j * rng.normal(size=(nrow, n, npol))).astype(np.complex64)
    uvw = rng.uniform(-800.0, 800.0, size=(nrow, 3))
    return dict(uvw=uvw, vis=vis, weight=np.ones((nrow, npol), np.float32), flag=flag, chan_freq=freq,
                chan_width=None if width is None else np.asarray(width, np.float64), l=l, m=m, z=z)


def _compare(o, b, scale):
    assert np.array_equal(o["flag"], b["flag"])
    assert np.max(np.abs(o["vis"] - b["vis"])) <= 1e-12 * scale
    assert np.max(np.abs(o["wsum"] - b["wsum"])) <= 1e-13
    assert np.array_equal(o["uvw"], b["uvw"])


@pytest.mark.parametrize("variant", ["plain", "descending", "jitter_width", "single_channel", "flags_heavy"])
@pytest.mark.parametrize("where", ["line", "low_edge", "high_edge", "wide"])
def test_rebin_brute_force_matches_oracle(variant, where):
    """A second implementation of the per-row definition on tiny random targets, with
    windows that fit, overhang either band edge, or are wider than the band."""
    cfg = synth.config("tiny")
    kw = {}
    if variant == "descending":
        kw = dict(descending=True)
    elif variant == "jitter_width":
        kw = dict(chan_jitter=0.4, with_width=True)
    elif variant == "single_channel":
        kw = dict(nchan=1, with_width=True)
    elif variant == "flags_heavy":
        cfg = synth.config("tiny", flag_frac=0.5)
    t = synth.make_target(cfg, 1, **kw)
    h = t.numpy()
    g = synth.make_grid(cfg)
    dfreq = g["dfreq"]
    nout = {"line": 6, "low_edge": 5, "high_edge": 5, "wide": 4 * len(h["chan_freq"]) + 3}[where]
    opz = 1.0 + float(h["z"])
    band_lo = float(np.min(h["chan_freq"])) * opz
    band_hi = float(np.max(h["chan_freq"])) * opz
    central = {"line": cfg.line_rest, "low_edge": band_lo - 3 * dfreq, "high_edge": band_hi + 3 * dfreq,
               "wide": cfg.line_rest}[where]
    lo_o = oracle.rebin_window(h, central, dfreq, nout)
    lo_b = brute.rebin_window(h["chan_freq"], h["chan_width"], float(h["z"]), central, dfreq, nout)
    assert lo_o == lo_b
    o = oracle.rebin_rows(h, lo_o, dfreq, nout)
    b = brute.rebin_rows(h, lo_o, dfreq, nout)
    _compare(o, b, float(np.max(np.abs(h["vis"]))))
    assert (o["flag"] == 0).any()


def test_rebin_aligned_channels_give_back_the_input():
    """Output channels equal to the rest-frame input channels (z = 1: observed 0.5 MHz
    channels become 1 MHz) and no offset: every output is its input channel, bit for bit,
    and a flagged input leaves its output flagged and zero."""
    freq = np.arange(50e6, 55e6, 0.5e6)
    flag = np.zeros((4, 10, 2), np.uint8)
    flag[1, 3, 0] = 1
    flag[2, :, 1] = 1
    t = _dict_target(freq, None, 1.0, nrow=4, flag=flag)
    o = oracle.rebin_rows(t, 99.5e6, 1e6, 10)
    want = t["vis"].astype(np.complex128)
    keep = flag == 0
    assert np.array_equal(o["vis"][keep], want[keep])
    assert np.array_equal(o["flag"], flag)
    assert np.all(o["vis"][~keep] == 0)
    assert np.all(o["wsum"][keep] == 1.0) and np.all(o["wsum"][~keep] == 0.0)


def test_rebin_half_shifted_channels_average_neighbours():
    """Output channels shifted by half an input channel: each interior output channel is
    the mean of its two input channels (f = 1/2 each); with one of them flagged, it is the
    other one alone.  The two outermost output channels see half a channel each."""
    freq = np.arange(100e6, 110e6, 1e6)          # rest edges 99.5 .. 109.5 MHz at z = 0
    flag = np.zeros((3, 10, 1), np.uint8)
    flag[0, 4, 0] = 1
    t = _dict_target(freq, None, 0.0, nrow=3, npol=1, flag=flag)
    o = oracle.rebin_rows(t, 99.0e6, 1e6, 11)    # output edges 99, 100, ..., 110 MHz
    v = t["vis"].astype(np.complex128)
    for r in range(3):
        for j in range(1, 10):
            a, b = v[r, j - 1, 0], v[r, j, 0]
            fa, fb = flag[r, j - 1, 0] == 0, flag[r, j, 0] == 0
            want = (a + b) / 2 if (fa and fb) else (a if fa else b)
            assert abs(o["vis"][r, j, 0] - want) <= 1e-15 * abs(want) + 1e-300
        assert o["vis"][r, 0, 0] == v[r, 0, 0] or flag[r, 0, 0]
        assert o["vis"][r, 10, 0] == v[r, 9, 0] or flag[r, 9, 0]
    assert o["wsum"][1, 5, 0] == 1.0 and o["wsum"][1, 0, 0] == 0.5
    assert o["wsum"][0, 4, 0] == 0.5 and o["wsum"][0, 5, 0] == 0.5   # one of the pair flagged


def test_rebin_constant_spectrum_is_preserved():
    """Eq. 3 is a normalised mean: a spectrum constant along the channels stays that
    constant in every output channel any unflagged input reaches, for irregular channel
    widths, any z and any flags."""
    rng = np.random.default_rng(3)
    freq = 40e9 + np.cumsum(rng.uniform(5e6, 9e6, size=40))
    width = rng.uniform(4e6, 9e6, size=40)
    c = (rng.normal(size=(6, 1, 2)) + 1j * rng.normal(size=(6, 1, 2))).astype(np.complex64)
    vis = np.broadcast_to(c, (6, 40, 2)).copy()
    flag = (rng.uniform(size=(6, 40, 2)) < 0.3).astype(np.uint8)
    t = _dict_target(freq, width, 1.7, nrow=6, vis=vis, flag=flag)
    lo = oracle.rebin_window(t, 40.15e9 * 2.7, 11e6 * 2.7, 24)
    o = oracle.rebin_rows(t, lo, 11e6 * 2.7, 24)
    keep = o["flag"] == 0
    assert keep.sum() > 100
    want = np.broadcast_to(c.astype(np.complex128), o["vis"].shape)
    assert np.max(np.abs(o["vis"] - want)[keep] / np.abs(want)[keep]) < 1e-14


@pytest.mark.parametrize("lm", [(10e-6, -4e-6), (0.01, -0.007)])
def test_rebin_point_source_stays_real(lm):
    """A noiseless point source at (l, m), shifted to (l, m) by Eq. 2 and rebinned by Eq. 3,
    is real in every output channel: Eq. 3's weights are real and the shift removes the
    whole phase (its sign and w-term included)."""
    cfg = synth.config("small", gauss_frac=0.0)
    t = synth.make_target(cfg, 2, noiseless=True, offset_lm=lm, no_flags=True)
    g = synth.make_grid(cfg)
    lo = oracle.rebin_window(t, cfg.line_rest, g["dfreq"], 40)
    o = oracle.rebin_rows(t, lo, g["dfreq"], 40)
    big = np.abs(o["vis"]) > 1e-3 * cfg.peak
    assert big.sum() > 100
    assert np.max(np.abs(o["vis"].imag)[big] / np.abs(o["vis"])[big]) < 1e-6
    assert np.all(o["vis"].real[big] > 0)


def test_rebin_window_placement_closed_forms():
    """Channels 100 .. 109 MHz of width 1 MHz at z = 1: rest band [199, 219] MHz.  Windows
    of 2 MHz channels: one that fits stays centred; one overhanging the top moves down to
    end at 219; one overhanging the bottom moves up to start at 199; one wider than the
    band starts at 199."""
    t = _dict_target(np.arange(100e6, 110e6, 1e6), None, 1.0)
    cases = [(210e6, 4, 206e6), (217e6, 4, 211e6), (200e6, 4, 199e6), (210e6, 20, 199e6)]
    for central, nout, want in cases:
        assert oracle.rebin_window(t, central, 2e6, nout) == want
        assert brute.rebin_window(t["chan_freq"], None, 1.0, central, 2e6, nout) == want


def test_rebin_uvw_is_the_rest_frame_baseline():
    """Eq. 1 without the rotation: the output baseline is the observed one over 1 + z, so in
    wavelengths at the rest frequency nu (1 + z) it equals the observed baseline at nu."""
    t = _dict_target(np.arange(100e6, 110e6, 1e6), None, 2.5)
    o = oracle.rebin_rows(t, 340e6, 3.5e6, 8)
    nu = 105e6
    lam_rest = o["uvw"] * (nu * 3.5) / 299792458.0
    lam_obs = t["uvw"] * nu / 299792458.0
    assert np.max(np.abs(lam_rest - lam_obs) / np.abs(lam_obs)) < 1e-15


def test_rebin_validation():
    t = _dict_target(np.arange(100e6, 110e6, 1e6), None, 1.0)
    with pytest.raises(ValueError):
        oracle.rebin_rows(t, 199e6, 2e6, 0)
    with pytest.raises(ValueError):
        oracle.rebin_rows(t, 199e6, 0.0, 4)
    with pytest.raises(ValueError):
        oracle.rebin_window(t, 210e6, -1.0, 4)
    with pytest.raises(ValueError):
        oracle.rebin_window(t, math.nan, 2e6, 4)
