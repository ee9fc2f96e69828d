"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-derived values
(tests/golden), closed forms (Eq. 2 phase shift of a point or Gaussian source, Eq. 4
overlap fractions), invariants (conservation of weight and flux through the
rebinning, z-independence of the uv cell), textbook special cases (plain
nearest-grid-point gridding), brute force on tiny inputs, and a direct-DFT image of a
stack.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import brute
from synth.configs import C_LIGHT, F_CO10

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "handworked.json")


def _golden_target(t):
    re = np.asarray(t["vis_re"], np.float32)
    im = np.asarray(t["vis_im"], np.float32)
    return dict(uvw=np.asarray(t["uvw"], np.float64), vis=(re + 1j * im).astype(np.complex64),
                weight=np.asarray(t["weight"], np.float32), flag=np.asarray(t["flag"], np.uint8),
                chan_freq=np.asarray(t["chan_freq"], np.float64), chan_width=t["chan_width"],
                l=t["l"], m=t["m"], z=t["z"])


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_golden_handworked(case):
    g = case["grid"]
    o = oracle.stack(g, [_golden_target(case["target"])])
    nz = np.argwhere(o["N"] > 0)
    assert len(nz) == len(case["expect"])
    for e in case["expect"]:
        c = (e["j"], e["iv"], e["iu"])
        assert o["S"][c] == complex(e["S_re"], e["S_im"])
        assert o["W"][c] == e["W"]
        assert int(o["N"][c]) == e["N"]
        a = sum(wf * math.sqrt(m2) for wf, m2 in e["A_terms"])
        assert abs(o["A"][c] - a) <= 1e-14 * a
    assert o["stats"] == case["stats"]


def _brute_vs_oracle(grid, targets):
    hs = [t.numpy() for t in targets]
    b = brute.stack(grid, hs)
    o = oracle.stack(grid, targets)
    assert o["stats"] == b["stats"]
    nz = {tuple(int(x) for x in c) for c in np.argwhere(o["N"] > 0)}
    assert nz == set(b["cells"].keys())
    for key, (S, W, A, N) in b["cells"].items():
        assert int(o["N"][key]) == N
        assert abs(o["S"][key] - S) <= 1e-13 * max(A, 1e-300)
        assert abs(o["W"][key] - W) <= 1e-13 * W
        assert abs(o["A"][key] - A) <= 1e-13 * A


@pytest.mark.parametrize("variant", ["plain", "descending", "jitter_width", "perchan_badw", "nearest",
                                     "odd_small_grid"])
def test_brute_force_matches_oracle(variant):
    """T1: a second implementation of the definition on tiny random inputs."""
    cfg = synth.config("tiny")
    kw = {}
    flags = 0
    grid = synth.make_grid(cfg)
    if variant == "descending":
        kw = dict(descending=True)
    elif variant == "jitter_width":
        kw = dict(chan_jitter=0.4, with_width=True)
    elif variant == "perchan_badw":
        kw = dict(weight_per_chan=True, bad_weight_frac=0.2)
    elif variant == "nearest":
        flags = oracle.F_SPECTRAL_NEAREST
        grid = synth.make_grid(cfg, flags)
    elif variant == "odd_small_grid":
        # a grid smaller than the uv coverage and a rest band narrower than the data
        grid = dict(grid, nu=7, nv=5, du=grid["du"] * 1.3, nchan=5,
                    freq_lo=grid["freq_lo"] + 2 * grid["dfreq"])
    targets = synth.make_targets(cfg, **kw)
    _brute_vs_oracle(grid, targets)


def test_single_channel_with_width():
    cfg = synth.config("tiny")
    t = synth.make_target(cfg, 0, nchan=1, with_width=True)
    assert t.chan_width is not None
    _brute_vs_oracle(synth.make_grid(cfg), [t])


def test_zero_offset_is_identity():
    """T2: with l = m = 0 the Eq. 2 phasor is exactly 1 and V' is bit-identical to V."""
    t = synth.make_target("small", 1, offset_lm=(0.0, 0.0))
    rot = oracle.rotate(t)
    v = t.vis.numpy().astype(np.complex128)
    assert np.array_equal(rot, v)


def _line(cfg, nu_rest):
    vel = C_LIGHT * (cfg.line_rest - nu_rest) / cfg.line_rest / 1e3
    return cfg.peak * np.exp(-4.0 * math.log(2.0) * (vel / cfg.fwhm_kms) ** 2)


@pytest.mark.parametrize("lm", [(10e-6, -4e-6), (0.01, -0.007), (-0.2, 0.15)])
def test_point_source_becomes_real_constant(lm):
    """T3: a noiseless point source at (l, m) rotates to the real spectrum S(nu).

    Checks the sign of the Eq. 2 exponent and the w-term: at the larger offsets
    w (n-1) is many turns, so dropping or mis-signing any term leaves a phase.
    """
    cfg = synth.config("small", gauss_frac=0.0)
    t = synth.make_target(cfg, 2, noiseless=True, offset_lm=lm, no_flags=True)
    rot = oracle.rotate(t)
    spec = _line(cfg, t.chan_freq * (1.0 + t.z))
    mask = spec > 1e-3 * cfg.peak
    ref = np.broadcast_to(spec[None, :, None], rot.shape)
    err = np.abs(rot - ref)[:, mask, :] / ref[:, mask, :]
    assert err.max() < 1e-6, err.max()


def test_gaussian_source_becomes_real_gaussian():
    """T4: a noiseless Gaussian source rotates to S(nu) exp(-pi^2 theta^2 |u|^2 / (4 ln 2))."""
    cfg = synth.config("small", gauss_frac=1.0, gauss_fwhm=2.0 * synth.configs.ARCSEC)
    t = synth.make_target(cfg, 0, noiseless=True, offset_lm=(3e-4, 2e-4), no_flags=True)
    rot = oracle.rotate(t)
    uvw = t.uvw.numpy()
    lam_inv = t.chan_freq / C_LIGHT
    q = (uvw[:, 0:1] ** 2 + uvw[:, 1:2] ** 2) * lam_inv[None, :] ** 2
    th = cfg.gauss_fwhm
    ref = _line(cfg, t.chan_freq * (1.0 + t.z))[None, :] * np.exp(-math.pi ** 2 * th * th * q / (4 * math.log(2)))
    ref = ref[:, :, None]
    big = np.broadcast_to(ref > 1e-3 * cfg.peak, rot.shape)
    assert (np.abs(rot - ref)[big] / np.broadcast_to(ref, rot.shape)[big]).max() < 1e-6


def test_conservation_of_weight_and_flux():
    """T5: every channel inside the band splits with fractions summing to one, so
    sum over cells of W equals the sum of usable weights, and sum of S equals the sum
    of w V' over usable samples."""
    cfg = synth.config("c1")
    ts = synth.make_targets(cfg, n=3)
    g = synth.make_grid(cfg)
    o = oracle.stack(g, ts)
    wsum = 0.0
    ssum = 0.0 + 0.0j
    for t in ts:
        tab = oracle.channel_table(g, t)
        fsum = np.add.reduceat(tab["f"], tab["start"][:-1])
        assert np.allclose(fsum, 1.0, rtol=0, atol=1e-12)
        w = np.broadcast_to(t.weight.numpy()[:, None, :], t.vis.shape).astype(np.float64)
        use = t.flag.numpy() == 0
        wsum += w[use].sum()
        ssum += (w * oracle.rotate(t))[use].sum()
    assert abs(o["W"].sum() - wsum) <= 1e-12 * wsum
    assert abs(o["S"].sum() - ssum) <= 1e-12 * o["A"].sum()
    assert int(o["N"].sum()) == o["stats"]["n_contrib"]
    st = o["stats"]
    assert st["n_samples"] == sum(st[k] for k in ("n_flagged", "n_bad_weight", "n_outside_uv",
                                                    "n_outside_band", "n_used"))


def _one_chan_target(freq, width, z, uvw=((10.0, 5.0, 1.0),)):
    freq = np.asarray(freq, np.float64)
    n = freq.shape[0]
    return dict(uvw=np.asarray(uvw, np.float64), vis=np.ones((len(uvw), n, 1), np.complex64),
                weight=np.ones((len(uvw), 1), np.float32), flag=None, chan_freq=freq,
                chan_width=None if width is None else np.asarray(width, np.float64), l=0.0, m=0.0, z=z)


def test_overlap_closed_forms():
    """T6: Eq. 4 on aligned, half-shifted, touching and sliver channels; rest scaling."""
    g = dict(nu=8, nv=8, du=1.0, dv=1.0, nchan=10, freq_lo=99.5e6, dfreq=1e6, flags=0)
    # aligned: rest channels coincide with output channels -> one pair, f = 1
    tab = oracle.channel_table(g, _one_chan_target(np.arange(100e6, 110e6, 1e6), None, 0.0))
    assert np.array_equal(np.diff(tab["start"]), np.ones(10, np.int32))
    assert np.array_equal(tab["j"], np.arange(10)) and np.all(tab["f"] == 1.0)
    # half shift -> (0.5, 0.5) in two neighbouring channels, except the top one (half outside)
    tab = oracle.channel_table(g, _one_chan_target(np.arange(100.5e6, 109.5e6, 1e6), None, 0.0))
    assert np.array_equal(np.diff(tab["start"]), np.full(9, 2, np.int32))
    assert np.all(tab["f"] == 0.5)
    # rest frame: observed 50 MHz channels of width 0.5 MHz at z = 1 -> rest 1 MHz, aligned
    tab = oracle.channel_table(g, _one_chan_target(np.arange(50e6, 55e6, 0.5e6), None, 1.0))
    assert np.array_equal(tab["j"], np.arange(10)) and np.all(tab["f"] == 1.0)
    assert np.all(tab["hi"] - tab["lo"] == 1e6)
    # touching: a channel ending exactly at freq_lo contributes nothing
    tab = oracle.channel_table(g, _one_chan_target([99.0e6], [1e6], 0.0))
    assert tab["start"][-1] == 0
    # sliver: overlap of 1e-10 of the width is dropped, 1e-8 is kept
    for frac, keep in ((1e-10, 0), (1e-8, 1)):
        tab = oracle.channel_table(g, _one_chan_target([99.0e6 + frac * 1e6], [1e6], 0.0))
        assert tab["start"][-1] == keep
    # centred finite-difference widths of a non-uniform axis, one-sided at the ends
    f = np.array([100e6, 100.5e6, 101.5e6, 103.5e6])
    tab = oracle.channel_table(g, _one_chan_target(f, None, 0.0))
    assert np.array_equal(tab["width"], [0.5e6, 0.75e6, 1.5e6, 2e6])


def test_textbook_gridding_special_case():
    """T7: z = 0, l = m = 0 and output channels equal to the input channels reduce the
    stack to nearest-grid-point gridding: add w V at (k, rint(v/dv)+n/2, rint(u/du)+n/2)."""
    cfg = synth.config("small")
    t = synth.make_target(cfg, 3, z=0.0, offset_lm=(0.0, 0.0))
    nch = t.nchan
    dnu = t.chan_freq[1] - t.chan_freq[0]
    du = 2.0 ** round(math.log2(synth.make_grid(cfg)["du"]))     # exact reciprocal
    n = 64
    g = dict(nu=n, nv=n, du=du, dv=du, nchan=nch, freq_lo=t.chan_freq[0] - 0.5 * dnu, dfreq=dnu,
             flags=oracle.F_SPECTRAL_NEAREST)
    o = oracle.stack(g, [t])
    h = t.numpy()
    lam = h["chan_freq"] / C_LIGHT
    iu = np.rint(h["uvw"][:, 0:1] * lam[None, :] / du).astype(np.int64) + n // 2
    iv = np.rint(h["uvw"][:, 1:2] * lam[None, :] / du).astype(np.int64) + n // 2
    inside = (iu >= 0) & (iu < n) & (iv >= 0) & (iv < n)
    S = np.zeros((nch, n, n), np.complex128)
    W = np.zeros((nch, n, n))
    N = np.zeros((nch, n, n), np.int64)
    kk = np.broadcast_to(np.arange(nch)[None, :], iu.shape)
    for p in range(h["vis"].shape[2]):
        use = inside & (h["flag"][:, :, p] == 0)
        w = np.broadcast_to(h["weight"][:, None, p].astype(np.float64), iu.shape)
        idx = (kk[use], iv[use], iu[use])
        np.add.at(S, idx, (w * h["vis"][:, :, p].astype(np.complex128))[use])
        np.add.at(W, idx, w[use])
        np.add.at(N, idx, 1)
    assert inside.sum() > 0.5 * inside.size
    assert np.array_equal(o["N"].astype(np.int64), N)
    assert np.allclose(o["S"], S, rtol=0, atol=1e-12 * np.abs(S).max())
    assert np.allclose(o["W"], W, rtol=1e-14, atol=0)


def test_uv_cell_is_independent_of_z():
    """T8: u_lambda = u_m nu_obs / c does not change with the redshift; only j moves."""
    cfg = synth.config("c1")
    g = synth.make_grid(cfg)
    t2 = synth.make_target(cfg, 0, z=2.1)
    t3 = synth.make_target(cfg, 0, z=2.1)
    t3.z = 2.8
    a = oracle.indices(g, t2)
    b = oracle.indices(g, t3)
    assert np.array_equal(a["iu"], b["iu"]) and np.array_equal(a["iv"], b["iv"])
    assert not np.array_equal(a["j0"], b["j0"])


def test_thread_count_and_slabs_do_not_change_results():
    cfg = synth.config("c1")
    ts = synth.make_targets(cfg, n=2)
    g = synth.make_grid(cfg)
    o1 = oracle.stack(g, ts, threads=1)
    o8 = oracle.stack(g, ts, threads=8)
    for k in ("S", "W", "A", "N"):
        assert np.array_equal(o1[k], o8[k])
    o = oracle.stack(g, ts, jlo=20, jhi=37, threads=3)
    for k in ("S", "W", "A", "N"):
        assert np.array_equal(o[k], o1[k][20:37])


def test_channel_slices_add_up():
    cfg = synth.config("small")
    t = synth.make_target(cfg, 1)
    g = synth.make_grid(cfg)
    full = oracle.stack(g, [t])
    cuts = [0, 17, 60, t.nchan]
    parts = [oracle.stack(g, [t.channel_slice(a, b)]) for a, b in zip(cuts[:-1], cuts[1:])]
    N = sum(p["N"] for p in parts)
    S = sum(p["S"] for p in parts)
    W = sum(p["W"] for p in parts)
    assert np.array_equal(N, full["N"])
    assert np.allclose(S, full["S"], rtol=0, atol=1e-12 * full["A"].max())
    assert np.allclose(W, full["W"], rtol=1e-12, atol=0)
    for k in oracle.STAT_NAMES:
        assert sum(p["stats"][k] for p in parts) == full["stats"][k]



@pytest.mark.parametrize("perchan", [False, True])
def test_strided_channel_view_equals_copied_slice(perchan):
    """A channel range read in place from the full data arrays (kdata = 0, kstride = nchan)
    gives the same bits as the same range copied out (an indexing change only)."""
    cfg = synth.config("small")
    t = synth.make_target(cfg, 2, weight_per_chan=perchan, bad_weight_frac=0.05 if perchan else 0.0)
    g = synth.make_grid(cfg)
    k0, k1 = 23, t.nchan - 31
    copied = oracle.stack(g, [t.channel_slice(k0, k1)])
    view = dict(t.numpy(), kbeg=k0, kend=k1, kdata=0, kstride=t.nchan)
    strided = oracle.stack(g, [view])
    for k in ("S", "W", "A", "N"):
        assert np.array_equal(strided[k], copied[k])
    assert strided["stats"] == copied["stats"]
    with pytest.raises(ValueError):
        oracle.stack(g, [dict(view, kdata=k0 + 1)])      # the view must hold [kbeg, kend)

def _stacked_line(cfg, n_targets=4):
    ts = synth.make_targets(cfg, n=n_targets, noiseless=True)
    g = synth.make_grid(cfg)
    return g, ts, oracle.stack(g, ts)


def test_rest_frame_line_lands_on_its_rest_channel():
    """Sec. 3.1: nu_rest = nu_obs (1+z).  Lines observed at different z stack at the
    rest frequency: the stacked spectrum peaks in the channel holding it."""
    cfg = synth.config("c1", gauss_frac=0.0)
    g, ts, o = _stacked_line(cfg)
    spec = o["S"].sum(axis=(1, 2)).real / np.maximum(o["W"].sum(axis=(1, 2)), 1e-300)
    j_line = (F_CO10 - g["freq_lo"]) / g["dfreq"]
    jp = int(np.argmax(spec))
    assert abs((jp + 0.5) - j_line) <= 1.0
    # the line centre sits on the edge between two rest channels: both hold the mean of
    # the profile over half a FWHM-sized channel (about 0.79 of the peak)
    jl = int(round(j_line))
    assert 0.95 < spec[jl - 1] / spec[jl] < 1.05
    assert spec[jp] > 0.7 * cfg.peak
    assert spec[jl + 4] < 0.1 * spec[jp] and spec[jl - 5] < 0.1 * spec[jp]


def _dft_image(g, S, W, pix, npix):
    """Direct DFT of the channel-summed grid: I(x, y) = Re sum S exp(2 pi i (u x + v y)) / sum W."""
    Ssum = S.sum(axis=0)
    Wsum = W.sum()
    iv, iu = np.nonzero(np.abs(Ssum) > 0)
    u = (iu - g["nu"] // 2) * g["du"]
    v = (iv - g["nv"] // 2) * g["dv"]
    s = Ssum[iv, iu]
    xs = (np.arange(npix) - npix // 2) * pix
    img = np.zeros((npix, npix))
    for a, y in enumerate(xs):
        for b, x in enumerate(xs):
            img[a, b] = (s * np.exp(2j * np.pi * (u * x + v * y))).real.sum() / Wsum
    return img, xs


@pytest.mark.parametrize("noisy", [False, True])
def test_dft_image_recovers_injected_source(noisy):
    """T17: a direct-DFT image of a small stack peaks at the phase centre, where every
    target's source was moved, with the injected flux (noiseless) or within 5 sigma."""
    cfg = synth.config("c1", gauss_frac=0.0, offset=8 * synth.configs.ARCSEC, peak=0.05,
                       sigma=0.02 if noisy else 1e-3)
    ts = synth.make_targets(cfg, n=4, noiseless=not noisy)
    g = synth.make_grid(cfg)
    # continuum-like: channels within the line core only
    o = oracle.stack(g, ts, jlo=28, jhi=36)
    fov = 1.0 / g["du"]
    pix = fov / 64
    img, xs = _dft_image(g, o["S"], o["W"], pix, 21)
    a, b = np.unravel_index(np.argmax(img), img.shape)
    assert abs(a - 10) <= 1 and abs(b - 10) <= 1
    spec = o["S"].sum(axis=(1, 2)).real / o["W"].sum(axis=(1, 2))
    expect = (o["W"].sum(axis=(1, 2)) * spec).sum() / o["W"].sum()
    if not noisy:
        assert abs(img[10, 10] - expect) <= 1e-6 * expect
        # the source sits at the centre only because of the rotation: with l, m negated
        # it lands twice as far away
        bad = [synth.make_target(cfg, i, noiseless=True) for i in range(4)]
        for t in bad:
            t.l, t.m = -t.l, -t.m
        ob = oracle.stack(g, bad, jlo=28, jhi=36)
        imb, _ = _dft_image(g, ob["S"], ob["W"], pix, 21)
        assert imb[10, 10] < 0.5 * img[10, 10]
    else:
        nvis = o["W"].sum() / (1.0 / cfg.sigma ** 2)
        sig = cfg.sigma / math.sqrt(nvis)
        assert abs(img[a, b] - cfg.peak * expect / cfg.peak) < 5 * sig + 0.05 * expect


def test_plan_spectral_grid_closed_form():
    """Sec. 3.1: Delta nu_new = max_i Delta nu_rf,i, grid centred on central_freq."""
    f1 = 30e9 + np.arange(64) * 15.625e6
    f2 = 40e9 + np.arange(200) * 7.8125e6
    lo, df = oracle.plan_spectral_grid([f1, f2], [None, None], [2.5, 3.0], F_CO10, 64)
    assert df == 15.625e6 * 3.5
    assert lo == F_CO10 - 32 * df


def test_validation():
    g = synth.make_grid("tiny")
    good = synth.make_target("tiny", 0).numpy()
    assert oracle.check(g, [good])
    assert not oracle.check(g, [dict(good, z=-1.0)])
    assert not oracle.check(g, [dict(good, l=0.8, m=0.6)])
    one = dict(good, chan_freq=good["chan_freq"][:1], vis=good["vis"][:, :1], flag=good["flag"][:, :1])
    assert not oracle.check(g, [one])
    assert oracle.check(g, [dict(one, chan_width=np.array([1e6]))])
    assert not oracle.check(dict(g, du=0.0), [good])
