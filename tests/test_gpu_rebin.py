"""GPU per-row rebinned product vs the FP64 oracle, through the C ABI.

Window edges, output flags and output baselines must be identical to the oracle's; each
rebinned visibility within 1e-5 of it, relative to its own Eq. 3 terms: the same
fraction-weighted mean taken of the input magnitudes, sum_k f_kj |V_k| / sum_k f_kj (the
oracle's rebinning of |V| with no shift), which bounds the output and scales the rounding
of each term; the Eq. 3 normalisers within 1e-6.  Cases span several workgroups with ragged
tails (window widths above, below and not a multiple of a workgroup), every polarisation
count, descending and irregular channel axes, windows that fit, overhang an edge of the
band or exceed it, a target at the 65535-channel limit, and the bench's full-size shape on
sampled rows.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_01897_amd import vista  # noqa: E402

TOL = 1e-5


def _term_scale(h, lo, dfreq, nout):
    """Per output: sum_k f_kj |V_k| / sum_k f_kj over its unflagged inputs -- the oracle's
    Eq. 3 rebinning of the input magnitudes, unshifted (l = m = 0 makes the phase 1)."""
    mag = dataclasses.replace(h, vis=h.vis.abs().to(torch.complex64), l=0.0, m=0.0, rotate_uvw=False)
    return np.abs(oracle.rebin_rows(mag, lo, dfreq, nout)["vis"])


def _compare(h, out, lo, ora, lo_ora, dfreq):
    """h: host target (synth.Target); out: the GPU outputs of it; ora: oracle outputs of it."""
    assert lo == lo_ora
    gv = out["vis"].cpu().numpy().astype(np.complex128)
    if out.get("flag") is not None:
        assert np.array_equal(out["flag"].cpu().numpy(), ora["flag"])
    live = ora["flag"] == 0
    scale = _term_scale(h, lo_ora, dfreq, ora["vis"].shape[1])
    assert np.all(scale[live] > 0)
    err = np.abs(gv - ora["vis"])[live] / scale[live] if live.any() else np.zeros(1)
    assert err.max() <= TOL, "max |dV| / (sum f |V| / sum f) = %g" % err.max()
    assert np.all(gv[ora["flag"] == 1] == 0)
    if out.get("wsum") is not None:
        ws = out["wsum"].cpu().numpy()
        assert np.max(np.abs(ws - ora["wsum"]) / np.maximum(ora["wsum"], 1.0)) <= 1e-6
    if out.get("uvw") is not None:
        assert np.array_equal(out["uvw"].cpu().numpy(), ora["uvw"])
    return float(err.max())


def _run(hs, nout, dfreq, central, **kw):
    ds = [h.to("cuda") for h in hs]
    outs, los, tim = vista.rebin_rows(ds, nout, dfreq, central, **kw)
    torch.cuda.synchronize()
    return outs, los, tim


@pytest.mark.parametrize("variant", ["plain", "descending", "jitter_width", "npol1", "npol4", "no_flags"])
@pytest.mark.parametrize("window", ["line", "fine", "narrow", "edge", "wide"])
def test_rebin_matches_oracle(variant, window):
    cfg = synth.config("small")
    kw = {}
    if variant == "descending":
        kw = dict(descending=True)
    elif variant == "jitter_width":
        kw = dict(chan_jitter=0.4, with_width=True)
    elif variant == "npol1":
        cfg = synth.config("small", npol=1)
    elif variant == "npol4":
        cfg = synth.config("small", npol=4)
    elif variant == "no_flags":
        kw = dict(no_flags=True)
    hs = synth.make_targets(cfg, **kw)
    g = synth.make_grid(cfg)
    # the recipe's rest width fits about 48-96 output channels in a target's band: a window
    # that fits; one of 300 channels of a tenth of that width (several output channels per
    # input channel); a narrow one; one centred beyond the band's top; one wider than it
    nout, dfreq, central = {"line": (40, g["dfreq"], cfg.line_rest),
                            "fine": (300, g["dfreq"] / 10, cfg.line_rest),
                            "narrow": (7, g["dfreq"], cfg.line_rest),
                            "edge": (40, g["dfreq"], cfg.line_rest * 1.05),
                            "wide": (300, g["dfreq"], cfg.line_rest)}[window]
    outs, los, tim = _run(hs, nout, dfreq, central)
    assert tim["accum_ms"] > 0
    for h, out, lo in zip(hs, outs, los):
        lo_ora = oracle.rebin_window(h, central, dfreq, nout)
        ora = oracle.rebin_rows(h, lo_ora, dfreq, nout)
        _compare(h, out, lo, ora, lo_ora, dfreq)
        assert (ora["flag"] == 0).any()


@pytest.mark.parametrize("window", ["line", "fine"])
def test_rebin_channel_axis_at_its_limit(window):
    """A target of 65535 channels, the most one target may have: each output channel
    averages hundreds ("fine") or thousands ("line") of input channels."""
    cfg = synth.config("small")
    g = synth.make_grid(cfg)
    h = synth.make_target(cfg, 1, nchan=65535, n_int=2)
    nout, dfreq = {"line": (40, g["dfreq"]), "fine": (300, g["dfreq"] / 10)}[window]
    outs, los, _ = _run([h], nout, dfreq, cfg.line_rest)
    lo_ora = oracle.rebin_window(h, cfg.line_rest, dfreq, nout)
    ora = oracle.rebin_rows(h, lo_ora, dfreq, nout)
    print(window, _compare(h, outs[0], los[0], ora, lo_ora, dfreq))
    assert (ora["flag"] == 0).any()


def test_rebin_mixed_polarisations_and_empty_target():
    """Targets with 1, 2 and 4 polarisations and one without rows in one call."""
    g = synth.make_grid("small")
    hs = [synth.make_target(synth.config("small", npol=p), i) for i, p in ((0, 1), (1, 2), (2, 4))]
    empty = synth.make_target("small", 3)
    empty = dataclasses.replace(empty, uvw=empty.uvw[:0], vis=empty.vis[:0], weight=empty.weight[:0],
                                flag=empty.flag[:0])
    hs.insert(1, empty)
    cfg = synth.config("small")
    outs, los, tim = _run(hs, 130, g["dfreq"], cfg.line_rest)
    assert tim["n_accum_launches"] == 3
    for h, out, lo in zip(hs, outs, los):
        lo_ora = oracle.rebin_window(h, cfg.line_rest, g["dfreq"], 130)
        if h.nrow == 0:
            assert out["vis"].numel() == 0
            continue
        _compare(h, out, lo, oracle.rebin_rows(h, lo_ora, g["dfreq"], 130), lo_ora, g["dfreq"])


def test_rebin_optional_outputs():
    """Only the visibilities are required; flags, normalisers and baselines are skipped."""
    cfg = synth.config("small")
    g = synth.make_grid(cfg)
    hs = synth.make_targets(cfg, n=2)
    outs, los, _ = _run(hs, 200, g["dfreq"], cfg.line_rest, want=("vis",))
    for h, out, lo in zip(hs, outs, los):
        assert out["flag"] is None and out["wsum"] is None and out["uvw"] is None
        ora = oracle.rebin_rows(h, lo, g["dfreq"], 200)
        _compare(h, out, lo, ora, oracle.rebin_window(h, cfg.line_rest, g["dfreq"], 200), g["dfreq"])


@pytest.mark.parametrize("lm", [(10e-6, -4e-6), (0.01, -0.007)])
def test_rebin_point_source_is_real(lm):
    """A noiseless point source at (l, m) comes out real in every output channel."""
    cfg = synth.config("small", gauss_frac=0.0)
    h = synth.make_target(cfg, 2, noiseless=True, offset_lm=lm, no_flags=True)
    g = synth.make_grid(cfg)
    outs, los, _ = _run([h], 60, g["dfreq"], cfg.line_rest)
    v = outs[0]["vis"].cpu().numpy()
    big = np.abs(v) > 1e-3 * cfg.peak
    assert big.sum() > 100
    assert np.max(np.abs(v.imag)[big] / np.abs(v)[big]) < 2e-6


def test_rebin_full_size_sampled_rows():
    """The bench's shape (the 50-target workload's targets, 903 baselines x 120 integrations
    x 960 channels x 2 pols, 480-channel windows of the common rest width around the line):
    every row computed on the GPU, 256 sampled rows of each of 4 targets checked against the
    oracle."""
    cfg = synth.config("c2")
    g = synth.make_grid(cfg)
    idx = [0, 17, 33, 49]
    ds = [synth.make_target(cfg, i, device="cuda") for i in idx]
    outs, los, tim = vista.rebin_rows(ds, 480, g["dfreq"], cfg.line_rest)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    for d, out, lo in zip(ds, outs, los):
        rows = np.sort(rng.choice(d.nrow, 256, replace=False))
        rt = torch.from_numpy(rows).to("cuda")
        sub = dataclasses.replace(d, uvw=d.uvw[rt].cpu(), vis=d.vis[rt].cpu(), weight=d.weight[rt].cpu(),
                                  flag=d.flag[rt].cpu())
        lo_ora = oracle.rebin_window(sub, cfg.line_rest, g["dfreq"], 480)
        ora = oracle.rebin_rows(sub, lo_ora, g["dfreq"], 480)
        o = {k: (None if v is None else v[rt]) for k, v in out.items()}
        _compare(sub, o, lo, ora, lo_ora, g["dfreq"])
        assert (ora["flag"] == 0).mean() > 0.9
