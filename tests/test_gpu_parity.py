"""GPU path vs the FP64 oracle, through the C ABI.

Indices and counts must be identical; stacked sums within 1e-5 of the oracle (relative to
the cell scale A = sum |w f V'| for S, and to W for W).  Cases span several tiles and
rest-channel blocks with ragged edges, the edge layouts of the channel axis, every
accumulation mode, and the batched form.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_01897_amd import vista  # noqa: E402
from tests.gpu_util import compare, compare_fp32_plain, gpu_stack, targets_on_gpu  # noqa: E402

MODES = {"atomic": 0, "deterministic": vista.F_DETERMINISTIC, "kahan": vista.F_KAHAN,
         "deterministic_kahan": vista.F_DETERMINISTIC | vista.F_KAHAN, "plain_fp32": vista.F_PLAIN_FP32}


@pytest.mark.parametrize("mode", list(MODES))
def test_c1_matches_oracle(mode):
    """The 8-target correctness workload, every accumulation mode."""
    cfg = synth.config("c1")
    hs, ds = targets_on_gpu(cfg)
    g = synth.make_grid(cfg)
    o = oracle.stack(g, hs)
    out, st = gpu_stack(g, ds, flags=MODES[mode])
    err = compare(o, out, st=st)
    print(mode, err)


def test_debug_indices_bit_exact():
    """Cell (iu, iv), first rest channel and overlap count per (row, channel)."""
    cfg = synth.config("small")
    g = synth.make_grid(cfg)
    for i in range(2):
        h = synth.make_target(cfg, i, chan_jitter=0.3)
        gi = vista.debug_indices(g, h.to("cuda"))
        oi = oracle.indices(g, h)
        assert np.array_equal(gi["iu"].astype(np.int64), oi["iu"])
        assert np.array_equal(gi["iv"].astype(np.int64), oi["iv"])
        assert np.array_equal(gi["j0"], oi["j0"])
        assert np.array_equal(gi["nj"], oi["nj"])


def test_long_channel_axes():
    """Targets of 2500 and 4100 channels next to a short one.  Binning stages a block's
    channel scales in LDS only up to 2048 channels, so these rows search the channel table
    in global memory instead."""
    cfg = synth.config("small")
    g = synth.make_grid(cfg)
    hs = [synth.make_target(cfg, 0, nchan=2500, n_int=8), synth.make_target(cfg, 1, nchan=4100, n_int=6),
          synth.make_target(cfg, 2)]
    o = oracle.stack(g, hs)
    out, st = gpu_stack(g, [h.to("cuda") for h in hs])
    err = compare(o, out, st=st)
    print(err)


@pytest.mark.parametrize("mode", ["atomic", "deterministic"])
def test_channel_axis_at_its_limit(mode):
    """A target of 65535 channels, the most one target may have (a record's channel bounds
    then reach 65535), next to a short one; thousands of its channels overlap each rest
    channel."""
    cfg = synth.config("small")
    g = synth.make_grid(cfg)
    hs = [synth.make_target(cfg, 1, nchan=65535, n_int=2), synth.make_target(cfg, 2)]
    o = oracle.stack(g, hs)
    out, st = gpu_stack(g, [h.to("cuda") for h in hs], flags=MODES[mode])
    compare(o, out, st=st)


def test_boundary_samples_bit_exact():
    """Samples placed exactly on cell edges and one ulp either side of them."""
    cfg = synth.config("small")
    g = dict(synth.make_grid(cfg))
    h = synth.make_target(cfg, 0)
    a = h.chan_freq / 299792458.0
    uvw = h.uvw.numpy().copy()
    k = h.nchan // 2
    # u_lambda exactly (i + 1/2) du at channel k, and nudged by +-1 ulp in metres
    for r in range(min(uvw.shape[0], 300)):
        half = ((r % 40) - 20 + 0.5) * g["du"] / a[k]
        uvw[r, 0] = np.nextafter(half, np.inf * ((r // 40) % 3 - 1)) if (r // 40) % 3 != 1 else half
        uvw[r, 1] = -half
    h.uvw = torch.from_numpy(uvw)
    gi = vista.debug_indices(g, h.to("cuda"))
    oi = oracle.indices(g, h)
    assert np.array_equal(gi["iu"].astype(np.int64), oi["iu"])
    assert np.array_equal(gi["iv"].astype(np.int64), oi["iv"])
    o = oracle.stack(g, [h])
    out, st = gpu_stack(g, [h.to("cuda")])
    compare(o, out, st=st)


@pytest.mark.parametrize("mode", ["atomic", "plain_fp32", "deterministic"])
def test_channels_cut_by_the_rest_grid(mode):
    """A rest grid that covers only the middle of the targets' bands, its edges at a
    fraction of a rest channel: the channels at both ends overlap the grid only in part,
    so their second overlap fraction is not one minus the first (Eq. 4), and the kernels
    must take it from the table, not derive it."""
    cfg = synth.config("small")
    g = dict(synth.make_grid(cfg))
    hs = synth.make_targets(cfg, n=4)
    g["freq_lo"] = g["freq_lo"] + (g["nchan"] // 4 + 0.37) * g["dfreq"]
    g["nchan"] = g["nchan"] // 2
    o = oracle.stack(g, hs)
    assert o["stats"]["n_outside_band"] > 0
    out, st = gpu_stack(g, [h.to("cuda") for h in hs], flags=MODES[mode])
    if mode == "plain_fp32":
        compare_fp32_plain(o, out)
    else:
        compare(o, out, st=st)


def test_zero_offset_rotation_is_identity():
    h = synth.make_target("small", 1, offset_lm=(0.0, 0.0))
    d = h.to("cuda")
    rot = vista.debug_rotate(synth.make_grid("small"), d)
    assert torch.equal(rot, d.vis)


@pytest.mark.parametrize("lm", [(10e-6, -4e-6), (0.01, -0.007)])
def test_point_source_rotates_to_real_constant(lm):
    cfg = synth.config("small", gauss_frac=0.0)
    h = synth.make_target(cfg, 2, noiseless=True, offset_lm=lm, no_flags=True)
    rot = vista.debug_rotate(synth.make_grid(cfg), h.to("cuda")).cpu().numpy().astype(np.complex128)
    ref = oracle.rotate(h)
    big = np.abs(ref) > 1e-3 * cfg.peak
    err = (np.abs(rot - ref)[big] / np.abs(ref[big]))
    assert err.max() < 2e-6, err.max()


def test_phase_fp32_ablation_loses_cycles():
    """With the phase argument formed in FP32, large offsets on long baselines decorrelate
    the rotated point source; the FP64 argument does not."""
    cfg = synth.config("c3", n_int=6, gauss_frac=0.0)
    h = synth.make_target(cfg, 0, noiseless=True, offset_lm=(2.9e-4, -2.9e-4), no_flags=True)
    g = synth.make_grid(cfg)
    ref = oracle.rotate(h)
    d = h.to("cuda")
    big = np.abs(ref) > 1e-2 * cfg.peak
    e64 = np.abs(vista.debug_rotate(g, d).cpu().numpy() - ref)[big] / np.abs(ref[big])
    e32 = np.abs(vista.debug_rotate(g, d, flags=vista.F_PHASE_FP32).cpu().numpy() - ref)[big] / np.abs(ref[big])
    assert e64.max() < 2e-6
    assert e32.max() > 1e-3


@pytest.mark.parametrize("variant", ["descending", "jitter_width", "perchan_badw", "nearest", "odd_small_grid",
                                     "npol1", "npol4", "no_flags"])
@pytest.mark.parametrize("mode", ["atomic", "deterministic_kahan", "plain_fp32"])
def test_edge_layouts(variant, mode):
    cfg = synth.config("small")
    kw = {}
    g = synth.make_grid(cfg)
    if variant == "descending":
        kw = dict(descending=True)
    elif variant == "jitter_width":
        kw = dict(chan_jitter=0.4, with_width=True)
    elif variant == "perchan_badw":
        kw = dict(weight_per_chan=True, bad_weight_frac=0.1)
    elif variant == "nearest":
        g = synth.make_grid(cfg, vista.F_SPECTRAL_NEAREST)
    elif variant == "odd_small_grid":
        g = dict(g, nu=37, nv=29, du=g["du"] * 1.7, nchan=61, freq_lo=g["freq_lo"] + 40 * g["dfreq"])
    elif variant == "npol1":
        cfg = synth.config("small", npol=1)
    elif variant == "npol4":
        cfg = synth.config("small", npol=4)
    elif variant == "no_flags":
        kw = dict(no_flags=True)
    hs, ds = targets_on_gpu(cfg, **kw)
    o = oracle.stack(g, hs)
    out, st = gpu_stack(g, ds, flags=g.get("flags", 0) | MODES[mode])
    compare(o, out, st=st)


@pytest.mark.parametrize("axis", ["u", "v"])
@pytest.mark.parametrize("mode", ["atomic", "deterministic_kahan"])
def test_maximum_grid_side(axis, mode):
    """One grid side at its limit of 65535 cells (a ragged last tile of 8192 or 16384 along
    it), the other 3 cells wide: each row's track crosses hundreds of cells and tiles of the
    long axis, and every sample lands inside the grid."""
    cfg = synth.config("small")
    g = synth.make_grid(cfg)
    fine, coarse = g["du"] * g["nu"] / 65535, g["du"] * g["nu"]
    if axis == "u":
        g = dict(g, nu=65535, nv=3, du=fine, dv=coarse)
    else:
        g = dict(g, nu=3, nv=65535, du=coarse, dv=fine)
    hs, ds = targets_on_gpu(cfg)
    o = oracle.stack(g, hs)
    assert o["stats"]["n_outside_uv"] == 0
    out, st = gpu_stack(g, ds, flags=MODES[mode])
    compare(o, out, st=st)


def test_empty_and_single_channel_targets():
    cfg = synth.config("small")
    g = synth.make_grid(cfg)
    h0 = synth.make_target(cfg, 0)
    h1 = synth.make_target(cfg, 1, nchan=1, with_width=True)
    h2 = synth.make_target(cfg, 2, n_int=1)
    empty = synth.make_target(cfg, 3)
    empty.uvw = empty.uvw[:0]
    empty.vis = empty.vis[:0]
    empty.weight = empty.weight[:0]
    empty.flag = empty.flag[:0]
    hs = [h0, empty, h1, h2]
    o = oracle.stack(g, hs)
    for flags in (0, vista.F_DETERMINISTIC | vista.F_KAHAN):
        out, st = gpu_stack(g, [h.to("cuda") for h in hs], flags=flags)
        compare(o, out, st=st)


def _one_tile_one_channel(cfg, g, i, k=None):
    """Target i of cfg reduced to its channel k (None: one channel spanning the band), every
    row moved into the 8 x 8 cells at the grid centre (u, v >= 0, under four cells)."""
    import dataclasses
    if k is None:
        h = synth.make_target(cfg, i, nchan=1, with_width=True, n_int=96)
    else:
        h = synth.make_target(cfg, i, n_int=96)
        width = np.full(1, abs(h.chan_freq[1] - h.chan_freq[0]))
        sl = lambda x: None if x is None else x[:, k:k + 1].contiguous()
        h = dataclasses.replace(h, vis=sl(h.vis), flag=sl(h.flag), chan_freq=h.chan_freq[k:k + 1].copy(),
                                chan_width=width)
    a = float(np.max(h.chan_freq)) / 299792458.0
    uv = h.uvw[:, :2].abs()
    h.uvw[:, :2] = uv * (3.5 * g["du"] / (float(uv.max()) * a))
    return h


@pytest.mark.parametrize("waves", [1, 4, 16])
@pytest.mark.parametrize("wide", [False, True])
def test_long_runs_of_one_channel_records(wide, waves):
    """Units whose sample streams are thousands of one-channel records in a row (one-channel
    targets, every row in one uv tile): windows of 64 records then end exactly where a
    chunk starts, and the walk must resume at the record past the window."""
    cfg = synth.config("small")
    g = synth.make_grid(cfg)
    # narrow: a channel whose overlap set is rest channel 64 alone (the first of block 1);
    # wide: one channel spanning the band (dozens of rest channels, two blocks)
    hs = [_one_tile_one_channel(cfg, g, i, None if wide else k) for i, k in ((0, 110), (1, 117), (2, 36))]
    o = oracle.stack(g, hs)
    assert o["stats"]["n_outside_uv"] == 0 and o["stats"]["n_outside_band"] == 0
    cells = np.argwhere(o["N"] > 0)
    assert cells[:, 1].min() >= 48 and cells[:, 1].max() < 56 and cells[:, 2].min() >= 48 and cells[:, 2].max() < 56
    out, st = gpu_stack(g, [h.to("cuda") for h in hs], tuning=dict(tile_u=8, tile_v=8, jblock=64, waves=waves))
    compare(o, out, st=st)
    out, st = gpu_stack(g, [h.to("cuda") for h in hs], flags=vista.F_KAHAN,
                        tuning=dict(tile_u=8, tile_v=8, jblock=64, waves=waves))
    compare(o, out, st=st)
    # the ordered kernel: chunks of 64 one-channel records whose rows share a few cells, so
    # lanes of one phase meet in a cell and take many turns
    out, st = gpu_stack(g, [h.to("cuda") for h in hs], flags=vista.F_DETERMINISTIC | vista.F_KAHAN,
                        tuning=dict(tile_u=8, tile_v=8, jblock=64, waves=waves))
    compare(o, out, st=st)


def test_no_targets_gives_zero_grid():
    g = synth.make_grid("small")
    out, st = gpu_stack(g, [])
    assert not out["count"].any() and not out["sum_w"].any()
    assert st["n_samples"] == 0


PACKED_SHAPES = [(8, 8, 64), (16, 4, 64), (16, 8, 32), (8, 4, 128), (16, 2, 128), (4, 4, 256), (8, 2, 256),
                 (4, 2, 512), (4, 4, 128), (8, 4, 64), (8, 2, 128), (4, 2, 256), (16, 2, 160), (8, 2, 320),
                 (8, 4, 160)]
ORDERED_SHAPES = [(2, 2, 64), (2, 1, 128), (1, 2, 128), (1, 1, 256), (2, 2, 128), (2, 1, 256), (2, 2, 256),
                  (4, 2, 256), (2, 2, 512), (4, 2, 512), (8, 4, 128), (8, 8, 64)]
PACKED_SHAPES_F32 = [(8, 4, 288), (16, 4, 144), (8, 8, 144), (16, 2, 288), (4, 4, 576), (8, 2, 576), (16, 8, 64),
                     (8, 4, 128), (8, 4, 144), (16, 4, 64)]


@pytest.fixture(scope="module")
def small_case():
    cfg = synth.config("small")
    hs, ds = targets_on_gpu(cfg)
    g = synth.make_grid(cfg)
    return g, ds, oracle.stack(g, hs)


@pytest.fixture(params=["direct", "aggregated"])
def lds_updates(request, monkeypatch):
    """Both forms of the packed kernel's LDS updates, forced on the same data."""
    monkeypatch.setenv("VISTA_AGGREGATE", "1" if request.param == "aggregated" else "0")
    return request.param


@pytest.mark.parametrize("waves", [4, 8, 16])
@pytest.mark.parametrize("shape", PACKED_SHAPES)
def test_every_tile_shape_matches(shape, waves, small_case, lds_updates):
    """The autotuner's candidates change only speed: counts identical, sums in tolerance
    (plain and compensated; the ordered kernel on the shapes it is built for), with 4
    wavefronts per workgroup, with 8 (two workgroups per compute unit, as the batched
    recipe's tuned shape runs) and with the 16 whose per-wavefront stream split the
    default workload's benchmark runs."""
    g, ds, o = small_case
    tu = dict(tile_u=shape[0], tile_v=shape[1], jblock=shape[2], waves=waves)
    out, st = gpu_stack(g, ds, tuning=tu)
    compare(o, out, st=st)
    out, st = gpu_stack(g, ds, flags=vista.F_KAHAN, tuning=tu)
    compare(o, out, st=st)
    if shape in ORDERED_SHAPES and waves == 4:
        out, st = gpu_stack(g, ds, flags=vista.F_DETERMINISTIC | vista.F_KAHAN, tuning=tu)
        compare(o, out, st=st)


@pytest.mark.parametrize("waves", [1, 4, 16])
@pytest.mark.parametrize("shape", ORDERED_SHAPES)
def test_every_ordered_shape_matches(shape, waves, small_case):
    """The deterministic form in every launch shape built for it, compensated and not, with
    one wavefront per workgroup (its default: the wavefront owns the whole block), four and
    sixteen (slices of the block per wavefront)."""
    g, ds, o = small_case
    tu = dict(tile_u=shape[0], tile_v=shape[1], jblock=shape[2], waves=waves)
    for flags in (vista.F_DETERMINISTIC, vista.F_DETERMINISTIC | vista.F_KAHAN):
        out, st = gpu_stack(g, ds, flags=flags, tuning=tu)
        compare(o, out, st=st)


@pytest.mark.parametrize("waves", [4, 8, 16])
@pytest.mark.parametrize("shape", PACKED_SHAPES_F32)
def test_every_fp32_tile_shape_matches(shape, waves, small_case, lds_updates):
    """The plain FP32 form's shapes (FP32 per-tile sums, 16 B of LDS per cell)."""
    g, ds, o = small_case
    tu = dict(tile_u=shape[0], tile_v=shape[1], jblock=shape[2], waves=waves)
    out, st = gpu_stack(g, ds, flags=vista.F_PLAIN_FP32, tuning=tu)
    compare(o, out, st=st)


@pytest.mark.parametrize("npol", [2, 1, 4])
@pytest.mark.parametrize("mode", ["atomic", "kahan", "plain_fp32", "deterministic_kahan"])
def test_fine_channels_match_oracle(mode, npol, lds_updates):
    """Targets of 3000 channels over a band whose rest channels each take dozens of them
    (and whose uv cells change slowly along the channel axis): lanes hold long runs of
    samples adding to one cell, the case the aggregated LDS updates are for; both update
    forms against the oracle, with a coarse target mixed in.  The ordered kernel (which has
    one update form) meets the same runs as dozens of phases per chunk."""
    cfg = synth.config("small", npol=npol)
    g = synth.make_grid(cfg)
    hs = [synth.make_target(cfg, 0, nchan=3000, n_int=6), synth.make_target(cfg, 1, nchan=2500, n_int=6,
                                                                            descending=True),
          synth.make_target(cfg, 2)]
    o = oracle.stack(g, hs)
    out, st = gpu_stack(g, [h.to("cuda") for h in hs], flags=MODES[mode])
    if mode == "plain_fp32":
        from tests.gpu_util import compare_fp32_plain
        compare_fp32_plain(o, out)
        assert st == o["stats"]
    else:
        compare(o, out, st=st)


def test_plain_fp32_rejects_compensated_flags():
    g = synth.make_grid("small")
    for extra in (vista.F_KAHAN, vista.F_DETERMINISTIC):
        with pytest.raises(vista.VistaError) as e:
            vista.Stack(g, flags=vista.F_PLAIN_FP32 | extra)
        assert e.value.code == vista.VISTA_E_ARG


def test_deterministic_mode_is_bit_identical():
    cfg = synth.config("small")
    _, ds = targets_on_gpu(cfg)
    g = synth.make_grid(cfg)
    ref, _ = gpu_stack(g, ds, flags=vista.F_DETERMINISTIC)
    for _ in range(4):
        out, _ = gpu_stack(g, ds, flags=vista.F_DETERMINISTIC)
        for k in ("sum_wvis", "sum_w", "count"):
            assert np.array_equal(out[k].view(np.uint8), ref[k].view(np.uint8))


@pytest.mark.parametrize("flags", [vista.F_DETERMINISTIC, vista.F_DETERMINISTIC | vista.F_KAHAN], ids=["fp64", "kahan"])
def test_deterministic_fine_channels_are_bit_identical(flags):
    """Fine channels (thousands of input channels per rest channel), where the ordered kernel
    sums each run of lanes with the same cells before one bid per run: the same bits from
    run to run, and the oracle's sums."""
    cfg = synth.config("small")
    g = synth.make_grid(cfg)
    hs = [synth.make_target(cfg, 1, nchan=65535, n_int=2), synth.make_target(cfg, 2, nchan=20000, n_int=3)]
    ds = [h.to("cuda") for h in hs]
    ref, st = gpu_stack(g, ds, flags=flags)
    compare(oracle.stack(g, hs), ref, st=st)
    for _ in range(3):
        out, _ = gpu_stack(g, ds, flags=flags)
        for k in ("sum_wvis", "sum_w", "count"):
            assert np.array_equal(out[k].view(np.uint8), ref[k].view(np.uint8))


@pytest.mark.parametrize("flags", ["kahan", "deterministic_kahan"])
def test_kahan_fp64_outputs(flags):
    """The FP64 outputs (FP64 tile sums, or s - c of the compensated FP32 tile sums) are
    much closer to the oracle than the 1e-5 of the FP32 outputs."""
    cfg = synth.config("small")
    hs, ds = targets_on_gpu(cfg)
    g = synth.make_grid(cfg)
    o = oracle.stack(g, hs)
    out, st = gpu_stack(g, ds, flags=MODES[flags], fp64=True)
    nz = o["N"] > 0
    e = np.abs(out["sum_wvis64"] - o["S"])[nz] / o["A"][nz]
    assert e.max() < 1e-6
    ew = np.abs(out["sum_w64"] - o["W"])[nz] / o["W"][nz]
    assert ew.max() < 1e-6


def test_host_memory_targets_and_outputs():
    cfg = synth.config("small")
    hs = synth.make_targets(cfg)
    g = synth.make_grid(cfg)
    o = oracle.stack(g, hs)
    s = vista.Stack(g)
    for h in hs:
        s.add(h)                       # pageable host tensors: copied at add time
    out = vista.alloc_outputs(g, device="cpu")
    st = s.finalize(out)
    s.close()
    compare(o, {k: v.numpy() for k, v in out.items()}, st=st)


def test_batch_equals_plain():
    """Several stacks with different grids and target counts in one launch."""
    grids, hs_all = [], []
    for i, name in enumerate(["small", "tiny", "c1"]):
        cfg = synth.config(name)
        grids.append(synth.make_grid(cfg))
        hs_all.append(synth.make_targets(cfg, n=min(cfg.n_targets, 3 + i)))
    b = vista.Batch(grids)
    dev = [[h.to("cuda") for h in hs] for hs in hs_all]
    for s, ds in enumerate(dev):
        for d in ds:
            b.add(s, d)
    b.run()
    for s, g in enumerate(grids):
        out = vista.alloc_outputs(g)
        st = b.finalize(s, out)
        o = oracle.stack(g, hs_all[s])
        compare(o, {k: v.cpu().numpy() for k, v in out.items()}, st=st)
    b.close()


def test_batch_of_many_small_stacks():
    """150 stacks in one launch, each one target on a grid of its own size (5 to 24 cells a
    side, 3 to 12 rest channels): the stack of every row and unit is looked up among many,
    and the work list orders units of many stacks by size."""
    cfg = synth.config("tiny")
    base = synth.make_grid(cfg)
    rng = np.random.default_rng(150)
    grids, hs_all = [], []
    for s in range(150):
        nu, nv, nch = int(rng.integers(5, 25)), int(rng.integers(5, 25)), int(rng.integers(3, 13))
        grids.append(dict(base, nu=nu, nv=nv, du=base["du"] * base["nu"] / nu, dv=base["dv"] * base["nv"] / nv,
                          nchan=nch, dfreq=base["dfreq"] * base["nchan"] / nch))
        hs_all.append([synth.make_target(cfg, s % cfg.n_targets)])
    b = vista.Batch(grids)
    for s, hs in enumerate(hs_all):
        b.add(s, hs[0].to("cuda"))
    b.run()
    for s, g in enumerate(grids):
        out = vista.alloc_outputs(g)
        st = b.finalize(s, out)
        compare(oracle.stack(g, hs_all[s]), {k: v.cpu().numpy() for k, v in out.items()}, st=st)
    b.close()


@pytest.mark.parametrize("n16", [1, 1000, 256 * 256 * 256 * 4 + 5])
def test_copy_kernel_copies_every_vector(n16):
    """The plain copy kernel (bandwidth measurement, counter calibration): every 16-byte
    vector copied, including the unrolled path at the largest grid and a ragged tail."""
    src = torch.randint(0, 256, (n16 * 16,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    vista.debug_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_workspace_reuse_across_sizes_shapes_and_streams():
    """Consecutive stacks on one thread reuse the cached launch workspace (device buffers,
    and the host buffers the channel tables are built in): a larger launch after a smaller
    one (buffers grow), a smaller one after it, another launch shape (a second workspace),
    another stream, and a release in between all give the oracle's result."""
    small_cfg, big_cfg = synth.config("tiny"), synth.config("small")
    cases = []
    for cfg in (small_cfg, big_cfg, small_cfg):
        hs, ds = targets_on_gpu(cfg)
        cases.append((synth.make_grid(cfg), hs, ds))
    for g, hs, ds in cases:
        out, st = gpu_stack(g, ds)
        compare(oracle.stack(g, hs), out, st=st)
    g, hs, ds = cases[1]
    o = oracle.stack(g, hs)
    out, st = gpu_stack(g, ds, tuning=dict(tile_u=16, tile_v=2, jblock=160, waves=16))
    compare(o, out, st=st)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out, st = vista.stack(g, ds)
    s.synchronize()
    compare(o, {k: v.cpu().numpy() for k, v in out.items()}, st=st)
    vista.release_workspace()
    out, st = gpu_stack(g, ds)
    compare(o, out, st=st)


def test_two_threads_stack_at_once():
    """Different handles on different host threads, each on a stream of its own, at the
    same time (each thread keeps its own workspace; the planning pool is shared): both
    results equal the oracle's, several times over."""
    import threading
    jobs = []
    for name in ("small", "c1"):
        cfg = synth.config(name)
        hs, ds = targets_on_gpu(cfg)
        g = synth.make_grid(cfg)
        jobs.append((g, hs, ds, oracle.stack(g, hs)))
    results = [[None] * 3 for _ in jobs]
    errors = []

    def work(i):
        g, hs, ds, o = jobs[i]
        try:
            s = torch.cuda.Stream()
            for rep in range(3):
                with torch.cuda.stream(s):
                    out, st = vista.stack(g, ds)
                s.synchronize()
                results[i][rep] = ({k: v.cpu().numpy() for k, v in out.items()}, st)
        except Exception as e:          # reported by the main thread
            errors.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(jobs))]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=240)
    assert not any(t.is_alive() for t in th), "a stacking thread did not finish"
    assert not errors, errors
    for (g, hs, ds, o), res in zip(jobs, results):
        for out, st in res:
            compare(o, out, st=st)
