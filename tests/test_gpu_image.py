"""Dirty images of stacked grids on the GPU vs the oracle's direct Fourier inversion.

Every pixel within 1e-5 log2(nu nv) ||S_j||_2 / W_j of the oracle -- the norm-wise rounding
bound of an FFT of that length on that input, spread evenly, with room for the hardware
twiddles -- plus an absolute 1e-30 (noiseless line wings reach FP32's denormal range, which
the device flushes to zero); the beam within 1e-5 (it is normalised to 1).  A single cell
dropped from a 512 x 512 channel moves its pixels by about ||S_j||_2 / (512 W_j), over ten
times the bound; grids of every shape class the FFT handles (axes of 2, rectangular,
each transform length of 64 to 1024 points both in registers and in LDS, lengths of 1024
on sampled pixels, and sampled pixels of axes up to 4096), 65535 channels, a grid stacked
by the library, a weight array that is not 16-byte aligned, and the bench's full-size grid
(512 x 512 x 960) on sampled pixels.
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

TOL = 1e-5
ATOL = 1e-30          # FP32 denormals are flushed on the device


def _scale(Sj, Wsum):
    """log2(cells) ||S_j||_2 / W_j: the per-pixel error scale of the channel's FFT."""
    n = Sj.size
    return max(1.0, np.log2(n)) * np.sqrt(np.sum(np.abs(Sj) ** 2)) / Wsum


def _check(S, W, img, beam=None):
    ref, rb = oracle.image(S, W, beam=True)
    for j in range(S.shape[0]):
        wt = W[j].sum()
        if wt <= 0:
            assert np.all(img[j] == 0)
            continue
        assert np.max(np.abs(img[j] - ref[j])) <= TOL * _scale(S[j], wt) + ATOL
        if beam is not None:
            assert np.max(np.abs(beam[j] - rb[j])) <= TOL
    return ref


def test_channel_count_at_its_limit():
    """65535 channels of a 4 x 8 grid, the most one call takes (the row pass puts the
    channels on the second dimension of its launch grid), with an empty channel."""
    rng = np.random.default_rng(65535)
    nchan, nv, nu = 65535, 4, 8
    S = (rng.normal(size=(nchan, nv, nu)) + 1j * rng.normal(size=(nchan, nv, nu))).astype(np.complex64)
    W = rng.uniform(0.0, 2.0, size=(nchan, nv, nu)).astype(np.float32)
    W[nchan // 2] = 0.0
    g = dict(nu=nu, nv=nv, du=1.0, dv=1.0, nchan=nchan, freq_lo=1e9, dfreq=1e6)
    img, beam, _ = vista.image(g, torch.from_numpy(S).cuda(), torch.from_numpy(W).cuda(), beam=True)
    torch.cuda.synchronize()
    _check(S.astype(np.complex128), W.astype(np.float64), img.cpu().numpy(), beam.cpu().numpy())


# (nv, nu): transforms of 64 to 1024 points are held in registers when a tile fits (columns:
# nu >= 32, or 16 at nv = 1024; rows: nv >= 8 to 32 rows by length), the rest use the LDS
# Stockham passes; these shapes take each length both ways.  With register rows (64 <= nu
# <= 1024) and 128 <= nv <= 2048 the real part is formed from half the staging (the
# Hermitian path): (128, 64) and (256, 256) here, more in the sampled tests below
@pytest.mark.parametrize("shape", [(2, 2), (2, 8), (16, 4), (32, 32), (16, 64), (64, 8), (64, 128), (128, 16),
                                   (128, 32), (256, 256), (512, 16), (512, 32), (128, 64)])
def test_random_grids_match_oracle(shape):
    nv, nu = shape
    rng = np.random.default_rng(nv * 1000 + nu)
    nchan = 5
    S = (rng.normal(size=(nchan, nv, nu)) + 1j * rng.normal(size=(nchan, nv, nu))).astype(np.complex64)
    W = rng.uniform(0.0, 2.0, size=(nchan, nv, nu)).astype(np.float32)
    W[3] = 0.0
    g = dict(nu=nu, nv=nv, du=1.0, dv=1.0, nchan=nchan, freq_lo=1e9, dfreq=1e6)
    img, beam, tim = vista.image(g, torch.from_numpy(S).cuda(), torch.from_numpy(W).cuda(), beam=True)
    torch.cuda.synchronize()
    _check(S.astype(np.complex128), W.astype(np.float64), img.cpu().numpy(), beam.cpu().numpy())
    assert tim["accum_ms"] > 0


def test_stacked_grid_image_matches_oracle():
    """The library's own stack of the correctness workload, imaged on the GPU; a noiseless
    point source lands on the centre pixel."""
    cfg = synth.config("c1", gauss_frac=0.0, offset=8 * synth.configs.ARCSEC, peak=0.05)
    hs = synth.make_targets(cfg, n=4, noiseless=True)
    g = synth.make_grid(cfg)
    out, st = vista.stack(g, [h.to("cuda") for h in hs])
    img, beam, _ = vista.image(g, out["sum_wvis"], out["sum_w"], beam=True)
    torch.cuda.synchronize()
    S = out["sum_wvis"].cpu().numpy().astype(np.complex128)
    W = out["sum_w"].cpu().numpy().astype(np.float64)
    _check(S, W, img.cpu().numpy(), beam.cpu().numpy())
    im = img.cpu().numpy()
    j = int(np.argmax(S.sum(axis=(1, 2)).real / np.maximum(W.sum(axis=(1, 2)), 1e-30)))
    a, b = np.unravel_index(np.argmax(im[j]), im[j].shape)
    assert (a, b) == (g["nv"] // 2, g["nu"] // 2)


def test_full_size_grid_sampled_pixels():
    """The bench's 512 x 512 x 960 stacked grid (12 of its 50 targets), every channel imaged
    on the GPU; 64 pixels of each of 6 channels checked by direct inversion."""
    cfg = synth.config("c2")
    g = synth.make_grid(cfg)
    ds = [synth.make_target(cfg, i, device="cuda") for i in range(12)]
    out, st = vista.stack(g, ds)
    img, _, tim = vista.image(g, out["sum_wvis"], out["sum_w"])
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    for j in (0, 300, 470, 480, 700, 959):
        S = out["sum_wvis"][j].cpu().numpy().astype(np.complex128)
        W = out["sum_w"][j].cpu().numpy().astype(np.float64)
        q = rng.integers(0, g["nv"], 64)
        p = rng.integers(0, g["nu"], 64)
        q[0], p[0] = g["nv"] // 2, g["nu"] // 2
        ref = oracle.image_pixels(S, W, q, p)
        got = img[j].cpu().numpy()[q, p]
        wt = W.sum()
        scale = _scale(S, wt) if wt > 0 else 1.0
        assert np.max(np.abs(got - ref)) <= TOL * scale + ATOL


def _sampled(S, W, img, beam, rng, npix):
    nchan, nv, nu = S.shape
    for j in range(nchan):
        wt = W[j].sum()
        q = rng.integers(0, nv, npix)
        p = rng.integers(0, nu, npix)
        q[0], p[0] = nv // 2, nu // 2
        ref = oracle.image_pixels(S[j], W[j], q, p)
        assert np.max(np.abs(img[j][q, p] - ref)) <= TOL * _scale(S[j], wt) + ATOL
        if beam is not None:
            rb = oracle.image_pixels(W[j].astype(np.complex128), W[j], q, p)
            assert np.max(np.abs(beam[j][q, p] - rb)) <= TOL


@pytest.mark.parametrize("shape,nchan", [((4, 4096), 3), ((4096, 2), 3), ((2048, 8), 2), ((1024, 64), 3),
                                         ((64, 1024), 3), ((1024, 1024), 2), ((4096, 4096), 1), ((2048, 64), 2),
                                         ((2048, 1024), 1), ((128, 512), 2), ((256, 1024), 2), ((512, 128), 2)])
def test_longest_axes_sampled_pixels(shape, nchan):
    """Axes up to the 4096 limit, where one row or one column fills a whole tile; and
    sizes of the Hermitian path (register rows, 128 <= nv <= 2048) up to its longest."""
    nv, nu = shape
    rng = np.random.default_rng(nv + 7 * nu)
    S = (rng.normal(size=(nchan, nv, nu)) + 1j * rng.normal(size=(nchan, nv, nu))).astype(np.complex64)
    W = rng.uniform(0.0, 2.0, size=(nchan, nv, nu)).astype(np.float32)
    g = dict(nu=nu, nv=nv, du=1.0, dv=1.0, nchan=nchan, freq_lo=1e9, dfreq=1e6)
    img, beam, _ = vista.image(g, torch.from_numpy(S).cuda(), torch.from_numpy(W).cuda(), beam=True)
    torch.cuda.synchronize()
    _sampled(S.astype(np.complex128), W.astype(np.float64), img.cpu().numpy(), beam.cpu().numpy(), rng,
             16 if nu * nv > 1 << 20 else 48)


def test_weights_not_16_byte_aligned():
    """A weight array that starts 4 bytes into its allocation takes the scalar summing path;
    the image is the same as the oracle's."""
    nchan, nv, nu = 3, 64, 32
    rng = np.random.default_rng(5)
    S = (rng.normal(size=(nchan, nv, nu)) + 1j * rng.normal(size=(nchan, nv, nu))).astype(np.complex64)
    W = rng.uniform(0.0, 2.0, size=(nchan, nv, nu)).astype(np.float32)
    buf = torch.zeros(W.size + 1, dtype=torch.float32, device="cuda")
    w_dev = buf[1:].view(nchan, nv, nu)
    w_dev.copy_(torch.from_numpy(W))
    assert w_dev.data_ptr() % 16 != 0
    g = dict(nu=nu, nv=nv, du=1.0, dv=1.0, nchan=nchan, freq_lo=1e9, dfreq=1e6)
    img, beam, _ = vista.image(g, torch.from_numpy(S).cuda(), w_dev, beam=True)
    torch.cuda.synchronize()
    _check(S.astype(np.complex128), W.astype(np.float64), img.cpu().numpy(), beam.cpu().numpy())
