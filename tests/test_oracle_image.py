"""Pins of the oracle's dirty image of a stacked grid (CPU only).

The oracle inverts each rest channel of the grid by a direct Fourier sum.  Pinned by closed
forms (one filled cell gives a constant or a pure cosine pattern; the pixel sum picks out
the centre cell; the dirty beam is 1 at the centre), by the special case that reduces to a
library routine (numpy's inverse FFT with centring shifts), and by a stacked point source
landing on the centre pixel with its flux.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _cell_grid(nchan, nv, nu, cells):
    S = np.zeros((nchan, nv, nu), np.complex128)
    W = np.zeros((nchan, nv, nu), np.float64)
    for j, iv, iu, s, w in cells:
        S[j, iv, iu] += s
        W[j, iv, iu] += w
    return S, W


@pytest.mark.parametrize("shape", [(8, 8), (16, 4), (6, 10), (5, 7)])
def test_single_cell_closed_forms(shape):
    nv, nu = shape
    cu, cv = nu // 2, nv // 2
    s, w = 0.7 - 0.4j, 2.5
    # centre cell: a constant image Re(s) / w
    S, W = _cell_grid(1, nv, nu, [(0, cv, cu, s, w)])
    img = oracle.image(S, W)
    assert np.max(np.abs(img - s.real / w)) < 1e-15
    # one off-centre cell: Re(s exp(2 pi i (du (p - cu) / nu + dv (q - cv) / nv))) / w
    iu, iv = (cu + 1) % nu, (cv + nv - 1) % nv
    S, W = _cell_grid(1, nv, nu, [(0, iv, iu, s, w)])
    img = oracle.image(S, W)
    p, q = np.meshgrid(np.arange(nu), np.arange(nv))
    ph = 2 * np.pi * ((iu - cu) * (p - cu) / nu + (iv - cv) * (q - cv) / nv)
    assert np.max(np.abs(img[0] - (s * np.exp(1j * ph)).real / w)) < 1e-14


def test_pixel_sum_and_beam_peak():
    """Summed over all pixels, every cell but the centre one cancels; the dirty beam is
    exactly 1 at the centre pixel; a channel without weight images to zero."""
    rng = np.random.default_rng(1)
    nchan, nv, nu = 3, 12, 16
    S = rng.normal(size=(nchan, nv, nu)) + 1j * rng.normal(size=(nchan, nv, nu))
    W = rng.uniform(0.5, 2.0, size=(nchan, nv, nu))
    W[2] = 0.0
    img, beam = oracle.image(S, W, beam=True)
    for j in range(2):
        wt = W[j].sum()
        assert abs(img[j].sum() - nu * nv * S[j, nv // 2, nu // 2].real / wt) < 1e-10
        assert abs(beam[j, nv // 2, nu // 2] - 1.0) < 1e-14
    assert np.all(img[2] == 0) and np.all(beam[2] == 0)


@pytest.mark.parametrize("shape", [(8, 8), (32, 16), (6, 10)])
def test_matches_centred_inverse_fft(shape):
    """The direct sum equals numpy's inverse FFT with the centring shifts (for even sizes
    the centre index n/2 is where ifftshift puts frequency 0)."""
    nv, nu = shape
    rng = np.random.default_rng(2)
    S = rng.normal(size=(2, nv, nu)) + 1j * rng.normal(size=(2, nv, nu))
    W = rng.uniform(0.1, 1.0, size=(2, nv, nu))
    img = oracle.image(S, W)
    for j in range(2):
        ref = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(S[j]))).real * nu * nv / W[j].sum()
        assert np.max(np.abs(img[j] - ref)) < 1e-12 * np.max(np.abs(ref))


def test_stacked_point_source_lands_on_the_centre_pixel():
    """A noiseless point source stacked at the phase centre: every line channel's dirty
    image peaks at the centre pixel with the channel's mean flux."""
    cfg = synth.config("c1", gauss_frac=0.0, offset=8 * synth.configs.ARCSEC, peak=0.05)
    ts = synth.make_targets(cfg, n=3, noiseless=True)
    g = synth.make_grid(cfg)
    o = oracle.stack(g, ts, jlo=28, jhi=36)
    img = oracle.image(o["S"], o["W"])
    for j in range(img.shape[0]):
        flux = o["S"][j].sum().real / o["W"][j].sum()
        if flux < 0.2 * cfg.peak:
            continue
        a, b = np.unravel_index(np.argmax(img[j]), img[j].shape)
        assert (a, b) == (g["nv"] // 2, g["nu"] // 2)
        assert abs(img[j, a, b] - flux) < 1e-12 * flux


def test_pixels_agree_with_full_image():
    rng = np.random.default_rng(3)
    S = rng.normal(size=(1, 16, 16)) + 1j * rng.normal(size=(1, 16, 16))
    W = rng.uniform(0.1, 1.0, size=(1, 16, 16))
    img = oracle.image(S, W)
    q = np.array([0, 3, 8, 15]); p = np.array([5, 8, 0, 15])
    px = oracle.image_pixels(S[0], W[0], q, p)
    assert np.max(np.abs(px - img[0, q, p])) < 1e-15 * max(1.0, np.max(np.abs(img)))
    assert math.isfinite(px.sum())
