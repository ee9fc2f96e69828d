"""Seeded generator of synthetic targets (one target = one dataset selection).

Geometry (antennas, uvw, channel frequencies, redshift, source offset) is drawn with
NumPy's PCG64 from a per-target ``SeedSequence.spawn`` child of the recipe seed.  The
bulk arrays (visibilities, flags, weights) are drawn with a ``torch.Generator`` on the
requested device, in fixed row blocks, so a recipe's data is identical for a given
device.  Nothing here depends on the stacking library or on the oracle.

uvw follows the standard earth-rotation synthesis relations (Thompson, Moran &
Swenson, *Interferometry and Synthesis in Radio Astronomy*, eqs. 4.1 and 4.15): local
(E, N, U) baselines are turned into equatorial (X, Y, Z) at the array latitude and
projected for hour angle H and declination delta.  Rows are time-major (all baselines
of integration 0, then integration 1, ...), as in a Measurement Set.

The model visibility of a source at direction cosines (l0, m0) with spectrum S and
shape G is  V = S(nu_rest) * G(u, v) * exp(-2 pi i (nu/c) (u l0 + v m0 + w (n0 - 1)))
with n0 = sqrt(1 - l0^2 - m0^2), plus complex Gaussian noise of rms sigma per part.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import torch

from .configs import C_LIGHT, Config, config as _config, grid_for

LATITUDE = math.radians(-23.02)     # array latitude
DECLINATION = math.radians(-30.0)   # source declination
SIDEREAL_DAY = 86164.0905           # [s]
ROW_BLOCK = 8192                    # rows per bulk-generation block (fixes the draw order)


@dataclasses.dataclass
class Target:
    """One target dataset.  Array fields are torch tensors on one device."""
    uvw: torch.Tensor            # [nrow, 3] float64, metres
    vis: torch.Tensor            # [nrow, nchan, npol] complex64
    weight: torch.Tensor         # [nrow, npol] (or [nrow, nchan, npol]) float32
    flag: Optional[torch.Tensor]  # [nrow, nchan, npol] uint8, or None
    chan_freq: np.ndarray        # [nchan] float64, observed Hz
    chan_width: Optional[np.ndarray]
    l: float
    m: float
    z: float
    weight_per_chan: bool = False
    meta: dict = dataclasses.field(default_factory=dict)
    # the phase centre (ra0, dec0) and the stacking position (ra1, dec1) [rad], consistent
    # with (l, m); rotate_uvw asks the stack to apply Eq. 1's rotation between them
    ra0: float = 0.0
    dec0: float = 0.0
    ra1: float = 0.0
    dec1: float = 0.0
    rotate_uvw: bool = False

    @property
    def nrow(self) -> int:
        return int(self.uvw.shape[0])

    @property
    def nchan(self) -> int:
        return int(self.chan_freq.shape[0])

    @property
    def npol(self) -> int:
        return int(self.vis.shape[2])

    def to(self, device) -> "Target":
        mv = lambda x: None if x is None else x.to(device)
        return dataclasses.replace(self, uvw=mv(self.uvw), vis=mv(self.vis), weight=mv(self.weight),
                                   flag=mv(self.flag))

    def numpy(self) -> dict:
        """Host copies as plain NumPy arrays (for the CPU oracle)."""
        cp = lambda x: None if x is None else x.detach().cpu().numpy()
        return dict(uvw=cp(self.uvw), vis=cp(self.vis), weight=cp(self.weight), flag=cp(self.flag),
                    chan_freq=self.chan_freq, chan_width=self.chan_width, l=self.l, m=self.m,
                    z=self.z, weight_per_chan=self.weight_per_chan, rotate_uvw=self.rotate_uvw,
                    ra0=self.ra0, dec0=self.dec0, ra1=self.ra1, dec1=self.dec1)

    def channel_slice(self, k0: int, k1: int) -> dict:
        """Host copy of channels [k0, k1) of every row, with the full frequency axis."""
        cp = lambda x: None if x is None else x[:, k0:k1].contiguous().cpu().numpy()
        d = dict(uvw=self.uvw.cpu().numpy(), vis=cp(self.vis),
                 weight=(cp(self.weight) if self.weight_per_chan else self.weight.cpu().numpy()),
                 flag=cp(self.flag), chan_freq=self.chan_freq, chan_width=self.chan_width,
                 l=self.l, m=self.m, z=self.z, weight_per_chan=self.weight_per_chan,
                 kbeg=k0, kend=k1, rotate_uvw=self.rotate_uvw, ra0=self.ra0, dec0=self.dec0, ra1=self.ra1,
                 dec1=self.dec1)
        return d


def _antennas(rng: np.random.Generator, n: int, diameter: float) -> np.ndarray:
    r = 0.5 * diameter * np.sqrt(rng.random(n))
    th = 2.0 * np.pi * rng.random(n)
    return np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n)], axis=1)  # E, N, U


def _uvw(enu: np.ndarray, n_int: int, t_int: float) -> np.ndarray:
    i, j = np.triu_indices(enu.shape[0], k=1)
    b = enu[j] - enu[i]                                    # baseline E, N, U
    sl, cl = math.sin(LATITUDE), math.cos(LATITUDE)
    X = -sl * b[:, 1] + cl * b[:, 2]
    Y = b[:, 0]
    Z = cl * b[:, 1] + sl * b[:, 2]
    ha = (np.arange(n_int) - 0.5 * (n_int - 1)) * t_int * 2.0 * math.pi / SIDEREAL_DAY
    sh, ch = np.sin(ha)[:, None], np.cos(ha)[:, None]
    sd, cd = math.sin(DECLINATION), math.cos(DECLINATION)
    u = sh * X + ch * Y
    v = -sd * ch * X + sd * sh * Y + cd * Z
    w = cd * ch * X - cd * sh * Y + sd * Z
    return np.stack([u, v, w], axis=-1).reshape(-1, 3)   # time-major rows


def _channels(rng, nchan, band_width, nu_c, descending, jitter, with_width):
    dnu = band_width / nchan
    f = nu_c + (np.arange(nchan) - 0.5 * (nchan - 1)) * dnu
    if jitter > 0.0:
        f = f + jitter * dnu * (rng.random(nchan) - 0.5)
    width = np.full(nchan, dnu) if (with_width or nchan == 1) else None
    if descending:
        f = f[::-1].copy()
        width = None if width is None else width[::-1].copy()
    return f, width


def make_target(cfg: Config | str, index: int, device="cpu", *, noiseless: bool | None = None,
                descending: bool = False, chan_jitter: float = 0.0, with_width: bool = False,
                weight_per_chan: bool = False, bad_weight_frac: float = 0.0,
                nchan: int | None = None, n_int: int | None = None, z: float | None = None,
                offset_lm: tuple | None = None, no_flags: bool = False) -> Target:
    """Draw target ``index`` of recipe ``cfg`` on ``device``.

    Keyword overrides produce the edge cases the tests need (descending or jittered
    channels, explicit widths, per-channel weights, bad weights, fixed z or offset).
    """
    if isinstance(cfg, str):
        cfg = _config(cfg)
    noiseless = cfg.noiseless if noiseless is None else noiseless
    ss = np.random.SeedSequence(cfg.seed).spawn(index + 1)[index]
    rng = np.random.Generator(np.random.PCG64(ss))
    n_ant = int(rng.integers(cfg.n_ant[0], cfg.n_ant[1] + 1))
    enu = _antennas(rng, n_ant, cfg.array_diameter)
    nch = int(rng.choice(np.asarray(cfg.nchan)))
    zz = float(rng.uniform(*cfg.z_range))
    lm = rng.uniform(-cfg.offset, cfg.offset, 2)
    gauss = bool(rng.random() < cfg.gauss_frac)
    bulk_seed = int(rng.integers(0, 2**62))
    nch = nchan if nchan is not None else nch
    zz = z if z is not None else zz
    l0, m0 = (float(lm[0]), float(lm[1])) if offset_lm is None else (float(offset_lm[0]), float(offset_lm[1]))
    nint = n_int if n_int is not None else cfg.n_int

    uvw = _uvw(enu, nint, cfg.t_int)
    nu_c = cfg.line_rest / (1.0 + zz)
    freq, width = _channels(rng, nch, cfg.band_width, nu_c, descending, chan_jitter, with_width)

    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(bulk_seed)
    nrow, npol = uvw.shape[0], cfg.npol
    uvw_t = torch.from_numpy(uvw).to(dev)
    freq_t = torch.from_numpy(np.ascontiguousarray(freq)).to(dev)
    vis = torch.empty((nrow, nch, npol), dtype=torch.complex64, device=dev)
    flag = None if no_flags else torch.empty((nrow, nch, npol), dtype=torch.uint8, device=dev)
    wshape = (nrow, nch, npol) if weight_per_chan else (nrow, npol)
    w0 = 1.0 / (cfg.sigma * cfg.sigma)
    g = torch.randn(wshape, generator=gen, device=dev, dtype=torch.float32)
    weight = (w0 * torch.exp(cfg.weight_scatter * g)).to(torch.float32)
    if bad_weight_frac > 0.0:
        bad = torch.rand(wshape, generator=gen, device=dev) < bad_weight_frac
        kind = torch.randint(0, 4, wshape, generator=gen, device=dev)
        badv = torch.tensor([0.0, -1.0, float("nan"), float("inf")], device=dev, dtype=torch.float32)
        weight = torch.where(bad, badv[kind], weight)

    # Spectrum: Gaussian line in rest radio velocity.
    nu_rest = freq_t * (1.0 + zz)
    vel = C_LIGHT * (cfg.line_rest - nu_rest) / cfg.line_rest / 1e3
    spec = cfg.peak * torch.exp(-4.0 * math.log(2.0) * (vel / cfg.fwhm_kms) ** 2)   # [nch] f64
    n0m1 = math.sqrt(1.0 - l0 * l0 - m0 * m0) - 1.0
    theta = cfg.gauss_fwhm if gauss else 0.0
    for r0 in range(0, nrow, ROW_BLOCK):
        r1 = min(nrow, r0 + ROW_BLOCK)
        u = uvw_t[r0:r1, 0:1]
        v = uvw_t[r0:r1, 1:2]
        w = uvw_t[r0:r1, 2:3]
        lam_inv = (freq_t / C_LIGHT)[None, :]
        turns = (u * l0 + v * m0 + w * n0m1) * lam_inv                  # [B, nch] f64
        amp = spec[None, :].expand(r1 - r0, nch)
        if theta > 0.0:
            q = (u * u + v * v) * lam_inv * lam_inv
            amp = amp * torch.exp(-(math.pi ** 2) * theta * theta * q / (4.0 * math.log(2.0)))
        ph = -2.0 * math.pi * turns
        re = (amp * torch.cos(ph))[:, :, None].expand(r1 - r0, nch, npol)
        im = (amp * torch.sin(ph))[:, :, None].expand(r1 - r0, nch, npol)
        if not noiseless:
            nz = torch.randn((r1 - r0, nch, npol, 2), generator=gen, device=dev, dtype=torch.float32)
            re = re + cfg.sigma * nz[..., 0].double()
            im = im + cfg.sigma * nz[..., 1].double()
        vis[r0:r1] = torch.complex(re.float(), im.float())
        if flag is not None:
            fl = torch.rand((r1 - r0, nch, npol), generator=gen, device=dev) < cfg.flag_frac
            flag[r0:r1] = fl.to(torch.uint8)
    meta = dict(n_ant=n_ant, gaussian=gauss, theta=theta, seed=bulk_seed, index=index, cfg=cfg.name,
                peak=cfg.peak)
    ra1, dec1 = radec_of_offset(0.0, DECLINATION, l0, m0)
    return Target(uvw=uvw_t, vis=vis, weight=weight, flag=flag, chan_freq=freq, chan_width=width,
                  l=l0, m=m0, z=zz, weight_per_chan=weight_per_chan, meta=meta, ra0=0.0, dec0=DECLINATION,
                  ra1=ra1, dec1=dec1)


def radec_of_offset(ra0: float, dec0: float, l: float, m: float) -> tuple:
    """(R.A., Dec.) of the direction with direction cosines (l, m) about the phase centre
    (ra0, dec0): l along the centre's east axis, m along its north axis."""
    n = math.sqrt(1.0 - l * l - m * m)
    sr, cr, sd, cd = math.sin(ra0), math.cos(ra0), math.sin(dec0), math.cos(dec0)
    x = -l * sr - m * sd * cr + n * cd * cr
    y = l * cr - m * sd * sr + n * cd * sr
    zc = m * cd + n * sd
    return math.atan2(y, x), math.asin(max(-1.0, min(1.0, zc)))


def make_targets(cfg: Config | str, device="cpu", n: int | None = None, **kw) -> list:
    if isinstance(cfg, str):
        cfg = _config(cfg)
    n = cfg.n_targets if n is None else n
    return [make_target(cfg, i, device, **kw) for i in range(n)]


def make_grid(cfg: Config | str, flags: int = 0) -> dict:
    if isinstance(cfg, str):
        cfg = _config(cfg)
    return grid_for(cfg, flags)


def batch_stack_sizes(n_stacks: int, seed: int, lo: int = 5, hi: int = 500, mu: float = math.log(40.0),
                      s: float = 1.0) -> list:
    """Targets per stack for the batched recipe: clip(round(lognormal(mu, s)), lo, hi)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    return [int(np.clip(round(x), lo, hi)) for x in rng.lognormal(mu, s, n_stacks)]
