"""Workload recipes.

Each recipe stands in for the paper's mock Measurement Sets (Sec. 4.3: heterogeneous
redshifts, arrays and channel layouts per dataset).  Values are the workload
sizes used for the measurements; the reasons for each choice are recorded in
the design notes, not here.

Units: metres, seconds, Hz, Jy, radians.
"""
from __future__ import annotations

import dataclasses
import math

C_LIGHT = 299792458.0
ARCSEC = math.pi / (180.0 * 3600.0)
F_CO10 = 115.2712018e9      # CO(1-0) rest frequency
F_CII = 1900.5369e9          # [CII] 158 um rest frequency


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n_targets: int
    n_ant: tuple            # (lo, hi) antennas per target, inclusive, uniform
    array_diameter: float   # antennas uniform in a disc of this diameter [m]
    n_int: int              # integrations
    t_int: float            # integration time [s]
    nchan: tuple            # channel counts to draw from (uniform)
    band_width: float       # total contiguous bandwidth of a target [Hz]
    line_rest: float        # rest frequency the band is centred on [Hz]
    z_range: tuple          # z ~ U(lo, hi)
    npol: int
    peak: float             # line peak [Jy]
    fwhm_kms: float         # line FWHM, rest radio velocity [km/s]
    gauss_frac: float       # fraction of targets with a Gaussian source
    gauss_fwhm: float       # Gaussian source FWHM [rad]
    offset: float           # offsets l, m ~ U(-offset, offset) [rad]
    sigma: float            # noise per real/imag part [Jy]
    weight_scatter: float   # w = sigma^-2 * exp(weight_scatter * N(0,1))
    flag_frac: float
    grid_nu: int
    grid_nchan: int
    seed: int
    noiseless: bool = False

    def dfreq(self) -> float:
        """Rest channel width: the widest rest-frame input channel the recipe can draw."""
        return self.band_width / min(self.nchan) * (1.0 + self.z_range[1])

    def nu_obs_max(self) -> float:
        return self.line_rest / (1.0 + self.z_range[0]) + 0.5 * self.band_width

    def cell(self) -> float:
        """uv cell [wavelengths]: the grid spans +-1.02 u_max, so no sample leaves it."""
        u_max = self.array_diameter * self.nu_obs_max() / C_LIGHT
        return 2.0 * 1.02 * u_max / self.grid_nu


def _c(name, **kw):
    return Config(name=name, **kw)


CONFIGS = {
    # 8 targets, 10 antennas within 500 m, 60 x 10 s, 1 spw of 64 x 15.625 MHz at
    # 115.27 GHz/(1+z), z ~ U(2,3), 2 pols, 0.5 mJy / 300 km/s line, sigma 1 mJy,
    # 2% flags, grid 128^2 x 64.
    "c1": _c("c1", n_targets=8, n_ant=(10, 10), array_diameter=500.0, n_int=60, t_int=10.0,
             nchan=(64,), band_width=64 * 15.625e6, line_rest=F_CO10, z_range=(2.0, 3.0), npol=2,
             peak=0.5e-3, fwhm_kms=300.0, gauss_frac=0.0, gauss_fwhm=0.0, offset=10 * ARCSEC,
             sigma=1e-3, weight_scatter=0.0, flag_frac=0.02, grid_nu=128, grid_nchan=64,
             seed=20260901 + 1),
    # ALMA scale: 50 targets, 43 antennas within 2 km, 120 x 10 s, 4 x 240 x 7.8125 MHz,
    # z ~ U(1.5,3.5), point or 0.3" Gaussian at up to 15", sigma 2 mJy, weights with 20%
    # lognormal scatter, grid 512^2 x 960.
    "c2": _c("c2", n_targets=50, n_ant=(43, 43), array_diameter=2000.0, n_int=120, t_int=10.0,
             nchan=(960,), band_width=960 * 7.8125e6, line_rest=F_CO10, z_range=(1.5, 3.5), npol=2,
             peak=0.5e-3, fwhm_kms=300.0, gauss_frac=0.5, gauss_fwhm=0.3 * ARCSEC,
             offset=15 * ARCSEC, sigma=2e-3, weight_scatter=0.2, flag_frac=0.02, grid_nu=512,
             grid_nchan=960, seed=20260901 + 2),
    # Precision variant: 20 targets, baselines up to 16 km, 345 GHz band ([CII] at
    # z ~ U(4.4,4.8)), 4 x 480 x 3.90625 MHz, offsets up to 60", grid 512^2 x 1920.
    "c3": _c("c3", n_targets=20, n_ant=(43, 43), array_diameter=16000.0, n_int=60, t_int=10.0,
             nchan=(1920,), band_width=1920 * 3.90625e6, line_rest=F_CII, z_range=(4.4, 4.8), npol=2,
             peak=0.5e-3, fwhm_kms=300.0, gauss_frac=0.0, gauss_fwhm=0.0, offset=60 * ARCSEC,
             sigma=1e-3, weight_scatter=0.0, flag_frac=0.02, grid_nu=512, grid_nchan=1920,
             seed=20260901 + 3),
    # Batched variant: one stack of the 64; target count per stack is drawn in
    # make_batch_sizes().  12-50 antennas, channels from {128,480,960,3840} over 7.5 GHz,
    # z ~ U(0.5,4), data as c1, grid 256^2 x 256.
    "c4": _c("c4", n_targets=40, n_ant=(12, 50), array_diameter=2000.0, n_int=60, t_int=10.0,
             nchan=(128, 480, 960, 3840), band_width=7.5e9, line_rest=F_CO10, z_range=(0.5, 4.0),
             npol=2, peak=0.5e-3, fwhm_kms=300.0, gauss_frac=0.0, gauss_fwhm=0.0,
             offset=10 * ARCSEC, sigma=1e-3, weight_scatter=0.0, flag_frac=0.02, grid_nu=256,
             grid_nchan=256, seed=20260901 + 4),
    # Full-scale batched + compensated: per stack 200..1000 targets of 43 antennas,
    # 60 x 10 s, 4 x 960 x 1.953125 MHz, z ~ U(1.5,3.5), grid 1024^2 x 1920.
    "c5": _c("c5", n_targets=200, n_ant=(43, 43), array_diameter=2000.0, n_int=60, t_int=10.0,
             nchan=(3840,), band_width=3840 * 1.953125e6, line_rest=F_CO10, z_range=(1.5, 3.5),
             npol=2, peak=0.5e-3, fwhm_kms=300.0, gauss_frac=0.0, gauss_fwhm=0.0,
             offset=15 * ARCSEC, sigma=1e-3, weight_scatter=0.0, flag_frac=0.02, grid_nu=1024,
             grid_nchan=1920, seed=20260901 + 5),
    # Small cases for tests (not workloads).
    "tiny": _c("tiny", n_targets=3, n_ant=(4, 6), array_diameter=300.0, n_int=5, t_int=60.0,
               nchan=(7, 16, 33), band_width=0.6e9, line_rest=F_CO10, z_range=(1.0, 3.0), npol=2,
               peak=1e-3, fwhm_kms=300.0, gauss_frac=0.5, gauss_fwhm=1.0 * ARCSEC,
               offset=10 * ARCSEC, sigma=1e-3, weight_scatter=0.2, flag_frac=0.1, grid_nu=17,
               grid_nchan=9, seed=7),
    "small": _c("small", n_targets=4, n_ant=(8, 12), array_diameter=1500.0, n_int=24, t_int=30.0,
                nchan=(96, 200, 333), band_width=3.0e9, line_rest=F_CO10, z_range=(1.0, 3.0),
                npol=2, peak=1e-3, fwhm_kms=300.0, gauss_frac=0.5, gauss_fwhm=0.5 * ARCSEC,
                offset=20 * ARCSEC, sigma=1e-3, weight_scatter=0.2, flag_frac=0.03, grid_nu=96,
                grid_nchan=150, seed=11),
}


def config(name: str, **overrides) -> Config:
    """Return a recipe, optionally with fields replaced (e.g. n_targets for a subset)."""
    cfg = CONFIGS[name]
    return dataclasses.replace(cfg, **overrides) if overrides else cfg


def grid_for(cfg: Config, flags: int = 0) -> dict:
    """Common output grid of a recipe: rest channels centred on the line.

    The rest channel width is the recipe's widest possible rest-frame input channel
    (its channel width times 1 + the top of its z range), so every drawn target fits.
    """
    dfreq = cfg.dfreq()
    n = cfg.grid_nchan
    du = cfg.cell()
    return dict(nu=cfg.grid_nu, nv=cfg.grid_nu, du=du, dv=du, nchan=n,
                freq_lo=cfg.line_rest - 0.5 * n * dfreq, dfreq=dfreq, flags=int(flags))
