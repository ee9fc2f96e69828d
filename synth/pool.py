"""Targets that share their bulk data through a pool of datasets.

The batched and streamed recipes hold more input than any memory can (terabytes), so
their targets draw on a pool of distinct datasets: target i uses the rows of pool entry
e_i -- its uvw, visibilities, weights and flags, unchanged -- and carries its own
redshift, offset (l, m) and channel frequencies (the entry's channel count, centred on the
line at that redshift).  Every target's bytes are still read in full when it is stacked.
The visibilities then no longer follow the target's own source model; that changes
nothing the stacking computes or costs.  Nothing here depends on the stacking library or
on the oracle.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .configs import Config, config as _config
from .generate import Target, _channels, make_target


def make_pool(cfg: Config | str, n_entries: int, device="cpu", seed: int | None = None,
              cycle_nchan: bool = True) -> list:
    """n_entries distinct datasets of recipe cfg.  With cycle_nchan, entry e has the
    recipe's channel count number e modulo their number (every count appears)."""
    if isinstance(cfg, str):
        cfg = _config(cfg)
    if seed is not None:
        cfg = dataclasses.replace(cfg, seed=int(seed))
    out = []
    for e in range(n_entries):
        kw = dict(nchan=int(cfg.nchan[e % len(cfg.nchan)])) if cycle_nchan else {}
        out.append(make_target(cfg, e, device, **kw))
    return out


def pool_targets(cfg: Config | str, pool: list, n: int, seed: int) -> list:
    """n targets drawing on the pool: entry, z ~ U(z_range), l, m ~ U(-offset, offset) and
    contiguous channels of the entry's count over the recipe's band centred on
    line_rest / (1 + z), from a PCG64 stream of `seed`."""
    if isinstance(cfg, str):
        cfg = _config(cfg)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(int(seed))))
    out = []
    for _ in range(n):
        e = int(rng.integers(len(pool)))
        z = float(rng.uniform(*cfg.z_range))
        lm = rng.uniform(-cfg.offset, cfg.offset, 2)
        src: Target = pool[e]
        nch = src.nchan
        freq, width = _channels(rng, nch, cfg.band_width, cfg.line_rest / (1.0 + z), False, 0.0, False)
        meta = dict(src.meta, pool_entry=e)
        out.append(dataclasses.replace(src, chan_freq=freq, chan_width=width, l=float(lm[0]), m=float(lm[1]),
                                       z=z, meta=meta, rotate_uvw=False))
    return out
