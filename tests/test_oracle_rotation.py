"""Pins of the oracle's Eq. 1 rotation (CPU only).

With a target's rotation switched on, the uv cell comes from the baseline rotated from the
phase centre (ra0, dec0) to the stacking position (ra1, dec1), and (l, m) are the stacking
position's direction cosines.  Pinned here by the mathematics of the rotation (orthonormal,
proper, identity for equal centres, inverse by swapping them, third row = the closed-form
direction cosines, w' - w = the Eq. 2 turns), a closed-form case (both centres on the
equator: a rotation about the v axis, checked down to the cell indices), a pure-Python
second implementation built from the closed-form matrix elements, and agreement with the
unrotated path where the rotation is the identity.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import brute


def _rotated(t, ra0=None, dec0=None, ra1=None, dec1=None):
    kw = dict(rotate_uvw=True)
    for k, v in (("ra0", ra0), ("dec0", dec0), ("ra1", ra1), ("dec1", dec1)):
        if v is not None:
            kw[k] = v
    return dataclasses.replace(t, **kw)


CENTRES = [(0.0, -0.52, 0.01, -0.5), (1.3, 0.7, 1.1, 0.95), (4.0, -1.2, 4.6, -1.3), (2.0, 0.0, 2.0, 0.0),
           (0.3, 1.55, 2.9, 1.5)]


@pytest.mark.parametrize("centres", CENTRES)
def test_rotation_is_proper_orthonormal_with_closed_form_third_row(centres):
    t = _rotated(synth.make_target("tiny", 0), *centres)
    R, l, m, nm1 = oracle.rotation(t)
    assert np.max(np.abs(R @ R.T - np.eye(3))) < 1e-15
    assert abs(np.linalg.det(R) - 1.0) < 1e-15
    ra0, dec0, ra1, dec1 = centres
    d = ra1 - ra0
    lc = math.cos(dec1) * math.sin(d)
    mc = math.sin(dec1) * math.cos(dec0) - math.cos(dec1) * math.sin(dec0) * math.cos(d)
    nc = math.sin(dec1) * math.sin(dec0) + math.cos(dec1) * math.cos(dec0) * math.cos(d)
    assert np.max(np.abs(R[2] - [lc, mc, nc])) < 1e-15
    assert (l, m) == (R[2, 0], R[2, 1])
    assert abs(nm1 - (nc - 1.0)) < 1e-15


@pytest.mark.parametrize("centres", CENTRES)
def test_rotation_inverse_and_phase_identity(centres):
    """Swapping the centres inverts R; the rotated w minus the original w is exactly the
    Eq. 2 turns u l + v m + w (n - 1) the shift removes."""
    ra0, dec0, ra1, dec1 = centres
    t = synth.make_target("tiny", 0)
    R, l, m, nm1 = oracle.rotation(_rotated(t, ra0, dec0, ra1, dec1))
    Ri, _, _, _ = oracle.rotation(_rotated(t, ra1, dec1, ra0, dec0))
    assert np.max(np.abs(Ri @ R - np.eye(3))) < 1e-15
    uvw = t.uvw.numpy()
    w_rot = uvw @ R[2]
    turns = uvw[:, 0] * l + uvw[:, 1] * m + uvw[:, 2] * nm1
    assert np.max(np.abs((w_rot - uvw[:, 2]) - turns)) <= 1e-12 * np.max(np.abs(uvw))


def test_rotation_identity_when_centres_coincide():
    """Equal centres: R is the identity and the stack equals the unrotated one with
    l = m = 0 (cells, counts and sums)."""
    cfg = synth.config("tiny")
    g = synth.make_grid(cfg)
    ts = synth.make_targets(cfg)
    rot = [_rotated(t, t.ra0, t.dec0, t.ra0, t.dec0) for t in ts]
    for t in rot:
        R, l, m, _ = oracle.rotation(t)
        assert np.max(np.abs(R - np.eye(3))) < 1e-16 and l == 0.0 and abs(m) < 1e-16
    plain = [dataclasses.replace(t, l=0.0, m=0.0) for t in ts]
    a, b = oracle.stack(g, rot), oracle.stack(g, plain)
    assert np.array_equal(a["N"], b["N"])
    assert np.max(np.abs(a["S"] - b["S"])) <= 1e-15 * max(1.0, np.max(a["A"]))


@pytest.mark.parametrize("theta", [0.05, -0.3, 1.0])
def test_equatorial_rotation_closed_form_cells(theta):
    """Both centres on the equator, the stacking position theta east of the phase centre:
    R rotates about the v axis, u' = cos(theta) u - sin(theta) w, v' = v; the oracle's
    cells are rint(u' a_k / du) + nu/2 exactly."""
    cfg = synth.config("tiny")
    g = synth.make_grid(cfg)
    t = _rotated(synth.make_target(cfg, 1), 0.0, 0.0, theta, 0.0)
    R, _, _, _ = oracle.rotation(t)
    assert np.array_equal(R, [[math.cos(theta), 0.0, -math.sin(theta)], [0.0, 1.0, 0.0],
                              [math.sin(theta), 0.0, math.cos(theta)]])
    uvw = t.uvw.numpy()
    up = math.cos(theta) * uvw[:, 0] + 0.0 * uvw[:, 1] + (-math.sin(theta)) * uvw[:, 2]
    vp = 0.0 * uvw[:, 0] + 1.0 * uvw[:, 1] + 0.0 * uvw[:, 2]
    a = t.chan_freq / 299792458.0
    iu = np.rint((up[:, None] * a[None, :]) * (1.0 / g["du"])).astype(np.int64) + g["nu"] // 2
    iv = np.rint((vp[:, None] * a[None, :]) * (1.0 / g["dv"])).astype(np.int64) + g["nv"] // 2
    oi = oracle.indices(g, t)
    assert np.array_equal(oi["iu"], iu) and np.array_equal(oi["iv"], iv)


@pytest.mark.parametrize("variant", ["plain", "descending", "jitter_width"])
def test_rotation_brute_force_matches_oracle(variant):
    """The pure-Python second implementation (R from its closed-form elements) agrees on
    tiny random stacks with the rotation on, and on the rebinned rows' baselines."""
    cfg = synth.config("tiny", offset=0.3)        # offsets large enough for R to move cells
    kw = {"plain": {}, "descending": dict(descending=True), "jitter_width": dict(chan_jitter=0.4,
                                                                                  with_width=True)}[variant]
    g = synth.make_grid(cfg)
    ts = [_rotated(t) for t in synth.make_targets(cfg, **kw)]
    moved = sum(int(np.sum(oracle.indices(g, t)["iu"] != oracle.indices(g, dataclasses.replace(
        t, rotate_uvw=False))["iu"])) for t in ts)
    assert moved > 0                               # the rotation changes some cells here
    hs = [t.numpy() for t in ts]
    b = brute.stack(g, hs)
    o = oracle.stack(g, ts)
    assert o["stats"] == b["stats"]
    nz = {tuple(int(x) for x in c) for c in np.argwhere(o["N"] > 0)}
    assert nz == set(b["cells"].keys())
    for key, (S, W, A, N) in b["cells"].items():
        assert int(o["N"][key]) == N
        assert abs(o["S"][key] - S) <= 1e-12 * max(A, 1e-300)
    h = hs[0]
    lo = oracle.rebin_window(h, cfg.line_rest, g["dfreq"], 6)
    ob = oracle.rebin_rows(h, lo, g["dfreq"], 6)
    bb = brute.rebin_rows(h, lo, g["dfreq"], 6)
    assert np.max(np.abs(ob["uvw"] - bb["uvw"])) <= 1e-15 * np.max(np.abs(h["uvw"]))
    assert np.array_equal(ob["flag"], bb["flag"])
    assert np.max(np.abs(ob["vis"] - bb["vis"])) <= 1e-12 * float(np.max(np.abs(h["vis"])))


def test_rotation_validation():
    t = synth.make_target("tiny", 0)
    with pytest.raises(ValueError):                # the stacking position behind the phase centre
        oracle.indices(synth.make_grid("tiny"), _rotated(t, 0.0, 0.0, math.pi, 0.0))
    with pytest.raises(ValueError):
        oracle.indices(synth.make_grid("tiny"), _rotated(t, 0.0, float("nan"), 0.1, 0.0))
