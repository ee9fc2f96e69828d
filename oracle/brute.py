"""Pure-Python brute force of the stacking definition, for tiny inputs only.

TEST INFRASTRUCTURE ONLY.  A second, independently written implementation of the same
definition as ``vista_oracle.c`` (scalar ``math`` in double precision, dictionaries for
the grid), used to check the C oracle on small random cases.  It follows the paper's
steps directly: rest-frame edges (Sec. 3.1), the Eq. 2 phase shift with
(dl, dm, dn) = (-l, -m, 1-n), the Eq. 3-4 overlap fractions with centred-difference
widths, and a nearest-cell (u, v, nu_rest) accumulation.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299792458.0


def _widths(freq, width):
    n = len(freq)
    if width is not None:
        return [float(x) for x in width]
    out = []
    for k in range(n):
        if k == 0:
            out.append(abs(freq[1] - freq[0]))
        elif k == n - 1:
            out.append(abs(freq[n - 1] - freq[n - 2]))
        else:
            out.append(abs(freq[k + 1] - freq[k - 1]) / 2.0)
    return out


def overlap_pairs(grid, freq, width, z):
    """For each input channel the list of (j, f_kj) with f_kj > 1e-9 (Eq. 4)."""
    opz = 1.0 + z
    Ws = _widths([float(x) for x in freq], width)
    pairs = []
    for k, nu in enumerate(freq):
        nu = float(nu)
        if grid.get("flags", 0) & 4:
            x = math.floor((nu * opz - grid["freq_lo"]) / grid["dfreq"])
            pairs.append([(int(x), 1.0)] if 0 <= x < grid["nchan"] else [])
            continue
        lo = (nu - 0.5 * Ws[k]) * opz
        hi = (nu + 0.5 * Ws[k]) * opz
        wr = Ws[k] * opz
        lst = []
        for j in range(grid["nchan"]):
            ej = grid["freq_lo"] + float(j) * grid["dfreq"]
            ej1 = grid["freq_lo"] + float(j + 1) * grid["dfreq"]
            ov = min(hi, ej1) - max(lo, ej)
            if ov / wr > 1e-9:
                lst.append((j, ov / wr))
        pairs.append(lst)
    return pairs


def rotation(t: dict):
    """Eq. 1's rotation written from its closed-form elements (d = ra1 - ra0):
    rows (east, north, towards) of the stacking position's uvw frame dotted with those of
    the phase centre's.  Returns (R, l, m); R is None without the rotation."""
    if not t.get("rotate_uvw"):
        return None, float(t["l"]), float(t["m"])
    a0, d0, a1, d1 = float(t["ra0"]), float(t["dec0"]), float(t["ra1"]), float(t["dec1"])
    d = a1 - a0
    sd0, cd0, sd1, cd1 = math.sin(d0), math.cos(d0), math.sin(d1), math.cos(d1)
    R = [[math.cos(d), sd0 * math.sin(d), -cd0 * math.sin(d)],
         [-sd1 * math.sin(d), sd1 * sd0 * math.cos(d) + cd1 * cd0, cd1 * sd0 - sd1 * cd0 * math.cos(d)],
         [cd1 * math.sin(d), sd1 * cd0 - cd1 * sd0 * math.cos(d), sd1 * sd0 + cd1 * cd0 * math.cos(d)]]
    return R, R[2][0], R[2][1]


def _rot(R, u, v, w):
    if R is None:
        return u, v, w
    return tuple(R[i][0] * u + R[i][1] * v + R[i][2] * w for i in range(3))


def stack(grid: dict, targets) -> dict:
    """Returns {(j, iv, iu): [S (complex), W, A, N]} and the sample classification."""
    cells = {}
    st = dict(n_samples=0, n_flagged=0, n_bad_weight=0, n_outside_uv=0, n_outside_band=0, n_used=0,
              n_contrib=0)
    nu_, nv_ = grid["nu"], grid["nv"]
    for t in targets:
        uvw = np.asarray(t["uvw"], np.float64)
        vis = np.asarray(t["vis"])
        if not np.iscomplexobj(vis):
            vis = vis.view(np.complex64)[..., 0] if vis.shape[-1] == 2 else vis
        flag = t.get("flag")
        weight = np.asarray(t["weight"], np.float32)
        freq = [float(x) for x in t["chan_freq"]]
        pairs = overlap_pairs(grid, freq, t.get("chan_width"), float(t["z"]))
        R, l, m = rotation(t)
        n_minus_1 = -(l * l + m * m) / (1.0 + math.sqrt(1.0 - (l * l + m * m)))
        npol = vis.shape[2]
        for r in range(uvw.shape[0]):
            ur, vr, _ = _rot(R, float(uvw[r, 0]), float(uvw[r, 1]), float(uvw[r, 2]))
            for k in range(len(freq)):
                a = freq[k] / C_LIGHT
                u, v, w = float(uvw[r, 0]) * a, float(uvw[r, 1]) * a, float(uvw[r, 2]) * a
                ru = round_half_even((ur * a) * (1.0 / grid["du"]))
                rv = round_half_even((vr * a) * (1.0 / grid["dv"]))
                inside = (-(nu_ // 2) <= ru < nu_ - nu_ // 2) and (-(nv_ // 2) <= rv < nv_ - nv_ // 2)
                turns = u * l + v * m + w * n_minus_1
                ph = 2.0 * math.pi * (turns - round_half_even(turns))
                rot = complex(math.cos(ph), math.sin(ph))
                for p in range(npol):
                    st["n_samples"] += 1
                    if not pairs[k]:
                        st["n_outside_band"] += 1
                        continue
                    if not inside:
                        st["n_outside_uv"] += 1
                        continue
                    if flag is not None and flag[r, k, p]:
                        st["n_flagged"] += 1
                        continue
                    wt = float(weight[r, k, p] if t.get("weight_per_chan") else weight[r, p])
                    if not (wt > 0.0 and math.isfinite(wt)):
                        st["n_bad_weight"] += 1
                        continue
                    st["n_used"] += 1
                    vv = complex(float(vis[r, k, p].real), float(vis[r, k, p].imag)) * rot
                    for j, f in pairs[k]:
                        key = (j, int(rv) + nv_ // 2, int(ru) + nu_ // 2)
                        c = cells.setdefault(key, [0j, 0.0, 0.0, 0])
                        c[0] += wt * f * vv
                        c[1] += wt * f
                        c[2] += wt * f * abs(vv)
                        c[3] += 1
                        st["n_contrib"] += 1
    return dict(cells=cells, stats=st)


def round_half_even(x: float) -> float:
    """IEEE round-to-nearest-even of a double (math.floor based, exact for |x| < 2^52)."""
    if not math.isfinite(x):
        return x
    f = math.floor(x)
    d = x - f
    if d > 0.5:
        return f + 1.0
    if d < 0.5:
        return f
    return f if (f % 2.0) == 0.0 else f + 1.0


def rebin_window(freq, width, z, central_freq, dfreq, nout):
    """The target's own output window (Sec. 3.1): centred on central_freq, moved to the
    nearest edge of the rest-frame band when it does not fit; returns its lower edge."""
    opz = 1.0 + z
    freq = [float(x) for x in freq]
    Ws = _widths(freq, width)
    lo = min((nu - 0.5 * W) * opz for nu, W in zip(freq, Ws))
    hi = max((nu + 0.5 * W) * opz for nu, W in zip(freq, Ws))
    span = float(nout) * dfreq
    start = central_freq - 0.5 * span
    if start + span > hi:
        start = hi - span
    if start < lo:
        start = lo
    return start


def rebin_rows(t: dict, freq_lo: float, dfreq: float, nout: int) -> dict:
    """Eq. 3 per row and polarisation on the window [freq_lo + j dfreq, freq_lo + (j+1) dfreq):
    the Eq. 4-weighted mean of the Eq. 2-rotated unflagged inputs; flagged (and 0) where
    nothing unflagged overlaps; uvw divided by 1 + z."""
    grid = dict(freq_lo=freq_lo, dfreq=dfreq, nchan=nout, flags=0)
    uvw = np.asarray(t["uvw"], np.float64)
    vis = np.asarray(t["vis"])
    flag = t.get("flag")
    freq = [float(x) for x in t["chan_freq"]]
    z = float(t["z"])
    pairs = overlap_pairs(grid, freq, t.get("chan_width"), z)
    R, l, m = rotation(t)
    n_minus_1 = -(l * l + m * m) / (1.0 + math.sqrt(1.0 - (l * l + m * m)))
    nrow, npol = uvw.shape[0], vis.shape[2]
    out = np.zeros((nrow, nout, npol), np.complex128)
    oflag = np.ones((nrow, nout, npol), np.uint8)
    wsum = np.zeros((nrow, nout, npol), np.float64)
    for r in range(nrow):
        num = {}
        den = {}
        for k in range(len(freq)):
            a = freq[k] / C_LIGHT
            turns = (float(uvw[r, 0]) * a * l + float(uvw[r, 1]) * a * m + float(uvw[r, 2]) * a * n_minus_1)
            ph = 2.0 * math.pi * (turns - round_half_even(turns))
            rot = complex(math.cos(ph), math.sin(ph))
            for j, f in pairs[k]:
                for p in range(npol):
                    if flag is not None and flag[r, k, p]:
                        continue
                    vv = complex(float(vis[r, k, p].real), float(vis[r, k, p].imag)) * rot
                    num[(j, p)] = num.get((j, p), 0j) + f * vv
                    den[(j, p)] = den.get((j, p), 0.0) + f
        for (j, p), d in den.items():
            if d > 0.0:
                out[r, j, p] = num[(j, p)] / d
                oflag[r, j, p] = 0
                wsum[r, j, p] = d
    ruvw = np.array([_rot(R, *[float(x) for x in uvw[r]]) for r in range(nrow)], np.float64).reshape(nrow, 3)
    return dict(vis=out, flag=oflag, wsum=wsum, uvw=ruvw / (1.0 + z))
