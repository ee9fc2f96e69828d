"""Helpers shared by the GPU parity tests: comparison of a GPU stack with the oracle."""
import numpy as np
import torch

import oracle
import synth
from paper_2609_01897_amd import vista

# Stacked sums must agree with the FP64 oracle to 1e-5, relative to the cell's scale
# A = sum |w f V'| for S (noise cancels inside S, so |S| itself can be tiny) and to W.
TOL = 1e-5


def targets_on_gpu(cfg, n=None, **kw):
    """Targets drawn on the host (so the oracle sees the same bytes), moved to the GPU."""
    ts = synth.make_targets(cfg, n=n, **kw)
    return ts, [t.to("cuda") for t in ts]


def gpu_stack(grid, dts, flags=None, fp64=False, tuning=None):
    out, st = vista.stack(grid, dts, flags=flags, fp64=fp64, tuning=tuning)
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in out.items()}
    return host, st


def compare(o, g, jlo=0, jhi=None, tol=TOL, check_stats=True, st=None):
    """Assert GPU output g (host arrays) equals oracle output o on rest channels [jlo, jhi)."""
    jhi = o["N"].shape[0] + jlo if jhi is None else jhi
    N = g["count"][jlo:jhi].astype(np.int64)
    assert np.array_equal(N, o["N"].astype(np.int64)), "counts differ in %d cells" % int(
        (N != o["N"].astype(np.int64)).sum())
    S = g["sum_wvis"][jlo:jhi].astype(np.complex128)
    W = g["sum_w"][jlo:jhi].astype(np.float64)
    A = o["A"]
    nz = o["N"] > 0
    es = np.abs(S - o["S"])[nz] / A[nz] if nz.any() else np.zeros(1)
    ew = np.abs(W - o["W"])[nz] / o["W"][nz] if nz.any() else np.zeros(1)
    # empty cells must be exactly zero
    assert np.all(S[~nz] == 0) and np.all(W[~nz] == 0)
    assert es.max() <= tol, "max |dS|/A = %g" % es.max()
    assert ew.max() <= tol, "max |dW|/W = %g" % ew.max()
    if check_stats and st is not None:
        assert st == o["stats"], (st, o["stats"])
    return dict(max_dS_over_A=float(es.max()), median_dS_over_A=float(np.median(es)),
                max_dW_over_W=float(ew.max()), median_dW_over_W=float(np.median(ew)))


def data_free(t):
    """A data-free host view of a target: enough for its channel table."""
    npol = int(t.vis.shape[2])
    return dict(uvw=np.zeros((0, 3)), vis=np.zeros((0, int(t.vis.shape[1]), npol), np.complex64),
                weight=np.zeros((0, npol), np.float32), flag=None, chan_freq=t.chan_freq,
                chan_width=t.chan_width, l=t.l, m=t.m, z=t.z, weight_per_chan=False)


def reaching(grid, t, jlo, jhi):
    """Channel range [k0, k1) of target t whose Eq. 4 overlap sets meet rest channels
    [jlo, jhi) (None if no channel does).  The channel-to-rest map is monotonic, so the
    range is contiguous and every cell of the slab depends on nothing else."""
    tab = oracle.channel_table(grid, data_free(t))
    n = len(tab["start"]) - 1
    kq = np.repeat(np.arange(n), np.diff(tab["start"]))
    m = (tab["j"] >= jlo) & (tab["j"] < jhi)
    if not m.any():
        return None
    ks = np.unique(kq[m])
    k0, k1 = int(ks[0]), int(ks[-1]) + 1
    assert ks.size == k1 - k0
    return k0, k1


def host_arrays(t):
    """Host NumPy views (or copies, for device tensors) of a target's bulk arrays."""
    cp = lambda x: None if x is None else x.detach().cpu().numpy()
    return dict(uvw=cp(t.uvw), vis=cp(t.vis), weight=cp(t.weight), flag=cp(t.flag),
                weight_per_chan=bool(t.weight_per_chan))


def oracle_view(t, bulk, k0, k1):
    """The oracle's input for channels [k0, k1) of a pooled target: its own channel axis,
    redshift and offset over the pool entry's arrays, read in place."""
    return dict(bulk, chan_freq=t.chan_freq, chan_width=t.chan_width, l=t.l, m=t.m, z=t.z,
                kbeg=k0, kend=k1, kdata=0, kstride=int(t.nchan))


def compare_fp32_plain(o, g, jlo=0, jhi=None):
    """Comparison for the plain FP32 form: counts exact; each sum within the first-order
    bound of recursive FP32 summation, (n + 2) 2^-24 of its cell scale (n contributions,
    plus the rounding of each term), on top of the usual 1e-5."""
    jhi = o["N"].shape[0] + jlo if jhi is None else jhi
    N = g["count"][jlo:jhi].astype(np.int64)
    assert np.array_equal(N, o["N"].astype(np.int64))
    nz = o["N"] > 0
    n = o["N"][nz].astype(np.float64)
    bound = TOL + (n + 2.0) * 2.0 ** -24
    S = g["sum_wvis"][jlo:jhi].astype(np.complex128)
    W = g["sum_w"][jlo:jhi].astype(np.float64)
    es = np.abs(S - o["S"])[nz] / o["A"][nz]
    ew = np.abs(W - o["W"])[nz] / o["W"][nz]
    assert np.all(es <= bound), "max excess |dS|/A %g" % float((es - bound).max())
    assert np.all(ew <= bound), "max excess |dW|/W %g" % float((ew - bound).max())
    return dict(max_dS_over_A=float(es.max()), median_dS_over_A=float(np.median(es)),
                max_dW_over_W=float(ew.max()), max_count=int(n.max()))
