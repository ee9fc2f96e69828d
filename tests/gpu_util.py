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
