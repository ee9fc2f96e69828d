"""Precision matrix on the precision recipe (baselines to 16 km at 345 GHz, offsets to
60 arcsec): the FP32-argument ablation against the FP64-argument paths (plain,
compensated, deterministic compensated), each against the FP64 oracle on a slab of rest
channels around the line, with max and median relative errors per grid quantity.

Run with -s to see the table (one JSON line)."""
import json

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_01897_amd import vista  # noqa: E402
from tests.gpu_util import TOL  # noqa: E402

N_TARGETS = 4          # of the recipe's 20: all rows and channels of each
SLAB = 96              # rest channels compared, centred on the line


def _errors(o, g, jlo, jhi):
    nz = o["N"] > 0
    S = g["sum_wvis"][jlo:jhi].astype(np.complex128)[nz]
    W = g["sum_w"][jlo:jhi].astype(np.float64)[nz]
    es = np.abs(S - o["S"][nz]) / o["A"][nz]
    ew = np.abs(W - o["W"][nz]) / o["W"][nz]
    r = dict(counts_equal=bool(np.array_equal(g["count"][jlo:jhi].astype(np.uint64), o["N"])),
             S_max=float(es.max()), S_median=float(np.median(es)),
             W_max=float(ew.max()), W_median=float(np.median(ew)))
    if "sum_wvis64" in g:
        e64 = np.abs(g["sum_wvis64"][jlo:jhi][nz] - o["S"][nz]) / o["A"][nz]
        w64 = np.abs(g["sum_w64"][jlo:jhi][nz] - o["W"][nz]) / o["W"][nz]
        r.update(S64_max=float(e64.max()), S64_median=float(np.median(e64)),
                 W64_max=float(w64.max()), W64_median=float(np.median(w64)))
    return r


def test_precision_matrix():
    cfg = synth.config("c3")
    g = synth.make_grid(cfg)
    hs = synth.make_targets(cfg, n=N_TARGETS)
    jlo = int(g["nchan"]) // 2 - SLAB // 2
    jhi = jlo + SLAB
    o = oracle.stack(g, hs, jlo=jlo, jhi=jhi)
    ds = [t.to("cuda") for t in hs]
    paths = {
        "fp32_argument": vista.F_PHASE_FP32,
        "fp32_argument_kahan": vista.F_PHASE_FP32 | vista.F_KAHAN,
        "fp64_argument": 0,
        "fp64_argument_kahan": vista.F_KAHAN,
        "fp64_argument_deterministic_kahan": vista.F_DETERMINISTIC | vista.F_KAHAN,
    }
    table = {}
    for name, fl in paths.items():
        out, st = vista.stack(g, ds, flags=fl, fp64=bool(fl & vista.F_KAHAN))
        host = {k: v[jlo:jhi].cpu().numpy() for k, v in out.items()}
        del out
        table[name] = _errors(o, host, 0, SLAB)
    torch.cuda.empty_cache()
    print(json.dumps({"precision_matrix": table, "workload": "precision recipe, %d of 20 targets, rest "
                      "channels [%d, %d) of %d" % (N_TARGETS, jlo, jhi, int(g["nchan"]))}))
    for name in ("fp64_argument", "fp64_argument_kahan", "fp64_argument_deterministic_kahan"):
        r = table[name]
        assert r["counts_equal"]
        assert r["S_max"] <= TOL and r["W_max"] <= TOL, (name, r)
    for name in ("fp64_argument_kahan", "fp64_argument_deterministic_kahan"):
        assert table[name]["S64_max"] < 1e-6, table[name]
    # forming the argument in FP32 decorrelates long baselines at large offsets
    assert table["fp32_argument"]["S_max"] > 100 * table["fp64_argument"]["S_max"]
