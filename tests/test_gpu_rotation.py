"""Eq. 1's rotation on the GPU vs the oracle, through the C ABI.

With a target's rotation on, the uv cells come from the rotated baseline: the GPU's
(iu, iv) must equal the oracle's bit for bit (the rotation is built from the same angles
by the same FP64 sequence on both sides), and the stacks and rebinned rows must meet the
same bar as without it.  The offsets (up to 0.3 rad) are large enough for the rotation to
move cells.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_01897_amd import vista  # noqa: E402
from tests.test_gpu_rebin import _term_scale  # noqa: E402
from tests.gpu_util import compare, gpu_stack  # noqa: E402

MODES = {"atomic": 0, "kahan": vista.F_KAHAN, "deterministic": vista.F_DETERMINISTIC,
         "deterministic_kahan": vista.F_DETERMINISTIC | vista.F_KAHAN}


def _targets(name="small", offset=0.3, **kw):
    cfg = synth.config(name, offset=offset)
    return cfg, [dataclasses.replace(t, rotate_uvw=True) for t in synth.make_targets(cfg, **kw)]


def test_rotated_indices_bit_exact():
    cfg, hs = _targets()
    g = synth.make_grid(cfg)
    moved = 0
    for h in hs:
        gi = vista.debug_indices(g, h.to("cuda"))
        oi = oracle.indices(g, h)
        assert np.array_equal(gi["iu"].astype(np.int64), oi["iu"])
        assert np.array_equal(gi["iv"].astype(np.int64), oi["iv"])
        moved += int(np.sum(oi["iu"] != oracle.indices(g, dataclasses.replace(h, rotate_uvw=False))["iu"]))
    assert moved > 0


@pytest.mark.parametrize("mode", list(MODES))
def test_rotated_stack_matches_oracle(mode):
    cfg, hs = _targets()
    g = synth.make_grid(cfg)
    o = oracle.stack(g, hs)
    out, st = gpu_stack(g, [h.to("cuda") for h in hs], flags=MODES[mode])
    compare(o, out, st=st)


def test_rotated_stack_descending_and_mixed():
    """Descending channels, and rotated targets mixed with unrotated ones in one stack."""
    cfg, hs = _targets(descending=True)
    plain = synth.make_targets(synth.config("small"), n=2)
    hs = hs[:2] + plain
    g = synth.make_grid(cfg)
    o = oracle.stack(g, hs)
    out, st = gpu_stack(g, [h.to("cuda") for h in hs])
    compare(o, out, st=st)


def test_rotated_rebin_rows_match_oracle():
    cfg, hs = _targets()
    g = synth.make_grid(cfg)
    ds = [h.to("cuda") for h in hs]
    outs, los, _ = vista.rebin_rows(ds, 40, g["dfreq"], cfg.line_rest)
    torch.cuda.synchronize()
    for h, out, lo in zip(hs, outs, los):
        ora = oracle.rebin_rows(h, lo, g["dfreq"], 40)
        assert lo == oracle.rebin_window(h, cfg.line_rest, g["dfreq"], 40)
        assert np.array_equal(out["uvw"].cpu().numpy(), ora["uvw"])
        assert np.array_equal(out["flag"].cpu().numpy(), ora["flag"])
        # each output relative to its own Eq. 3 terms (the magnitudes' fraction-weighted mean)
        live = ora["flag"] == 0
        scale = _term_scale(h, lo, g["dfreq"], 40)
        err = np.abs(out["vis"].cpu().numpy().astype(np.complex128) - ora["vis"])[live] / scale[live]
        assert err.max() <= 1e-5
