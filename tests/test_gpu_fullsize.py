"""Parity at the benchmark's full size (c2: 50 targets x 903 baselines x 120 integrations
x 960 channels x 2 pols, grid 512 x 512 x 960), in the launch shapes the bench times: the
autotuner's usual pick (8 x 4 cells x 160 rest channels, 16 wavefronts), its runner-up
(16 x 2 x 160), the default (8 x 4 x 128), and the plain FP32 form's default
(8 x 4 x 288).

The oracle cannot stack the whole workload in a test, so it checks sampled outputs:
slabs of rest channels (two across rest-channel block boundaries -- the one at 768 is
reached by a single input channel of some targets, so its units stream long runs of
one-channel records --, one on the line, the last one), each computed by the oracle from
only the input channels whose Eq. 4 overlap sets reach the slab -- every cell of the slab
depends on nothing else -- plus identities the statistics and the count grid satisfy at
any size.  The plain FP32 form is held to the first-order bound of FP32 recursive
summation, which grows with each cell's contribution count."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_01897_amd import vista  # noqa: E402
from tests.gpu_util import compare, compare_fp32_plain, reaching  # noqa: E402

SLABS = [(124, 132), (476, 484), (764, 772), (952, 960)]
SHAPES = {
    "tuned_8x4x160": (0, dict(tile_u=8, tile_v=4, jblock=160, waves=16)),
    "tuned_16x2x160": (0, dict(tile_u=16, tile_v=2, jblock=160, waves=16)),
    "default_8x4x128": (0, dict(tile_u=8, tile_v=4, jblock=128, waves=16)),
    "plain_fp32_8x4x288": (vista.F_PLAIN_FP32, dict(tile_u=8, tile_v=4, jblock=288, waves=16)),
}


@pytest.fixture(scope="module")
def c2():
    cfg = synth.config("c2")
    g = synth.make_grid(cfg)
    ts = [synth.make_target(cfg, i, device="cuda") for i in range(cfg.n_targets)]
    refs = []
    for jlo, jhi in SLABS:
        parts = []
        for t in ts:
            r = reaching(g, t, jlo, jhi)
            if r is not None:
                parts.append(t.channel_slice(*r))
        refs.append(oracle.stack(g, parts, jlo=jlo, jhi=jhi, stats=False))
    yield g, ts, refs
    del ts
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", list(SHAPES))
def test_c2_full_size_sampled_slabs(name, c2):
    g, ts, refs = c2
    flags, shape = SHAPES[name]
    out, st = vista.stack(g, ts, flags=flags, tuning=shape)
    torch.cuda.synchronize()

    # identities at any size
    n = sum(int(t.vis.numel()) for t in ts)
    assert st["n_samples"] == n
    assert (st["n_flagged"] + st["n_bad_weight"] + st["n_outside_uv"] + st["n_outside_band"] + st["n_used"]
            == st["n_samples"])
    assert int(out["count"].sum(dtype=torch.int64).item()) == st["n_contrib"]

    for (jlo, jhi), o in zip(SLABS, refs):
        host = {k: v[jlo:jhi].cpu().numpy() for k, v in out.items()}
        if flags & vista.F_PLAIN_FP32:
            err = compare_fp32_plain(o, host)
        else:
            err = compare(o, host, check_stats=False)
        print(name, (jlo, jhi), err, flush=True)
    del out
    torch.cuda.empty_cache()
