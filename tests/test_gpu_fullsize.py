"""Parity at the benchmark's full size (c2: 50 targets x 903 baselines x 120 integrations
x 960 channels x 2 pols, grid 512 x 512 x 960), in the launch shape the bench times.

The oracle cannot stack the whole workload in a test, so it checks sampled outputs:
slabs of rest channels (two across rest-channel block boundaries -- the one at 768 is
reached by a single input channel of some targets, so its units stream long runs of
one-channel records --, one on the line, the last one), each computed by the oracle from only the input channels whose Eq. 4 overlap
sets reach the slab -- every cell of the slab depends on nothing else -- plus identities
the statistics and the count grid satisfy at any size."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_01897_amd import vista  # noqa: E402
from tests.gpu_util import compare  # noqa: E402

BENCH_SHAPE = dict(tile_u=8, tile_v=4, jblock=128, waves=16)
SLABS = [(124, 132), (476, 484), (764, 772), (952, 960)]


def _meta(t):
    """A data-free host view of a target: enough for its channel table."""
    npol = int(t.vis.shape[2])
    return dict(uvw=np.zeros((0, 3)), vis=np.zeros((0, int(t.vis.shape[1]), npol), np.complex64),
                weight=np.zeros((0, npol), np.float32), flag=None, chan_freq=t.chan_freq,
                chan_width=t.chan_width, l=t.l, m=t.m, z=t.z, weight_per_chan=False)


def _reaching(tab, jlo, jhi):
    """Channel range [k0, k1) whose overlap sets meet rest channels [jlo, jhi)."""
    ks = [k for k in range(len(tab["start"]) - 1)
          if np.any((tab["j"][tab["start"][k]:tab["start"][k + 1]] >= jlo) &
                    (tab["j"][tab["start"][k]:tab["start"][k + 1]] < jhi))]
    if not ks:
        return None
    assert ks[-1] - ks[0] + 1 == len(ks)          # monotonic channel -> rest map
    return ks[0], ks[-1] + 1


def test_c2_full_size_sampled_slabs():
    cfg = synth.config("c2")
    g = synth.make_grid(cfg)
    ts = [synth.make_target(cfg, i, device="cuda") for i in range(cfg.n_targets)]
    out, st = vista.stack(g, ts, tuning=BENCH_SHAPE)
    torch.cuda.synchronize()

    # identities at any size
    n = sum(int(t.vis.numel()) for t in ts)
    assert st["n_samples"] == n
    assert (st["n_flagged"] + st["n_bad_weight"] + st["n_outside_uv"] + st["n_outside_band"] + st["n_used"]
            == st["n_samples"])
    assert int(out["count"].to(torch.int64).sum().item()) == st["n_contrib"]

    tabs = [oracle.channel_table(g, _meta(t)) for t in ts]
    for jlo, jhi in SLABS:
        parts = []
        for t, tab in zip(ts, tabs):
            r = _reaching(tab, jlo, jhi)
            if r is not None:
                parts.append(t.channel_slice(*r))
        o = oracle.stack(g, parts, jlo=jlo, jhi=jhi, stats=False)
        host = {k: v[jlo:jhi].cpu().numpy() for k, v in out.items()}
        err = compare(o, host, check_stats=False)
        print((jlo, jhi), len(parts), err)
