"""Parity on the batched and streamed recipes at their own shapes.

Batched recipe: 64 stacks of lognormal target counts (clip(round(lognormal(ln 40, 1)),
5, 500)), 12-50 antennas, 60 integrations, channel counts from {128, 480, 960, 3840},
z ~ U(0.5, 4), grids of 256 x 256 x 256.  A seeded subset of 4 of the 64 stacks runs as
one batch (one captured launch sequence), and every stack of it is checked against the
oracle.  Streamed recipe: one stack of 200 targets of 903 baselines x 60 integrations x
3840 channels x 2 polarisations (666 GB) streamed from pinned host memory in waves with
the compensated state carried across them, grid 1024 x 1024 x 1920.

Both recipes hold more input than any memory, so their targets draw on a pool of distinct
datasets, each target with its own redshift, offset and channel axis.  The oracle cannot
stack them whole in a test: it computes slabs of rest channels from only the input
channels that reach them (the channel-to-rest map is monotonic), reading the pool in
place; the statistics and the count grid are checked whole by identities that hold at
any size."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_01897_amd import vista  # noqa: E402
from tests.gpu_util import compare, host_arrays, oracle_view, reaching  # noqa: E402

C4_SIZES_SEED = 20260904          # stack sizes of the 64-stack recipe
C4_PICK_SEED = 20260914           # which 4 of the 64 stacks the test runs
C4_POOL = 24                      # distinct datasets (about 19 GB)
C5_POOL = 8                       # distinct pinned datasets (about 30 GB)
C5_TARGETS = 200


def _identities(st, out, targets):
    n = sum(int(t.vis.numel()) for t in targets)
    assert st["n_samples"] == n
    assert (st["n_flagged"] + st["n_bad_weight"] + st["n_outside_uv"] + st["n_outside_band"] + st["n_used"]
            == st["n_samples"])
    cnt = out["count"].view(torch.int32)               # counts stay far below 2^31
    assert int(cnt.sum(dtype=torch.int64).item()) == st["n_contrib"]


def _slab_check(grid, targets, bulk_of, out, jlo, jhi, tol_fn=compare):
    views = []
    for t in targets:
        r = reaching(grid, t, jlo, jhi)
        if r is not None:
            views.append(oracle_view(t, bulk_of(t), *r))
    o = oracle.stack(grid, views, jlo=jlo, jhi=jhi, stats=False)
    host = {k: v[jlo:jhi].cpu().numpy() for k, v in out.items()}
    err = tol_fn(o, host, check_stats=False)
    print("slab", (jlo, jhi), "targets reaching", len(views), err, flush=True)
    return err


@pytest.mark.parametrize("tuning", [None, dict(tile_u=8, tile_v=4, jblock=64, waves=8)],
                         ids=["default_shape", "tuned_shape"])
def test_c4_seeded_subset_in_one_batch(tuning):
    """Four seeded stacks of the batched recipe in one batch, in the library's default
    launch shape and in the one the autotuner picks for the whole recipe (8 x 4 x 64,
    8 wavefronts), each stack against the oracle."""
    cfg = synth.config("c4")
    sizes = synth.batch_stack_sizes(64, seed=C4_SIZES_SEED)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(C4_PICK_SEED)))
    pick = sorted(int(i) for i in rng.choice(64, 4, replace=False))
    pool = synth.make_pool(cfg, C4_POOL, device="cuda")
    stacks = [synth.pool_targets(cfg, pool, sizes[s], seed=C4_SIZES_SEED * 100 + s) for s in pick]
    print("stacks", pick, "targets", [len(x) for x in stacks], flush=True)
    grid = synth.make_grid(cfg)
    outs = [vista.alloc_outputs(grid) for _ in stacks]
    b = vista.Batch([grid] * len(stacks), tuning=tuning)
    for s, ts in enumerate(stacks):
        for t in ts:
            b.add(s, t)
        b.set_output(s, outs[s])
    b.run()
    tim = b.timings()
    sts = [b.finalize(s) for s in range(len(stacks))]
    b.close()
    torch.cuda.synchronize()
    assert tim["n_waves"] == 1
    print("batch", tim, flush=True)
    hosts = [host_arrays(e) for e in pool]
    bulk_of = lambda t: hosts[t.meta["pool_entry"]]
    # a slab across the block edge at 128, one each side of the line, one reached only by
    # the more distant targets
    slabs = [(124, 132), (96, 104), (150, 158), (70, 78)]
    for s, ts in enumerate(stacks):
        _identities(sts[s], outs[s], ts)
        _slab_check(grid, ts, bulk_of, outs[s], *slabs[s])


def test_c5_stack_streamed_from_pinned_memory():
    cfg = synth.config("c5")
    grid = synth.make_grid(cfg, vista.F_KAHAN)
    pin = lambda x: None if x is None else torch.empty(x.shape, dtype=x.dtype, pin_memory=True).copy_(x)
    pool = []
    for e in synth.make_pool(cfg, C5_POOL, device="cuda"):
        import dataclasses
        pool.append(dataclasses.replace(e, uvw=pin(e.uvw), vis=pin(e.vis), weight=pin(e.weight), flag=pin(e.flag)))
        del e
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    targets = synth.pool_targets(cfg, pool, C5_TARGETS, seed=cfg.seed * 100 + 1)
    out = vista.alloc_outputs(grid)
    b = vista.Batch([grid])
    for t in targets:
        b.add(0, t)
    b.set_output(0, out)
    b.run()
    tim = b.timings()
    st = b.finalize(0)
    b.close()
    torch.cuda.synchronize()
    print("streamed", tim, flush=True)
    assert tim["n_waves"] >= 4, tim
    _identities(st, out, targets)
    hosts = [host_arrays(e) for e in pool]                 # pinned: read in place
    bulk_of = lambda t: hosts[t.meta["pool_entry"]]
    _slab_check(grid, targets, bulk_of, out, 840, 1080)
