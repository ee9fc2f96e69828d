"""Host-side logic of bench.py (no GPU): the one-GPU guard, launch-shape parsing, the
algorithmic byte count, and the rule that a committed counter reading is used only while
the kernel source, workload and launch shape it was taken on are the current ones."""
import hashlib
import json
import os
import subprocess
import sys
import types

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_parse_tuning():
    assert bench.parse_tuning("") is None
    assert bench.parse_tuning("8,4,64,8") == dict(tile_u=8, tile_v=4, jblock=64, waves=8)


def test_algorithmic_bytes():
    """9 B per sample with flags (8 without), 24 + 4 npol B per row (per-channel weights: 24 B
    a row and 4 B a sample), 16 B per grid cell per grid."""
    def target(nrow, nch, npol, flags=True, wpc=False):
        return types.SimpleNamespace(vis=np.zeros((nrow, nch, npol, 1)), flag=np.zeros(1) if flags else None,
                                     weight_per_chan=wpc)
    grid = dict(nu=4, nv=2, nchan=3)
    nb, ns = bench.algorithmic_bytes([target(10, 5, 2)], grid)
    assert ns == 100 and nb == 100 * 9 + 10 * (24 + 8) + 24 * 16
    nb, ns = bench.algorithmic_bytes([target(10, 5, 2, flags=False, wpc=True), target(1, 1, 4)], grid, ngrids=2)
    assert ns == 104 and nb == (100 * 8 + 10 * 24 + 100 * 4) + (4 * 9 + 1 * (24 + 16)) + 2 * 24 * 16


def _profile(tmp_path, src_bytes, **fields):
    src = tmp_path / "kernel.hip"
    src.write_bytes(src_bytes)
    prof = tmp_path / "profile.json"
    prof.write_text(json.dumps(dict(kernel_sha256=hashlib.sha256(src_bytes).hexdigest(), **fields)))
    return str(src), str(prof)


def test_counter_traffic_needs_the_profiled_source_workload_and_shape(tmp_path, monkeypatch):
    shape = dict(tile_u=8, tile_v=4, jblock=160, waves=16)
    src, prof = _profile(tmp_path, b"kernel v1", config="c2", launch_shape=shape, hbm_bytes_per_launch=123.0)
    monkeypatch.setattr(bench, "KERNEL_SRC", src)
    monkeypatch.setattr(bench, "PROFILE_COUNTERS", prof)
    monkeypatch.setattr(bench, "PROFILE_BATCHED", prof)
    assert bench.counter_traffic("c2", dict(shape)) == 123.0
    assert bench.counter_traffic("c3", dict(shape)) is None                        # another workload
    assert bench.counter_traffic("c2", dict(shape, jblock=128)) is None            # another shape
    assert bench.counter_traffic("c2", None) is None
    with open(src, "wb") as f:                                                     # the source changed
        f.write(b"kernel v2")
    assert bench.counter_traffic("c2", dict(shape)) is None


def test_ordered_counter_traffic_reads_its_own_summary(tmp_path, monkeypatch):
    """The deterministic form's traffic comes from the ordered kernel's summary, never from
    the packed kernel's (same source file, workload and test, another launch shape)."""
    shape = dict(tile_u=2, tile_v=2, jblock=64, waves=1)
    src, prof = _profile(tmp_path, b"kernel", config="c2", launch_shape=shape, hbm_bytes_per_launch=9.0)
    monkeypatch.setattr(bench, "KERNEL_SRC", src)
    monkeypatch.setattr(bench, "PROFILE_COUNTERS", str(tmp_path / "missing.json"))
    assert bench.counter_traffic("c2", dict(shape), prof) == 9.0
    assert bench.counter_traffic("c2", dict(shape)) is None
    assert bench.counter_traffic("c2", dict(shape, waves=16), prof) is None


def test_batched_counter_traffic_needs_the_profiled_shape(tmp_path, monkeypatch):
    shape = dict(tile_u=8, tile_v=4, jblock=64, waves=8)
    src, prof = _profile(tmp_path, b"kernel", config="c4", launch_shape=shape, hbm_bytes_per_launch=7.0)
    monkeypatch.setattr(bench, "KERNEL_SRC", src)
    monkeypatch.setattr(bench, "PROFILE_BATCHED", prof)
    assert bench.batched_counter_traffic(dict(shape, source="autotuned")) == 7.0   # extra keys ignored
    assert bench.batched_counter_traffic(dict(shape, waves=16)) is None
    assert bench.batched_counter_traffic(None) is None


def test_image_and_rebin_traffic_follow_their_sources(tmp_path, monkeypatch):
    src, prof = _profile(tmp_path, b"image", config="c2", hbm_bytes_per_call=5.0)
    monkeypatch.setattr(bench, "IMAGE_SRC", src)
    monkeypatch.setattr(bench, "PROFILE_IMAGE", prof)
    assert bench.image_counter_traffic("c2") == 5.0
    assert bench.image_counter_traffic("c1") is None
    src, prof = _profile(tmp_path, b"rebin", config="c2", nout=480, hbm_bytes_per_launch=3.0)
    monkeypatch.setattr(bench, "REBIN_SRC", src)
    monkeypatch.setattr(bench, "PROFILE_REBIN", prof)
    assert bench.rebin_counter_traffic("c2", 480) == 3.0
    assert bench.rebin_counter_traffic("c2", 240) is None


def test_roofline_fields():
    r = bench.roofline(8e9, 2.0, traffic=1.5e10)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["achieved"] - 4000.0) < 1e-9 and abs(r["frac"] - 0.5) < 1e-12 and r["traffic"] == 1.5e10
