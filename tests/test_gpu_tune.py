"""Autotuner on the GPU: picks a valid tiling, caches it, and the tuned plan
keeps parity with the oracle."""
import os
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2203_14906_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_autotune_cache_and_parity(tmp_path):
    assert torch.cuda.is_available()
    from paper_2203_14906_amd import hodmas
    f = ph.config_frame(1)
    cache = str(tmp_path / "tune.jsonl")
    t0 = time.perf_counter()
    til = hodmas.autotune(f.geometry, f.grid, 1024, "f32", 4, cache_path=cache)
    first = time.perf_counter() - t0
    tx, tz, split, chunk = til
    assert tx * tz * split in (256, 512) and split in (1, 2, 4) and chunk >= 1
    assert os.path.exists(cache) and til == tuple(__import__("json").loads(open(cache).readline())["tiling"])
    t0 = time.perf_counter()
    again = hodmas.autotune(f.geometry, f.grid, 1024, "f32", 4, cache_path=cache)
    assert again == til and time.perf_counter() - t0 < first
    plan = hodmas.Plan(f.geometry, f.grid, 1024, "f32", max_order=4, tiling=til)
    arr = ph.to_fp32(f.rf)
    img = plan.beamform(torch.from_numpy(arr).cuda(), 4).cpu().numpy().astype(np.float64)
    ref = O.beamform(arr, f.geometry, f.grid, 4)
    assert np.linalg.norm(img - ref) / np.linalg.norm(ref) <= 1e-5
    plan.close()


def test_autotune_mirror_pairs(tmp_path):
    """With HODMAS_FLAG_MIRROR the tuner keeps only tilings the pairing accepts
    (whole, even tile columns), caches them under their own key, and the tuned
    paired plan keeps parity."""
    assert torch.cuda.is_available()
    from paper_2203_14906_amd import hodmas
    f = ph.config_frame(1)
    cache = str(tmp_path / "tune.jsonl")
    plain = hodmas.autotune(f.geometry, f.grid, 1024, "f32", 2, cache_path=cache)
    til = hodmas.autotune(f.geometry, f.grid, 1024, "f32", 2, flags=hodmas.FLAG_MIRROR, cache_path=cache)
    tx = til[0]
    assert f.grid.nx % tx == 0 and (f.grid.nx // tx) % 2 == 0
    keys = [__import__("json").loads(l)["key"] for l in open(cache)]
    assert len(keys) == 2 and keys[0] != keys[1]
    assert hodmas.autotune(f.geometry, f.grid, 1024, "f32", 2, cache_path=cache) == plain
    plan = hodmas.Plan(f.geometry, f.grid, 1024, "f32", max_order=2, tiling=til, flags=hodmas.FLAG_MIRROR)
    arr = ph.to_fp32(f.rf)
    img = plan.beamform(torch.from_numpy(arr).cuda(), 2).cpu().numpy().astype(np.float64)
    ref = O.beamform(arr, f.geometry, f.grid, 2)
    assert np.linalg.norm(img - ref) / np.linalg.norm(ref) <= 1e-5
    plan.close()


def test_autotune_batch_mirror_pairs(tmp_path):
    """HODMAS_FLAG_TUNE_BATCH | HODMAS_FLAG_MIRROR (the mixed batch's tuning):
    a 256-thread tiling the pairing accepts; a batch of the tuned paired plan
    gives the plan's own images bit for bit."""
    assert torch.cuda.is_available()
    from paper_2203_14906_amd import hodmas
    f = ph.config_frame(1)
    cache = str(tmp_path / "tune.jsonl")
    til = hodmas.autotune(f.geometry, f.grid, 1024, "f16", 6,
                          flags=hodmas.FLAG_TUNE_BATCH | hodmas.FLAG_MIRROR, cache_path=cache)
    tx, tz, split, _ = til
    assert tx * tz * split == 256
    assert f.grid.nx % tx == 0 and (f.grid.nx // tx) % 2 == 0
    plan = hodmas.Plan(f.geometry, f.grid, 1024, "f16", max_order=6, tiling=til, flags=hodmas.FLAG_MIRROR)
    rf = torch.from_numpy(ph.to_fp16(f.rf)).cuda()
    own = [plan.beamform(rf, k).cpu().numpy() for k in (1, 6)]
    bt = hodmas.Batch(max_frames=2, max_units=2 * plan.info().n_tiles, max_lds_bytes=plan.info().lds_bytes)
    outs = [torch.empty((f.grid.nz, f.grid.nx), dtype=torch.float32, device="cuda") for _ in range(2)]
    bt.set([plan, plan], [rf, rf], [1, 6], outs)
    bt.launch()
    torch.cuda.synchronize()
    for o, ref in zip(outs, own):
        assert np.array_equal(o.cpu().numpy(), ref)
    bt.close()
    plan.close()


def test_batch_tuning_times_batches(tmp_path):
    """HODMAS_FLAG_TUNE_BATCH times candidates as a batch runs them: on a
    small grid, where a single frame favours element splits, the tuned tiling
    runs a many-frame batch at least about as fast as the plan's default."""
    assert torch.cuda.is_available()
    from paper_2203_14906_amd import hodmas
    f = ph.config_frame(1)
    cache = str(tmp_path / "tune.jsonl")
    til = hodmas.autotune(f.geometry, f.grid, 1024, "f32", 2, flags=hodmas.FLAG_TUNE_BATCH, cache_path=cache)
    assert til[0] * til[1] * til[2] == 256
    rf = torch.from_numpy(ph.to_fp32(f.rf)).cuda()
    n = 256
    outs = [torch.empty((f.grid.nz, f.grid.nx), dtype=torch.float32, device="cuda") for _ in range(n)]

    def batch_ms(tiling):
        plan = hodmas.Plan(f.geometry, f.grid, 1024, "f32", max_order=2, tiling=tiling)
        bt = hodmas.Batch(max_frames=n, max_units=n * plan.info().n_tiles, max_lds_bytes=plan.info().lds_bytes)
        bt.set([plan] * n, [rf] * n, [2] * n, outs)
        ts = []
        for _ in range(7):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            bt.launch()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        bt.close()
        plan.close()
        return sorted(ts)[3]

    default = hodmas.Plan(f.geometry, f.grid, 1024, "f32", max_order=2).info().tiling
    default = (default.tile_x, default.tile_z, default.split, default.chunk)
    t_tuned, t_default = batch_ms(til), batch_ms(default)
    print("batch-tuned %s %.3f ms, default %s %.3f ms" % (til, t_tuned, default, t_default))
    assert t_tuned <= 1.1 * t_default
