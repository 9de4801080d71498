"""Batched form on the GPU: a mixed batch in one persistent launch gives every
frame bitwise the image of its own per-frame launch (so parity carries over),
graph replays match the eager launch, and bad work lists are refused."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2203_14906_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2203_14906_amd import hodmas
    return hodmas


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


SPECS = [  # (N, S, nx, nz, order, dtype)
    (64, 1024, 96, 80, 1, "f32"), (128, 2048, 128, 128, 6, "f16"), (32, 512, 37, 53, 3, "i16"),
    (64, 1024, 64, 64, 4, "f16"), (16, 600, 40, 24, 2, "f32"), (128, 1024, 200, 100, 5, "i16"),
    (256, 2048, 64, 96, 2, "f16"), (8, 300, 17, 19, 6, "f32"), (64, 2048, 150, 150, 3, "f32"),
    (4, 256, 12, 12, 6, "f16"),  # order above the element count: zero image
]


def make_batch_inputs(hd, specs, seed0=500):
    plans, rfs, outs, orders, frames = [], [], [], [], []
    for i, (n, S, nx, nz, k, dt) in enumerate(specs):
        f = ph.make_frame(n, S, nx, nz, n_points=5, n_lines=1, snr_db=15.0, seed=seed0 + i)
        if dt == "f32":
            arr, scale = ph.to_fp32(f.rf), 1.0
        elif dt == "f16":
            arr, scale = ph.to_fp16(f.rf), 1.0
        else:
            arr, scale = ph.to_int16(f.rf, seed0 + i)
        plans.append(hd.Plan(f.geometry, f.grid, S, dt, max_order=6, dequant_scale=float(scale)))
        rfs.append(torch.from_numpy(arr).cuda())
        outs.append(torch.full((nz, nx), float("nan"), dtype=torch.float32, device="cuda"))
        orders.append(k)
        frames.append((f, arr, float(scale)))
    return plans, rfs, outs, orders, frames


def test_mixed_batch_equals_per_frame_launches(hd):
    plans, rfs, outs, orders, frames = make_batch_inputs(hd, SPECS)
    alone = [p.beamform(r, k) for p, r, k in zip(plans, rfs, orders)]
    torch.cuda.synchronize()
    batch = hd.Batch(max_frames=32, max_units=100000)
    batch.set(plans, rfs, orders, outs)
    inf = batch.info()
    say("batch: %d frames, %d units, grid %d, lds %d" % (inf.n_frames, inf.n_units, inf.grid, inf.lds_bytes))
    batch.launch()
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(alone, outs)):
        assert torch.equal(a, b), "frame %d differs between the batch and its own launch" % i
    # spot parity of two members against the oracle
    for i in (1, 5):
        f, arr, scale = frames[i]
        o = O.beamform(arr, f.geometry, f.grid, orders[i], dequant_scale=scale if arr.dtype == np.int16 else None)
        g = outs[i].cpu().numpy().astype(np.float64)
        err = np.linalg.norm(g - o) / np.linalg.norm(o)
        say("batch member %d (order %d, %s) rel L2 %.3e" % (i, orders[i], arr.dtype, err))
        assert err <= 2e-5
    assert torch.all(outs[-1] == 0)
    batch.close()
    for p in plans:
        p.close()


def test_graph_replays_and_reset_work_list(hd):
    plans, rfs, outs, orders, _ = make_batch_inputs(hd, SPECS[:6], seed0=700)
    alone = [p.beamform(r, k).clone() for p, r, k in zip(plans, rfs, orders)]
    batch = hd.Batch(max_frames=16, max_units=50000)
    batch.set(plans, rfs, orders, outs)
    batch.capture()
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))
        # unrelated eager work between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        batch.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i, (a, b) in enumerate(zip(alone, outs)):
            assert torch.equal(a, b), "replay %d frame %d" % (rep, i)
    # a new work list (other orders, reversed frames) is read by the same graph
    orders2 = [(k % 6) + 1 for k in orders][::-1]
    plans2, rfs2, outs2 = plans[::-1], rfs[::-1], outs[::-1]
    batch.set(plans2, rfs2, orders2, outs2)
    batch.replay()
    torch.cuda.synchronize()
    for p, r, k, o in zip(plans2, rfs2, orders2, outs2):
        assert torch.equal(p.beamform(r, k), o)
    batch.close()
    for p in plans:
        p.close()


def test_graph_replays_follow_changing_kind_mixes(hd):
    """Replays fit the instantiated graph to each work list (absent kinds
    switched off, grids cut to the unit count): a kind that leaves and comes
    back, a single tiny frame, and back-to-back replays without a host wait
    all give every frame its own launch's image."""
    plans, rfs, outs, orders, _ = make_batch_inputs(hd, SPECS, seed0=900)
    alone = [p.beamform(r, k).clone() for p, r, k in zip(plans, rfs, orders)]
    batch = hd.Batch(max_frames=16, max_units=100000)
    batch.set(plans, rfs, orders, outs)
    batch.capture()
    picks = [list(range(len(SPECS))), [2, 8], [9], [4, 0], list(range(len(SPECS))), [7]]
    for step, idx in enumerate(picks):
        for i in idx:
            outs[i].fill_(float("nan"))
        batch.set([plans[i] for i in idx], [rfs[i] for i in idx], [orders[i] for i in idx],
                  [outs[i] for i in idx])
        for _ in range(3):                       # replays queued back to back
            batch.replay()
        torch.cuda.synchronize()
        for i in idx:
            assert torch.equal(alone[i], outs[i]), "step %d frame %d" % (step, i)
        say("replay step %d (frames %s) ok" % (step, idx))
    batch.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("comp", [True, False])
def test_batch_multi_chunk_split_and_batch_lds(hd, comp):
    # units of several chunks, split tilings (combined through LDS between
    # units) and orders above the element count, one after another in a
    # persistent workgroup
    flags = 0 if comp else hd.FLAG_ACC_PLAIN
    cases = [  # (N, S, nx, nz, order, dtype, tiling, extra flags)
        (32, 512, 40, 36, 3, "f32", (16, 16, 1, 5), 0), (24, 400, 33, 29, 6, "f16", (8, 8, 4, 7), 0),
        (48, 700, 45, 50, 2, "i16", (16, 8, 2, 9), 0), (128, 2048, 96, 96, 5, "f32", (8, 8, 4, 43), 0),
        (256, 2048, 64, 64, 4, "f16", (8, 8, 4, 19), 0), (20, 300, 16, 16, 6, "f32", (16, 16, 1, 3), 0),
        (64, 1024, 48, 48, 1, "i16", (16, 16, 1, 64), 0), (5, 200, 18, 18, 6, "f16", (8, 8, 4, 2), 0),
    ]
    plans, rfs, outs, orders = [], [], [], []
    for i, (n, S, nx, nz, k, dt, til, fl) in enumerate(cases):
        f = ph.make_frame(n, S, nx, nz, n_points=4, n_lines=1, snr_db=15.0, seed=900 + i)
        if dt == "f32":
            arr, scale = ph.to_fp32(f.rf), 1.0
        elif dt == "f16":
            arr, scale = ph.to_fp16(f.rf), 1.0
        else:
            arr, scale = ph.to_int16(f.rf, 900 + i)
        p = hd.Plan(f.geometry, f.grid, S, dt, max_order=6, dequant_scale=float(scale), tiling=til,
                    flags=flags | fl)
        t = p.info().tiling
        say("case %d: N=%d %dx%d k=%d %s tiling %s" % (i, n, nx, nz, k, dt, (t.tile_x, t.tile_z, t.split, t.chunk)))
        plans.append(p)
        rfs.append(torch.from_numpy(arr).cuda())
        outs.append(torch.full((nz, nx), float("nan"), dtype=torch.float32, device="cuda"))
        orders.append(k)
    alone = [p.beamform(r, k).clone() for p, r, k in zip(plans, rfs, orders)]
    lds = max(p.info().lds_bytes for p in plans)
    batch = hd.Batch(max_frames=16, max_units=100000, max_lds_bytes=lds, flags=flags)
    batch.set(plans, rfs, orders, outs)
    batch.launch()
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(alone, outs)):
        assert torch.equal(a, b), "case %d differs between the batch and its own launch" % i
    batch.close()
    for p in plans:
        p.close()


def test_batch_rejects_bad_work_lists(hd):
    f = ph.make_frame(16, 256, 20, 20, n_points=2, seed=3)
    p4 = hd.Plan(f.geometry, f.grid, 256, "f32", max_order=4)
    plain = hd.Plan(f.geometry, f.grid, 256, "f32", max_order=6, flags=hd.FLAG_ACC_PLAIN)
    host = hd.Plan(f.geometry, f.grid, 256, "f32", max_order=6, flags=hd.FLAG_HOST_ONLY)
    rf = torch.from_numpy(ph.to_fp32(f.rf)).cuda()
    out = torch.empty((20, 20), dtype=torch.float32, device="cuda")
    b = hd.Batch(max_frames=2, max_units=10000)
    with pytest.raises(hd.HodmasError) as e:
        b.set([p4], [rf], [5], [out])
    assert e.value.status == hd.EUNSUPPORTED
    with pytest.raises(hd.HodmasError) as e:
        b.set([plain], [rf], [2], [out])
    assert e.value.status == hd.EINVAL
    with pytest.raises(hd.HodmasError) as e:
        b.set([host], [rf], [2], [out])
    assert e.value.status == hd.EINVAL
    with pytest.raises(hd.HodmasError) as e:
        b.set([p4, p4, p4], [rf] * 3, [1] * 3, [out] * 3)
    assert e.value.status == hd.EINVAL
    small = hd.Batch(max_frames=2, max_units=1)
    with pytest.raises(hd.HodmasError) as e:
        small.set([p4], [rf], [1], [out])
    assert e.value.status == hd.EINVAL
    tiny_lds = hd.Batch(max_frames=2, max_units=10000, max_lds_bytes=256)
    with pytest.raises(hd.HodmasError) as e:
        tiny_lds.set([p4], [rf], [1], [out])
    assert e.value.status == hd.EINVAL
    with pytest.raises(hd.HodmasError) as e:
        b.launch()                      # nothing set yet
    assert e.value.status == hd.EINVAL
    pl = hd.Batch(max_frames=2, max_units=10000, flags=hd.FLAG_ACC_PLAIN)
    pl.set([plain], [rf], [3], [out])
    pl.launch()
    torch.cuda.synchronize()
    assert torch.equal(out, plain.beamform(rf, 3))
    for x in (b, small, tiny_lds, pl):
        x.close()
    for x in (p4, plain, host):
        x.close()


def test_each_kind_gets_its_own_lds_and_grid(hd):
    """A kind runs with the LDS of its own largest plan, so a small-LDS work
    list gets a larger persistent grid than a large-LDS one in the same batch;
    graph replays refit the nodes' LDS and grid when the list changes, and
    every image stays bitwise its own launch."""
    f = ph.config_frame(1)
    arr = ph.to_fp32(f.rf)
    dev = torch.from_numpy(arr).cuda()
    S = arr.shape[1]
    big = hd.Plan(f.geometry, f.grid, S, "f32", max_order=4, tiling=(16, 16, 1, 64))
    small = hd.Plan(f.geometry, f.grid, S, "f32", max_order=4, tiling=(16, 16, 1, 4))
    lb, ls = big.info().lds_bytes, small.info().lds_bytes
    assert ls < lb
    bt = hd.Batch(max_frames=4, max_units=4 * big.info().n_tiles, max_lds_bytes=64 * 1024)
    outs = [torch.full((f.grid.nz, f.grid.nx), float("nan"), dtype=torch.float32, device="cuda")
            for _ in range(4)]
    ref = {(id(p), k): p.beamform(dev, k).cpu().numpy() for p in (big, small) for k in (2, 4)}
    captured = False
    for rep, plan in enumerate([big, small, big, small]):
        for o in outs:
            o.fill_(float("nan"))
        bt.set([plan] * 4, [dev] * 4, [2, 4, 2, 4], outs)
        inf = bt.info()
        assert inf.lds_bytes == plan.info().lds_bytes
        if plan is small:
            grid_small = inf.grid
        else:
            grid_big = inf.grid
        if not captured:
            bt.launch()
            bt.capture()
            captured = True
        else:
            bt.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            assert np.array_equal(o.cpu().numpy(), ref[(id(plan), [2, 4][i % 2])]), (rep, i)
    say("per-kind LDS: big %d B -> grid %d, small %d B -> grid %d" % (lb, grid_big, ls, grid_small))
    assert grid_small >= grid_big
    bt.close()
    big.close()
    small.close()


def test_graph_gains_kinds_after_capture(hd):
    """A graph captured for one kind holds only that kind's kernel; a later
    work list with other kinds has it rebuilt at the next replay, and every
    frame still gets its own launch's image (also when the list shrinks back)."""
    plans, rfs, outs, orders, _ = make_batch_inputs(hd, SPECS, seed0=950)
    alone = [p.beamform(r, k).clone() for p, r, k in zip(plans, rfs, orders)]
    batch = hd.Batch(max_frames=16, max_units=100000)
    first = [0]
    for step, idx in enumerate([first, list(range(len(SPECS))), first, [len(SPECS) - 1, 1]]):
        for i in idx:
            outs[i].fill_(float("nan"))
        batch.set([plans[i] for i in idx], [rfs[i] for i in idx], [orders[i] for i in idx],
                  [outs[i] for i in idx])
        if step == 0:
            batch.capture()
        for _ in range(2):
            batch.replay()
        torch.cuda.synchronize()
        for i in idx:
            assert torch.equal(alone[i], outs[i]), "step %d frame %d" % (step, i)
    batch.close()
    for p in plans:
        p.close()
