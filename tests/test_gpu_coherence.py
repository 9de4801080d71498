"""Coherence-factor weighting in the per-frame and batched kernels against the
FP64 oracle (same stored values): relative L2 within 1e-5 for FP32 storage
and 2e-5 on the same stored values for FP16 / int16, plus the exact
constant-channel cases and the entry points that refuse weighted plans."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2203_14906_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f16": 2e-5, "i16": 2e-5}


@pytest.fixture(scope="module")
def hd():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2203_14906_amd import hodmas
    return hodmas


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(g, o):
    n = np.linalg.norm(o)
    return np.linalg.norm(g - o) / n if n > 0 else np.linalg.norm(g)


def stored(rf, dtype, seed=0):
    if dtype == "f32":
        return ph.to_fp32(rf), 1.0
    if dtype == "f16":
        return ph.to_fp16(rf), 1.0
    codes, scale = ph.to_int16(rf, seed)
    return codes, float(scale)


@pytest.mark.parametrize("tiling", [None, (16, 16, 1, 64), (16, 8, 2, 5), (8, 8, 4, 3)])
@pytest.mark.parametrize("dtype", ["f32", "f16", "i16"])
def test_weighted_small_ragged_frames(hd, tiling, dtype):
    f = ph.make_frame(13, 300, 37, 53, n_points=6, n_lines=1, snr_db=15.0, seed=17)
    grid = ph.Grid(nx=37, nz=53, x0_m=-3e-3, dx_m=0.17e-3, z0_m=0.2e-3, dz_m=0.21e-3)
    arr, scale = stored(f.rf, dtype, seed=17)
    plan = hd.Plan(f.geometry, grid, arr.shape[1], dtype, max_order=6, dequant_scale=scale, tiling=tiling,
                   flags=hd.FLAG_CF)
    dev = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    for k in range(1, 7):
        g = plan.beamform(dev, k).cpu().numpy().astype(np.float64)
        o = O.beamform(arr, f.geometry, grid, k, dequant_scale=scale if dtype == "i16" else None,
                       weighting="cf")
        err = rel_l2(g, o)
        say("CF small %s %s k=%d rel L2 %.2e" % (dtype, tiling, k, err))
        assert err <= TOL[dtype]
    plan.close()


@pytest.mark.parametrize("cfg,orders", [(1, (1, 2, 3, 4)), (2, (1, 3, 6))])
def test_weighted_configs(hd, cfg, orders):
    f = ph.config_frame(cfg)
    arr = ph.to_fp32(f.rf)
    dev = torch.from_numpy(arr).cuda()
    for flags in (hd.FLAG_CF, hd.FLAG_CF | hd.FLAG_ACC_PLAIN):
        plan = hd.Plan(f.geometry, f.grid, arr.shape[1], "f32", max_order=6, flags=flags)
        for k in orders:
            g = plan.beamform(dev, k).cpu().numpy().astype(np.float64)
            o = O.beamform(arr, f.geometry, f.grid, k, weighting="cf")
            err = rel_l2(g, o)
            say("CF config %d flags %d k=%d rel L2 %.2e" % (cfg, flags, k, err))
            assert err <= 1e-5
        plan.close()


def test_constant_channels_and_refusals(hd):
    n, S = 16, 400
    geom = ph.Geometry(n)
    grid = ph.Grid(nx=9, nz=7, x0_m=-1e-3, dx_m=0.25e-3, z0_m=3e-3, dz_m=0.3e-3)
    same = np.full((n, S), 0.7, dtype=np.float32)
    alt = np.repeat(np.array([0.7 if i % 2 == 0 else -0.7 for i in range(n)], dtype=np.float32)[:, None], S, axis=1)
    wplan = hd.Plan(geom, grid, S, "f32", max_order=4, flags=hd.FLAG_CF)
    plan = hd.Plan(geom, grid, S, "f32", max_order=4)
    for k in (1, 2, 4):
        a = wplan.beamform(torch.from_numpy(same).cuda(), k).cpu().numpy()
        b = plan.beamform(torch.from_numpy(same).cuda(), k).cpu().numpy()
        np.testing.assert_allclose(a, b, rtol=1e-6)           # fully coherent: CF = 1
        z = wplan.beamform(torch.from_numpy(alt).cuda(), k).cpu().numpy()
        assert np.abs(z).max() <= 1e-6 * np.abs(b).max()      # cancelling aperture: CF = 0
    torch.cuda.synchronize()
    # weighted plans are refused where the kernels carry no weighting
    out = torch.empty((7, 9), dtype=torch.float32, device="cuda")
    ptrs = (ctypes.c_void_p * 2)(out.data_ptr(), out.data_ptr())
    rf = torch.from_numpy(same).cuda()
    assert hd.lib.hodmas_beamform_orders(wplan.handle, ctypes.c_void_p(rf.data_ptr()), 2, ptrs, None) == \
        hd.EUNSUPPORTED
    # the weighted batch kinds accumulate compensated: a plain-accumulation
    # batch refuses a weighted plan
    pplan = hd.Plan(geom, grid, S, "f32", max_order=4, tiling=(16, 16, 1, 0), flags=hd.FLAG_CF | hd.FLAG_ACC_PLAIN)
    batch = hd.Batch(max_frames=2, max_units=1000, flags=hd.FLAG_ACC_PLAIN)
    with pytest.raises(hd.HodmasError) as ei:
        batch.set([pplan], [rf], [1], [out])
    assert ei.value.status == hd.EUNSUPPORTED
    batch.close()
    pplan.close()
    wplan.close()
    plan.close()


@pytest.mark.parametrize("dtype", ["f32", "f16", "i16"])
def test_weighted_plans_in_the_batch(hd, dtype):
    """Coherence-weighted plans (unpaired and mirror-paired) mixed with
    unweighted ones of several orders in one batch: every image equals the
    frame's own hodmas_beamform launch bit for bit (direct launch and graph
    replays), and the weighted images match the oracle's weighted image."""
    sym = ph.Grid(nx=64, nz=53, x0_m=-(64 - 1) / 2.0 * 0.17e-3, dx_m=0.17e-3, z0_m=0.2e-3, dz_m=0.21e-3)
    ragged = ph.Grid(nx=37, nz=53, x0_m=-3e-3, dx_m=0.17e-3, z0_m=0.2e-3, dz_m=0.21e-3)
    # (elements, seed, grid, flags, order): weighted frames from the per-frame tests' phantoms
    specs = [(13, 17, ragged, hd.FLAG_CF, 6), (16, 9, sym, hd.FLAG_CF | hd.FLAG_MIRROR, 3),
             (13, 17, ragged, 0, 6), (16, 9, sym, hd.FLAG_CF | hd.FLAG_MIRROR, 1),
             (13, 17, ragged, hd.FLAG_CF, 2), (16, 9, sym, hd.FLAG_MIRROR, 6)]
    plans, devs, data, outs, orders = [], [], [], [], []
    for n_el, seed, grid, flags, k in specs:
        f = ph.make_frame(n_el, 300, grid.nx, grid.nz, n_points=6, n_lines=1, snr_db=15.0, seed=seed)
        arr, scale = stored(f.rf, dtype, seed=seed)
        plans.append(hd.Plan(f.geometry, grid, 300, dtype, max_order=6, dequant_scale=scale, flags=flags,
                             tiling=(16, 16, 1, 8)))
        devs.append(torch.from_numpy(np.ascontiguousarray(arr)).cuda())
        data.append((f, arr, scale, grid))
        outs.append(torch.full((grid.nz, grid.nx), float("nan"), dtype=torch.float32, device="cuda"))
        orders.append(k)
    own = [p.beamform(d, k).cpu().numpy() for p, d, k in zip(plans, devs, orders)]
    bt = hd.Batch(max_frames=len(plans), max_units=sum(p.info().n_tiles for p in plans),
                  max_lds_bytes=max(p.info().lds_bytes for p in plans))
    bt.set(plans, devs, orders, outs)
    bt.launch()
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), own[i]), "frame %d differs from its own launch" % i
    bt.capture()
    for rep in range(2):
        for o in outs:
            o.fill_(float("nan"))
        bt.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            assert np.array_equal(o.cpu().numpy(), own[i]), "replay %d frame %d" % (rep, i)
    for i, ((f, arr, scale, grid), (_, _, _, flags, k)) in enumerate(zip(data, specs)):
        o = O.beamform(arr, f.geometry, grid, k, dequant_scale=scale if dtype == "i16" else None,
                       weighting="cf" if flags & hd.FLAG_CF else None)
        err = rel_l2(own[i].astype(np.float64), o)
        say("CF batch %s frame %d flags %d k=%d rel L2 %.2e" % (dtype, i, flags, k, err))
        assert err <= TOL[dtype]
    bt.close()
    for p in plans:
        p.close()
