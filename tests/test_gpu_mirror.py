"""Mirror pairing (HODMAS_FLAG_MIRROR): one workgroup forms a tile and its
mirror image about x = 0 from one set of delays.  Images are checked against
the FP64 oracle to the same bars as the unpaired kernel (relative L2 1e-5 for
FP32 storage, 2e-5 on the same stored values for FP16 / int16) and against the
unpaired launch (rounding-level differences only), over ragged grids, several
tilings, multi-chunk staging, record-boundary checks, coherence weighting and
odd and even element counts -- per frame and as pair units in the batch."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2203_14906_amd import phantom as ph
from sign_band import MAX_FLAGGED_SHARE, band_rel_l2, plan_eps

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


def symmetric_grid(nx, nz, dx, z0, dz):
    return ph.Grid(nx=nx, nz=nz, x0_m=-(nx - 1) / 2.0 * dx, dx_m=dx, z0_m=z0, dz_m=dz)


@pytest.mark.parametrize("n_elem", [13, 16])
@pytest.mark.parametrize("tiling", [None, (16, 16, 1, 64), (16, 8, 2, 5), (8, 8, 4, 3), (16, 16, 2, 0)])
@pytest.mark.parametrize("dtype", ["f32", "f16", "i16"])
def test_mirror_small_ragged_frames(hd, n_elem, tiling, dtype):
    f = ph.make_frame(n_elem, 300, 64, 53, n_points=6, n_lines=1, snr_db=15.0, seed=21)
    grid = symmetric_grid(64, 53, 0.17e-3, 0.2e-3, 0.21e-3)
    arr, scale = stored(f.rf, dtype, seed=21)
    kw = dict(max_order=6, dequant_scale=scale, tiling=tiling)
    plan = hd.Plan(f.geometry, grid, arr.shape[1], dtype, flags=hd.FLAG_MIRROR, **kw)
    ref = hd.Plan(f.geometry, grid, arr.shape[1], dtype, **kw)
    dev = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    say("mirror small n=%d %s %s chunk %d" % (n_elem, dtype, tiling, plan.info().tiling.chunk))
    for k in range(1, 7):
        g = plan.beamform(dev, k).cpu().numpy().astype(np.float64)
        u = ref.beamform(dev, k).cpu().numpy().astype(np.float64)
        o = O.beamform(arr, f.geometry, grid, k, dequant_scale=scale if dtype == "i16" else None)
        err, err_u = rel_l2(g, o), rel_l2(g, u)
        say("  k=%d rel L2 vs oracle %.2e, vs unpaired %.2e" % (k, err, err_u))
        assert err <= TOL[dtype]
        assert err_u <= TOL[dtype]
    plan.close()
    ref.close()


def test_mirror_record_checks_and_skipped_elements(hd):
    """Deep pixels run past the record (per-sample checks, elements left out of
    tiles); FORCE_CHECK runs the checks everywhere."""
    S = 330
    f = ph.make_frame(24, S, 64, 45, n_points=8, n_lines=1, snr_db=20.0, seed=5)
    grid = ph.make_grid(64, 45, 24 * 0.3e-3 * 1.5, 14e-3)
    arr = ph.to_fp32(f.rf)
    dev = torch.from_numpy(arr).cuda()
    for flags in (hd.FLAG_MIRROR, hd.FLAG_MIRROR | hd.FLAG_FORCE_CHECK, hd.FLAG_MIRROR | hd.FLAG_ACC_PLAIN):
        for tiling in ((16, 16, 1, 8), (8, 8, 4, 3)):
            plan = hd.Plan(f.geometry, grid, S, "f32", max_order=6, tiling=tiling, flags=flags)
            for k in (1, 2, 4, 6):
                g = plan.beamform(dev, k).cpu().numpy().astype(np.float64)
                o = O.beamform(arr, f.geometry, grid, k)
                err = rel_l2(g, o)
                say("mirror deep flags %d %s k=%d rel L2 %.2e" % (flags, tiling, k, err))
                assert err <= 1e-5
            plan.close()


@pytest.mark.parametrize("cfg,orders", [(1, (1, 2, 3, 4)), (2, (1, 2, 3, 4, 5, 6))])
def test_mirror_configs(hd, cfg, orders):
    f = ph.config_frame(cfg)
    arr = ph.to_fp32(f.rf)
    dev = torch.from_numpy(arr).cuda()
    for tiling in (None, (16, 8, 2, 0)):
        plan = hd.Plan(f.geometry, f.grid, arr.shape[1], "f32", max_order=6, tiling=tiling,
                       flags=hd.FLAG_MIRROR)
        for k in orders:
            g = plan.beamform(dev, k).cpu().numpy().astype(np.float64)
            o = O.beamform(arr, f.geometry, f.grid, k)
            err = rel_l2(g, o)
            say("mirror config %d %s k=%d rel L2 %.2e" % (cfg, tiling, k, err))
            assert err <= 1e-5
        plan.close()


def test_mirror_with_coherence_factor(hd):
    f = ph.make_frame(16, 300, 64, 53, n_points=6, n_lines=1, snr_db=15.0, seed=9)
    grid = symmetric_grid(64, 53, 0.17e-3, 0.2e-3, 0.21e-3)
    arr = ph.to_fp32(f.rf)
    dev = torch.from_numpy(arr).cuda()
    for tiling in (None, (8, 8, 4, 3)):
        plan = hd.Plan(f.geometry, grid, 300, "f32", max_order=6, tiling=tiling,
                       flags=hd.FLAG_MIRROR | hd.FLAG_CF)
        for k in (1, 2, 3, 6):
            g = plan.beamform(dev, k).cpu().numpy().astype(np.float64)
            o = O.beamform(arr, f.geometry, grid, k, weighting="cf")
            err = rel_l2(g, o)
            say("mirror CF %s k=%d rel L2 %.2e" % (tiling, k, err))
            assert err <= 1e-5
        plan.close()


def test_mirror_symmetric_input_gives_symmetric_image(hd):
    """Channel records mirrored about the array centre make a mirror-symmetric
    image; the paired kernel forms both halves from the same delays."""
    f = ph.make_frame(32, 512, 64, 64, n_points=6, n_lines=0, snr_db=30.0, seed=2)
    rf = 0.5 * (f.rf + f.rf[::-1])
    arr = ph.to_fp32(rf)
    grid = symmetric_grid(64, 64, 0.15e-3, 1e-3, 0.15e-3)
    plan = hd.Plan(f.geometry, grid, 512, "f32", max_order=6, flags=hd.FLAG_MIRROR)
    dev = torch.from_numpy(arr).cuda()
    for k in (1, 3, 6):
        g = plan.beamform(dev, k).cpu().numpy()
        say("mirror symmetry k=%d max |left - right| %.3g" % (k, np.abs(g - g[:, ::-1]).max()))
        # the mirrored rows hold the same samples, read at the same delays,
        # summed in the same order: the halves agree bit for bit
        assert np.array_equal(g, g[:, ::-1])
    plan.close()


def test_mirror_plan_in_other_entry_points(hd):
    """The all-orders pass runs a mirror plan unpaired (same images)."""
    f = ph.config_frame(1)
    arr = ph.to_fp32(f.rf)
    dev = torch.from_numpy(arr).cuda()
    plan = hd.Plan(f.geometry, f.grid, arr.shape[1], "f32", max_order=4, flags=hd.FLAG_MIRROR)
    imgs = plan.beamform_orders(dev, 4)
    for k in range(1, 5):
        o = O.beamform(arr, f.geometry, f.grid, k)
        err = rel_l2(imgs[k - 1].cpu().numpy().astype(np.float64), o)
        say("mirror plan, all-orders pass k=%d rel L2 %.2e" % (k, err))
        assert err <= 1e-5
    plan.close()


@pytest.mark.parametrize("dtype", ["f32", "f16", "i16"])
def test_mirror_pairs_in_the_batch(hd, dtype):
    """Mirror plans in a batch run as pair units of their own kinds, mixed with
    unpaired plans of the same and other orders: every image equals the
    frame's own hodmas_beamform launch bit for bit (direct launch and graph
    replays), and the mirror images match the oracle."""
    grid = symmetric_grid(64, 53, 0.17e-3, 0.2e-3, 0.21e-3)
    frames, plans, devs, orders, scales = [], [], [], [], []
    for i, (n_elem, flags, k) in enumerate([(16, hd.FLAG_MIRROR, 6), (13, hd.FLAG_MIRROR, 3), (16, 0, 6),
                                            (13, hd.FLAG_MIRROR, 1), (16, hd.FLAG_MIRROR, 6), (13, 0, 2)]):
        f = ph.make_frame(n_elem, 300, 64, 53, n_points=6, n_lines=1, snr_db=15.0, seed=40 + i)
        arr, scale = stored(f.rf, dtype, seed=40 + i)
        plans.append(hd.Plan(f.geometry, grid, 300, dtype, max_order=6, dequant_scale=scale, flags=flags,
                             tiling=(16, 16, 1, 8) if i == 4 else None))
        frames.append((f, arr))
        devs.append(torch.from_numpy(np.ascontiguousarray(arr)).cuda())
        orders.append(k)
        scales.append(scale)
    ref = [p.beamform(d, k).cpu().numpy() for p, d, k in zip(plans, devs, orders)]
    lds = max(p.info().lds_bytes for p in plans)
    units = sum(p.info().n_tiles for p in plans)
    bt = hd.Batch(max_frames=len(plans), max_units=units, max_lds_bytes=lds)
    outs = [torch.full((grid.nz, grid.nx), float("nan"), dtype=torch.float32, device="cuda") for _ in plans]
    bt.set(plans, devs, orders, outs)
    paired = sum(p.info().n_tiles // (2 if p.info().flags & hd.FLAG_MIRROR else 1) for p in plans)
    assert bt.info().n_units == paired
    bt.launch()
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), ref[i]), "frame %d differs from its own launch" % i
    bt.capture()
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        bt.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            assert np.array_equal(o.cpu().numpy(), ref[i]), "replay %d frame %d" % (rep, i)
    # this frame set holds sign-change pixels (frame 0: a sample 5e-9 from zero,
    # where one float32 delay ulp moves e_6 by ten percent), so the error is
    # taken from the oracle's delay-uncertainty band there
    for i, (p, (f, arr)) in enumerate(zip(plans, frames)):
        mirror = bool(p.info().flags & hd.FLAG_MIRROR)
        eps = plan_eps(p, f.geometry, grid, mirror=mirror)
        err, flagged = band_rel_l2(ref[i], arr, f.geometry, grid, orders[i],
                                   dequant_scale=scales[i] if dtype == "i16" else None, eps=eps)
        say("batch %s frame %d mirror %d k=%d rel L2 from the band %.2e (half-width %.2e, %d sign-change pixels)"
            % (dtype, i, mirror, orders[i], err, eps, flagged))
        assert err <= TOL[dtype]
        assert flagged <= max(2, MAX_FLAGGED_SHARE * grid.nx * grid.nz)
    bt.close()
    for p in plans:
        p.close()


def test_mirror_batch_config2_matches_oracle_samples(hd):
    """Config 2 as the bench's step runs it: eight frames of mirror plans in one
    batched launch per order; each image equals its own paired launch bit for
    bit, and sampled pixels match the oracle."""
    p = ph.CONFIGS[2]
    fr = [ph.make_frame(p["n_elements"], p["n_samples"], p["nx"], p["nz"], n_points=p["n_points"],
                        n_lines=p["n_lines"], snr_db=p["snr_db"], seed=2000 + b) for b in range(2)]
    grid = fr[0].grid
    plan = hd.Plan(fr[0].geometry, grid, p["n_samples"], "f32", max_order=6, flags=hd.FLAG_MIRROR)
    devs = [torch.from_numpy(ph.to_fp32(f.rf)).cuda() for f in fr] * 4
    bt = hd.Batch(max_frames=8, max_units=8 * plan.info().n_tiles, max_lds_bytes=plan.info().lds_bytes)
    outs = [torch.empty((grid.nz, grid.nx), dtype=torch.float32, device="cuda") for _ in range(8)]
    rng = np.random.default_rng(7)
    # both halves of the image, the centre columns and the corners
    ix = np.concatenate([rng.integers(0, grid.nx, 40), [0, grid.nx - 1, grid.nx // 2 - 1, grid.nx // 2]])
    iz = np.concatenate([rng.integers(0, grid.nz, 40), [0, grid.nz - 1, 0, grid.nz - 1]])
    for k in (1, 3, 6):
        bt.set([plan] * 8, devs, [k] * 8, outs)
        bt.launch()
        own = [plan.beamform(devs[j], k).cpu().numpy() for j in range(2)]
        for j, o in enumerate(outs):
            assert np.array_equal(o.cpu().numpy(), own[j % 2])
        arr = ph.to_fp32(fr[0].rf)
        ref = O.beamform(arr, fr[0].geometry, grid, k, pixels=(ix, iz))
        got = own[0][iz, ix].astype(np.float64)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        say("config 2 mirror batch k=%d sampled rel L2 %.2e" % (k, err))
        assert err <= 1e-5
    bt.close()
    plan.close()


@pytest.mark.parametrize("dtype", ["i16", "f16"])
def test_mirror_config3_reduced_storage(hd, dtype):
    """Config 3 at full size (256 elements, 2048 samples, 1024x1024) with
    mirror pairs, as the reduced-precision bench times it: sampled pixels of
    both halves against the oracle fed the same stored values."""
    f = ph.config_frame(3)
    arr, scale = stored(f.rf, dtype, seed=3000)
    plan = hd.Plan(f.geometry, f.grid, arr.shape[1], dtype, max_order=6, dequant_scale=scale, flags=hd.FLAG_MIRROR)
    dev = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    rng = np.random.default_rng(11)
    ix = np.concatenate([rng.integers(0, f.grid.nx, 1500), [0, f.grid.nx - 1, f.grid.nx // 2 - 1, f.grid.nx // 2]])
    iz = np.concatenate([rng.integers(0, f.grid.nz, 1500), [0, f.grid.nz - 1, 0, f.grid.nz - 1]])
    for k in (1, 3, 6):
        g = plan.beamform(dev, k).cpu().numpy().astype(np.float64)[iz, ix]
        o = O.beamform(arr, f.geometry, f.grid, k, dequant_scale=scale if dtype == "i16" else None,
                       pixels=(ix, iz))
        err = rel_l2(g, o)
        say("config 3 mirror %s k=%d sampled rel L2 %.2e" % (dtype, k, err))
        assert err <= TOL[dtype]
    plan.close()


def test_mirror_batch_at_config4_sizes(hd):
    """Paired FP16 plans of config-4 shapes (up to 256 elements, 4096 samples,
    1024x1024) and mixed orders in one batch, as the mixed-batch bench runs
    them: every image bitwise its own paired launch, sampled pixels within the
    reduced-storage bar of the oracle on the same stored values."""
    shapes = [(256, 4096, 1024, 6), (64, 1024, 256, 1), (128, 2048, 768, 4), (256, 2048, 512, 3)]
    plans, devs, outs, orders, meta = [], [], [], [], []
    for i, (n, S, side, k) in enumerate(shapes):
        f = ph.make_frame(n, S, 8, 8, n_points=50, n_lines=3, snr_db=10.0, seed=4100 + i)
        w, d = ph.field_of_view(n, S)
        grid = ph.make_grid(side, side, w, d)
        arr = ph.to_fp16(f.rf)
        plans.append(hd.Plan(ph.Geometry(n), grid, S, "f16", max_order=6, flags=hd.FLAG_MIRROR))
        devs.append(torch.from_numpy(arr).cuda())
        outs.append(torch.empty((side, side), dtype=torch.float32, device="cuda"))
        orders.append(k)
        meta.append((arr, ph.Geometry(n), grid))
    own = [p.beamform(d, k).cpu().numpy() for p, d, k in zip(plans, devs, orders)]
    bt = hd.Batch(max_frames=len(plans), max_units=sum(p.info().n_tiles for p in plans),
                  max_lds_bytes=max(p.info().lds_bytes for p in plans))
    bt.set(plans, devs, orders, outs)
    bt.capture()
    bt.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    for i, (o, ref) in enumerate(zip(outs, own)):
        img = o.cpu().numpy()
        assert np.array_equal(img, ref), "frame %d differs from its own launch" % i
        arr, geom, grid = meta[i]
        ix, iz = rng.integers(0, grid.nx, 600), rng.integers(0, grid.nz, 600)
        want = O.beamform(arr, geom, grid, orders[i], pixels=(ix, iz))
        err = rel_l2(img[iz, ix].astype(np.float64), want)
        say("config-4 shape %s k=%d mirror batch sampled rel L2 %.2e" % (shapes[i][:3], orders[i], err))
        assert err <= TOL["f16"]
    bt.close()
    for p in plans:
        p.close()
