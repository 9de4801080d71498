"""Host logic of the plan (no GPU): argument validation and the float64 tables
(delay anchors, LDS windows, skipped elements) checked against exact delays."""
import ctypes
import math

import numpy as np
import pytest

from paper_2203_14906_amd import hodmas, phantom as ph

C, FS = 1540.0, 40e6
LAM = C / FS


def _plan(geom, grid, S, dtype="f32", **kw):
    kw.setdefault("flags", 0)
    kw["flags"] |= hodmas.FLAG_HOST_ONLY
    return hodmas.Plan(geom, grid, S, dtype, **kw)


def _status(fn):
    with pytest.raises(hodmas.HodmasError) as ei:
        fn()
    return ei.value.status


def test_argument_validation():
    g = ph.Geometry(16)
    grid = ph.make_grid(20, 20, 16 * 0.3e-3, 5e-3)
    ok = _plan(g, grid, 256)
    ok.close()
    E = hodmas.EINVAL
    assert _status(lambda: _plan(ph.Geometry(0), grid, 256)) == E
    assert _status(lambda: _plan(ph.Geometry(16, sound_speed_m_s=0.0), grid, 256)) == E
    assert _status(lambda: _plan(ph.Geometry(16, fs_hz=float("nan")), grid, 256)) == E
    assert _status(lambda: _plan(ph.Geometry(16, pitch_m=-1.0), grid, 256)) == E
    assert _status(lambda: _plan(ph.Geometry(16, element_x_m=[0.0] * 15 + [float("inf")]), grid, 256)) == E
    assert _status(lambda: _plan(g, ph.Grid(0, 4, 0.0, 1e-4, 1e-3, 1e-4), 256)) == E
    assert _status(lambda: _plan(g, ph.Grid(4, 4, 0.0, -1e-4, 1e-3, 1e-4), 256)) == E
    assert _status(lambda: _plan(g, ph.Grid(4, 4, 0.0, 1e-4, 0.0, 1e-4), 256)) == E      # z0 = 0
    assert _status(lambda: _plan(g, ph.Grid(4, 4, 0.0, 1e-4, 1e-3, 0.0), 256)) == E
    assert _status(lambda: _plan(g, ph.Grid(16385, 4, 0.0, 1e-4, 1e-3, 1e-4), 256)) == E
    assert _status(lambda: _plan(g, grid, 0)) == E
    assert _status(lambda: _plan(g, grid, 256, channel_stride=255)) == E
    assert _status(lambda: _plan(g, grid, 256, dtype=7)) == E
    assert _status(lambda: _plan(g, grid, 256, "i16", dequant_scale=0.0)) == E
    assert _status(lambda: _plan(g, grid, 256, frame_max=-1.0)) == E
    assert _status(lambda: _plan(g, grid, 256, max_order=0)) == E
    assert _status(lambda: _plan(g, grid, 256, max_order=7)) == E
    assert _status(lambda: _plan(g, grid, 256, tiling=(16, 16, 3, 64))) == E
    assert _status(lambda: _plan(g, grid, 256, tiling=(16, 8, 1, 64))) == E
    assert _status(lambda: _plan(g, grid, 256, tiling=(16, 16, 4, 64))) == E     # 1024 threads
    _plan(g, grid, 256, tiling=(16, 16, 2, 64)).close()                         # 512 threads
    # delays beyond float32's exact-integer range are refused
    assert _status(lambda: _plan(g, ph.Grid(4, 4, 0.0, 1e-4, 1e4, 1e-4), 256)) == E


def test_null_pointers_and_destroy():
    L = hodmas.lib
    out = ctypes.c_void_p()
    assert L.hodmas_plan(None, None, None, 1, 0, None, ctypes.byref(out)) == hodmas.EINVAL
    assert L.hodmas_destroy(None) == hodmas.OK
    assert L.hodmas_beamform(None, None, 1, None, None) == hodmas.EINVAL
    p = _plan(ph.Geometry(8), ph.make_grid(8, 8, 2.4e-3, 3e-3), 128)
    # a host-only plan has no device tables to launch with
    assert L.hodmas_beamform(p.handle, ctypes.c_void_p(16), 1, ctypes.c_void_p(16), None) == hodmas.EINVAL
    imgs = (ctypes.c_void_p * 6)(*([16] * 6))
    assert L.hodmas_beamform_orders(None, ctypes.c_void_p(16), 2, imgs, None) == hodmas.EINVAL
    assert L.hodmas_beamform_orders(p.handle, ctypes.c_void_p(16), 2, imgs, None) == hodmas.EINVAL
    assert L.hodmas_plan_get_info(p.handle, None) == hodmas.EINVAL
    p.close()


def _exact_delays(ex, grid, t0s, ix, iz):
    xp = (grid.x0_m + ix * grid.dx_m) / LAM
    zp = (grid.z0_m + iz * grid.dz_m) / LAM
    return np.sqrt((xp[:, None] - ex[None, :] / LAM) ** 2 + zp[:, None] ** 2) - t0s


def _f32(x):
    return np.float32(x)


@pytest.mark.parametrize("case", ["deep", "shallow_t0", "irregular", "coarse"])
def test_tables_cover_every_delay(case):
    S = 400
    if case == "deep":           # far corners run past the record: skips and checks
        g = ph.Geometry(24)
        grid = ph.make_grid(41, 37, 24 * 0.3e-3 * 3, 20e-3)
        tiling = (16, 16, 1, 8)
    elif case == "shallow_t0":   # t0 pushes near pixels before the record start
        g = ph.Geometry(16, t0_s=2e-6)
        grid = ph.make_grid(30, 50, 16 * 0.3e-3, 8e-3)
        tiling = (16, 8, 2, 5)
    elif case == "irregular":    # non-uniform element positions, ragged tiles
        rng = np.random.default_rng(3)
        g = ph.Geometry(13, element_x_m=np.sort(rng.uniform(-3e-3, 3e-3, 13)))
        grid = ph.Grid(nx=19, nz=23, x0_m=-2e-3, dx_m=0.21e-3, z0_m=0.5e-3, dz_m=0.33e-3)
        tiling = (8, 8, 4, 3)
    else:                        # coarse pixels: long windows
        g = ph.Geometry(32)
        grid = ph.make_grid(24, 24, 32 * 0.3e-3, 12e-3)
        tiling = (16, 16, 1, 64)
    plan = _plan(g, grid, S, tiling=tiling)
    info = plan.info()
    tiles, entries, stage = plan.tables()
    ex = g.positions()
    t0s = g.t0_s * FS
    chunk = info.tiling.chunk
    covered = np.zeros((grid.nz, grid.nx), dtype=int)
    n_checked_tiles = 0
    for td in tiles:
        covered[td.iz0:td.iz0 + td.nz, td.ix0:td.ix0 + td.nx] += 1
        ixs, izs = np.meshgrid(np.arange(td.ix0, td.ix0 + td.nx), np.arange(td.iz0, td.iz0 + td.nz))
        ixs, izs = ixs.ravel(), izs.ravel()
        t = _exact_delays(ex, grid, t0s, ixs, izs)                     # [pixels, elements]
        active = [st.channel for st in stage[td.first_entry:td.first_entry + td.n_active]]
        assert active == sorted(active)
        for i in range(len(ex)):
            if i not in active:                                        # skipped: never in the record
                assert np.all((t[:, i] < 0) | (t[:, i] > S - 1)), (td.ix0, td.iz0, i)
        if not td.check:
            assert np.all(t[:, active] >= 0.5) and np.all(t[:, active] <= S - 1.5)
        else:
            n_checked_tiles += 1
        assert td.window <= info.max_window
        ia, ja = td.ix0 + (td.nx - 1) // 2, td.iz0 + (td.nz - 1) // 2
        assert td.xa == pytest.approx((grid.x0_m + ia * grid.dx_m) / LAM, rel=1e-15)
        assert td.za == pytest.approx((grid.z0_m + ja * grid.dz_m) / LAM, rel=1e-15)
        u = (grid.x0_m + ixs * grid.dx_m) / LAM - td.xa
        w = (grid.z0_m + izs * grid.dz_m) / LAM - td.za
        u2 = (2.0 * u).astype(np.float32)
        q = (u * u + w * (w + 2.0 * td.za)).astype(np.float32)
        tile_entries = entries[td.first_entry:td.first_entry + td.n_active]
        by_elem = {e.channel: e for e in tile_entries}
        assert len(by_elem) == td.n_active
        # constants of each chunk are grouped by split group: slots g, g+split, ...
        split = info.tiling.split
        order = []
        for c0 in range(0, td.n_active, chunk):
            nch = min(chunk, td.n_active - c0)
            for gq in range(split):
                order += list(range(c0 + gq, c0 + nch, split))
        assert [e.channel for e in tile_entries] == [stage[td.first_entry + sl].channel for sl in order]
        for slot in range(td.n_active):
            st = stage[td.first_entry + slot]
            i = st.channel
            e = by_elem[i]
            T0 = int(round(-e.lo))
            assert e.hi == pytest.approx(S - 1 - T0, abs=0)
            ta = math.sqrt((td.xa - ex[i] / LAM) ** 2 + td.za ** 2) - t0s
            assert T0 == math.floor(ta) and e.frac0 == pytest.approx(ta - T0, abs=1e-6)
            assert e.off == 4 * (T0 - st.first_sample + (slot % chunk) * (td.window + 2))
            # float32 reconstruction of each pixel's delay, as the kernel forms it
            num = (u2.astype(np.float64) * np.float64(e.a) + q).astype(np.float32)
            d = np.sqrt(np.abs(np.float64(e.d0sq) + num)).astype(np.float32)
            r = (1.0 / (d.astype(np.float64) + np.float64(e.d0))).astype(np.float32)
            trel = (num.astype(np.float64) * r + np.float64(e.frac0)).astype(np.float32)
            exact = t[:, i] - T0
            assert np.max(np.abs(trel - exact)) < 1e-3
            j = np.floor(trel).astype(np.int64) + T0 - st.first_sample     # window position
            assert j.min() >= 0 and j.max() + 1 <= td.window - 1
    assert np.all(covered == 1)
    if case in ("deep", "shallow_t0"):
        assert n_checked_tiles > 0
    plan.close()


def test_default_tiling_and_info():
    f = ph.config_frame(2)
    p = _plan(f.geometry, f.grid, 2048)
    inf = p.info()
    assert (inf.tiling.tile_x, inf.tiling.tile_z, inf.tiling.split) == (16, 16, 1)
    assert inf.n_tiles == 32 * 32
    assert inf.active_pairs == 32 * 32 * 128           # no element is out of the record here
    # rows of the window and two floats more (the first row's hold the zeros
    # that delays outside the record read)
    # (plus, as the plan shares delays along translated pixels, 48 eight-byte
    # entries per row of 16 lanes)
    staged = inf.tiling.chunk * (inf.max_window + 2) * 4
    assert inf.flags & hodmas.INFO_SHARED_DELAYS
    assert inf.lds_bytes == (staged + 7) // 8 * 8 + 16 * 48 * 8
    full = _plan(f.geometry, f.grid, 2048, flags=hodmas.FLAG_NO_SHARE)
    assert full.info().lds_bytes == staged
    full.close()
    small = _plan(ph.config_frame(1).geometry, ph.config_frame(1).grid, 1024)
    assert small.info().tiling.split in (2, 4)
    p.close()
    small.close()


def test_batch_argument_validation_without_device():
    L = hodmas.lib
    h = ctypes.c_void_p()
    assert L.hodmas_batch_create(0, 10, 0, 0, ctypes.byref(h)) == hodmas.EINVAL
    assert L.hodmas_batch_create(4, 0, 0, 0, ctypes.byref(h)) == hodmas.EINVAL
    assert L.hodmas_batch_create(4, 10, -1, 0, ctypes.byref(h)) == hodmas.EINVAL
    assert L.hodmas_batch_create(4, 10, 1 << 30, 0, ctypes.byref(h)) == hodmas.EINVAL
    assert L.hodmas_batch_create(4, 10, 0, 0x80, ctypes.byref(h)) == hodmas.EINVAL
    assert L.hodmas_batch_create(4, 10, 0, 0, None) == hodmas.EINVAL
    assert L.hodmas_batch_destroy(None) == hodmas.OK
    assert L.hodmas_batch_launch(None, None) == hodmas.EINVAL
    assert L.hodmas_batch_replay(None, None) == hodmas.EINVAL
    assert L.hodmas_batch_capture(None) == hodmas.EINVAL
    assert L.hodmas_batch_set(None, None, None, None, None, 1, None) == hodmas.EINVAL


def test_autotune_argument_validation_without_device():
    L = hodmas.lib
    t = hodmas.Tiling()
    g = hodmas.Geometry(8, 0.3e-3, 1540.0, 40e6, 0.0, None)
    gr = hodmas.Grid(8, 8, -1e-3, 0.3e-3, 1e-3, 0.3e-3)
    rd = hodmas.RfDesc(0, 128, 128, 1.0, 0.0)
    assert L.hodmas_autotune(None, ctypes.byref(gr), ctypes.byref(rd), 1, 0, None, ctypes.byref(t)) == hodmas.EINVAL
    assert L.hodmas_autotune(ctypes.byref(g), ctypes.byref(gr), ctypes.byref(rd), 7, 0, None, ctypes.byref(t)) == hodmas.EINVAL
    assert L.hodmas_autotune(ctypes.byref(g), ctypes.byref(gr), ctypes.byref(rd), 1, hodmas.FLAG_HOST_ONLY, None,
                             ctypes.byref(t)) == hodmas.EINVAL
    assert L.hodmas_autotune(ctypes.byref(g), ctypes.byref(gr), ctypes.byref(rd), 1, 0, None, None) == hodmas.EINVAL


def test_mirror_validation_and_default_tiling():
    M, E = hodmas.FLAG_MIRROR, hodmas.EINVAL
    g = ph.Geometry(24)
    grid = ph.make_grid(64, 40, 24 * 0.3e-3, 10e-3)
    p = _plan(g, grid, 512, flags=M)
    inf = p.info()
    assert inf.flags & M
    assert inf.tiling.tile_x == 16 and (64 // 16) % 2 == 0
    p.close()
    # 48 columns: 16-wide tiles would give an odd count, so the default is 8 wide
    p = _plan(g, ph.make_grid(48, 40, 24 * 0.3e-3, 10e-3), 512, flags=M)
    assert p.info().tiling.tile_x == 8
    p.close()
    # a grid off centre by a tenth of a pixel, a shifted or uneven array, tiles
    # that do not divide the grid or give an odd column count: refused
    off = ph.Grid(64, 40, grid.x0_m + 0.1 * grid.dx_m, grid.dx_m, grid.z0_m, grid.dz_m)
    assert _status(lambda: _plan(g, off, 512, flags=M)) == E
    ex = g.positions()
    assert _status(lambda: _plan(ph.Geometry(24, element_x_m=ex + 1e-5), grid, 512, flags=M)) == E
    bent = ex.copy()
    bent[3] += 1e-5
    assert _status(lambda: _plan(ph.Geometry(24, element_x_m=bent), grid, 512, flags=M)) == E
    assert _status(lambda: _plan(g, ph.make_grid(60, 40, 24 * 0.3e-3, 10e-3), 512, flags=M,
                                 tiling=(16, 16, 1, 0))) == E     # 16 does not divide 60
    assert _status(lambda: _plan(g, ph.make_grid(48, 40, 24 * 0.3e-3, 10e-3), 512, flags=M,
                                 tiling=(16, 16, 1, 0))) == E     # three columns
    # an explicitly symmetric array given element by element is accepted
    _plan(ph.Geometry(24, element_x_m=ex), grid, 512, flags=M).close()


def test_mirror_lds_holds_both_rows():
    f = ph.config_frame(2)
    plain = _plan(f.geometry, f.grid, 2048)
    mir = _plan(f.geometry, f.grid, 2048, flags=hodmas.FLAG_MIRROR)
    a, b = plain.info(), mir.info()
    assert b.max_window == a.max_window
    assert b.lds_bytes == 2 * b.tiling.chunk * (b.max_window + 2) * 4 <= 40 * 1024
    assert b.tiling.chunk <= a.tiling.chunk
    # the automatic chunk splits the 128 elements into equal chunks
    assert b.tiling.chunk == 64
    plain.close()
    mir.close()


def test_automatic_chunks_are_balanced():
    """When the LDS cap needs several chunks, they are of equal size (the last
    one at most one element short), and no more of them than the cap needs."""
    for n, S in ((128, 2048), (192, 2048), (256, 2048), (100, 1500)):
        g = ph.Geometry(n)
        w, d = ph.field_of_view(n, S)
        for nx, flags in ((256, 0), (256, hodmas.FLAG_MIRROR), (64, 0)):
            grid = ph.make_grid(nx, nx, w, d)
            p = _plan(g, grid, S, flags=flags)
            inf = p.info()
            rows = 2 if flags else 1
            c, win = inf.tiling.chunk, inf.max_window
            n_chunks = -(-n // c)
            staged = c * (win + 2) * 4 * rows
            assert inf.lds_bytes >= staged
            assert staged <= 40 * 1024
            assert n - (n_chunks - 1) * c >= c - n_chunks       # last chunk nearly full
            largest = max(1, 40 * 1024 // ((win + 2) * 4 * rows))
            assert n_chunks == -(-n // min(n, largest))         # no more chunks than the cap needs
            p.close()


@pytest.mark.parametrize("n_elem,tiling", [(24, (16, 16, 1, 8)), (13, (8, 8, 4, 3)), (32, (16, 8, 2, 0))])
def test_mirror_pixels_read_the_mirrored_delays(n_elem, tiling):
    """Each lane forms its pixel P from its tile's constants and, with the same
    float32 delay, the mirror pixel P' at element n-1-i from the mirrored LDS
    row.  Check on the host that this delay is P''s own delay to the mirrored
    element, that the mirrored row's sample window covers it, and that an
    element the tile skips contributes nothing to P' either."""
    S = 330                                                        # deep pixels run past the record
    g = ph.Geometry(n_elem)
    grid = ph.make_grid(64, 45, n_elem * 0.3e-3 * 1.5, 14e-3)       # wider than the array, ragged in z
    plan = _plan(g, grid, S, tiling=tiling, flags=hodmas.FLAG_MIRROR)
    info = plan.info()
    tiles, entries, stage = plan.tables()
    ex = g.positions()
    n = len(ex)
    tx = info.tiling.tile_x
    ntx = grid.nx // tx
    n_checked = n_skipped = 0
    for td in tiles:
        if td.ix0 // tx >= ntx // 2:
            continue                                               # right half: formed as mirrors
        assert td.nx == tx
        ixs, izs = np.meshgrid(np.arange(td.ix0, td.ix0 + td.nx), np.arange(td.iz0, td.iz0 + td.nz))
        ixs, izs = ixs.ravel(), izs.ravel()
        tm = _exact_delays(ex, grid, 0.0, grid.nx - 1 - ixs, izs)   # mirror pixels, every element
        u = (grid.x0_m + ixs * grid.dx_m) / LAM - td.xa
        w = (grid.z0_m + izs * grid.dz_m) / LAM - td.za
        u2 = (2.0 * u).astype(np.float32)
        q = (u * u + w * (w + 2.0 * td.za)).astype(np.float32)
        active = {st.channel for st in stage[td.first_entry:td.first_entry + td.n_active]}
        for i in range(n):
            if i not in active:
                assert np.all((tm[:, n - 1 - i] < 0) | (tm[:, n - 1 - i] > S - 1))
        by_elem = {e.channel: e for e in entries[td.first_entry:td.first_entry + td.n_active]}
        for slot in range(td.n_active):
            st = stage[td.first_entry + slot]
            e = by_elem[st.channel]
            T0 = int(round(-e.lo))
            num = (u2.astype(np.float64) * np.float64(e.a) + q).astype(np.float32)
            d = np.sqrt(np.abs(np.float64(e.d0sq) + num)).astype(np.float32)
            r = (1.0 / (d.astype(np.float64) + np.float64(e.d0))).astype(np.float32)
            trel = (num.astype(np.float64) * r + np.float64(e.frac0)).astype(np.float32)
            exact = tm[:, n - 1 - st.channel] - T0
            assert np.max(np.abs(trel - exact)) < 1e-3
            if not td.check:
                j = np.floor(trel).astype(np.int64) + T0 - st.first_sample
                assert j.min() >= 0 and j.max() + 1 <= td.window - 1
            n_checked += int(td.check)
            n_skipped += n - td.n_active
    assert n_checked > 0                                           # tiles at the record's end
    assert n_skipped > 0 or n_elem == 24                           # elements left out of tiles
    plan.close()


class _DeviceTensorStub:
    """Stands for a GPU tensor in the binding's argument checks (no device here)."""

    def __init__(self, shape, dtype, is_cuda=True):
        import torch
        self.shape = shape
        self.dtype = dtype
        self.is_cuda = is_cuda
        self._t = torch.empty(shape, dtype=dtype)

    def dim(self):
        return len(self.shape)

    def stride(self, i):
        return self._t.stride(i)

    def is_contiguous(self):
        return True

    def numel(self):
        return self._t.numel()

    def data_ptr(self):
        raise AssertionError("the binding passed a pointer before rejecting the arguments")


def test_batch_set_rejects_host_images_before_any_launch():
    """A host (CPU) image would hand the persistent kernel a host address; the
    binding refuses it before any library call."""
    import torch
    f = ph.make_frame(8, 128, 16, 16, n_points=2, n_lines=0, snr_db=20.0, seed=1)
    plan = _plan(f.geometry, f.grid, 128)
    bt = hodmas.Batch.__new__(hodmas.Batch)          # no device: the library handle is never used
    bt._h = ctypes.c_void_p()
    bt._keep = None
    rf = _DeviceTensorStub((8, 128), torch.float32)
    host_img = torch.empty((16, 16), dtype=torch.float32)
    with pytest.raises(ValueError, match="GPU tensor"):
        bt.set([plan], [rf], [1], [host_img])
    wrong = _DeviceTensorStub((16, 16), torch.float64)
    with pytest.raises(ValueError, match="GPU tensor"):
        bt.set([plan], [rf], [1], [wrong])
    plan.close()


def test_shared_delays_only_where_the_translation_holds():
    """Delays are shared along translated pixels only when consecutive
    elements are exactly four pixel columns apart, tiles are 16 columns wide
    with one element group, nx is a multiple of 16 and the plan forms pixels
    one per lane without weighting."""
    f = ph.config_frame(2)                  # pitch 0.3 mm = 4 x 0.075 mm columns
    g, gr = f.geometry, f.grid

    def shared(geom=g, grid=gr, **kw):
        p = _plan(geom, grid, 2048, **kw)
        on = bool(p.info().flags & hodmas.INFO_SHARED_DELAYS)
        p.close()
        return on

    assert shared()
    assert shared(dtype="f16")
    assert not shared(flags=hodmas.FLAG_NO_SHARE)
    assert not shared(flags=hodmas.FLAG_MIRROR)          # pairs take another path
    assert not shared(flags=hodmas.FLAG_CF)
    assert not shared(tiling=(32, 8, 1, 0))
    assert not shared(tiling=(16, 8, 2, 0))
    # pitch of two columns (config 1), and a grid 8 columns narrower
    assert not shared(ph.config_frame(1).geometry, ph.config_frame(1).grid)
    narrow = ph.Grid(nx=gr.nx - 8, nz=gr.nz, x0_m=gr.x0_m + 4 * gr.dx_m, dx_m=gr.dx_m, z0_m=gr.z0_m, dz_m=gr.dz_m)
    assert not shared(grid=narrow)
    # element positions given explicitly: shared while uniform at four columns, not once one moves
    x = (np.arange(g.n_elements) - (g.n_elements - 1) / 2.0) * g.pitch_m
    assert shared(ph.Geometry(g.n_elements, element_x_m=x))
    x[40] += 1e-9
    assert not shared(ph.Geometry(g.n_elements, element_x_m=x))
    # 1024^2 (config 3): 4096 tiles, 3 rounds over 256 CUs at six workgroups
    # per CU; the buffers' LDS would leave five, and four rounds
    f3 = ph.config_frame(3)
    p3 = _plan(f3.geometry, f3.grid, 2048, "f16")
    assert not p3.info().flags & hodmas.INFO_SHARED_DELAYS
    p3.close()


def test_automatic_chunk_takes_fewer_rounds_at_1024():
    """A 1024^2 grid has 4096 tiles (2048 mirror pairs): at the 40 KB chunk a
    one-frame launch would need several rounds of workgroups over 256 CUs, so
    the plan takes equal chunks within 20 KB instead (eight workgroups per
    CU); config 2's 1024 tiles fit one round either way and keep the 40 KB
    chunk."""
    f3 = ph.config_frame(3)
    for flags in (0, hodmas.FLAG_MIRROR):
        p = _plan(f3.geometry, f3.grid, 2048, "f16", flags=flags)
        inf = p.info()
        rows = 2 if flags else 1
        staged = inf.tiling.chunk * (inf.max_window + 2) * 4 * rows
        assert staged <= 20 * 1024 and inf.lds_bytes == staged
        n_chunks = -(-256 // inf.tiling.chunk)
        assert n_chunks >= 2 and inf.tiling.chunk == -(-256 // n_chunks)      # equal chunks
        # the 40 KB cap alone would have taken bigger chunks
        assert (40 * 1024) // ((inf.max_window + 2) * 4 * rows) > inf.tiling.chunk
        p.close()
    f2 = ph.config_frame(2)
    p = _plan(f2.geometry, f2.grid, 2048, flags=hodmas.FLAG_NO_SHARE)
    inf = p.info()
    assert inf.tiling.chunk == 128 and inf.lds_bytes > 20 * 1024
    p.close()
