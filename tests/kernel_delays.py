"""Host emulation of the beamforming kernel's float32 delay arithmetic, from
a plan's own tables (test infrastructure: it bounds the delay error that the
sign-change band must cover; see tests/sign_band.py).

Per tile the kernel forms, for a pixel at offset (u, w) samples from the
tile's anchor, in float32:
    u2 = 2u,  q = u^2 + w (w + 2 z_a)          (float64, rounded once)
    num = fma(u2, a, q)
    d = sqrt(|d0^2 + num|),  r = 1 / (d + d0)
    t = fma(num, r, frac0)                     (relative to floor(anchor delay))
with a, d0^2, d0, frac0 the table's float32 constants.  Here every step is
rounded to float32 exactly as written (fma through float64, whose product of
two float32 values is exact); the hardware square root and reciprocal are
within one ulp of the rounded values, which `bound` adds as |num r| 2^-22 (the
reciprocal's ulp and the square root's, carried into r, together).
A mirror-paired plan's right half takes each left pixel's delay to element i
as its mirror pixel's delay to element n-1-i.  A plan that shares delays along
translated pixels (element pitch = four pixel columns) also forms every
element's delay at the pixel four columns to the left, which serves the next
element at the lane's own pixel."""
import numpy as np

from oracle import oracle as O


def _r32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def delay_errors(plan, geometry, grid, mirror=False):
    """(max |float32 kernel delay - exact delay|, max of that plus the
    hardware allowance) over every pixel and active element of the plan."""
    from paper_2203_14906_amd import hodmas
    info = plan.info()
    tiles, entries, stage = plan.tables()
    lam = geometry.sound_speed_m_s / geometry.fs_hz
    ex = O.element_positions(info.n_elements, geometry.pitch_m, getattr(geometry, "element_x_m", None))
    t0s = geometry.t0_s * geometry.fs_hz
    n = info.n_elements
    tx = info.tiling.tile_x
    paired = mirror and (info.flags & hodmas.FLAG_MIRROR)
    worst = worst_b = 0.0
    shared = bool(info.flags & hodmas.INFO_SHARED_DELAYS)
    # samples of delay by which element i + 1 four columns on may differ from element i
    pitch_dev = float(np.abs(np.diff(ex) - 4.0 * grid.dx_m).max()) / lam if shared else 0.0
    for td in tiles:
        if paired and td.ix0 // tx >= (grid.nx // tx) // 2:
            continue                      # right half: formed from the left tiles' delays
        ixs, izs = np.meshgrid(np.arange(td.ix0, td.ix0 + td.nx), np.arange(td.iz0, td.iz0 + td.nz))
        ixs, izs = ixs.ravel(), izs.ravel()
        # the kernel's pixel terms (float64 grid in samples, as in FrameArgs)
        x0s, dxs, z0s, dzs = grid.x0_m / lam, grid.dx_m / lam, grid.z0_m / lam, grid.dz_m / lam
        u = x0s + ixs * dxs - td.xa
        w = z0s + izs * dzs - td.za
        u2 = _r32(2.0 * u)
        q = _r32(u * u + w * (w + 2.0 * td.za))
        ent = entries[td.first_entry:td.first_entry + td.n_active]
        a = np.array([e.a for e in ent])[:, None]
        d0sq = np.array([e.d0sq for e in ent])[:, None]
        d0 = np.array([e.d0 for e in ent])[:, None]
        frac0 = np.array([e.frac0 for e in ent])[:, None]
        T0 = np.array([-e.lo for e in ent])[:, None]
        ch = np.array([e.channel for e in ent])
        num = _r32(u2[None, :] * a + q[None, :])
        d = _r32(np.sqrt(np.abs(_r32(d0sq + num))))
        r = _r32(1.0 / _r32(d + d0))
        t = _r32(num * r + frac0)
        if paired:
            # the mirror pixel (nx-1-ix) to element n-1-i has this delay too
            pix = [(ixs, ch), (grid.nx - 1 - ixs, n - 1 - ch)]
        else:
            pix = [(ixs, ch)]
        for px, el in pix:
            xp = grid.x0_m + px * grid.dx_m
            zp = grid.z0_m + izs * grid.dz_m
            dx = xp[None, :] - ex[el][:, None]
            exact = geometry.fs_hz * (np.sqrt(dx * dx + zp[None, :] ** 2) / geometry.sound_speed_m_s) - t0s
            err = np.abs(T0 + t - exact)
            worst = max(worst, float(err.max()))
            worst_b = max(worst_b, float((err + np.abs(num * r) * 2.0 ** -22).max()))
        # (tiles whose first row lies shallower than 16 pixel columns compute every delay)
        if shared and not td.check and grid.z0_m + td.iz0 * grid.dz_m >= 16.0 * grid.dx_m:
            # delays shared along translated pixels: every element's delay is
            # also formed at the pixel four columns to the left and handed to
            # the pixel / element pair it equals exactly (one element on, four
            # columns on), up to the array's deviation from a 4-column pitch
            uf = u - 4.0 * dxs
            u2f = _r32(2.0 * uf)
            qf = _r32(uf * uf + w * (w + 2.0 * td.za))
            num = _r32(u2f[None, :] * a + qf[None, :])
            d = _r32(np.sqrt(np.abs(_r32(d0sq + num))))
            r = _r32(1.0 / _r32(d + d0))
            t = _r32(num * r + frac0)
            xp = grid.x0_m + (ixs - 4) * grid.dx_m
            zp = grid.z0_m + izs * grid.dz_m
            dx = xp[None, :] - ex[ch][:, None]
            exact = geometry.fs_hz * (np.sqrt(dx * dx + zp[None, :] ** 2) / geometry.sound_speed_m_s) - t0s
            err = np.abs(T0 + t - exact) + pitch_dev
            worst = max(worst, float(err.max()))
            worst_b = max(worst_b, float((err + np.abs(num * r) * 2.0 ** -22).max()))
    return worst, worst_b
