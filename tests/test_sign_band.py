"""Pins of the sign-change band (tests/sign_band.py), on the CPU with the
oracle only: the band is zero for the oracle's own image, leaves errors at
ordinary pixels whole, and covers the documented case -- a 16-element frame
whose pixel (iz 6, ix 19) holds a sample 5e-9 from zero, where a delay change
of 1e-6 samples moves e_6 by more than ten percent."""
import numpy as np

from oracle import oracle as O
from paper_2203_14906_amd import phantom as ph
from sign_band import EPS_SAMPLES, band_rel_l2

GRID = ph.Grid(nx=64, nz=53, x0_m=-(64 - 1) / 2.0 * 0.17e-3, dx_m=0.17e-3, z0_m=0.2e-3, dz_m=0.21e-3)


def _frame():
    f = ph.make_frame(16, 300, 64, 53, n_points=6, n_lines=1, snr_db=15.0, seed=40)
    return f, ph.to_fp32(f.rf)


def _pixel_value(arr, geom, iz, ix, order, shift=None):
    """e_order at one pixel from the oracle's steps, with one element's delay
    optionally moved: shift = (element, samples)."""
    x = arr.astype(np.float64)
    ex = O.element_positions(arr.shape[0], geom.pitch_m)
    xp, zp = GRID.x0_m + ix * GRID.dx_m, GRID.z0_m + iz * GRID.dz_m
    v = []
    for i in range(arr.shape[0]):
        t = O.tof(ex[i], xp, zp, geom.sound_speed_m_s, geom.fs_hz, geom.t0_s)
        if shift is not None and shift[0] == i:
            t += shift[1]
        v.append(O.sample(x[i], t))
    return O.esym([O.signed_root(a, order) for a in v], order), v


def test_sign_change_pixel_is_delay_sensitive():
    f, arr = _frame()
    e0, v = _pixel_value(arr, f.geometry, 6, 19, 6)
    ref = O.beamform(arr, f.geometry, GRID, 6, pixels=(np.array([19]), np.array([6])))[0]
    assert abs(e0 - ref) <= 1e-12 * abs(ref)
    assert abs(v[1]) < 1e-8                      # element 1 sits on a zero crossing
    lo, _ = _pixel_value(arr, f.geometry, 6, 19, 6, shift=(1, -1e-6))
    assert abs(lo - e0) > 0.1 * abs(e0)          # a quarter of a float32 ulp of the delay


def test_band_is_zero_for_the_oracle_and_flags_that_pixel():
    f, arr = _frame()
    ref = O.beamform(arr, f.geometry, GRID, 6)
    err, flagged = band_rel_l2(ref, arr, f.geometry, GRID, 6)
    assert err == 0.0
    assert flagged >= 1


def test_band_covers_the_shifted_delay_but_not_ordinary_errors():
    f, arr = _frame()
    ref = O.beamform(arr, f.geometry, GRID, 6)
    # the sign-change pixel evaluated at a delay error inside the band: no error
    got = ref.copy()
    got[6, 19] = _pixel_value(arr, f.geometry, 6, 19, 6, shift=(1, 0.5 * EPS_SAMPLES))[0]
    assert band_rel_l2(got, arr, f.geometry, GRID, 6)[0] == 0.0
    plain = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert plain > 1e-5                          # the plain metric fails this image
    # the same size of error at an ordinary pixel is counted whole
    got = ref.copy()
    got[30, 10] += 0.2
    err, _ = band_rel_l2(got, arr, f.geometry, GRID, 6)
    assert abs(err - 0.2 / np.linalg.norm(ref)) < 1e-12


def test_vectorised_band_matches_the_pixel_loop():
    """SignBand (vectorised flags) against the pixel-by-pixel definition."""
    from sign_band import band_rel_l2_loop
    f, arr = _frame()
    for order in (3, 6):
        ref = O.beamform(arr, f.geometry, GRID, order)
        got = ref.copy()
        got[6, 19] = _pixel_value(arr, f.geometry, 6, 19, order, shift=(1, 3e-5))[0]
        got[30, 10] += 0.05
        for eps in (1e-5, 4e-5):
            fast = band_rel_l2(got, arr, f.geometry, GRID, order, eps=eps)
            slow = band_rel_l2_loop(got, arr, f.geometry, GRID, order, eps=eps)
            assert fast[1] == slow[1] >= 1
            assert abs(fast[0] - slow[0]) <= 1e-15 + 1e-12 * slow[0]


def test_kernel_delay_emulation_follows_float32_steps():
    """tests/kernel_delays.py: one (pixel, element) by hand in float32, step by
    step (numpy float32 scalars; the FMAs through float64), and the worst
    error over a plan -- a few float32 ulps of delays of tens of samples."""
    import kernel_delays as KD
    from paper_2203_14906_amd import hodmas
    f, arr = _frame()
    plan = hodmas.Plan(f.geometry, GRID, 300, "f32", max_order=6, flags=hodmas.FLAG_HOST_ONLY)
    tiles, entries, _ = plan.tables()
    td, e = tiles[5], entries[tiles[5].first_entry + 3]
    lam = f.geometry.sound_speed_m_s / f.geometry.fs_hz
    ix, iz = td.ix0 + 2, td.iz0 + 1
    u = GRID.x0_m / lam + ix * (GRID.dx_m / lam) - td.xa
    w = GRID.z0_m / lam + iz * (GRID.dz_m / lam) - td.za
    u2, q = np.float32(2.0 * u), np.float32(u * u + w * (w + 2.0 * td.za))
    num = np.float32(np.float64(u2) * np.float64(e.a) + np.float64(q))
    d = np.float32(np.sqrt(np.float32(np.float32(e.d0sq) + num)))
    r = np.float32(1.0) / np.float32(d + np.float32(e.d0))
    t = np.float32(np.float64(num) * np.float64(r) + np.float64(e.frac0))
    ex = O.element_positions(16, f.geometry.pitch_m)
    exact = O.tof(ex[e.channel], GRID.x0_m + ix * GRID.dx_m, GRID.z0_m + iz * GRID.dz_m,
                  f.geometry.sound_speed_m_s, f.geometry.fs_hz, 0.0)
    worst, bound = KD.delay_errors(plan, f.geometry, GRID)
    assert abs(-e.lo + float(t) - exact) <= worst
    assert 1e-7 < worst < bound < 1e-4
    plan.close()


def test_plan_eps_covers_the_documented_pixel():
    """The band half-width derived for the frame's default plan covers the
    documented pixel's delay sensitivity (a shift of 1e-6 samples moved e_6 by
    ten percent there)."""
    from paper_2203_14906_amd import hodmas
    from sign_band import plan_eps
    f, arr = _frame()
    plan = hodmas.Plan(f.geometry, GRID, 300, "f32", max_order=6, flags=hodmas.FLAG_HOST_ONLY)
    eps = plan_eps(plan, f.geometry, GRID)
    assert EPS_SAMPLES <= eps < 1e-4
    ref = O.beamform(arr, f.geometry, GRID, 6)
    got = ref.copy()
    got[6, 19] = _pixel_value(arr, f.geometry, 6, 19, 6, shift=(1, -0.9 * eps))[0]
    assert band_rel_l2(got, arr, f.geometry, GRID, 6, eps=eps)[0] == 0.0
    plan.close()
