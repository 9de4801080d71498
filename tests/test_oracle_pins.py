"""Pins of the FP64 oracle against facts fixed outside it: the paper's own
definitions and closed forms, hand-worked values, brute force over subsets,
closed-form special cases, invariants and the focusing property of delay-and-sum.
None of these re-evaluates the oracle's own expansion."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2203_14906_amd import phantom as ph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
C, FS = 1540.0, 40e6
LAM = C / FS                                   # metres per sample of one-way delay


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([part.strip() for part in line.split(";")])
    return rows


def brute_esym(y, k):
    """Sum over all k-subsets of the product of their members (exact for ints)."""
    return sum(math.prod(c) for c in itertools.combinations(list(y), k))


def real_root(v, k):
    return math.copysign(abs(v) ** (1.0 / k), v) if v != 0 else 0.0


# ---------------------------------------------------------------- e_k stage
def test_golden_worked_example():
    for ys, k, want in _golden("esym_worked_example.txt"):
        y = [float(v) for v in ys.split()]
        assert O.esym(y, int(k)) == float(want)


def test_esym_matches_subset_enumeration_exactly():
    rng = np.random.default_rng(11)
    for _ in range(300):
        n = int(rng.integers(1, 11))
        y = rng.integers(-4, 5, size=n)
        for k in range(1, 8):
            want = brute_esym([int(v) for v in y], k)      # python ints, exact
            got = O.esym(y.astype(np.float64), k)
            assert got == float(want), (list(y), k, got, want)


def test_esym_special_cases():
    y = np.array([0.5, -2.0, 3.0, 0.25])
    assert O.esym(y, 4) == pytest.approx(np.prod(y), rel=1e-15)        # k = N: the product
    assert O.esym(y, 5) == 0.0                                          # k > N: no subset
    assert O.esym(y, 1) == pytest.approx(y.sum(), rel=1e-15)            # k = 1: DAS sum
    # a zero channel is the same as removing the channel
    for k in range(1, 5):
        assert O.esym(np.append(y, 0.0), k) == pytest.approx(O.esym(y, k), rel=1e-14, abs=1e-14)
    # order of channels does not matter
    for k in range(1, 5):
        assert O.esym(y[::-1].copy(), k) == pytest.approx(O.esym(y, k), rel=1e-14)


# ---------------------------------------------------------------- signed roots
def test_golden_signed_roots():
    for v, k, want in _golden("signed_roots.txt"):
        assert O.signed_root(float(v), int(k)) == pytest.approx(float(want), rel=1e-14, abs=0)


# ------------------------------------------- the paper's definitions, Eqs. 2, 4-6
def _paper_definition(s, k):
    """Eq. 2 (k=2), Eq. 4 (k=3), Eq. 5 (k=4), Eq. 6 (k=5) exactly as printed:
    the root is taken of the product of the k delayed samples."""
    total = 0.0
    for comb in itertools.combinations(s, k):
        prod = math.prod(comb)
        if k in (2, 4):       # signed even root of the product, Eqs. 2 and 5
            total += math.copysign(abs(prod) ** (1.0 / k), prod) if prod != 0 else 0.0
        else:                 # real odd root of the product, Eqs. 4 and 6
            total += real_root(prod, k)
    return total


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_oracle_equals_paper_definitions(k):
    rng = np.random.default_rng(100 + k)
    for _ in range(20):
        n = int(rng.integers(k, 9))
        s = rng.uniform(-1.0, 1.0, size=n) * rng.choice([1e-3, 1.0, 7.0])
        want = _paper_definition(list(s), k)
        got = O.esym([O.signed_root(v, k) for v in s], k)
        scale = max(1e-300, sum(abs(math.prod(c)) ** (1.0 / k) for c in itertools.combinations(s, k)))
        assert abs(got - want) <= 1e-12 * scale, (k, got, want)


# ------------------------------------------- the paper's O(N) forms, Eqs. 3, 7, 8, 9
def _eq3(s):
    a = sum(math.copysign(math.sqrt(abs(v)), v) for v in s)
    return (a * a - sum(abs(v) for v in s)) / 2.0


def _eq7(s):
    r = [real_root(v, 3) for v in s]
    a, b = sum(r), sum(x * x for x in r)
    return (a ** 3 + 2.0 * sum(s) - 3.0 * a * b) / 6.0


def _eq8(s):
    q = [math.copysign(abs(v) ** 0.25, v) if v else 0.0 for v in s]
    a = sum(q)
    h = sum(math.sqrt(abs(v)) for v in s)
    cube = sum(math.copysign(abs(v) ** 0.25, v) ** 3 if v else 0.0 for v in s)
    return (a ** 4 - 6.0 * sum(abs(v) for v in s) + 3.0 * h * h - 6.0 * h * a * a
            + 8.0 * cube * a) / 24.0


def _eq9(s):
    r = [real_root(v, 5) for v in s]
    p1 = sum(r)
    p2 = sum(x ** 2 for x in r)
    p3 = sum(x ** 3 for x in r)
    p4 = sum(x ** 4 for x in r)
    return (p1 ** 5 + 24.0 * sum(s) - 30.0 * p1 * p4 + 20.0 * p3 * p1 ** 2 - 20.0 * p3 * p2
            + 15.0 * p2 ** 2 * p1 - 10.0 * p2 * p1 ** 3) / 120.0


@pytest.mark.parametrize("k,form", [(2, _eq3), (3, _eq7), (4, _eq8), (5, _eq9)])
def test_oracle_equals_paper_closed_forms(k, form):
    rng = np.random.default_rng(7 * k)
    for _ in range(50):
        n = int(rng.integers(1, 40))
        s = rng.uniform(-1.0, 1.0, size=n) * rng.choice([1e-6, 1.0, 300.0])
        y = [O.signed_root(v, k) for v in s]
        got = O.esym(y, k)
        want = form(list(s))
        # the closed forms cancel terms of size ~ (sum|y|)^k / k!; allow their rounding
        scale = max(sum(abs(v) for v in y) ** k, 1e-300)
        assert abs(got - want) <= 1e-13 * scale, (k, n, got, want)


# ------------------------------------------- invariants over whole channel sets
@pytest.mark.parametrize("k", range(1, 7))
def test_identical_channels(k):
    # N identical samples s give C(N,k) sign(s)^k |s| (each of the C(N,k)
    # products is (sign(s) |s|^(1/k))^k)
    for n in (1, 3, 8, 17):
        for s in (0.37, -0.37, 2.5, -2.5):
            got = O.esym([O.signed_root(s, k) for _ in range(n)], k)
            want = math.comb(n, k) * (math.copysign(1.0, s) ** k) * abs(s)
            assert got == pytest.approx(want, rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("k", range(1, 7))
def test_sign_flip_and_homogeneity(k):
    rng = np.random.default_rng(50 + k)
    s = rng.uniform(-1, 1, size=13)
    base = O.esym([O.signed_root(v, k) for v in s], k)
    flip = O.esym([O.signed_root(-v, k) for v in s], k)
    assert flip == pytest.approx((-1) ** k * base, rel=1e-12, abs=1e-14)
    for a in (0.001, 3.0, 1e5):
        scaled = O.esym([O.signed_root(a * v, k) for v in s], k)
        assert scaled == pytest.approx(a * base, rel=1e-11, abs=1e-14 * a)


# ---------------------------------------------------------------- delays
def test_tof_hand_values():
    # element at x = 0, pixel 3 samples across and 4 deep: 5 samples of flight
    assert O.tof(0.0, 3 * LAM, 4 * LAM, C, FS) == pytest.approx(5.0, rel=1e-14)
    assert O.tof(-2 * LAM, LAM, 4 * LAM, C, FS) == pytest.approx(5.0, rel=1e-14)
    # t0 shifts the origin: one sample later start gives one sample less
    assert O.tof(0.0, 3 * LAM, 4 * LAM, C, FS, 1.0 / FS) == pytest.approx(4.0, rel=1e-14)
    # on axis: 1.54 mm at 1540 m/s is 1 microsecond, 40 samples at 40 MHz
    assert O.tof(0.0, 0.0, 1.54e-3, 1540.0, 40e6) == pytest.approx(40.0, rel=1e-14)


# ---------------------------------------------------------------- interpolation
def test_sample_rules():
    s = 3.0 * np.arange(10) + 1.0                     # ramp: interpolation is exact
    for t in (0.0, 0.25, 3.5, 7.75, 8.999, 9.0):
        assert O.sample(s, t) == pytest.approx(3.0 * t + 1.0, rel=1e-15)
    assert O.sample(s, 4.0) == s[4]                    # integer index: the stored sample
    assert O.sample(s, 9.0) == s[9]                    # t == S-1: last sample
    assert O.sample(s, 9.0 + 1e-9) == 0.0              # past the record: 0
    assert O.sample(s, -1e-12) == 0.0                  # before the record: 0
    assert O.sample(s, float("nan")) == 0.0
    assert O.sample(np.array([2.5]), 0.0) == 2.5       # single-sample record
    # the last sample is used without reading past the record (NaN sentinel after it)
    guarded = np.append(s, np.nan)
    assert O.sample(guarded[:10], 9.0) == s[9]
    q = np.arange(6, dtype=np.float64) ** 2            # secant of a parabola: j^2 + f(2j+1)
    assert O.sample(q, 2.25) == pytest.approx(4.0 + 0.25 * 5.0, rel=1e-15)


# ---------------------------------------------------------------- whole frames
def _geom(ex, t0=0.0):
    return ph.Geometry(n_elements=len(ex), pitch_m=0.0, sound_speed_m_s=C, fs_hz=FS, t0_s=t0,
                       element_x_m=np.asarray(ex, dtype=np.float64))


@pytest.mark.parametrize("k", range(1, 7))
def test_integer_delay_frame(k):
    """Elements at x = -9, -5, 0, 5, 9, 16 samples and a pixel 12 samples deep on
    axis: flight times 15, 13, 12, 13, 15, 20 samples (Pythagorean triples).
    Samples there are y_i^k with signs, so the pixel value is e_k(y) exactly."""
    ex = np.array([-9, -5, 0, 5, 9, 16], dtype=np.float64) * LAM
    delays = [15, 13, 12, 13, 15, 20]
    y = [2.0, -1.0, 3.0, 1.0, -2.0, 1.0]
    rng = np.random.default_rng(5)
    rf = rng.uniform(-50, 50, size=(6, 32))
    for i, (d, v) in enumerate(zip(delays, y)):
        rf[i, d] = math.copysign(abs(v) ** k, v)
    grid = ph.Grid(nx=1, nz=1, x0_m=0.0, dx_m=LAM, z0_m=12 * LAM, dz_m=LAM)
    got = O.beamform(rf, _geom(ex), grid, k)[0, 0]
    want = brute_esym(y, k)
    assert got == pytest.approx(want, rel=1e-9, abs=1e-9)


def test_ramp_rf_das_and_channel_rows():
    """Per-channel ramps s_i[t] = a_i t + b_i are interpolated exactly, so DAS at a
    pixel is sum_i (a_i t_i + b_i); distinct a_i, b_i catch channel-row mix-ups."""
    n, S = 7, 400
    ex = (np.arange(n) - 3.0) * 0.3e-3
    a = np.linspace(0.5, 2.0, n)
    b = np.linspace(-3.0, 1.0, n)
    rf = a[:, None] * np.arange(S)[None, :] + b[:, None]
    grid = ph.Grid(nx=5, nz=4, x0_m=-1e-3, dx_m=0.4e-3, z0_m=2e-3, dz_m=0.7e-3)
    img = O.beamform(rf, _geom(ex), grid, 1)
    for iz in range(4):
        for ix in range(5):
            xp, zp = -1e-3 + ix * 0.4e-3, 2e-3 + iz * 0.7e-3
            t = FS * np.sqrt((xp - ex) ** 2 + zp ** 2) / C
            assert img[iz, ix] == pytest.approx(np.sum(a * t + b), rel=1e-12)


def test_out_of_record_pixels_are_zero():
    ex = (np.arange(4) - 1.5) * 0.3e-3
    rf = np.ones((4, 50))
    # 40 mm deep is ~1039 samples of flight, far past a 50-sample record
    grid = ph.Grid(nx=3, nz=2, x0_m=0.0, dx_m=1e-4, z0_m=40e-3, dz_m=1e-4)
    for k in (1, 2, 3):
        assert np.all(O.beamform(rf, _geom(ex), grid, k) == 0.0)
    # with t0 pushing every delay below zero the result is 0 as well
    grid2 = ph.Grid(nx=2, nz=2, x0_m=0.0, dx_m=1e-4, z0_m=1e-3, dz_m=1e-4)
    assert np.all(O.beamform(rf, _geom(ex, t0=1e-3), grid2, 1) == 0.0)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_point_source_focuses_at_its_pixel(k):
    """Delay-and-sum aligns a point source's arrivals at the source position
    (Sec. II-A), so the image peaks on the pixel holding the source.  The RF is a
    Gaussian pulse centred on each element's arrival time r_i / c."""
    n, S = 32, 1024
    ex = (np.arange(n) - (n - 1) / 2.0) * 0.3e-3
    grid = ph.make_grid(48, 40, n * 0.3e-3, 12e-3)
    src_ix, src_iz = 33, 27                              # off axis, asymmetric
    xs = grid.x0_m + src_ix * grid.dx_m
    zs = grid.z0_m + src_iz * grid.dz_m
    arrival = FS * np.sqrt((xs - ex) ** 2 + zs ** 2) / C
    t = np.arange(S)[None, :]
    rf = np.exp(-0.5 * ((t - arrival[:, None]) / 1.5) ** 2)
    img = O.beamform(rf, _geom(ex), grid, k)
    iz, ix = np.unravel_index(np.argmax(img), img.shape)
    assert (ix, iz) == (src_ix, src_iz)


def test_stride_and_pixels_api():
    rng = np.random.default_rng(3)
    n, S = 5, 64
    rf = rng.standard_normal((n, S))
    ex = (np.arange(n) - 2.0) * 0.3e-3
    grid = ph.Grid(nx=6, nz=5, x0_m=-0.6e-3, dx_m=0.2e-3, z0_m=0.3e-3, dz_m=0.15e-3)
    full = O.beamform(rf, _geom(ex), grid, 3)
    # padded rows: the row stride is larger than the record length
    padded = np.zeros((n, S + 11))
    padded[:, :S] = rf
    L = O.lib()
    out = np.zeros((grid.nz, grid.nx))
    rc = L.hodmas_oracle_beamform(n, O._pd(ex), C, FS, 0.0, S, O._pd(padded), S + 11,
                                  grid.nx, grid.nz, grid.x0_m, grid.dx_m, grid.z0_m, grid.dz_m,
                                  3, O._pd(out))
    assert rc == 0
    np.testing.assert_array_equal(out, full)
    ix = np.array([0, 5, 3, 2], dtype=np.int32)
    iz = np.array([0, 4, 1, 3], dtype=np.int32)
    pix = O.beamform(rf, _geom(ex), grid, 3, pixels=(ix, iz))
    np.testing.assert_array_equal(pix, full[iz, ix])


def test_widening_is_exact():
    codes = np.array([[-8191, -1, 0, 1, 8191]], dtype=np.int16)
    scale = np.float32(1.0 / (0.7 * 8191))
    w = O.widen(codes, scale)
    assert w.dtype == np.float64
    np.testing.assert_array_equal(w, codes.astype(np.float64) * float(scale))
    h = np.array([[0.1, -0.333, 65504.0]], dtype=np.float16)
    np.testing.assert_array_equal(O.widen(h), [[float(v) for v in h[0]]])
    with pytest.raises(ValueError):
        O.widen(codes)


def test_bad_arguments_rejected():
    L = O.lib()
    ex = np.zeros(2)
    rf = np.zeros((2, 4))
    out = np.zeros(1)
    # stride shorter than the record
    assert L.hodmas_oracle_beamform(2, O._pd(ex), C, FS, 0.0, 4, O._pd(rf), 3, 1, 1,
                                    0.0, 1.0, 0.0, 1.0, 1, O._pd(out)) == 1
    # order 0
    assert L.hodmas_oracle_beamform(2, O._pd(ex), C, FS, 0.0, 4, O._pd(rf), 4, 1, 1,
                                    0.0, 1.0, 0.0, 1.0, 0, O._pd(out)) == 1
