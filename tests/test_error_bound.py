"""Pins of the per-pixel error bound (tests/error_bound.py), on the CPU: a
float32 emulation of the kernel's steps -- a delay moved by up to eps,
float32 interpolation by one fused multiply-add, correctly rounded roots,
powers as float32 products, compensated float32 sums (pairwise fours, a plain
partial per 32 elements, Kahan steps), Newton's identities in float32 for
k <= 4 and float64 above -- stays within the bound at every pixel of a
16-element frame at every order, while each plausible mistake in that path
leaves it somewhere: a delay off by a few eps in one element, a term of
Newton's identities with the wrong sign, a dropped element, a root of the
wrong order, the interpolation's fraction dropped.  The bound is also pinned
from above (it is not vacuous): at DAS and DMAS it stays within 1e-4 of the
image's peak."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2203_14906_amd import phantom as ph
import error_bound as EB

GRID = ph.Grid(nx=64, nz=53, x0_m=-(64 - 1) / 2.0 * 0.17e-3, dx_m=0.17e-3, z0_m=0.2e-3, dz_m=0.21e-3)
EPS = 2e-5


def _f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def emulate(arr, geometry, grid, k, rng, delay_err=EPS, bad_element=None, bad_shift=0.0,
            flip_newton=False, drop_element=None, root_order=None, drop_fraction=False):
    """The kernel's order-k image in float32 steps, with optional mistakes."""
    x = np.asarray(arr, dtype=np.float32)
    n_el, n_s = x.shape
    ex = O.element_positions(n_el, geometry.pitch_m)
    shape = (grid.nz, grid.nx)
    ro = root_order or k
    s = np.zeros((k,) + shape, dtype=np.float32)
    c = np.zeros((k,) + shape, dtype=np.float32)
    part = np.zeros((k,) + shape, dtype=np.float32)
    group = []
    for i in range(n_el):
        t = EB._delays(ex[i], geometry, grid) + rng.uniform(-delay_err, delay_err, shape)
        if i == bad_element:
            t = t + bad_shift
        inside = (t >= 0.0) & (t <= n_s - 1)
        jj = np.clip(np.floor(t), 0, n_s - 2).astype(np.int64)
        f = _f32(t - jj)
        s0, s1 = x[i, jj], x[i, jj + 1]
        if drop_fraction:
            v = s0.copy()
        else:
            v = _f32(f.astype(np.float64) * _f32(s1 - s0).astype(np.float64) + s0.astype(np.float64))
        v = np.where(inside & (i != drop_element), v, np.float32(0))
        a = np.abs(v)
        r = _f32(np.abs(v.astype(np.float64)) ** (1.0 / ro))
        y = np.copysign(r, v)
        T = []
        yj = np.ones(shape, dtype=np.float32)
        for j in range(1, k + 1):
            yj = (yj * y).astype(np.float32)
            T.append(yj if j < k else (v if k % 2 else a))
        group.append(np.stack(T))
        if len(group) == 4 or i == n_el - 1:
            while len(group) < 4:
                group.append(np.zeros_like(group[0]))
            g = ((group[0] + group[1]) + (group[2] + group[3])).astype(np.float32)
            part = (part + g).astype(np.float32)
            group = []
            if (i + 1) % 32 == 0 or i == n_el - 1:
                yk = (part - c).astype(np.float32)          # Kahan step
                tk = (s + yk).astype(np.float32)
                c = ((tk - s) - yk).astype(np.float32)
                s = tk
                part = np.zeros_like(part)
    R = np.float32 if k <= 4 else np.float64
    p = (s.astype(R) - c.astype(R)).astype(R)
    e = [np.ones(shape, dtype=R)]
    for m in range(1, k + 1):
        acc = np.zeros(shape, dtype=R)
        for j in range(1, m + 1):
            term = (e[m - j] * p[j - 1]).astype(R)
            plus = bool(j % 2) != (flip_newton and j == 2)
            acc = (acc + term if plus else acc - term).astype(R)
        e.append((acc * R(1.0 / m)).astype(R))
    return e[k].astype(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def frame():
    f = ph.make_frame(16, 300, 64, 53, n_points=6, n_lines=1, snr_db=15.0, seed=41)
    arr = ph.to_fp32(f.rf)
    bounds = EB.pixel_bounds(arr, f.geometry, GRID, (1, 2, 3, 4, 5, 6), EPS)
    refs = {k: O.beamform(arr, f.geometry, GRID, k) for k in range(1, 7)}
    return f, arr, bounds, refs


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_float32_emulation_within_bound(frame, k):
    f, arr, bounds, refs = frame
    rng = np.random.default_rng(100 + k)
    got = emulate(arr, f.geometry, GRID, k, rng)
    q = EB.worst_ratio(got, refs[k], bounds[k])
    assert q <= 1.0, "order %d: error reaches %.2f of the bound" % (k, q)
    assert np.any(got != refs[k])            # the emulation does round


def test_bound_is_tight_at_low_orders(frame):
    f, arr, bounds, refs = frame
    for k in (1, 2):
        assert bounds[k].max() <= 1e-4 * np.abs(refs[k]).max()


@pytest.mark.parametrize("mistake", ["delay", "newton_sign", "dropped_element", "root_order", "no_fraction"])
def test_mistakes_leave_the_bound(frame, mistake):
    f, arr, bounds, refs = frame
    kw = {"delay": dict(bad_element=5, bad_shift=0.02),
          "newton_sign": dict(flip_newton=True),
          "dropped_element": dict(drop_element=9),
          "root_order": dict(root_order=5),
          "no_fraction": dict(drop_fraction=True)}[mistake]
    for k in ((2, 3, 4, 5, 6) if mistake != "root_order" else (6,)):
        got = emulate(arr, f.geometry, GRID, k, np.random.default_rng(7), **kw)
        q = EB.worst_ratio(got, refs[k], bounds[k])
        assert q > 1.0, "%s at order %d stays within the bound (%.2f)" % (mistake, k, q)


def test_zero_bound_without_rounding_or_delay_error(frame, monkeypatch):
    """With no delay error and no rounding the bound vanishes, except where a
    sample is exactly zero -- there is none here."""
    f, arr, _, refs = frame
    monkeypatch.setattr(EB, "U32", 0.0)
    monkeypatch.setattr(EB, "U64", 0.0)
    b = EB.pixel_bounds(arr, f.geometry, GRID, (3, 6), 0.0)
    assert b[3].max() == 0.0 and b[6].max() == 0.0
