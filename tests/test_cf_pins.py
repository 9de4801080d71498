"""Pins of the coherence-factor weighting in the oracle: closed forms of the
factor and frames whose weighted image is known exactly."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2203_14906_amd import phantom as ph


def test_coherence_closed_forms():
    assert O.coherence([2.5] * 7) == pytest.approx(1.0, abs=1e-15)          # all equal: fully coherent
    assert O.coherence([1.0, -1.0] * 8) == 0.0                              # cancels exactly
    assert O.coherence([0.0, 0.0, -3.0, 0.0, 0.0]) == pytest.approx(1 / 5)  # one element of five
    assert O.coherence([0.0] * 9) == 0.0                                     # nothing received
    assert O.coherence([1.0, 1.0, 0.0, 0.0]) == pytest.approx(4 / (4 * 2))   # (2)^2 / (4 * 2)


def test_coherence_bounds_and_scale_invariance():
    rng = np.random.default_rng(3)
    for _ in range(50):
        v = rng.standard_normal(rng.integers(1, 40))
        cf = O.coherence(v)
        assert -1e-15 <= cf <= 1.0 + 1e-15                                   # Cauchy-Schwarz
        assert O.coherence(v * 7.3) == pytest.approx(cf, rel=1e-12)
        assert O.coherence(-v) == pytest.approx(cf, rel=1e-12)


def _uniform_frame(values, n_samples=400):
    """Channel i holds the constant values[i]: every delay inside the record
    reads it exactly."""
    return np.repeat(np.asarray(values, dtype=np.float64)[:, None], n_samples, axis=1)


def test_weighted_images_on_constant_channels():
    n = 16
    geom = ph.Geometry(n)
    grid = ph.Grid(nx=9, nz=7, x0_m=-1e-3, dx_m=0.25e-3, z0_m=3e-3, dz_m=0.3e-3)   # all delays in record
    same = _uniform_frame([0.7] * n)
    for k in (1, 2, 3, 5):
        plain = O.beamform(same, geom, grid, k)
        np.testing.assert_allclose(O.beamform(same, geom, grid, k, weighting="cf"), plain, rtol=1e-13)
    alt = _uniform_frame([0.7 if i % 2 == 0 else -0.7 for i in range(n)])
    for k in (1, 2, 4):
        assert np.all(O.beamform(alt, geom, grid, k, weighting="cf") == 0.0)
    # one live element of sixteen: CF = 1/16 of the single-element image
    one = _uniform_frame([0.0] * 5 + [0.9] + [0.0] * 10)
    np.testing.assert_allclose(O.beamform(one, geom, grid, 1, weighting="cf"),
                               O.beamform(one, geom, grid, 1) / n, rtol=1e-13)


def test_weighting_refused_for_pixel_lists():
    f = ph.make_frame(8, 128, 4, 4, n_points=1, seed=1)
    with pytest.raises(ValueError):
        O.beamform(ph.to_fp32(f.rf), f.geometry, f.grid, 1, pixels=([0], [0]), weighting="cf")
