"""Pins of the image-quality metric oracle against closed forms and library
routines."""
import numpy as np
import pytest

from oracle import metrics as M

T = (2, 6, 3, 7)       # ix0, ix1, iz0, iz1
B = (10, 20, 0, 12)


def test_snr_cr_closed_forms():
    img = np.zeros((12, 20))
    img[3:7, 2:6] = 10.0                              # target: constant 10
    bg = np.tile([1.0, 3.0], 60).reshape(12, 10)      # background: mean 2, std 1 exactly
    img[:, 10:20] = bg
    snr, cr = M.snr_cr(img, T, B)
    assert snr == pytest.approx(20.0)                # 20 log10(10 / 1)
    assert cr == pytest.approx(20 * np.log10(5.0))   # 20 log10(10 / 2)


def test_gcnr_separated_and_identical():
    img = np.zeros((12, 20))
    img[3:7, 2:6] = 1.0
    img[:, 10:20] = 0.2
    assert M.gcnr(img, T, B) == 1.0                  # disjoint distributions
    same = np.full((12, 20), 0.5)
    assert M.gcnr(same, T, B) == 0.0                 # identical distributions


def test_gcnr_equals_library_histograms():
    rng = np.random.default_rng(4)
    img = rng.rayleigh(1.0, (40, 40))
    img[5:15, 5:15] += 2.5
    t, b = (5, 15, 5, 15), (20, 40, 0, 40)
    tv, bv = img[5:15, 5:15], img[0:40, 20:40]
    peak = max(tv.max(), bv.max())
    edges = np.linspace(0.0, 1.0, 65)
    ht, _ = np.histogram(tv / peak, bins=edges)
    hb, _ = np.histogram(bv / peak, bins=edges)
    ref = 1.0 - np.minimum(ht / tv.size, hb / bv.size).sum()
    assert M.gcnr(img, t, b, bins=64) == pytest.approx(ref, abs=1e-12)


def test_fwhm_of_gaussian_and_triangle():
    x = np.arange(201, dtype=np.float64)
    sigma = 7.0
    img = np.zeros((5, 201))
    img[2] = np.exp(-0.5 * ((x - 100.0) / sigma) ** 2)
    w = M.fwhm(img, (90, 110, 0, 5), dx_m=0.1e-3)
    exact = 2.0 * np.sqrt(2.0 * np.log(2.0)) * sigma * 0.1e-3
    assert w == pytest.approx(exact, rel=2e-3)       # linear interpolation on a sampled Gaussian
    tri = np.maximum(0.0, 1.0 - np.abs(x - 100.0) / 40.0)   # triangle: exact FWHM 40 samples
    img[2] = tri
    assert M.fwhm(img, (90, 110, 0, 5), dx_m=1.0) == pytest.approx(40.0, abs=1e-12)


def test_fwhm_runs_to_the_edge():
    img = np.ones((3, 10))
    img[1, 4] = 1.5                                   # half is 0.75: the row never gets there
    assert M.fwhm(img, (0, 10, 0, 3), dx_m=1.0) == pytest.approx(9.0)   # never halves: edges
