"""Pins of the display-chain oracle (band-pass, Hilbert envelope, log
compression) against closed forms and library routines -- nothing here
retypes the oracle's own formulas."""
import numpy as np
import pytest
import scipy.ndimage
import scipy.signal

from oracle import display as D


@pytest.mark.parametrize("numtaps,f_lo,f_hi,fs", [(31, 2e6, 8e6, 40e6), (65, 1e6, 3e6, 20.5e6),
                                                  (5, 3e6, 6e6, 30e6), (129, 4e6, 12e6, 41.07e6)])
def test_taps_equal_library_window_design(numtaps, f_lo, f_hi, fs):
    ref = scipy.signal.firwin(numtaps, [f_lo, f_hi], pass_zero=False, fs=fs, window="hamming", scale=True)
    np.testing.assert_allclose(D.bandpass_taps(numtaps, f_lo, f_hi, fs), ref, rtol=0, atol=1e-14)


def test_taps_reject_bad_designs():
    for args in [(30, 1e6, 2e6, 10e6), (31, 2e6, 1e6, 10e6), (31, 1e6, 6e6, 10e6), (31, 0.0, 1e6, 10e6)]:
        with pytest.raises(ValueError):
            D.bandpass_taps(*args)


def test_bandpass_equals_library_convolution():
    rng = np.random.default_rng(1)
    img = rng.standard_normal((200, 7))
    taps = D.bandpass_taps(41, 1.5e6, 6e6, 40e6)
    ref = scipy.ndimage.convolve1d(img, taps[::-1], axis=0, mode="constant", cval=0.0)
    np.testing.assert_allclose(D.bandpass(img, taps), ref, rtol=0, atol=1e-13)
    for j in range(img.shape[1]):
        np.testing.assert_allclose(D.bandpass(img[:, j:j + 1], taps)[:, 0], np.convolve(img[:, j], taps, "same"),
                                   rtol=0, atol=1e-13)


def test_bandpass_passes_centre_tone_and_stops_dc():
    fs, f_lo, f_hi = 40e6, 2e6, 8e6
    taps = D.bandpass_taps(65, f_lo, f_hi, fs)
    n = np.arange(2000)
    tone = np.cos(2 * np.pi * 0.5 * (f_lo + f_hi) / fs * n + 0.3)[:, None]
    out = D.bandpass(tone, taps)
    interior = slice(100, 1900)
    np.testing.assert_allclose(out[interior], tone[interior], atol=1e-12)   # unit gain, zero phase
    dc = D.bandpass(np.ones((2000, 1)), taps)
    assert np.abs(dc[interior]).max() < 10 ** (-40 / 20)                   # Hamming stop band


@pytest.mark.parametrize("n", [64, 256, 1024, 96, 81])
def test_envelope_of_pure_tones_is_the_amplitude(n):
    k = np.arange(n)
    rng = np.random.default_rng(n)
    cols = []
    amps = []
    for f in (1, 3, n // 4, n // 2 - 1):
        a, ph = rng.uniform(0.5, 2.0), rng.uniform(0, 2 * np.pi)
        cols.append(a * np.cos(2 * np.pi * f * k / n + ph))
        amps.append(a)
    env = D.envelope(np.stack(cols, axis=1))
    np.testing.assert_allclose(env, np.broadcast_to(amps, env.shape), rtol=1e-12)


def test_envelope_of_modulated_carrier_is_the_modulation():
    # a slow positive modulation times a faster carrier with separate spectra
    n = 512
    k = np.arange(n)
    mod = 1.0 + 0.6 * np.cos(2 * np.pi * 5 * k / n + 0.4)
    x = mod * np.cos(2 * np.pi * 60 * k / n)
    np.testing.assert_allclose(D.envelope(x[:, None])[:, 0], mod, rtol=1e-12)


def test_envelope_equals_library_hilbert():
    rng = np.random.default_rng(5)
    for n in (128, 333):
        x = rng.standard_normal((n, 4))
        np.testing.assert_allclose(D.envelope(x), np.abs(scipy.signal.hilbert(x, axis=0)), rtol=1e-12, atol=1e-12)


def test_log_compression():
    env = np.array([[2.0, 0.2, 0.02], [2e-4, 0.0, 1.0]])
    db = D.log_compress(env, 60.0)
    np.testing.assert_allclose(db[0], [0.0, -20.0, -40.0], atol=1e-12)
    assert db[1, 0] == -60.0 and db[1, 1] == -60.0
    np.testing.assert_allclose(db[1, 2], 20 * np.log10(0.5), atol=1e-12)
    assert np.all(D.log_compress(np.zeros((3, 3)), 45.0) == -45.0)


def test_display_chain_on_a_pulse_train():
    # band-limited pulses at known depths: the envelope peaks sit on them
    nz, fs = 1024, 40e6
    z = np.arange(nz)
    img = np.zeros((nz, 3))
    sigma = fs / (2 * np.pi * 5e6)
    for col, centre in enumerate((200, 500, 800)):
        u = (z - centre) / sigma
        img[:, col] = -u * np.exp(-0.5 * u * u)
    c, dz = 1540.0, 1540.0 / fs
    bp, env, db = D.display(img, dz, c, 2e6, 9e6, 63, 50.0)
    for col, centre in enumerate((200, 500, 800)):
        assert abs(int(np.argmax(env[:, col])) - centre) <= 1
    assert db.max() == 0.0 and db.min() >= -50.0
