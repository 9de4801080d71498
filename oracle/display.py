"""FP64 CPU oracle of the display chain (test infrastructure only).

The simulation study of the paper (Sec. III) band-passes the beamformed image,
takes its envelope with the Hilbert transform and log-compresses it before
display.  The paper gives no filter or dynamic-range values; the readings here
are:

- band-pass: a centred FIR along depth (the fast-time axis of a PA image), a
  Hamming-windowed difference of two ideal low-pass responses scaled to unit
  gain at the centre of the pass band; the depth step dz is dz/c seconds of
  one-way flight, so the filter's sampling rate is c/dz; samples beyond the
  image are zero;
- envelope: the magnitude of the analytic signal of each depth column, built
  from the length-nz DFT (keep bin 0 and the Nyquist bin, double the positive
  bins, drop the negative ones) -- the textbook discrete analytic signal;
- log compression: 20 log10(envelope / max envelope), clipped below at minus
  the dynamic range (an all-zero image maps to minus the dynamic range).

Plain numpy in float64, written from those definitions; only ``tests/`` and
the benchmark's CPU baseline use it.  Nothing here is shared with the HIP path.
"""
from __future__ import annotations

import numpy as np


def bandpass_taps(numtaps: int, f_lo_hz: float, f_hi_hz: float, fs_hz: float) -> np.ndarray:
    """Windowed-sinc band-pass taps (odd length, symmetric), unit gain at the
    centre frequency (f_lo + f_hi) / 2."""
    if numtaps < 1 or numtaps % 2 == 0:
        raise ValueError("numtaps must be odd and positive")
    if not (0.0 < f_lo_hz < f_hi_hz < fs_hz / 2.0):
        raise ValueError("need 0 < f_lo < f_hi < fs/2")
    m = np.arange(numtaps, dtype=np.float64) - (numtaps - 1) / 2.0
    lo, hi = f_lo_hz / fs_hz, f_hi_hz / fs_hz          # cycles per sample
    h = 2.0 * hi * np.sinc(2.0 * hi * m) - 2.0 * lo * np.sinc(2.0 * lo * m)
    if numtaps > 1:
        k = np.arange(numtaps, dtype=np.float64)
        h *= 0.54 - 0.46 * np.cos(2.0 * np.pi * k / (numtaps - 1))
    fc = 0.5 * (lo + hi)
    gain = np.sum(h * np.cos(2.0 * np.pi * fc * m))    # symmetric taps: H(fc) is real
    return h / gain


def bandpass(image: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """Centred FIR along axis 0 (depth), zero outside the image."""
    img = np.asarray(image, dtype=np.float64)
    nz = img.shape[0]
    half = (len(taps) - 1) // 2
    out = np.zeros_like(img)
    for k, h in enumerate(taps):
        shift = k - half                              # out[z] += h[k] * img[z + shift]
        lo, hi = max(0, -shift), min(nz, nz - shift)
        if lo < hi:
            out[lo:hi] += h * img[lo + shift:hi + shift]
    return out


def analytic_mask(n: int) -> np.ndarray:
    """Per-bin weights that turn a length-n DFT into the analytic signal's."""
    w = np.zeros(n)
    w[0] = 1.0
    if n % 2 == 0:
        w[1:n // 2] = 2.0
        w[n // 2] = 1.0
    else:
        w[1:(n + 1) // 2] = 2.0
    return w


def envelope(image: np.ndarray) -> np.ndarray:
    """|analytic signal| of every depth column (axis 0)."""
    x = np.asarray(image, dtype=np.float64)
    spec = np.fft.fft(x, axis=0)
    z = np.fft.ifft(spec * analytic_mask(x.shape[0])[:, None], axis=0)
    return np.abs(z)


def log_compress(env: np.ndarray, dynamic_range_db: float) -> np.ndarray:
    env = np.asarray(env, dtype=np.float64)
    peak = env.max() if env.size else 0.0
    if peak <= 0.0:
        return np.full(env.shape, -float(dynamic_range_db))
    with np.errstate(divide="ignore"):
        db = 20.0 * np.log10(env / peak)
    return np.maximum(db, -float(dynamic_range_db))


def display(image: np.ndarray, dz_m: float, sound_speed_m_s: float, f_lo_hz: float, f_hi_hz: float,
            numtaps: int, dynamic_range_db: float):
    """(band-passed image, envelope, dB image) for a beamformed image [nz][nx]."""
    taps = bandpass_taps(numtaps, f_lo_hz, f_hi_hz, sound_speed_m_s / dz_m)
    bp = bandpass(image, taps)
    env = envelope(bp)
    return bp, env, log_compress(env, dynamic_range_db)
