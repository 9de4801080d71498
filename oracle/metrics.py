"""FP64 CPU oracle of the image-quality metrics (test infrastructure only).

The paper scores its images with (Sec. IV):
- SNR = 20 log10(mu_in / sigma_out)  (Eq. 10),
- CR  = 20 log10(mu_in / mu_out)     (Eq. 11),
  with mu_in, mu_out the mean PA signal over a target and a background region
  and sigma_out the standard deviation over the background;
- gCNR = 1 - sum_x min(h_in(x), h_out(x))  (Eq. 12), h the distributions of
  the normalised signal amplitude x in the two regions;
- FWHM of a target's lateral profile.

Readings (the paper gives no further detail): the metrics are taken on the
envelope image (linear amplitude); regions are pixel rectangles
[ix0, ix1) x [iz0, iz1); sigma_out is the population standard deviation; the
amplitude is normalised by the largest value over both regions and binned
into B equal bins on [0, 1] (the top edge in the last bin, a negative value
-- not expected of an envelope -- in the first), each histogram divided by
its region's pixel count; the FWHM is taken along the image row
through the target region's maximum, walking left and right from the peak to
the first samples at or below half of it and interpolating linearly between
neighbouring pixels, times the pixel pitch (a side that never drops to half
ends at the image edge).

Plain numpy, written from those definitions; only ``tests/`` use it.
"""
from __future__ import annotations

import numpy as np


def region(img: np.ndarray, rect) -> np.ndarray:
    ix0, ix1, iz0, iz1 = rect
    return np.asarray(img, dtype=np.float64)[iz0:iz1, ix0:ix1]


def snr_cr(img, target, background):
    t, b = region(img, target), region(img, background)
    mu_in, mu_out, sd_out = t.mean(), b.mean(), b.std()
    return 20.0 * np.log10(mu_in / sd_out), 20.0 * np.log10(mu_in / mu_out)


def gcnr(img, target, background, bins: int = 256) -> float:
    t, b = region(img, target), region(img, background)
    peak = max(t.max(), b.max())
    if peak <= 0.0:
        return 0.0
    def hist(r):
        idx = np.clip((r / peak * bins).astype(np.int64), 0, bins - 1)
        return np.bincount(idx.ravel(), minlength=bins) / r.size
    return 1.0 - np.minimum(hist(t), hist(b)).sum()


def fwhm(img, target, dx_m: float) -> float:
    img = np.asarray(img, dtype=np.float64)
    t = region(img, target)
    iz_rel, ix_rel = np.unravel_index(np.argmax(t), t.shape)
    iz, ix = target[2] + iz_rel, target[0] + ix_rel
    row = img[iz]
    peak = row[ix]
    half = 0.5 * peak

    def walk(step):
        j = ix
        while 0 <= j + step < row.size:
            if row[j + step] <= half:
                # linear crossing between j and j + step
                return j + step * (row[j] - half) / (row[j] - row[j + step])
            j += step
        return float(j)

    return (walk(+1) - walk(-1)) * dx_m
