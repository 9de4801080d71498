"""Error of an image against the FP64 oracle, measured from the oracle's own
delay-uncertainty band where a delayed sample sits on a sign change.

The signed k-th root sign(v)|v|^(1/k) has unbounded slope at v = 0 (Sec. II,
the root step of the higher-order correlation).  Where an element's delayed
sample is so close to a zero crossing of its channel that moving its delay by
`eps` samples could change the sample's sign, e_k at that pixel is not fixed by
a float32 delay: rounding alone leaves a few 1e-6 samples of error in a delay of
tens of samples, and one such element can move e_6 by ten percent while every
other pixel of the image agrees to 1e-7.  At those pixels the oracle is
evaluated again with that element's delay moved by -eps and +eps (the other
elements unchanged); the smallest and largest of the values bound where a
kernel with that delay error may land.  The error there is the distance from
the band (zero inside it); everywhere else it is the plain difference.

Only the oracle is called here (test infrastructure)."""
import math

import numpy as np

from oracle import oracle as O

EPS_SAMPLES = 1e-5   # about two float32 ulps of a delay below 64 samples


def band_rel_l2(got, arr, geometry, grid, order, dequant_scale=None, eps=EPS_SAMPLES):
    """(relative L2 error of `got` [nz][nx] from the oracle with sign-change
    pixels measured from their band, number of such pixels)."""
    x = np.ascontiguousarray(O.widen(arr, dequant_scale))
    n_el, n_s = x.shape
    ex = O.element_positions(n_el, geometry.pitch_m, getattr(geometry, "element_x_m", None))
    c, fs, t0 = geometry.sound_speed_m_s, geometry.fs_hz, geometry.t0_s
    ref = O.beamform(arr, geometry, grid, order, dequant_scale=dequant_scale)
    got = np.asarray(got, dtype=np.float64)
    err = got - ref
    flagged = 0
    for iz in range(grid.nz):
        zp = grid.z0_m + iz * grid.dz_m
        for ix in range(grid.nx):
            xp = grid.x0_m + ix * grid.dx_m
            t = [O.tof(ex[i], xp, zp, c, fs, t0) for i in range(n_el)]
            near = []
            for i in range(n_el):
                j = math.floor(t[i])
                if 0 <= j < n_s - 1:
                    v = O.sample(x[i], t[i])
                    if abs(v) <= abs(x[i, j + 1] - x[i, j]) * eps:
                        near.append(i)
            if not near:
                continue
            v = [O.sample(x[i], t[i]) for i in range(n_el)]
            vals = [ref[iz, ix]]
            for i in near:
                for s in (-eps, eps):
                    w = list(v)
                    w[i] = O.sample(x[i], t[i] + s)
                    vals.append(O.esym([O.signed_root(a, order) for a in w], order))
            lo, hi = min(vals), max(vals)
            g = got[iz, ix]
            err[iz, ix] = 0.0 if lo <= g <= hi else (g - hi if g > hi else g - lo)
            flagged += 1
    n = np.linalg.norm(ref)
    return (np.linalg.norm(err) / n if n > 0 else np.linalg.norm(got)), flagged
