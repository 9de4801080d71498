"""Error of an image against the FP64 oracle, measured from the oracle's own
delay-uncertainty band where a delayed sample sits on a sign change.

The signed k-th root sign(v)|v|^(1/k) has unbounded slope at v = 0 (Sec. II,
the root step of the higher-order correlation).  Where an element's delayed
sample is so close to a zero crossing of its channel that moving its delay by
`eps` samples could change the sample's sign, e_k at that pixel is not fixed by
a float32 delay: rounding leaves a few 1e-6 samples of error in a delay of
tens of samples, and one such element can move e_6 by ten percent while every
other pixel of the image agrees to 1e-7.  At those pixels the oracle is
evaluated again with that element's delay moved by -eps and +eps (the other
elements unchanged); the smallest and largest of the values bound where a
kernel with that delay error may land.  The error there is the distance from
the band (zero inside it); everywhere else it is the plain difference.  A
sample between two equal stored values (flat runs of int16 codes, often
zeros) does not move with its delay and is not flagged: the test is strict,
|v| < |s[j+1] - s[j]| eps.

eps is not a free choice: `plan_eps` takes it from tests/kernel_delays.py,
which emulates the kernel's float32 delay arithmetic on the plan's own tables
and bounds its error over every pixel and element (plus the one-ulp
allowance of the hardware square root and reciprocal).  The flagged pixels
are counted; the GPU tests cap their share (MAX_FLAGGED_SHARE).

Only the oracle is called here (test infrastructure)."""
import math

import numpy as np

from oracle import oracle as O

EPS_SAMPLES = 1e-5         # default; the GPU tests use plan_eps(plan, ...)
MAX_FLAGGED_SHARE = 5e-3   # at most this share of an image's pixels may be flagged


def plan_eps(plan, geometry, grid, mirror=False):
    """The band half-width for images of `plan`: the bound on its kernels'
    float32 delay error (never below EPS_SAMPLES)."""
    from kernel_delays import delay_errors
    return max(EPS_SAMPLES, delay_errors(plan, geometry, grid, mirror=mirror)[1])


def _exact_delays(ex, geometry, grid):
    """[N][nz][nx] delays in samples, the oracle's formula in float64."""
    c, fs, t0 = geometry.sound_speed_m_s, geometry.fs_hz, geometry.t0_s
    xp = grid.x0_m + np.arange(grid.nx) * grid.dx_m
    zp = grid.z0_m + np.arange(grid.nz) * grid.dz_m
    out = np.empty((ex.shape[0], grid.nz, grid.nx))
    for i, xe in enumerate(ex):
        dx = xp[None, :] - xe
        out[i] = fs * (np.sqrt(dx * dx + zp[:, None] * zp[:, None]) / c - t0)
    return out


class SignBand:
    """The sign-change pixels of one stored frame (independent of the order)
    and the band evaluation at them for any order."""

    def __init__(self, arr, geometry, grid, dequant_scale=None, eps=EPS_SAMPLES):
        self.x = np.ascontiguousarray(O.widen(arr, dequant_scale))
        self.arr, self.geometry, self.grid, self.scale, self.eps = arr, geometry, grid, dequant_scale, eps
        n_el, n_s = self.x.shape
        self.ex = O.element_positions(n_el, geometry.pitch_m, getattr(geometry, "element_x_m", None))
        near = {}
        for i, xe in enumerate(self.ex):
            t = _exact_delays(np.array([xe]), geometry, grid)[0]
            j = np.floor(t)
            inside = (j >= 0) & (j < n_s - 1)
            jj = np.clip(j, 0, n_s - 2).astype(np.int64)
            f = t - jj
            s0, s1 = self.x[i, jj], self.x[i, jj + 1]
            v = (1.0 - f) * s0 + f * s1
            hit = inside & (np.abs(v) < np.abs(s1 - s0) * eps)
            for iz, ix in zip(*np.nonzero(hit)):
                near.setdefault((int(iz), int(ix)), []).append(i)
        self.near = near

    @property
    def flagged(self):
        return len(self.near)

    def _band(self, iz, ix, order, ref_value):
        g, gr = self.geometry, self.grid
        xp, zp = gr.x0_m + ix * gr.dx_m, gr.z0_m + iz * gr.dz_m
        c, fs, t0 = g.sound_speed_m_s, g.fs_hz, g.t0_s
        t = [O.tof(self.ex[i], xp, zp, c, fs, t0) for i in range(self.x.shape[0])]
        v = [O.sample(self.x[i], t[i]) for i in range(self.x.shape[0])]
        vals = [ref_value]
        for i in self.near[(iz, ix)]:
            for s in (-self.eps, self.eps):
                w = list(v)
                w[i] = O.sample(self.x[i], t[i] + s)
                vals.append(O.esym([O.signed_root(a, order) for a in w], order))
        return min(vals), max(vals)

    def rel_l2(self, got, order, ref=None):
        """Relative L2 error of `got` [nz][nx] from the oracle (computed here
        unless given), sign-change pixels measured from their band."""
        if ref is None:
            ref = O.beamform(self.arr, self.geometry, self.grid, order, dequant_scale=self.scale)
        got = np.asarray(got, dtype=np.float64)
        err = got - ref
        for (iz, ix) in self.near:
            lo, hi = self._band(iz, ix, order, ref[iz, ix])
            g = got[iz, ix]
            err[iz, ix] = 0.0 if lo <= g <= hi else (g - hi if g > hi else g - lo)
        n = np.linalg.norm(ref)
        return np.linalg.norm(err) / n if n > 0 else np.linalg.norm(got)


def band_rel_l2(got, arr, geometry, grid, order, dequant_scale=None, eps=EPS_SAMPLES):
    """(relative L2 error of `got` [nz][nx] from the oracle with sign-change
    pixels measured from their band, number of such pixels)."""
    sb = SignBand(arr, geometry, grid, dequant_scale, eps)
    return sb.rel_l2(got, order), sb.flagged


def band_rel_l2_loop(got, arr, geometry, grid, order, dequant_scale=None, eps=EPS_SAMPLES):
    """The same measure pixel by pixel through the oracle's scalar calls (the
    definition the vectorised SignBand is checked against on small frames)."""
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
                    if abs(v) < abs(x[i, j + 1] - x[i, j]) * eps:
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
