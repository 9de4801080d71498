"""A per-pixel bound on how far a kernel image may sit from the FP64 oracle's:
a forward (running) error analysis of the path's float32 steps, evaluated at
every pixel from the exact delayed samples (test infrastructure; only the
oracle's input helpers are called).

The steps and what each may add (u = 2^-24, float32's unit roundoff):
  1. delay (Eq. 1): the kernel's float32 delay is within `eps` samples of the
     exact one (tests/kernel_delays.py bounds it per plan), so the
     interpolated sample moves by at most eps |s[j+1] - s[j]|; a delay within
     eps of either end of the record may fall on either side of it (sample or
     zero), which adds the end samples' size;
  2. interpolation fma(f, s1 - s0, s0), or the mixed-precision form on FP16
     halves, and the int16 codes' rescaling: at most 4u (|s0| + |s1|);
  3. the signed k-th root (Eqs. 2, 4-6) of the moved sample: by the mean value
     theorem where the move dv is at most half of |v|, else by
     |r(v + dv) - r(v)| <= 2 (3 dv)^(1/k) (both roots are at most (3 dv)^(1/k));
     plus the root's own rounding -- square roots 2u (k = 2), 4u (k = 4), and
     2^(log2|v| / k) with the hardware log2 and exp2 (one ulp each) at most
     u (4 + (3 |log2 v| + 2) / k);
  4. the powers y^j, j < k, as products of the root: at most
     j (r + dr)^(j-1) dr + j (rel + u) (r + dr)^j; the k-th power is the
     sample itself (no root);
  5. power sums, compensated float32 (pairwise groups, a plain partial per 32
     elements, one Kahan step per partial): at most 12u sum_i |y_i^j|;
  6. Newton's identities (Eq. 9's general form) in float32 for k <= 4 and
     float64 for k >= 5: with e_m and p_j the exact values and E_m, d_j the
     bounds on their errors,
       E_m = (1/m) sum_j [E_{m-j} (|p_j| + d_j) + |e_{m-j}| d_j]
             + ((m + 1) u_R / m) sum_j (|e_{m-j}| + E_{m-j}) (|p_j| + d_j)
             + 2 u_R (|e_m| + E_m)
     (first order in the perturbations of p, exact in the propagation of
     E; the rounding of m products, m - 1 sums and the scaling by 1/m);
  7. the output scale and the float32 store: 2u (|e_k| + E_k).

The bound is first order only where step 3 uses the mean value theorem and is
otherwise rigorous up to the stated per-operation allowances.  It covers the
sign-change pixels on its own: there dv exceeds |v| and step 3 takes the
Holder form.  `margin` (the tests use 2) multiplies the whole.
"""
import math

import numpy as np

from oracle import oracle as O

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def _root_rel(a, k):
    """Step 3's rounding allowance of the kernel's k-th root, relative."""
    if k == 1:
        return np.zeros_like(a)
    if k == 2:
        return np.full_like(a, 2 * U32)
    if k == 4:
        return np.full_like(a, 4 * U32)
    with np.errstate(divide="ignore"):
        L = np.abs(np.log2(np.where(a > 0, a, 1.0)))
    return U32 * (4.0 + (3.0 * L + 2.0) / k)


def _delays(xe, geometry, grid, rows=None):
    """[rows][nx] exact delays (samples) to the element at xe (Eq. 1); every
    row of the grid unless `rows` lists some."""
    c, fs, t0 = geometry.sound_speed_m_s, geometry.fs_hz, geometry.t0_s
    xp = grid.x0_m + np.arange(grid.nx) * grid.dx_m
    zp = grid.z0_m + (np.arange(grid.nz) if rows is None else np.asarray(rows)) * grid.dz_m
    dx = xp[None, :] - xe
    return fs * (np.sqrt(dx * dx + zp[:, None] * zp[:, None]) / c - t0)


def pixel_bounds(arr, geometry, grid, orders, eps, dequant_scale=None, margin=2.0, rows=None):
    """{k: [nz][nx] bound on |kernel image - oracle image|} for the orders
    given, for RF `arr` (as stored) imaged with a plan whose float32 delays
    are within `eps` samples of the exact ones; [len(rows)][nx] when `rows`
    names image rows."""
    x = np.ascontiguousarray(O.widen(arr, dequant_scale))
    n_el, n_s = x.shape
    ex = O.element_positions(n_el, geometry.pitch_m, getattr(geometry, "element_x_m", None))
    shape = (grid.nz if rows is None else len(rows), grid.nx)
    p = {k: np.zeros((k,) + shape) for k in orders}     # exact power sums, signed
    d = {k: np.zeros((k,) + shape) for k in orders}     # bounds on their errors
    for i in range(n_el):
        t = _delays(ex[i], geometry, grid, rows)
        inside = (t >= 0.0) & (t <= n_s - 1)
        jj = np.clip(np.floor(t), 0, n_s - 2).astype(np.int64)
        f = t - jj
        s0, s1 = x[i, jj], x[i, jj + 1]
        v = np.where(inside, (1.0 - f) * s0 + f * s1, 0.0)
        dv = eps * np.abs(s1 - s0) + 4.0 * U32 * (np.abs(s0) + np.abs(s1))
        near0 = np.abs(t) <= eps
        near1 = np.abs(t - (n_s - 1)) <= eps
        dv = np.where(inside | near0 | near1, dv, 0.0)
        dv = dv + near0 * (abs(x[i, 0]) + abs(x[i, 1])) + near1 * (abs(x[i, -1]) + abs(x[i, -2]))
        a = np.abs(v)
        sg = np.sign(v)
        for k in orders:
            if k == 1:
                y, dr, rel = v, dv, np.zeros_like(a)
                r = a
            else:
                with np.errstate(divide="ignore", invalid="ignore"):
                    r = np.where(a > 0, np.exp2(np.log2(np.where(a > 0, a, 1.0)) / k), 0.0)
                    small = dv <= 0.5 * a
                    lo = np.where(small, a - dv, 1.0)
                    mvt = np.exp2(np.log2(lo) * (1.0 / k - 1.0)) * dv / k
                dr = np.where(small, mvt, 2.0 * np.exp2(np.log2(np.maximum(3.0 * dv, 1e-300)) / k))
                dr = np.where(dv > 0, dr, 0.0)
                rel = _root_rel(a, k)
                y = sg * r
            rr = r + dr
            yj = np.ones_like(a)
            rj = np.ones_like(a)          # rr^(j-1)
            for j in range(1, k + 1):
                yj = yj * y
                if j < k:
                    dT = j * rj * dr + j * (rel + U32) * rj * rr
                    mag = rj * rr
                else:
                    dT, mag = dv, a + dv
                p[k][j - 1] += yj
                d[k][j - 1] += dT + 12.0 * U32 * mag
                rj = rj * rr
    out = {}
    for k in orders:
        uR = U32 if k <= 4 else U64
        e, E = [np.ones(shape)], [np.zeros(shape)]
        for m in range(1, k + 1):
            acc = np.zeros(shape)
            err = np.zeros(shape)
            s_abs = np.zeros(shape)
            for j in range(1, m + 1):
                pj, dj = p[k][j - 1], d[k][j - 1]
                term = e[m - j] * pj
                acc = acc + term if j % 2 else acc - term
                err += E[m - j] * (np.abs(pj) + dj) + np.abs(e[m - j]) * dj
                s_abs += (np.abs(e[m - j]) + E[m - j]) * (np.abs(pj) + dj)
            em = acc / m
            Em = err / m + (m + 1) * uR * s_abs / m
            Em = Em + 2.0 * uR * (np.abs(em) + Em)
            e.append(em)
            E.append(Em)
        out[k] = margin * (E[k] + 2.0 * U32 * (np.abs(e[k]) + E[k]))
    return out


def worst_ratio(got, ref, bound):
    """max over pixels of |got - ref| / bound (pixels whose bound is zero
    count only if they differ)."""
    err = np.abs(np.asarray(got, dtype=np.float64) - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(bound > 0, err / bound, np.where(err > 0, math.inf, 0.0))
    return float(q.max())
