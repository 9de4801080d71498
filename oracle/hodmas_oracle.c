/*
 * hodmas_oracle.c -- plain FP64 CPU oracle for higher-order delay-multiply-and-sum
 * (HO-DMAS) photoacoustic beamforming.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously correct reference the
 * GPU library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the GPU library neither links nor
 * calls it, and the two share no source, header, table or helper.
 *
 * What is computed, for every pixel p of the image grid and a chosen order k
 * (the number of channels multiplied together):
 *
 *   1. the one-way time of flight from the pixel to element i, in samples,
 *      t_i(p) = fs * (|p - e_i| / c - t0)            (delay of Eq. 1, Sec. II-A);
 *   2. the delayed channel sample s_i = s_i[t_i(p)], linearly interpolated
 *      between neighbouring samples, and 0 when t_i(p) lies outside [0, S-1];
 *   3. the signed k-th root y_i = sign(s_i) |s_i|^(1/k)  (Eq. 2 and Eqs. 4-6:
 *      signed square and fourth roots, real cube and fifth roots);
 *   4. the image value S_k(p) = sum over all k-subsets I of the channels of
 *      prod_{i in I} y_i  (Eq. 1 for k = 1, Eq. 2 for k = 2, Eqs. 4-6 for
 *      k = 3..5, and the same definition for higher orders, Sec. VI).
 *
 * Step 4 is the k-th elementary symmetric polynomial of the y_i.  It is
 * evaluated here as the coefficient of x^k in prod_i (1 + y_i x), expanding the
 * product one channel at a time.  Every k-subset product appears exactly once
 * in that expansion, so this is the subset-sum definition reorganised as a
 * product of binomials; it is deliberately NOT the power-sum route (Eqs. 3, 7-9)
 * the fast path takes.
 *
 * Where the paper is silent (delay formula, interpolation, boundary, signs of
 * odd roots) each function below states the reading it follows.
 * Build: gcc -O2 -fopenmp -ffp-contract=off, no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Time of flight in samples from pixel (xp, zp) to an element at (xe, 0).
 * One-way propagation (the pixel is the source), time origin at the laser
 * shot shifted by t0 (Sec. II-A, Eq. 1: the per-element delay applied to
 * each channel before summation). */
double hodmas_oracle_tof(double xe, double xp, double zp, double c, double fs, double t0)
{
    double dx = xp - xe;
    double dist = sqrt(dx * dx + zp * zp);
    return fs * (dist / c - t0);
}

/* Channel sample at fractional index t: linear interpolation between s[j] and
 * s[j+1]; t outside [0, S-1] gives 0 (the channel drops out of every product);
 * t == S-1 gives s[S-1]; integer t gives s[t]. */
double hodmas_oracle_sample(const double *s, int64_t n_samples, double t)
{
    if (n_samples <= 0 || !(t >= 0.0) || t > (double)(n_samples - 1))
        return 0.0;
    if (n_samples == 1)
        return s[0];
    double fl = floor(t);
    int64_t j = (int64_t)fl;
    if (j > n_samples - 2)
        j = n_samples - 2;
    double f = t - (double)j;
    return (1.0 - f) * s[j] + f * s[j + 1];
}

/* Signed k-th root sign(v) |v|^(1/k), sign(0) = 0.  For odd k this is the real
 * root of Eqs. 4 and 6; for even k the signed root of Eqs. 2 and 5. */
double hodmas_oracle_signed_root(double v, int order)
{
    if (v == 0.0)
        return 0.0;
    if (order == 1)
        return v;
    double m = pow(fabs(v), 1.0 / (double)order);
    return v < 0.0 ? -m : m;
}

/* k-th elementary symmetric polynomial of y[0..n-1]: the coefficient of x^k in
 * prod_i (1 + y_i x).  e[j] holds the coefficient of x^j of the partial
 * product; multiplying by (1 + y_i x) adds y_i * e[j-1] to e[j], taken from
 * high j to low so every old coefficient is used once.  k > n gives 0. */
double hodmas_oracle_esym(const double *y, int n, int order)
{
    if (order < 0)
        return 0.0;
    if (order == 0)
        return 1.0;
    double *e = (double *)calloc((size_t)order + 1, sizeof(double));
    if (!e)
        return NAN;
    e[0] = 1.0;
    for (int i = 0; i < n; ++i) {
        int top = (i + 1 < order) ? i + 1 : order;
        for (int j = top; j >= 1; --j)
            e[j] += y[i] * e[j - 1];
    }
    double r = e[order];
    free(e);
    return r;
}

/* Coherence factor of the n delayed samples v_i (the weighting the paper
 * proposes to combine with its beamformers, Sec. VI; the factor itself is the
 * standard one of the weighting literature it cites in Sec. I):
 *   CF = (sum_i v_i)^2 / (n * sum_i v_i^2),
 * with n the number of array elements (samples outside the record count as
 * zeros); 0 when every sample is 0.  By Cauchy-Schwarz 0 <= CF <= 1. */
double hodmas_oracle_coherence(const double *v, int n)
{
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < n; ++i) {
        s1 += v[i];
        s2 += v[i] * v[i];
    }
    return s2 > 0.0 ? (s1 * s1) / ((double)n * s2) : 0.0;
}

/* One pixel: delays, interpolated samples, signed roots, symmetric sum;
 * weighting 1 multiplies the sum by the coherence factor of the samples.
 * y and v are caller scratch of n_el doubles each. */
static double beamform_pixel(int n_el, const double *elem_x, double c, double fs, double t0,
                             int64_t n_samples, const double *rf, int64_t stride,
                             double xp, double zp, int order, int weighting, double *y, double *v)
{
    for (int i = 0; i < n_el; ++i) {
        double t = hodmas_oracle_tof(elem_x[i], xp, zp, c, fs, t0);
        v[i] = hodmas_oracle_sample(rf + (int64_t)i * stride, n_samples, t);
        y[i] = hodmas_oracle_signed_root(v[i], order);
    }
    double e = hodmas_oracle_esym(y, n_el, order);
    return weighting == 1 ? e * hodmas_oracle_coherence(v, n_el) : e;
}

static int check_args(int n_el, const double *elem_x, double c, double fs, int64_t n_samples,
                      const double *rf, int64_t stride, int order)
{
    if (n_el < 1 || !elem_x || !rf || !(c > 0.0) || !(fs > 0.0))
        return 1;
    if (n_samples < 1 || stride < n_samples || order < 1)
        return 1;
    return 0;
}

/* Whole image, row-major [nz][nx]; pixel (ix, iz) sits at
 * (x0 + ix*dx, z0 + iz*dz).  weighting: 0 none, 1 coherence factor.
 * Returns 0 on success, 1 on bad arguments, 2 when out of memory. */
int hodmas_oracle_beamform_weighted(int n_el, const double *elem_x, double c, double fs, double t0,
                                    int64_t n_samples, const double *rf, int64_t stride,
                                    int nx, int nz, double x0, double dx, double z0, double dz,
                                    int order, int weighting, double *image)
{
    if (check_args(n_el, elem_x, c, fs, n_samples, rf, stride, order) || nx < 0 || nz < 0 || !image ||
        weighting < 0 || weighting > 1)
        return 1;
    int64_t npix = (int64_t)nx * nz;
    int bad = 0;
#pragma omp parallel
    {
        double *y = (double *)malloc(sizeof(double) * 2 * (size_t)n_el);
        if (!y) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < npix; ++p) {
            if (!y)
                continue;
            int64_t iz = p / nx, ix = p % nx;
            image[p] = beamform_pixel(n_el, elem_x, c, fs, t0, n_samples, rf, stride,
                                      x0 + (double)ix * dx, z0 + (double)iz * dz, order, weighting,
                                      y, y + n_el);
        }
        free(y);
    }
    return bad ? 2 : 0;
}

int hodmas_oracle_beamform(int n_el, const double *elem_x, double c, double fs, double t0,
                           int64_t n_samples, const double *rf, int64_t stride,
                           int nx, int nz, double x0, double dx, double z0, double dz,
                           int order, double *image)
{
    return hodmas_oracle_beamform_weighted(n_el, elem_x, c, fs, t0, n_samples, rf, stride, nx, nz,
                                           x0, dx, z0, dz, order, 0, image);
}

/* A list of pixels (ix[j], iz[j]), j < npix, into out[j]. */
int hodmas_oracle_beamform_pixels(int n_el, const double *elem_x, double c, double fs, double t0,
                                  int64_t n_samples, const double *rf, int64_t stride,
                                  double x0, double dx, double z0, double dz, int order,
                                  int64_t npix, const int32_t *ix, const int32_t *iz, double *out)
{
    if (check_args(n_el, elem_x, c, fs, n_samples, rf, stride, order) || npix < 0 ||
        (npix > 0 && (!ix || !iz || !out)))
        return 1;
    int bad = 0;
#pragma omp parallel
    {
        double *y = (double *)malloc(sizeof(double) * 2 * (size_t)n_el);
        if (!y) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < npix; ++p) {
            if (!y)
                continue;
            out[p] = beamform_pixel(n_el, elem_x, c, fs, t0, n_samples, rf, stride,
                                    x0 + (double)ix[p] * dx, z0 + (double)iz[p] * dz, order, 0,
                                    y, y + n_el);
        }
        free(y);
    }
    return bad ? 2 : 0;
}

/* Number of threads a parallel region of this library runs with. */
int hodmas_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads later parallel regions of this library use (n >= 1); timing only,
 * the results do not depend on it. */
void hodmas_oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
