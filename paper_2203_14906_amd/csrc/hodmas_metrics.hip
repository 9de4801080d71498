// Image-quality metrics of a beamformed (envelope) image (Sec. IV): SNR
// (Eq. 10), CR (Eq. 11), gCNR (Eq. 12) over a target and a background
// rectangle, and the FWHM of the target's lateral profile.
//
// One workgroup does it all: the regions are small next to an image, and
// the statistics need each other in sequence (means, then deviations and the
// normalising peak, then histograms, then the half-maximum walk).  Sums are
// float64; the amplitude bins use a float64 division, so a pixel lands in
// the same bin as in a float64 reference.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "hodmas.h"

namespace {

constexpr int kMetBlock = 1024;
constexpr int kMaxBins = 4096;

struct Rect {
    int ix0, ix1, iz0, iz1;
    __device__ int count() const { return (ix1 - ix0) * (iz1 - iz0); }
    __device__ int64_t at(int q, int nx) const   // q-th pixel in row-major order
    {
        const int w = ix1 - ix0;
        return (int64_t)(iz0 + q / w) * nx + ix0 + q % w;
    }
};

// Block-wide sum of a double (every thread gets the result).
__device__ double block_sum(double v, double* sh)
{
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i)
        t += sh[i];
    return t;
}

__device__ double block_max(double v, double* sh)
{
    for (int off = 32; off >= 1; off >>= 1)
        v = fmax(v, __shfl_xor(v, off));
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        sh[w] = v;
    __syncthreads();
    double t = sh[0];
    for (int i = 1; i < nw; ++i)
        t = fmax(t, sh[i]);
    return t;
}

__device__ int block_min_int(int v, int* sh)
{
    for (int off = 32; off >= 1; off >>= 1)
        v = min(v, __shfl_xor(v, off));
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        sh[w] = v;
    __syncthreads();
    int t = sh[0];
    for (int i = 1; i < nw; ++i)
        t = min(t, sh[i]);
    return t;
}

__global__ __launch_bounds__(kMetBlock) void metrics_kernel(const float* __restrict__ img, int nx, Rect tr,
                                                            Rect br, int bins, double dx,
                                                            hodmas_metrics* __restrict__ out)
{
    __shared__ double sh[kMetBlock / 64];
    __shared__ int shi[kMetBlock / 64];
    __shared__ unsigned hist_t[kMaxBins], hist_b[kMaxBins];
    const int nt = tr.count(), nb = br.count();
    // means and maxima
    double st = 0.0, sb = 0.0, mt = -HUGE_VAL, mb = -HUGE_VAL;
    for (int q = threadIdx.x; q < nt; q += kMetBlock) {
        const double v = img[tr.at(q, nx)];
        st += v;
        mt = fmax(mt, v);
    }
    for (int q = threadIdx.x; q < nb; q += kMetBlock) {
        const double v = img[br.at(q, nx)];
        sb += v;
        mb = fmax(mb, v);
    }
    const double mu_in = block_sum(st, sh) / nt;
    const double mu_out = block_sum(sb, sh) / nb;
    const double max_t = block_max(mt, sh);
    const double max_b = block_max(mb, sh);
    // deviations from the background mean; the target's first maximum
    double dev = 0.0;
    for (int q = threadIdx.x; q < nb; q += kMetBlock) {
        const double d = (double)img[br.at(q, nx)] - mu_out;
        dev += d * d;
    }
    const double sigma_out = sqrt(block_sum(dev, sh) / nb);
    int first = nt;
    for (int q = threadIdx.x; q < nt; q += kMetBlock)
        if ((double)img[tr.at(q, nx)] == max_t)
            first = min(first, q);
    first = block_min_int(first, shi);
    if (first >= nt)
        first = 0;   // no pixel equals the maximum (NaNs): fall back to the first
    // histograms of the normalised amplitude
    for (int i = threadIdx.x; i < bins; i += kMetBlock) {
        hist_t[i] = 0u;
        hist_b[i] = 0u;
    }
    __syncthreads();
    const double peak = fmax(max_t, max_b);
    if (peak > 0.0) {
        for (int q = threadIdx.x; q < nt; q += kMetBlock) {
            const int k = min(max((int)((double)img[tr.at(q, nx)] / peak * bins), 0), bins - 1);
            atomicAdd(&hist_t[k], 1u);
        }
        for (int q = threadIdx.x; q < nb; q += kMetBlock) {
            const int k = min(max((int)((double)img[br.at(q, nx)] / peak * bins), 0), bins - 1);
            atomicAdd(&hist_b[k], 1u);
        }
    }
    __syncthreads();
    double overlap = 0.0;
    for (int i = threadIdx.x; i < bins; i += kMetBlock)
        overlap += fmin((double)hist_t[i] / nt, (double)hist_b[i] / nb);
    overlap = block_sum(overlap, sh);
    if (threadIdx.x == 0) {
        // FWHM along the row through the target's maximum
        const int64_t p = tr.at(first, nx);
        const int iz = (int)(p / nx), ix = (int)(p - (int64_t)iz * nx);
        const float* row = img + (int64_t)iz * nx;
        const double half = 0.5 * (double)row[ix];
        double edge[2];
        for (int side = 0; side < 2; ++side) {
            const int step = side ? 1 : -1;
            int j = ix;
            double e = (double)j;
            while (j + step >= 0 && j + step < nx) {
                const double a = row[j], b = row[j + step];
                if (b <= half) {
                    e = j + step * (a - half) / (a - b);
                    break;
                }
                j += step;
                e = (double)j;
            }
            edge[side] = e;
        }
        hodmas_metrics m;
        m.mu_in = mu_in;
        m.mu_out = mu_out;
        m.sigma_out = sigma_out;
        m.snr_db = 20.0 * log10(mu_in / sigma_out);
        m.cr_db = 20.0 * log10(mu_in / mu_out);
        m.gcnr = peak > 0.0 ? 1.0 - overlap : 0.0;
        m.fwhm_m = (edge[1] - edge[0]) * dx;
        *out = m;
    }
}

bool rect_ok(const hodmas_rect* r, int nx, int nz)
{
    return r && r->ix0 >= 0 && r->ix0 < r->ix1 && r->ix1 <= nx && r->iz0 >= 0 && r->iz0 < r->iz1 &&
           r->iz1 <= nz;
}

}  // namespace

extern "C" hodmas_status hodmas_image_metrics(const float* image_dev, int32_t nx, int32_t nz, double dx_m,
                                              const hodmas_rect* target, const hodmas_rect* background,
                                              int32_t bins, void* stream, hodmas_metrics* out)
{
    if (!image_dev || !out || nx < 1 || nz < 1 || !(dx_m > 0.0) || bins < 2 || bins > kMaxBins ||
        !rect_ok(target, nx, nz) || !rect_ok(background, nx, nz))
        return HODMAS_EINVAL;
    hodmas_metrics* d_out = nullptr;
    if (hipMalloc((void**)&d_out, sizeof(hodmas_metrics)) != hipSuccess) {
        (void)hipGetLastError();
        return HODMAS_ENOMEM;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Rect tr{target->ix0, target->ix1, target->iz0, target->iz1};
    const Rect br{background->ix0, background->ix1, background->iz0, background->iz1};
    hipLaunchKernelGGL(metrics_kernel, dim3(1), dim3(kMetBlock), 0, st, image_dev, nx, tr, br, bins, dx_m,
                       d_out);
    hodmas_metrics h;
    const bool ok = hipGetLastError() == hipSuccess &&
                    hipMemcpyAsync(&h, d_out, sizeof(h), hipMemcpyDeviceToHost, st) == hipSuccess &&
                    hipStreamSynchronize(st) == hipSuccess;
    (void)hipFree(d_out);
    if (!ok) {
        (void)hipGetLastError();
        return HODMAS_EDEVICE;
    }
    *out = h;
    return HODMAS_OK;
}
