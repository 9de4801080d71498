// Display chain of a beamformed image (Sec. III): band-pass along depth,
// envelope by the Hilbert transform, log compression.
//
// Kernel 1 takes a group of C depth columns per workgroup and keeps them in
// LDS as split real/imaginary arrays: the columns are read row by row (C
// consecutive floats per row), band-passed with the centred FIR into the real
// array, transformed by a radix-2 decimation-in-frequency FFT (natural order in,
// bit-reversed out), weighted by the analytic-signal mask in that bit-reversed
// order, and transformed back by a decimation-in-time inverse FFT
// (bit-reversed in, natural out) -- no permutation pass is needed.  It writes
// the envelope |z| and one maximum per workgroup.  Kernel 2 reduces those
// maxima and writes 20 log10(envelope / max), clipped at the dynamic range.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "hodmas.h"

namespace {

constexpr int kDispBlock = 256;
constexpr int kDispColsBudget = 8192;    // C columns x nz samples per workgroup (64 KB as re + im)
constexpr int kMaxNz = 8192;
constexpr int kMaxTaps = 255;
constexpr uint32_t kDisplayMagic = 0x44495350u;  // "DISP"

__device__ __forceinline__ int bit_reverse(int i, int log2n)
{
    return (int)(__builtin_bitreverse32((uint32_t)i) >> (32 - log2n));
}

// Images of one launch: the envelope kernel and the log compression take
// image blockIdx.y (up to kDisplayBatch per launch pair).
constexpr int kDisplayBatch = 16;
struct DisplayImages {
    const float* image[kDisplayBatch];
    float* env[kDisplayBatch];        // envelope out (the dB buffer when no envelope is wanted)
    float* db[kDisplayBatch];
};

__global__ __launch_bounds__(kDispBlock) void envelope_kernel(DisplayImages ims, int nx, int nz, int log2n,
                                                              int cols, const float* __restrict__ taps,
                                                              int numtaps, const float2* __restrict__ tw,
                                                              float* __restrict__ block_max, int n_blocks)
{
    extern __shared__ float lds[];
    const float* __restrict__ image = ims.image[blockIdx.y];
    float* __restrict__ env = ims.env[blockIdx.y];
    // column c at c * ld: the odd stride keeps the row-by-row transposing
    // passes free of bank conflicts
    const int ld = nz + 1;
    float* re = lds;                       // [cols][ld]
    float* im = lds + cols * ld;           // [cols][ld]
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * cols;
    const int nc = min(cols, nx - x0);     // columns of this group inside the image
    const int total = cols * nz;

    // 1. raw samples into im (row by row: the nc columns of a row are adjacent)
    for (int q = tid; q < total; q += kDispBlock) {
        const int z = q / cols, c = q - z * cols;
        im[c * ld + z] = c < nc ? image[(int64_t)z * nx + x0 + c] : 0.f;
    }
    __syncthreads();
    // 2. centred FIR along depth into re (zero beyond the image)
    const int half = (numtaps - 1) / 2;
    for (int q = tid; q < total; q += kDispBlock) {
        const int c = q / nz, z = q - c * nz;
        const float* col = im + c * ld;
        float acc = 0.f;
        for (int k = 0; k < numtaps; ++k) {
            const int zz = z + k - half;
            if (zz >= 0 && zz < nz)
                acc = __builtin_fmaf(taps[k], col[zz], acc);
        }
        re[c * ld + z] = acc;
    }
    __syncthreads();
    for (int q = tid; q < total; q += kDispBlock) {
        const int c = q / nz, z = q - c * nz;
        im[c * ld + z] = 0.f;
    }
    __syncthreads();
    // 3. forward DIF FFT: span n/2 down to 1; twiddle exp(-2 pi i pos / (2 span))
    const int n = nz, hb = n / 2;
    for (int span = hb; span >= 1; span >>= 1) {
        const int stride = hb / span;     // twiddle index step in the length-n/2 table
        for (int q = tid; q < cols * hb; q += kDispBlock) {
            const int c = q / hb, j = q - c * hb;
            const int pos = j & (span - 1);
            const int i0 = c * ld + ((j - pos) << 1) + pos, i1 = i0 + span;
            const float ar = re[i0], ai = im[i0], br = re[i1], bi = im[i1];
            const float2 w = tw[pos * stride];
            const float dr = ar - br, di = ai - bi;
            re[i0] = ar + br;
            im[i0] = ai + bi;
            re[i1] = dr * w.x - di * w.y;
            im[i1] = dr * w.y + di * w.x;
        }
        __syncthreads();
    }
    // 4. analytic-signal weights, at bit-reversed positions: keep bin 0 and the
    //    Nyquist bin, double bins 1..n/2-1, drop the rest; 1/n for the inverse
    const float inv_n = 1.f / (float)n;
    for (int q = tid; q < total; q += kDispBlock) {
        const int c = q / nz, p = q - c * nz;
        const int k = bit_reverse(p, log2n);
        const float wgt = (k == 0 || k == hb) ? inv_n : (k < hb ? 2.f * inv_n : 0.f);
        re[c * ld + p] *= wgt;
        im[c * ld + p] *= wgt;
    }
    __syncthreads();
    // 5. inverse DIT FFT: span 1 up to n/2; twiddle exp(+2 pi i pos / (2 span))
    for (int span = 1; span <= hb; span <<= 1) {
        const int stride = hb / span;
        for (int q = tid; q < cols * hb; q += kDispBlock) {
            const int c = q / hb, j = q - c * hb;
            const int pos = j & (span - 1);
            const int i0 = c * ld + ((j - pos) << 1) + pos, i1 = i0 + span;
            const float2 w = tw[pos * stride];
            const float br = re[i1], bi = im[i1];
            const float tr = br * w.x + bi * w.y;     // b * conj(w)
            const float ti = bi * w.x - br * w.y;
            const float ar = re[i0], ai = im[i0];
            re[i0] = ar + tr;
            im[i0] = ai + ti;
            re[i1] = ar - tr;
            im[i1] = ai - ti;
        }
        __syncthreads();
    }
    // 6. envelope out (row by row), and this group's maximum
    float m = 0.f;
    for (int q = tid; q < total; q += kDispBlock) {
        const int z = q / cols, c = q - z * cols;
        if (c < nc) {
            const float r = re[c * ld + z], i = im[c * ld + z];
            const float e = __builtin_sqrtf(r * r + i * i);
            env[(int64_t)z * nx + x0 + c] = e;
            m = fmaxf(m, e);
        }
    }
    for (int off = 32; off >= 1; off >>= 1)
        m = fmaxf(m, __shfl_xor(m, off));
    __syncthreads();                       // LDS reused for the cross-wave maximum
    if ((tid & 63) == 0)
        lds[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        float bm = 0.f;
        for (int w = 0; w < kDispBlock / 64; ++w)
            bm = fmaxf(bm, lds[w]);
        block_max[(int64_t)blockIdx.y * n_blocks + blockIdx.x] = bm;
    }
}

__global__ __launch_bounds__(kDispBlock) void log_compress_kernel(DisplayImages ims, int64_t count,
                                                                  const float* __restrict__ block_max,
                                                                  int n_blocks, float dyn_range_db)
{
    __shared__ float part[kDispBlock / 64];
    const float* env = ims.env[blockIdx.y];
    float* db = ims.db[blockIdx.y];
    block_max += (int64_t)blockIdx.y * n_blocks;
    float m = 0.f;
    for (int i = threadIdx.x; i < n_blocks; i += kDispBlock)
        m = fmaxf(m, block_max[i]);
    for (int off = 32; off >= 1; off >>= 1)
        m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = m;
    __syncthreads();
    float peak = 0.f;
    for (int w = 0; w < kDispBlock / 64; ++w)
        peak = fmaxf(peak, part[w]);
    const float floor_db = -dyn_range_db;
    const float inv_peak = peak > 0.f ? 1.f / peak : 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kDispBlock + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * kDispBlock) {
        float v = floor_db;
        if (peak > 0.f) {
            const float r = env[i] * inv_peak;
            v = r > 0.f ? fmaxf(20.f * log10f(r), floor_db) : floor_db;
        }
        db[i] = v;
    }
}

// ---------------------------------------------------------------------------
// Allocation-free form (hodmas_display_run_static).  Its band-pass taps, FFT
// twiddles and per-workgroup envelope maxima live in this file-scope device
// array instead of buffers a plan allocates.  Every GPU the library runs on
// holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for that device.
constexpr int kStaticTapFloats = 256;                   // taps (numtaps <= 255)
constexpr int kStaticTwiddles = kMaxNz / 2;             // float2 twiddles
constexpr int kStaticMaxBlocks = 65536;                 // one maximum per workgroup (nx <= 65536)
constexpr size_t kStaticTwiddleOffset = sizeof(float) * kStaticTapFloats;
constexpr size_t kStaticBlockMaxOffset = kStaticTwiddleOffset + sizeof(float2) * kStaticTwiddles;
constexpr size_t kStaticScratchBytes = kStaticBlockMaxOffset + sizeof(float) * kStaticMaxBlocks;
static_assert(kStaticTwiddleOffset % 8 == 0 && kStaticBlockMaxOffset % 4 == 0, "scratch regions aligned");

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Columns per envelope workgroup: as many as the LDS budget allows, but few
// enough that the grid still gives every CU two workgroups.
int display_cols(int nx, int nz, int cus)
{
    return std::max(1, std::min({16, kDispColsBudget / nz, nx / (2 * cus)}));
}

struct StaticTaps {
    float v[kMaxTaps];
};

// The taps (from the kernel arguments) and the twiddles exp(-2 pi i t / nz),
// t < nz / 2, evaluated in float64 and rounded to float as the plan does.
__global__ __launch_bounds__(kDispBlock) void static_tables_kernel(StaticTaps taps, int numtaps, int nz,
                                                                   float* __restrict__ d_taps,
                                                                   float2* __restrict__ d_tw)
{
    const int i = blockIdx.x * kDispBlock + threadIdx.x;
    if (i < numtaps)
        d_taps[i] = taps.v[i];
    if (i < nz / 2) {
        double sn, cs;
        sincospi(-2.0 * double(i) / double(nz), &sn, &cs);
        d_tw[i] = make_float2((float)cs, (float)sn);
    }
}

}  // namespace

struct hodmas_display_s {
    uint32_t magic = kDisplayMagic;
    hodmas_display_desc desc{};
    int log2n = 0, cols = 1, n_blocks = 0, device = -1;
    float* d_taps = nullptr;
    float2* d_tw = nullptr;
    float* d_block_max = nullptr;
};

extern "C" {

hodmas_status hodmas_display_taps(const hodmas_display_desc* d, double* taps)
{
    if (!d || !taps)
        return HODMAS_EINVAL;
    const int nt = d->numtaps;
    if (nt < 1 || nt > kMaxTaps || nt % 2 == 0 || !(d->dz_m > 0.0) || !(d->sound_speed_m_s > 0.0))
        return HODMAS_EINVAL;
    const double fs = d->sound_speed_m_s / d->dz_m;     // one-way flight: dz is dz/c seconds
    if (!(d->f_lo_hz > 0.0 && d->f_lo_hz < d->f_hi_hz && d->f_hi_hz < 0.5 * fs))
        return HODMAS_EINVAL;
    // difference of two Hamming-windowed ideal low-pass responses, scaled to
    // unit gain at the centre of the pass band
    const double lo = d->f_lo_hz / fs, hi = d->f_hi_hz / fs, mid = 0.5 * (nt - 1);
    const double pi = 3.14159265358979323846;
    auto sinc = [pi](double x) { return x == 0.0 ? 1.0 : std::sin(pi * x) / (pi * x); };
    double gain = 0.0;
    for (int k = 0; k < nt; ++k) {
        const double m = k - mid;
        double h = 2.0 * hi * sinc(2.0 * hi * m) - 2.0 * lo * sinc(2.0 * lo * m);
        if (nt > 1)
            h *= 0.54 - 0.46 * std::cos(2.0 * pi * k / (nt - 1));
        taps[k] = h;
        gain += h * std::cos(pi * (lo + hi) * m);
    }
    for (int k = 0; k < nt; ++k)
        taps[k] /= gain;
    return HODMAS_OK;
}

hodmas_status hodmas_display_plan(const hodmas_display_desc* d, hodmas_display_t* out)
{
    if (!d || !out)
        return HODMAS_EINVAL;
    *out = nullptr;
    if (d->nx < 1 || d->nz < 2 || d->nz > kMaxNz || (d->nz & (d->nz - 1)) != 0 || d->nx > 65536 ||
        !(d->dynamic_range_db > 0.f))
        return HODMAS_EINVAL;
    std::vector<double> taps(kMaxTaps);
    hodmas_status st = hodmas_display_taps(d, taps.data());
    if (st != HODMAS_OK)
        return st;
    hodmas_display_s* p = new (std::nothrow) hodmas_display_s;
    if (!p)
        return HODMAS_ENOMEM;
    p->desc = *d;
    while ((1 << p->log2n) < d->nz)
        ++p->log2n;
    int cus = 256;
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
    }
    p->cols = display_cols(d->nx, d->nz, cus);
    p->n_blocks = (d->nx + p->cols - 1) / p->cols;
    std::vector<float> ft(d->numtaps);
    for (int k = 0; k < d->numtaps; ++k)
        ft[k] = (float)taps[k];
    std::vector<float2> tw(d->nz / 2);
    for (int t = 0; t < d->nz / 2; ++t) {
        const double a = -2.0 * 3.14159265358979323846 * t / d->nz;
        tw[t] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    const size_t lds = sizeof(float) * 2 * (size_t)p->cols * (d->nz + 1);
    bool ok = hipGetDevice(&p->device) == hipSuccess &&
              (lds <= 64 * 1024 ||
               hipFuncSetAttribute((const void*)envelope_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds) == hipSuccess) &&
              hipMalloc((void**)&p->d_taps, sizeof(float) * ft.size()) == hipSuccess &&
              hipMalloc((void**)&p->d_tw, sizeof(float2) * tw.size()) == hipSuccess &&
              hipMalloc((void**)&p->d_block_max, sizeof(float) * p->n_blocks * kDisplayBatch) == hipSuccess &&
              hipMemcpy(p->d_taps, ft.data(), sizeof(float) * ft.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(p->d_tw, tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        hodmas_display_destroy(p);
        return HODMAS_ENOMEM;
    }
    *out = p;
    return HODMAS_OK;
}

}  // extern "C"

namespace {

// Launch the chain for n <= kDisplayBatch images of one shape.
hipError_t launch_display(const hodmas_display_desc& d, int log2n, int cols, int n_blocks, const float* taps,
                          const float2* tw, float* block_max, const DisplayImages& ims, int n, hipStream_t st)
{
    const size_t lds = sizeof(float) * 2 * (size_t)cols * (d.nz + 1);
    hipLaunchKernelGGL(envelope_kernel, dim3(n_blocks, n), dim3(kDispBlock), lds, st, ims, d.nx, d.nz, log2n,
                       cols, taps, d.numtaps, tw, block_max, n_blocks);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        const int64_t count = (int64_t)d.nx * d.nz;
        const int grid = (int)std::min<int64_t>((count + kDispBlock - 1) / kDispBlock, 4096);
        hipLaunchKernelGGL(log_compress_kernel, dim3(grid, n), dim3(kDispBlock), 0, st, ims, count, block_max,
                           n_blocks, d.dynamic_range_db);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

extern "C" {

hodmas_status hodmas_display_run_batch(hodmas_display_t p, const float* const* images_dev,
                                       float* const* envelopes_dev, float* const* dbs_dev, int32_t n,
                                       void* stream)
{
    if (!p || p->magic != kDisplayMagic || !images_dev || !dbs_dev || n < 1)
        return HODMAS_EINVAL;
    for (int32_t i = 0; i < n; ++i) {
        const float* env = envelopes_dev ? envelopes_dev[i] : nullptr;
        if (!images_dev[i] || !dbs_dev[i] || images_dev[i] == dbs_dev[i] || images_dev[i] == env)
            return HODMAS_EINVAL;
    }
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess)
        return HODMAS_EDEVICE;
    if (cur != p->device && hipSetDevice(p->device) != hipSuccess)
        return HODMAS_EDEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    for (int32_t i0 = 0; i0 < n && e == hipSuccess; i0 += kDisplayBatch) {
        const int m = std::min<int32_t>(kDisplayBatch, n - i0);
        DisplayImages ims{};
        for (int j = 0; j < m; ++j) {
            float* env = envelopes_dev ? envelopes_dev[i0 + j] : nullptr;
            ims.image[j] = images_dev[i0 + j];
            ims.db[j] = dbs_dev[i0 + j];
            ims.env[j] = env ? env : dbs_dev[i0 + j];     // the dB pass then works in place
        }
        e = launch_display(p->desc, p->log2n, p->cols, p->n_blocks, p->d_taps, p->d_tw, p->d_block_max, ims, m,
                           st);
    }
    if (cur != p->device)
        (void)hipSetDevice(cur);
    return e == hipSuccess ? HODMAS_OK : HODMAS_EDEVICE;
}

hodmas_status hodmas_display_run(hodmas_display_t p, const float* image_dev, float* envelope_dev, float* db_dev,
                                 void* stream)
{
    return hodmas_display_run_batch(p, &image_dev, envelope_dev ? &envelope_dev : nullptr, &db_dev, 1, stream);
}

}  // extern "C"

namespace {

constexpr int kMaxDevices = 64;

struct StaticDevice {
    bool ready = false;
    void* scratch = nullptr;      // device address of `scratch` on this device
    int cus = 256;
};

std::mutex g_static_mu;
StaticDevice g_static[kMaxDevices];

// First call on a device: the device address of its scratch array, its CU
// count, and the LDS limit of the envelope kernel.  Returns null on failure.
const StaticDevice* static_device(int dev)
{
    if (dev < 0 || dev >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticDevice& sd = g_static[dev];
    if (!sd.ready) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        const int lds_max = (int)(sizeof(float) * 2 * (size_t)(kDispColsBudget + 16));
        if (hipFuncSetAttribute((const void*)envelope_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                lds_max) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        sd.scratch = ptr;
        sd.cus = prop.multiProcessorCount;
        sd.ready = true;
    }
    return &sd;
}

}  // namespace

extern "C" {

hodmas_status hodmas_display_run_static(const hodmas_display_desc* d, const float* image_dev, float* envelope_dev,
                                        float* db_dev, void* stream)
{
    if (!d || !image_dev || !db_dev || image_dev == db_dev || image_dev == envelope_dev)
        return HODMAS_EINVAL;
    if (d->nx < 1 || d->nz < 2 || d->nz > kMaxNz || (d->nz & (d->nz - 1)) != 0 || !(d->dynamic_range_db > 0.f))
        return HODMAS_EINVAL;
    if (d->nx > kStaticMaxBlocks)
        return HODMAS_EUNSUPPORTED;             // more workgroup maxima than the scratch array holds
    double taps[kMaxTaps];
    const hodmas_status tst = hodmas_display_taps(d, taps);
    if (tst != HODMAS_OK)
        return tst;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess)
        return HODMAS_EDEVICE;
    const StaticDevice* sd = static_device(dev);
    if (!sd)
        return HODMAS_EDEVICE;
    int log2n = 0;
    while ((1 << log2n) < d->nz)
        ++log2n;
    const int cols = display_cols(d->nx, d->nz, sd->cus);
    const int n_blocks = (d->nx + cols - 1) / cols;
    if (n_blocks > kStaticMaxBlocks)
        return HODMAS_EUNSUPPORTED;
    StaticTaps ft;
    for (int k = 0; k < kMaxTaps; ++k)
        ft.v[k] = k < d->numtaps ? (float)taps[k] : 0.f;
    unsigned char* base = static_cast<unsigned char*>(sd->scratch);
    float* d_taps = reinterpret_cast<float*>(base);
    float2* d_tw = reinterpret_cast<float2*>(base + kStaticTwiddleOffset);
    float* d_block_max = reinterpret_cast<float*>(base + kStaticBlockMaxOffset);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n_tab = std::max(d->numtaps, d->nz / 2);
    hipLaunchKernelGGL(static_tables_kernel, dim3((n_tab + kDispBlock - 1) / kDispBlock), dim3(kDispBlock), 0, st,
                       ft, d->numtaps, d->nz, d_taps, d_tw);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        DisplayImages ims{};
        ims.image[0] = image_dev;
        ims.db[0] = db_dev;
        ims.env[0] = envelope_dev ? envelope_dev : db_dev;
        e = launch_display(*d, log2n, cols, n_blocks, d_taps, d_tw, d_block_max, ims, 1, st);
    }
    return e == hipSuccess ? HODMAS_OK : HODMAS_EDEVICE;
}

hodmas_status hodmas_display_destroy(hodmas_display_t p)
{
    if (!p)
        return HODMAS_OK;
    if (p->magic != kDisplayMagic)
        return HODMAS_EINVAL;
    if (p->d_taps) (void)hipFree(p->d_taps);
    if (p->d_tw) (void)hipFree(p->d_tw);
    if (p->d_block_max) (void)hipFree(p->d_block_max);
    p->magic = 0;
    delete p;
    return HODMAS_OK;
}

}  // extern "C"
