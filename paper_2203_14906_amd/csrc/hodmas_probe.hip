// Measured peaks of this device for the rooflines: issue rates of the VALU
// instruction forms the beamformer uses, and the HBM copy rate.
//
// Each rate kernel runs eight independent dependency chains per lane, with
// eight waves per SIMD, so neither latency nor occupancy limits it; the result
// is lane-operations per second (one wave64 instruction = 64 lane-operations).
// Packed FP32 is not measured: the library is built without it.
#include <hip/hip_runtime.h>

#include "hodmas.h"

namespace {

constexpr int kIters = 4096;
constexpr int kChains = 8;
constexpr int kBlock = 256;
constexpr int kBlocksPerCu = 8;   // 8 x 4 waves per CU = 8 waves per SIMD

enum Op { kAdd, kFma, kFmaSgpr, kExp2, kLog2, kSqrt, kRcp, kOps };

template <int OP>
__global__ __launch_bounds__(kBlock) void rate_kernel(float* __restrict__ out, float s)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    float x[kChains], y[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        x[i] = 0.5f + 1e-3f * float(tid + i);
        y[i] = 1.0f + 1e-7f * float(tid + 3 * i);
    }
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) {
            if constexpr (OP == kAdd) x[i] = x[i] + y[i];
            if constexpr (OP == kFma) x[i] = __builtin_fmaf(x[i], y[i], y[(i + 1) % kChains]);
            if constexpr (OP == kFmaSgpr) x[i] = __builtin_fmaf(x[i], s, y[i]);
            if constexpr (OP == kExp2) x[i] = __builtin_amdgcn_exp2f(x[i]);
            if constexpr (OP == kLog2) x[i] = __builtin_amdgcn_logf(x[i]);
            if constexpr (OP == kSqrt) x[i] = __builtin_amdgcn_sqrtf(x[i]);
            if constexpr (OP == kRcp) x[i] = __builtin_amdgcn_rcpf(x[i]);
        }
    }
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < kChains; ++i)
        acc += x[i];
    out[tid] = acc;   // keeps the chains alive
}

__global__ __launch_bounds__(kBlock) void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                      int64_t n)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

using RateFn = void (*)(float*, float);

const RateFn kRate[kOps] = {rate_kernel<kAdd>,  rate_kernel<kFma>,  rate_kernel<kFmaSgpr>, rate_kernel<kExp2>,
                            rate_kernel<kLog2>, rate_kernel<kSqrt>, rate_kernel<kRcp>};

// Median of three timed runs after one warm-up; milliseconds.
template <class Launch>
bool time_ms(hipStream_t st, hipEvent_t e0, hipEvent_t e1, Launch launch, float* ms)
{
    launch();
    float t[3];
    for (int r = 0; r < 3; ++r) {
        if (hipEventRecord(e0, st) != hipSuccess)
            return false;
        launch();
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t[r], e0, e1) != hipSuccess)
            return false;
    }
    const float a = t[0] < t[1] ? t[0] : t[1], b = t[0] < t[1] ? t[1] : t[0];
    *ms = t[2] < a ? a : (t[2] > b ? b : t[2]);
    return true;
}

}  // namespace

extern "C" hodmas_status hodmas_measure_peaks(hodmas_peaks* out, void* stream)
{
    if (!out)
        return HODMAS_EINVAL;
    int dev = -1;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return HODMAS_EDEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int blocks = prop.multiProcessorCount * kBlocksPerCu;
    const int64_t copy_bytes = int64_t(1) << 30;
    float* d_out = nullptr;
    float4 *src = nullptr, *dst = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (d_out) (void)hipFree(d_out);
        if (src) (void)hipFree(src);
        if (dst) (void)hipFree(dst);
    };
    if (hipMalloc((void**)&d_out, sizeof(float) * size_t(blocks) * kBlock) != hipSuccess ||
        hipMalloc((void**)&src, size_t(copy_bytes)) != hipSuccess ||
        hipMalloc((void**)&dst, size_t(copy_bytes)) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return HODMAS_ENOMEM;
    }
    double rate[kOps];
    const double lane_ops = double(blocks) * kBlock * kIters * kChains;
    for (int op = 0; op < kOps; ++op) {
        float ms = 0.f;
        const RateFn fn = kRate[op];
        const bool ok = time_ms(st, e0, e1, [&]() {
            hipLaunchKernelGGL(fn, dim3(blocks), dim3(kBlock), 0, st, d_out, 0.999f);
        }, &ms);
        if (!ok || !(ms > 0.f)) {
            (void)hipGetLastError();
            cleanup();
            return HODMAS_EDEVICE;
        }
        rate[op] = lane_ops / (double(ms) * 1e-3) / 1e12;
    }
    const int64_t n4 = copy_bytes / int64_t(sizeof(float4));
    float ms = 0.f;
    const bool ok = hipMemsetAsync(src, 0, size_t(copy_bytes), st) == hipSuccess &&
                    time_ms(st, e0, e1, [&]() {
                        hipLaunchKernelGGL(copy_kernel, dim3(prop.multiProcessorCount * 16), dim3(kBlock), 0, st,
                                           src, dst, n4);
                    }, &ms);
    cleanup();
    if (!ok || !(ms > 0.f)) {
        (void)hipGetLastError();
        return HODMAS_EDEVICE;
    }
    out->fp32_add = rate[kAdd];
    out->fp32_fma = rate[kFma];
    out->fp32_fma_sgpr = rate[kFmaSgpr];
    out->exp2 = rate[kExp2];
    out->log2 = rate[kLog2];
    out->sqrt = rate[kSqrt];
    out->rcp = rate[kRcp];
    out->hbm_copy_tb_s = 2.0 * double(copy_bytes) / (double(ms) * 1e-3) / 1e12;
    out->compute_units = prop.multiProcessorCount;
    return HODMAS_OK;
}
