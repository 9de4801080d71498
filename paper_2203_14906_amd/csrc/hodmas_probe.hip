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

enum Op { kAdd, kFma, kFmaSgpr, kExp2, kLog2, kSqrt, kRcp, kBfi, kFract, kOps };

template <int OP>
__global__ __launch_bounds__(kBlock) void rate_kernel(float* __restrict__ out, float s)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    float x[kChains], y[kChains];
    int mask = 0x7fffffff;
    asm volatile("v_mov_b32 %0, %0" : "+v"(mask));   // a VGPR operand for the bitwise probe
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
            if constexpr (OP == kBfi) {
                // integer / bitwise class (the copysign of the signed root)
                int b = __builtin_bit_cast(int, x[i]);
                asm volatile("v_bfi_b32 %0, %1, %0, %2" : "+v"(b) : "v"(mask), "v"(y[i]));
                x[i] = __builtin_bit_cast(float, b);
            }
            if constexpr (OP == kFract) x[i] = __builtin_amdgcn_fractf(x[i]);
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
                            rate_kernel<kLog2>, rate_kernel<kSqrt>, rate_kernel<kRcp>,     rate_kernel<kBfi>,
                            rate_kernel<kFract>};

// The beamformer's inner loop as an instruction mix: per element the delay
// (fma, add, sqrt, add, rcp, fma), the sample index and fraction (floor,
// fraction, address), the interpolation (a stand-in for the LDS gather, sub,
// fma), the signed sixth root (log2, scale, exp2, copysign), the powers and
// the six power-sum adds -- 27 VALU instructions, 4 of them transcendental --
// for four independent elements per iteration, with the per-element
// constants wave-uniform in SGPRs (as the kernel holds them) or in VGPRs.
constexpr int kLoopIters = 512;
constexpr int kLoopWavesPerSimd = 7;

#define HODMAS_PROBE_ELEMENT(CT)                                                                           \
    {                                                                                                      \
        float num, D, d, den, r, t, f, s0, s1, v, L, y, y2, y3, y4, y5;                                    \
        int fl, addr;                                                                                      \
        asm volatile("v_fma_f32 %0, %1, %2, %3" : "=v"(num) : "v"(u2), CT(ca), "v"(q));                 \
        asm volatile("v_add_f32 %0, %1, %2" : "=v"(D) : CT(cb), "v"(num));                               \
        asm volatile("v_sqrt_f32 %0, |%1|" : "=v"(d) : "v"(D));                                          \
        asm volatile("v_add_f32 %0, %1, %2" : "=v"(den) : CT(cc), "v"(d));                               \
        asm volatile("v_rcp_f32 %0, %1" : "=v"(r) : "v"(den));                                          \
        asm volatile("v_fma_f32 %0, %1, %2, %3" : "=v"(t) : "v"(num), "v"(r), CT(cd));                  \
        asm volatile("v_cvt_flr_i32_f32 %0, %1" : "=v"(fl) : "v"(t));                                   \
        asm volatile("v_fract_f32 %0, %1" : "=v"(f) : "v"(t));                                          \
        asm volatile("v_lshl_add_u32 %0, %1, 2, %2" : "=v"(addr) : "v"(fl), CT(off));                   \
        asm volatile("v_cvt_f32_i32 %0, %1" : "=v"(s0) : "v"(addr));                                    \
        asm volatile("v_add_f32 %0, 1.0, %1" : "=v"(s1) : "v"(s0));                                      \
        asm volatile("v_sub_f32 %0, %1, %2" : "=v"(v) : "v"(s1), "v"(s0));                              \
        asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(s0) : "v"(f), "v"(v));                              \
        asm volatile("v_log_f32 %0, |%1|" : "=v"(L) : "v"(s0));                                         \
        asm volatile("v_mul_f32 %0, 0x3e2aaaab, %1" : "=v"(L) : "v"(L));                                 \
        asm volatile("v_exp_f32 %0, %1" : "=v"(y) : "v"(L));                                            \
        asm volatile("v_mul_f32 %0, %1, %1" : "=v"(y2) : "v"(y));                                       \
        asm volatile("v_bfi_b32 %0, %1, %2, %3" : "=v"(y) : CT(mask), "v"(y), "v"(s0));                  \
        asm volatile("v_mul_f32 %0, %1, %2" : "=v"(y3) : "v"(y), "v"(y2));                              \
        asm volatile("v_mul_f32 %0, %1, %1" : "=v"(y4) : "v"(y2));                                      \
        asm volatile("v_mul_f32 %0, %1, %2" : "=v"(y5) : "v"(y3), "v"(y2));                             \
        asm volatile("v_add_f32 %0, %0, %1" : "+v"(p1) : "v"(y));                                       \
        asm volatile("v_add_f32 %0, %0, %1" : "+v"(p2) : "v"(y2));                                      \
        asm volatile("v_add_f32 %0, %0, %1" : "+v"(p3) : "v"(y3));                                      \
        asm volatile("v_add_f32 %0, %0, %1" : "+v"(p4) : "v"(y4));                                      \
        asm volatile("v_add_f32 %0, %0, %1" : "+v"(p5) : "v"(y5));                                      \
        asm volatile("v_add_f32_e64 %0, %0, |%1|" : "+v"(p6) : "v"(s0));                                \
    }
#define HODMAS_PROBE_SREG(x) "s"(x)
#define HODMAS_PROBE_VREG(x) "v"(x)

template <bool VGPR_CONSTANTS>
__global__ __launch_bounds__(kBlock) void loop_kernel(float* __restrict__ out, float a0, float b0, float c0, float d0,
                                                      int off0)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    float u2 = 1e-3f * (tid & 63), q = 2e-3f * (tid & 31);
    float p1 = 0.f, p2 = 0.f, p3 = 0.f, p4 = 0.f, p5 = 0.f, p6 = 0.f;
    float ca = a0, cb = b0, cc = c0, cd = d0;
    int off = off0, mask = 0x7fffffff;
    if constexpr (VGPR_CONSTANTS) {
        asm volatile("v_mov_b32 %0, %0" : "+v"(ca));
        asm volatile("v_mov_b32 %0, %0" : "+v"(cb));
        asm volatile("v_mov_b32 %0, %0" : "+v"(cc));
        asm volatile("v_mov_b32 %0, %0" : "+v"(cd));
        asm volatile("v_mov_b32 %0, %0" : "+v"(off));
        asm volatile("v_mov_b32 %0, %0" : "+v"(mask));
    }
    for (int it = 0; it < kLoopIters; ++it) {
        if constexpr (VGPR_CONSTANTS) {
            HODMAS_PROBE_ELEMENT(HODMAS_PROBE_VREG) HODMAS_PROBE_ELEMENT(HODMAS_PROBE_VREG)
            HODMAS_PROBE_ELEMENT(HODMAS_PROBE_VREG) HODMAS_PROBE_ELEMENT(HODMAS_PROBE_VREG)
        } else {
            HODMAS_PROBE_ELEMENT(HODMAS_PROBE_SREG) HODMAS_PROBE_ELEMENT(HODMAS_PROBE_SREG)
            HODMAS_PROBE_ELEMENT(HODMAS_PROBE_SREG) HODMAS_PROBE_ELEMENT(HODMAS_PROBE_SREG)
        }
    }
    out[tid] = p1 + p2 + p3 + p4 + p5 + p6;   // keeps the sums alive
}

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
    // the inner-loop mix: cycles per wave and element at 2.4 GHz
    double loop_cycles[2] = {0.0, 0.0};
    for (int var = 0; var < 2; ++var) {
        const int lblocks = prop.multiProcessorCount * kLoopWavesPerSimd;   // 4 waves per block
        float lms = 0.f;
        const bool lok = time_ms(st, e0, e1, [&]() {
            if (var)
                hipLaunchKernelGGL(loop_kernel<true>, dim3(lblocks), dim3(kBlock), 0, st, d_out, 0.5f, 400.f, 20.f,
                                   0.25f, 64);
            else
                hipLaunchKernelGGL(loop_kernel<false>, dim3(lblocks), dim3(kBlock), 0, st, d_out, 0.5f, 400.f, 20.f,
                                   0.25f, 64);
        }, &lms);
        if (!lok || !(lms > 0.f)) {
            (void)hipGetLastError();
            cleanup();
            return HODMAS_EDEVICE;
        }
        const double wave_elements = double(kLoopWavesPerSimd) * kLoopIters * 4;   // per SIMD
        loop_cycles[var] = double(lms) * 1e-3 * 2.4e9 / wave_elements;
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
    out->int_bfi = rate[kBfi];
    out->fract = rate[kFract];
    out->loop_cycles_sgpr = loop_cycles[0];
    out->loop_cycles_vgpr = loop_cycles[1];
    out->hbm_copy_tb_s = 2.0 * double(copy_bytes) / (double(ms) * 1e-3) / 1e12;
    out->compute_units = prop.multiProcessorCount;
    return HODMAS_OK;
}
