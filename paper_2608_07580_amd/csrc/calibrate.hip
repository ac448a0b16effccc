// Vector-ALU rate calibration: sustained lane-operations per second of the
// instructions the retrieval kernel's band loop is made of, so that the
// issue-slot roofline of that loop rests on measured weights (a 32-bit FMA
// is one issue slot; the exponential and reciprocal of the Planck term, the
// FP64 arithmetic of the residual and the conversions between them are
// measured against it).
//
// Each kernel runs eight independent dependency chains per lane (so latency
// is hidden at full occupancy) over a grid of many waves per SIMD, and writes
// every chain's value, so no operation is dead.
#include <hip/hip_runtime.h>

#include <vector>

#include "ff_internal.hpp"

namespace ff {
namespace {

constexpr int kChains = 8;
constexpr int kIters = 512;

enum CalOp : int { CAL_FMA32 = 0, CAL_EXP2_32 = 1, CAL_RCP32 = 2, CAL_FMA64 = 3, CAL_CVT = 4, CAL_NODE = 5 };

template <int OP>
__global__ void __launch_bounds__(256) cal_kernel(float seed, float* __restrict__ out32, double* __restrict__ out64)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const float s = seed + 1e-7f * (float)(tid & 1023);
    if constexpr (OP == CAL_FMA32) {
        float a[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = s + (float)c;
        for (int i = 0; i < kIters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) a[c] = __builtin_fmaf(a[c], 0.999999f, 1e-7f);
        }
        float t = 0.f;
#pragma unroll
        for (int c = 0; c < kChains; ++c) t += a[c];
        out32[tid] = t;
    } else if constexpr (OP == CAL_EXP2_32) {
        float a[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = 1e-3f * (s + (float)c);
        for (int i = 0; i < kIters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) a[c] = __builtin_amdgcn_exp2f(-a[c]);   // converges near 0.64
        }
        float t = 0.f;
#pragma unroll
        for (int c = 0; c < kChains; ++c) t += a[c];
        out32[tid] = t;
    } else if constexpr (OP == CAL_RCP32) {
        float a[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = 1.5f + s + (float)c;
        for (int i = 0; i < kIters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) a[c] = __builtin_amdgcn_rcpf(a[c]);      // x, 1/x, x, ...
        }
        float t = 0.f;
#pragma unroll
        for (int c = 0; c < kChains; ++c) t += a[c];
        out32[tid] = t;
    } else if constexpr (OP == CAL_FMA64) {
        double a[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = (double)s + c;
        for (int i = 0; i < kIters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) a[c] = fma(a[c], 0.999999, 1e-7);
        }
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < kChains; ++c) t += a[c];
        out64[tid] = t;
    } else if constexpr (OP == CAL_CVT) {
        // one widening and one narrowing conversion per step
        float a[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = s + (float)c;
        for (int i = 0; i < kIters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                double w = (double)a[c];
                asm volatile("" : "+v"(w));
                a[c] = (float)w;
                asm volatile("" : "+v"(a[c]));
            }
        }
        float t = 0.f;
#pragma unroll
        for (int c = 0; c < kChains; ++c) t += a[c];
        out32[tid] = t;
    } else {
        // the band loop's per-node body: x = a u, q = 1/(2^x - 1), three
        // quadrature sums (7 VALU + exp2 + rcp per node)
        float a = 1.0f + s, i0 = 0.f, m0 = 0.f, s0 = 0.f;
        float u[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) u[c] = 1e-3f * (1.0f + (float)c);
        for (int i = 0; i < kIters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                const float x = a * u[c];
                const float q = __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(x) - 1.0f);
                i0 = __builtin_fmaf(0.01f, q, i0);
                const float y = x * __builtin_fmaf(q, q, q);
                m0 = __builtin_fmaf(0.02f, y, m0);
                s0 = __builtin_fmaf(0.03f, y, s0);
            }
            asm volatile("" : "+v"(a) : "v"(i0), "v"(m0), "v"(s0));
        }
        out32[tid] = i0 + m0 + s0;
    }
}

template <int OP>
ff_status time_op(int blocks, float* o32, double* o64, hipEvent_t e0, hipEvent_t e1, hipStream_t s, double* ms)
{
    hipLaunchKernelGGL(cal_kernel<OP>, dim3(blocks), dim3(256), 0, s, 1.0f, o32, o64);   // warm-up
    FF_HIP_TRY(hipEventRecord(e0, s));
    hipLaunchKernelGGL(cal_kernel<OP>, dim3(blocks), dim3(256), 0, s, 1.0f, o32, o64);
    FF_HIP_TRY(hipEventRecord(e1, s));
    FF_HIP_TRY(hipGetLastError());
    FF_HIP_TRY(hipEventSynchronize(e1));
    float t = 0.f;
    FF_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    *ms = t;
    return FF_OK;
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" ff_status ff_valu_rates(double* rates_host, int32_t n_rates, void* stream)
{
    if (!rates_host || n_rates < 6) return set_error(FF_EINVAL, "ff_valu_rates: need room for 6 rates");
    int dev = 0, n_cu = 0;
    FF_HIP_TRY(hipGetDevice(&dev));
    FF_HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = n_cu * 32;     // 8 waves per SIMD for every SIMD
    const size_t lanes = (size_t)blocks * 256;
    float* o32 = nullptr;
    double* o64 = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMalloc(&o32, lanes * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&o64, lanes * sizeof(double));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    ff_status st = e == hipSuccess ? FF_OK : hip_error(e, "ff_valu_rates");
    // lane-operations per kernel: chains x iterations per lane; the node body
    // counts as one node (its operations are reported per node)
    const double ops = (double)lanes * kChains * kIters;
    double ms[6] = {0, 0, 0, 0, 0, 0};
    if (st == FF_OK) st = time_op<CAL_FMA32>(blocks, o32, o64, e0, e1, s, &ms[0]);
    if (st == FF_OK) st = time_op<CAL_EXP2_32>(blocks, o32, o64, e0, e1, s, &ms[1]);
    if (st == FF_OK) st = time_op<CAL_RCP32>(blocks, o32, o64, e0, e1, s, &ms[2]);
    if (st == FF_OK) st = time_op<CAL_FMA64>(blocks, o32, o64, e0, e1, s, &ms[3]);
    if (st == FF_OK) st = time_op<CAL_CVT>(blocks, o32, o64, e0, e1, s, &ms[4]);
    if (st == FF_OK) st = time_op<CAL_NODE>(blocks, o32, o64, e0, e1, s, &ms[5]);
    if (st == FF_OK) {
        for (int k = 0; k < 6; ++k) rates_host[k] = ops / (ms[k] * 1e-3);
        rates_host[4] *= 2.0;          // two conversions per step
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (o32) (void)hipFree(o32);
    if (o64) (void)hipFree(o64);
    if (st != FF_OK) return st;
    return clear_error();
}
