// Roofline calibration: the FP32 FMA rate this build's kernels can reach.
//
// Every kernel of the library is compiled with packed FP32 instructions
// disabled, so the VALU executes one wave64 FP32 instruction per SIMD every
// four cycles.  This kernel issues nothing but independent v_fma_f32 (eight
// chains per lane, enough waves to fill every SIMD) and reports the rate, the
// ceiling of any FP32 VALU-bound kernel here.
#include <hip/hip_runtime.h>

#include "pamd.h"

namespace {

constexpr int kFmaBlocks = 256 * 16, kFmaThreads = 256, kFmaIters = 20000, kFmaPerIter = 32;

__global__ __launch_bounds__(kFmaThreads) void k_fma_rate(float* out, int iters, float b, float c)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    float a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
        a[q] = tid * 1e-7f + q;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kFmaPerIter / 8; ++u) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                a[q] = fmaf(a[q], b, c);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        s += a[q];
    // a value no input produces: keeps the chains live, stores nothing
    if (s == -12345.0f)
        out[0] = s;
}

}  // namespace

extern "C" pamd_status pamd_fp32_fma_rate(float* d_sink, double* tflops, void* stream)
{
    if (!d_sink || !tflops)
        return PAMD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return PAMD_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return PAMD_ERR_HIP;
    }
    pamd_status st = PAMD_OK;
    double best = 0.0;
    for (int rep = 0; rep < 3 && st == PAMD_OK; ++rep) {
        hipEventRecord(e0, s);
        hipLaunchKernelGGL(k_fma_rate, dim3(kFmaBlocks), dim3(kFmaThreads), 0, s, d_sink, kFmaIters, 0.999f,
                           1e-3f);
        hipEventRecord(e1, s);
        float ms = 0.0f;
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.0f)) {
            st = PAMD_ERR_HIP;
            break;
        }
        const double flops = 2.0 * kFmaPerIter * (double)kFmaIters * kFmaBlocks * kFmaThreads;
        const double tf = flops / (ms * 1e-3) / 1e12;
        if (tf > best)
            best = tf;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *tflops = best;
    return st;
}
