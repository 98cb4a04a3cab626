// Microbenchmarks of the chip rates that the rooflines divide by: HBM copy
// bandwidth, the non-packed FP32 FMA issue rate, the v_exp_f32 issue rate
// (its cost in VALU slots is the ratio of the two) and the dense BF16 MFMA
// rate.  Each kernel writes a result that depends on every iteration so
// nothing is optimised away.
#include "gs_internal.hpp"

namespace gs {

__global__ __launch_bounds__(256) void k_peak_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                   int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
}

// 8 independent FMA chains per lane, `iters` steps each.
__global__ __launch_bounds__(256) void k_peak_fma(float *__restrict__ out, int iters, float x, float y) {
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = (float)(threadIdx.x + k) * 1e-3f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = fmaf(a[k], x, y);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += a[k];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// 8 independent chains of v_exp_f32 (a <- exp2(-a) stays in [0.5, 1]).
__global__ __launch_bounds__(256) void k_peak_exp(float *__restrict__ out, int iters) {
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = 0.5f + (float)((threadIdx.x + k) & 7) * 0.0625f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = __builtin_amdgcn_exp2f(-a[k]);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += a[k];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

typedef __bf16 pk_bf16x8 __attribute__((ext_vector_type(8)));
typedef float pk_f32x4 __attribute__((ext_vector_type(4)));

// 4 independent 16x16x32 BF16 MFMA accumulator chains per wave.
__global__ __launch_bounds__(256) void k_peak_mfma(float *__restrict__ out, int iters) {
    pk_bf16x8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = (__bf16)(1.0f + 0.125f * (float)((threadIdx.x + k) & 7));
        b[k] = (__bf16)(0.0078125f * (float)(1 + ((threadIdx.x * 3 + k) & 7)));
    }
    pk_f32x4 c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = pk_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[j], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

hipError_t measure_peaks(double *copy_bytes_per_s, double *fma_per_s, double *exp_per_s, double *mfma_flop_per_s,
                         void *scratch, size_t scratch_bytes, hipStream_t st) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        hipEventDestroy(e0);
        return e;
    }
    float ms = 0.0f;
    // copy: half the scratch to the other half
    const int64_t n4 = (int64_t)(scratch_bytes / 2 / sizeof(float4));
    const float4 *src = (const float4 *)scratch;
    float4 *dst = (float4 *)scratch + n4;
    const unsigned copy_blocks = 256u * 32u;
    hipLaunchKernelGGL(k_peak_copy, dim3(copy_blocks), dim3(256), 0, st, src, dst, n4);  // warm-up
    const int reps = 5;
    hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_peak_copy, dim3(copy_blocks), dim3(256), 0, st, src, dst, n4);
    hipEventRecord(e1, st);
    if ((e = hipEventSynchronize(e1)) == hipSuccess && (e = hipEventElapsedTime(&ms, e0, e1)) == hipSuccess)
        *copy_bytes_per_s = 2.0 * (double)n4 * sizeof(float4) * reps / (ms * 1e-3);
    // FMA, exp and MFMA: enough waves for every SIMD, many iterations
    const unsigned blocks = 256u * 16u;
    float *out = (float *)scratch;
    const int fma_iters = 4096, exp_iters = 2048, mfma_iters = 2048;
    hipLaunchKernelGGL(k_peak_fma, dim3(blocks), dim3(256), 0, st, out, 16, 0.999f, 1e-3f);
    hipEventRecord(e0, st);
    hipLaunchKernelGGL(k_peak_fma, dim3(blocks), dim3(256), 0, st, out, fma_iters, 0.999f, 1e-3f);
    hipEventRecord(e1, st);
    if (e == hipSuccess && (e = hipEventSynchronize(e1)) == hipSuccess &&
        (e = hipEventElapsedTime(&ms, e0, e1)) == hipSuccess)
        *fma_per_s = (double)blocks * 256.0 * 8.0 * fma_iters / (ms * 1e-3);
    hipLaunchKernelGGL(k_peak_exp, dim3(blocks), dim3(256), 0, st, out, 16);
    hipEventRecord(e0, st);
    hipLaunchKernelGGL(k_peak_exp, dim3(blocks), dim3(256), 0, st, out, exp_iters);
    hipEventRecord(e1, st);
    if (e == hipSuccess && (e = hipEventSynchronize(e1)) == hipSuccess &&
        (e = hipEventElapsedTime(&ms, e0, e1)) == hipSuccess)
        *exp_per_s = (double)blocks * 256.0 * 8.0 * exp_iters / (ms * 1e-3);
    hipLaunchKernelGGL(k_peak_mfma, dim3(blocks), dim3(256), 0, st, out, 16);
    hipEventRecord(e0, st);
    hipLaunchKernelGGL(k_peak_mfma, dim3(blocks), dim3(256), 0, st, out, mfma_iters);
    hipEventRecord(e1, st);
    if (e == hipSuccess && (e = hipEventSynchronize(e1)) == hipSuccess &&
        (e = hipEventElapsedTime(&ms, e0, e1)) == hipSuccess)
        // 4 waves per block, 4 MFMAs of 2 * 16 * 16 * 32 flops per iteration
        *mfma_flop_per_s = (double)blocks * 4.0 * 4.0 * mfma_iters * (2.0 * 16 * 16 * 32) / (ms * 1e-3);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return e;
}

}  // namespace gs
