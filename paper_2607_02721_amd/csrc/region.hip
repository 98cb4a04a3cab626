// Compact-region extension (Section 3.4: Assumption 2, the rho-net and
// Theorem 4): the reductions over per-ray renders at sampled camera poses of
// a region.  For K poses and P pixels (A and A_w as [K][P] float32):
//   - a pixel is kept when A > floor at every pose (Assumption 2 (iv) needs
//     A bounded away from zero on the region);
//   - per pair of poses (i < j), the largest |A_i - A_j| and |A_w,i - A_w,j|
//     over the kept pixels (the Lipschitz estimates divide them by the pose
//     distance on the host);
//   - the smallest A over kept pixels and poses, and the largest relative
//     error |A - A_w| / A over the representatives and over every pose.
// Maxima and minima of non-negative floats are taken on their bit patterns
// (integer atomics, order-free), so the results are deterministic.
#include "gs_internal.hpp"

namespace gs {

__device__ __forceinline__ float wave_max_f(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ float wave_min_f(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
    return v;
}

// keep[p]; out_bits: [0] min A (float bits, starts at +inf), [1] max error
// over the representatives, [2] over every pose; [3] kept pixel count.
__global__ __launch_bounds__(256) void k_region_pixels(const float *__restrict__ A, const float *__restrict__ Aw,
                                                       int K, int64_t P, float floor_, const int32_t *__restrict__ is_net,
                                                       uint8_t *__restrict__ keep, uint32_t *__restrict__ out_bits) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool ok = p < P;
    float amin = __builtin_inff(), enet = 0.0f, eall = 0.0f;
    if (ok) {
        for (int k = 0; k < K; ++k) ok = ok && A[(int64_t)k * P + p] > floor_;
    }
    if (ok) {
        for (int k = 0; k < K; ++k) {
            const float a = A[(int64_t)k * P + p], aw = Aw[(int64_t)k * P + p];
            const float e = fabsf(a - aw) / a;
            amin = fminf(amin, a);
            eall = fmaxf(eall, e);
            if (is_net[k]) enet = fmaxf(enet, e);
        }
    }
    if (p < P) keep[p] = ok ? 1 : 0;
    amin = wave_min_f(amin);
    enet = wave_max_f(enet);
    eall = wave_max_f(eall);
    const uint64_t bal = __ballot(ok);
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&out_bits[0], __float_as_uint(amin));
        atomicMax(&out_bits[1], __float_as_uint(enet));
        atomicMax(&out_bits[2], __float_as_uint(eall));
        if (bal) atomicAdd(&out_bits[3], (uint32_t)__popcll(bal));
    }
}

// One block per pair (i, j), i < j (pair index in row-major upper-triangle
// order): diff[2 pair] = max |A_i - A_j|, diff[2 pair + 1] = the same for A_w.
__global__ __launch_bounds__(256) void k_region_pairs(const float *__restrict__ A, const float *__restrict__ Aw,
                                                      int K, int64_t P, const uint8_t *__restrict__ keep,
                                                      const int32_t *__restrict__ pair_i,
                                                      const int32_t *__restrict__ pair_j, float *__restrict__ diff) {
    __shared__ float sh[2][4];
    const int pr = blockIdx.x;
    const int i = pair_i[pr], j = pair_j[pr];
    const float *a = A + (int64_t)i * P, *b = A + (int64_t)j * P;
    const float *aw = Aw + (int64_t)i * P, *bw = Aw + (int64_t)j * P;
    float d0 = 0.0f, d1 = 0.0f;
    for (int64_t p = threadIdx.x; p < P; p += 256) {
        if (keep[p]) {
            d0 = fmaxf(d0, fabsf(a[p] - b[p]));
            d1 = fmaxf(d1, fabsf(aw[p] - bw[p]));
        }
    }
    d0 = wave_max_f(d0);
    d1 = wave_max_f(d1);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = d0;
        sh[1][w] = d1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        diff[2 * pr] = fmaxf(fmaxf(sh[0][0], sh[0][1]), fmaxf(sh[0][2], sh[0][3]));
        diff[2 * pr + 1] = fmaxf(fmaxf(sh[1][0], sh[1][1]), fmaxf(sh[1][2], sh[1][3]));
    }
}

void launch_region_pixels(const float *A, const float *Aw, int K, int64_t P, float floor_, const int32_t *is_net,
                          uint8_t *keep, uint32_t *out_bits, hipStream_t st) {
    hipLaunchKernelGGL(k_region_pixels, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, A, Aw, K, P, floor_,
                       is_net, keep, out_bits);
}

void launch_region_pairs(const float *A, const float *Aw, int K, int64_t P, const uint8_t *keep, const int32_t *pi,
                         const int32_t *pj, int n_pairs, float *diff, hipStream_t st) {
    hipLaunchKernelGGL(k_region_pairs, dim3((unsigned)n_pairs), dim3(256), 0, st, A, Aw, K, P, keep, pi, pj, diff);
}

}  // namespace gs
