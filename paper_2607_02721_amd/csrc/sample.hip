// Sensitivity sampling (Algorithm 1, steps 3-5; proof of Theorem 2).
//
// p_i = s_i / S is realised exactly with integers: q_i = ceil(s_i 2^40)
// (exact, since s_i 2^40 is exact in float64 for a float32 s_i), C = inclusive
// prefix sum of q, Q = C[n-1].  Draw t uses the Philox4x32-10 block of
// counter (t, 0, 0) and key = seed, read as a 128-bit integer u, and picks
// the first index with C_i > floor(u Q / 2^128).  Weights are
// n_i Q / (m q_i), evaluated as two IEEE double products and one division
// (this file is built without floating-point contraction).
#include "gs_internal.hpp"

namespace gs {

// Accepted sensitivities: [0, 1 + 2^-10].  A share is at most 1, but its
// float32 value can exceed 1 by a few ulps (a Gaussian alone on a ray scores
// (c rho) (1/A) with 1/A rounded); with n <= 2^24 - 2^16 values of at most
// 2^40 + 2^30 each, Q stays below 2^64.
constexpr float kSensMax = 1.0009765625f;   // 1 + 2^-10

// q_i = ceil(s_i 2^40) (0 for s_i = 0 and for values outside the accepted
// range, which k_quantize reports).
__device__ __forceinline__ uint64_t quantum(float x) {
    return (x > 0.0f && x <= kSensMax) ? (uint64_t)ceil(ldexp((double)x, 40)) : 0ull;
}

// A sensitivity outside [0, 1 + 2^-10] (or NaN) could overflow Q: such a
// value gets q_i = 0 and raises *bad, which the host reads with Q and turns
// into an error.
__global__ void k_quantize(const float *__restrict__ s, int64_t n, uint64_t *__restrict__ q, uint32_t *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float x = i < n ? s[i] : 0.0f;
    const bool ok = x >= 0.0f && x <= kSensMax;
    if (i < n) q[i] = quantum(x);
    if (__ballot(!ok) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

void launch_quantize(const float *sens, int64_t n, uint64_t *q, uint32_t *bad, hipStream_t st) {
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sens, n, q, bad);
}

// Philox4x32-10 (Salmon et al., SC 2011): ten rounds of two 32x32->64
// multiplications with the round keys bumped by the golden-ratio and
// sqrt(3)-1 Weyl increments.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__global__ void k_draws(const uint64_t *__restrict__ C, int64_t n, int64_t m, uint64_t seed,
                        uint32_t *__restrict__ counts) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    uint32_t c[4] = {(uint32_t)t, (uint32_t)((uint64_t)t >> 32), 0u, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t Q = C[n - 1];
    const uint64_t u_lo = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
    const uint64_t u_hi = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
    // floor(u Q / 2^128) = hi word of (u_hi Q + floor(u_lo Q / 2^64))
    const uint64_t lo_hi = __umul64hi(u_lo, Q);
    const uint64_t hq_lo = u_hi * Q;
    const uint64_t hq_hi = __umul64hi(u_hi, Q);
    const uint64_t sum_lo = hq_lo + lo_hi;
    const uint64_t target = hq_hi + (sum_lo < hq_lo ? 1ull : 0ull);
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (C[mid] > target) hi = mid; else lo = mid + 1;
    }
    atomicAdd(&counts[lo], 1u);
}

void launch_draws(const uint64_t *C, int64_t n, int64_t m, uint64_t seed, uint32_t *counts, hipStream_t st) {
    hipLaunchKernelGGL(k_draws, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, C, n, m, seed, counts);
}

// With q null, q_i is recomputed from the sensitivities (same value).  The
// support count is summed per block of 1024 first: device-wide atomics on one
// address serialise, and one per wave cost about 0.15 ms at n = 10^6.
constexpr int kWeightThreads = 1024;

__global__ __launch_bounds__(kWeightThreads) void k_weights(const uint32_t *__restrict__ counts,
                                                            const uint64_t *__restrict__ q,
                                                            const float *__restrict__ sens,
                                                            const uint64_t *__restrict__ C, int64_t n, int64_t m,
                                                            double *__restrict__ w, int64_t *__restrict__ support) {
    __shared__ uint32_t wsup[kWeightThreads / 64];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = i < n;
    const uint32_t c = ok ? counts[i] : 0u;
    if (ok) {
        const double Q = (double)C[n - 1];
        const double num = (double)c * Q;
        const double den = (double)m * (double)(q ? q[i] : quantum(sens[i]));
        w[i] = c ? num / den : 0.0;
    }
    const uint64_t bal = __ballot(c > 0u);
    if ((threadIdx.x & 63) == 0) wsup[threadIdx.x >> 6] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kWeightThreads / 64; ++k) t += wsup[k];
        if (t) atomicAdd((unsigned long long *)support, (unsigned long long)t);
    }
}

void launch_weights(const uint32_t *counts, const uint64_t *q, const float *sens, const uint64_t *C, int64_t n,
                    int64_t m, double *weights, int64_t *support, hipStream_t st) {
    hipLaunchKernelGGL(k_weights, dim3((unsigned)((n + kWeightThreads - 1) / kWeightThreads)), dim3(kWeightThreads),
                       0, st, counts, q, sens, C, n, m, weights, support);
}

}  // namespace gs
