// Learned sampling proposal: an MLP 64 -> 256 -> 256 -> 256 -> 1 with SiLU
// that predicts log-sensitivity from per-Gaussian features.  The products run
// on the BF16 matrix cores of gfx950 (v_mfma_f32_16x16x32_bf16, FP32
// accumulation); activations are kept in BF16 between layers and in FP32
// (pre-activation) for the backward pass; parameters and Adam moments are
// FP32.
//
// Parameter vector (FP32, PyTorch Linear layout [out][in]):
//   W1[256][64] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] w4[256] b4
#include "gs_internal.hpp"

#include <math.h>

#include <cmath>

#include <algorithm>

namespace gs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// SiLU and its derivative with the hardware reciprocal (v_rcp_f32, 1 ulp)
// instead of an IEEE division: the same form in training and inference.
__device__ __forceinline__ float sigmoid_fast(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoid_fast(z); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = sigmoid_fast(z);
    return s * (1.0f + z * (1.0f - s));
}

// C[M][N] = A[M][K] * B[N][K]^T (row-major bf16, K contiguous), FP32 accumulate.
// Block = 4 waves computing a 64x64 tile (each wave 32x32 = 2x2 MFMA tiles of
// 16x16, K in steps of 32).  Fragment layout of v_mfma_f32_16x16x32_bf16:
// lane l holds row (l % 16) of A and column (l % 16) of B^T for the 8
// consecutive k at 8 (l / 16); the 16x16 result gives lane l the 4 rows
// 4 (l / 16) + r of column l % 16.
// Epilogues: 0 = store FP32 C; 1 = Z = C + bias -> store Z (FP32) and
// SiLU(Z) (BF16); 2 = store only SiLU(C + bias) (BF16).
// Requires M, N multiples of 64 and K a multiple of 32 (checked by the host).
// Element type of the training path: BF16 on the matrix cores (training),
// or FP32 through the same kernels (v_mfma_f32_16x16x4_f32; a precision mode
// for gradient checks).  Fragment loads are 8 consecutive k per lane either
// way.
template <typename T>
struct Frag8;
template <>
struct Frag8<__bf16> {
    bf16x8 v;
    __device__ __forceinline__ void load(const __bf16 *p) { v = *reinterpret_cast<const bf16x8 *>(p); }
};
template <>
struct Frag8<float> {
    float4 lo, hi;
    __device__ __forceinline__ void load(const float *p) {
        lo = *reinterpret_cast<const float4 *>(p);
        hi = *reinterpret_cast<const float4 *>(p + 4);
    }
};

// acc += A-fragment x B-fragment over one k step of 32.  BF16: one
// v_mfma_f32_16x16x32_bf16.  FP32: v_mfma_f32_16x16x4_f32 sums over the four
// 16-lane groups, so call e of 8 multiplies the k = 8 g + e of every group g:
// together the eight cover the same 32 k.
__device__ __forceinline__ void mma32(const Frag8<__bf16> &a, const Frag8<__bf16> &b, f32x4 &acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc, 0, 0, 0);
}
__device__ __forceinline__ void mma32(const Frag8<float> &a, const Frag8<float> &b, f32x4 &acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo.x, b.lo.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo.y, b.lo.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo.z, b.lo.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo.w, b.lo.w, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi.x, b.hi.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi.y, b.hi.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi.z, b.hi.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi.w, b.hi.w, acc, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ T to_elem(float x) { return static_cast<T>(x); }

// C[M][N] = A[M][K] * B[N][K]^T (row-major, K contiguous), FP32 accumulate.
// Block = 4 waves computing a 64x64 tile (each wave 32x32 = 2x2 MFMA tiles of
// 16x16, K in steps of 32).  Fragment layout of the 16x16 MFMAs: lane l
// holds row (l % 16) of A and column (l % 16) of B^T for the 8 consecutive k
// at 8 (l / 16); the 16x16 result gives lane l the 4 rows 4 (l / 16) + r of
// column l % 16.
// Split K: block z multiplies k in [z kchunk, min(K, (z + 1) kchunk)) and
// stores its partial product at C + z czstride (epilogue 0 only).
// Epilogues: 0 = store FP32 C; 1 = Z = C + bias -> store Z (FP32) and
// SiLU(Z) (T); 2 = store only SiLU(C + bias) (T).
// Requires M, N multiples of 64 and K, kchunk multiples of 32 (checked by the host).
template <int kEpi, typename T>
__global__ __launch_bounds__(256) void k_gemm_nt(const T *__restrict__ A, int lda, const T *__restrict__ B, int ldb,
                                                 int K, int kchunk, float *__restrict__ C, int ldc, int64_t czstride,
                                                 const float *__restrict__ bias, T *__restrict__ H, int ldh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row0 = blockIdx.x * 64 + (w & 1) * 32;
    const int col0 = blockIdx.y * 64 + (w >> 1) * 32;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    C += (int64_t)blockIdx.z * czstride;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const T *a0 = A + (int64_t)(row0 + fr) * lda + fk;
    const T *a1 = A + (int64_t)(row0 + 16 + fr) * lda + fk;
    const T *b0 = B + (int64_t)(col0 + fr) * ldb + fk;
    const T *b1 = B + (int64_t)(col0 + 16 + fr) * ldb + fk;
    for (int k0 = kb; k0 < ke; k0 += 32) {
        Frag8<T> fa0, fa1, fb0, fb1;
        fa0.load(a0 + k0);
        fa1.load(a1 + k0);
        fb0.load(b0 + k0);
        fb1.load(b1 + k0);
        mma32(fa0, fb0, acc[0][0]);
        mma32(fa0, fb1, acc[0][1]);
        mma32(fa1, fb0, acc[1][0]);
        mma32(fa1, fb1, acc[1][1]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + i * 16 + (lane >> 4) * 4 + r;
                const int col = col0 + j * 16 + fr;
                float v = acc[i][j][r];
                if (kEpi == 0) {
                    C[(int64_t)row * ldc + col] = v;
                } else {
                    v += bias[col];
                    if (kEpi == 1) C[(int64_t)row * ldc + col] = v;
                    H[(int64_t)row * ldh + col] = to_elem<T>(silu(v));
                }
            }
}

template <typename T>
static void gemm_nt(int epi, const T *A, int lda, const T *B, int ldb, int M, int N, int K, float *C, int ldc,
                    const float *bias, T *H, int ldh, hipStream_t st) {
    dim3 grid(M / 64, N / 64);
    if (epi == 0)
        hipLaunchKernelGGL((k_gemm_nt<0, T>), grid, dim3(256), 0, st, A, lda, B, ldb, K, K, C, ldc, (int64_t)0, bias,
                           H, ldh);
    else if (epi == 1)
        hipLaunchKernelGGL((k_gemm_nt<1, T>), grid, dim3(256), 0, st, A, lda, B, ldb, K, K, C, ldc, (int64_t)0, bias,
                           H, ldh);
    else
        hipLaunchKernelGGL((k_gemm_nt<2, T>), grid, dim3(256), 0, st, A, lda, B, ldb, K, K, C, ldc, (int64_t)0, bias,
                           H, ldh);
}

// Weight gradients are M x N = 256 x {256, 64} products over K = the batch
// rows: a 4 x 4 (or 4 x 1) grid of tiles would leave most of the 256 CUs
// idle, so K is split into up to kMaxSplits ranges of at least 512 rows, each
// tile of each range is one block, and a second kernel sums the partial
// products in range order (fixed, so the result is deterministic).
constexpr int kMaxSplits = 32;
static int split_count(int64_t K) { return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxSplits, K / 512)); }

__global__ void k_sum_splits(const float *__restrict__ part, int splits, int64_t count, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = part[i];
    for (int z = 1; z < splits; ++z) s += part[(int64_t)z * count + i];
    out[i] = s;
}

template <typename T>
static void gemm_nt_splitk(const T *A, int lda, const T *B, int ldb, int M, int N, int K, float *part, float *C,
                           hipStream_t st) {
    const int S = split_count(K);
    const int kchunk = (int)(((int64_t)K + S - 1) / S + 31) / 32 * 32;
    const int used = (K + kchunk - 1) / kchunk;
    dim3 grid(M / 64, N / 64, used);
    hipLaunchKernelGGL((k_gemm_nt<0, T>), grid, dim3(256), 0, st, A, lda, B, ldb, K, kchunk, part, N,
                       (int64_t)M * N, (const float *)nullptr, (T *)nullptr, 0);
    const int64_t count = (int64_t)M * N;
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, part, used, count, C);
}

// ---------------------------------------------------------------------------
// Elementwise and small kernels.

// X0[r][c] = T((feat[r][c] - mean[c]) * inv_std[c]); rows >= n are zero.
template <typename T>
__global__ void k_standardize(const float *__restrict__ feat, const float *__restrict__ norm, int64_t n,
                              int64_t rows, T *__restrict__ X0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * kMlpIn) return;
    const int64_t r = i / kMlpIn;
    const int c = (int)(i % kMlpIn);
    const float v = r < n ? (feat[i] - norm[c]) * norm[kMlpIn + c] : 0.0f;
    X0[i] = to_elem<T>(v);
}

// T copies of the weights: Wk[out][in] and their transposes Wk^T[in][out].
template <typename T>
__global__ void k_weights_cast(const float *__restrict__ P, T *__restrict__ W1, T *__restrict__ W2,
                               T *__restrict__ W3, T *__restrict__ W2t, T *__restrict__ W3t, T *__restrict__ W1t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMlpH * kMlpIn) {
        const int o = i / kMlpIn, c = i % kMlpIn;
        const T v = to_elem<T>(P[kOffW1 + i]);
        W1[i] = v;
        W1t[c * kMlpH + o] = v;
    }
    if (i < kMlpH * kMlpH) {
        const int o = i / kMlpH, c = i % kMlpH;
        const T v2 = to_elem<T>(P[kOffW2 + i]), v3 = to_elem<T>(P[kOffW3 + i]);
        W2[i] = v2;
        W3[i] = v3;
        W2t[c * kMlpH + o] = v2;
        W3t[c * kMlpH + o] = v3;
    }
}

// y[r] = H3[r] . w4 + b4 (w4 rounded to T like the other weights), one wave per row.
template <typename T>
__global__ __launch_bounds__(256) void k_head(const T *__restrict__ H3, const float *__restrict__ P, int64_t n,
                                              float *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < kMlpH / 64; ++k) {
        const int c = k * 64 + lane;
        acc += (float)H3[r * kMlpH + c] * (float)to_elem<T>(P[kOffW4 + c]);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) y[r] = acc + P[kOffB4];
}

// Loss and head backward.  dy = 2 (yhat - y) / n; per row r < n:
//   dZ3[r][c] = dy w4[c] silu'(Z3[r][c])  (T, also transposed into dZ3t).
// Block b (64 rows) writes its sums over those rows to part[b][0..257]:
// grad(w4)[c] (c < 256), grad(b4) (256) and the loss (257); k_head_sums adds
// the blocks in order (no float atomics: the result is deterministic).
constexpr int kHeadCols = kMlpH + 2;
template <typename T>
__global__ __launch_bounds__(256) void k_head_backward(const float *__restrict__ yhat, const float *__restrict__ y,
                                                       int64_t n, int64_t rows, const float *__restrict__ Z3,
                                                       const T *__restrict__ H3, const float *__restrict__ P,
                                                       T *__restrict__ dZ3, T *__restrict__ dZ3t,
                                                       float *__restrict__ part) {
    // one block per 64 rows; thread c handles column c of those rows
    const int c = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const float w4 = (float)to_elem<T>(P[kOffW4 + c]);
    float gw = 0.0f, gb = 0.0f, ls = 0.0f;
    for (int k = 0; k < 64; ++k) {
        const int64_t r = r0 + k;
        float dz = 0.0f;
        if (r < n) {
            const float e = yhat[r] - y[r];
            const float dy = 2.0f * e / (float)n;
            dz = dy * w4 * silu_grad(Z3[r * kMlpH + c]);
            gw += dy * (float)H3[r * kMlpH + c];
            if (c == 0) {
                gb += dy;
                ls += e * e / (float)n;
            }
        }
        const T b = to_elem<T>(dz);
        dZ3[r * kMlpH + c] = b;
        dZ3t[(int64_t)c * rows + r] = b;
    }
    float *out = part + (int64_t)blockIdx.x * kHeadCols;
    out[c] = gw;
    if (c == 0) {
        out[kMlpH] = gb;
        out[kMlpH + 1] = ls;
    }
}

// G[kOffW4 + c] (c <= 256: w4 then b4) and the loss from the per-block
// partials, summed over blocks in order.
// 64 columns per block; the four waves sum the blocks b = q, q + 4, ... in
// order (eight loads in flight), and their sums are added in wave order.
__global__ __launch_bounds__(256) void k_head_sums(const float *__restrict__ part, int nblocks,
                                                   float *__restrict__ G, float *__restrict__ loss) {
    __shared__ float sh[4][64];
    const int l = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + l;
    float s = 0.0f;
    if (c < kHeadCols) {
        int b = q;
        for (; b + 28 < nblocks; b += 32) {
            float x[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = part[(int64_t)(b + 4 * k) * kHeadCols + c];
#pragma unroll
            for (int k = 0; k < 8; ++k) s += x[k];
        }
        for (; b < nblocks; b += 4) s += part[(int64_t)b * kHeadCols + c];
    }
    sh[q][l] = s;
    __syncthreads();
    if (q == 0 && c < kHeadCols) {
        const float t = ((sh[0][l] + sh[1][l]) + sh[2][l]) + sh[3][l];
        if (c < kMlpH + 1)
            G[kOffW4 + c] = t;
        else
            *loss = t;
    }
}

// dZ = dH * silu'(Z) for a hidden layer; writes T dZ and its transpose.
template <typename T>
__global__ void k_act_backward(const float *__restrict__ dH, const float *__restrict__ Z, int64_t n, int64_t rows,
                               T *__restrict__ dZ, T *__restrict__ dZt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * kMlpH) return;
    const int64_t r = i / kMlpH;
    const int c = (int)(i % kMlpH);
    const float v = r < n ? dH[i] * silu_grad(Z[i]) : 0.0f;
    const T b = to_elem<T>(v);
    dZ[i] = b;
    dZt[(int64_t)c * rows + r] = b;
}

// out[c][r] = in[r][c] for a rows x cols matrix.
template <typename T>
__global__ void k_transpose(const T *__restrict__ in, int64_t rows, int cols, T *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    const int64_t r = i / cols;
    const int c = (int)(i % cols);
    out[(int64_t)c * rows + r] = in[i];
}

// grad(b)[c] = sum_r dZt[c][r]: one block per output c, fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_bias_grad(const T *__restrict__ dZt, int64_t rows, float *__restrict__ g) {
    __shared__ float sh[256];
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int64_t r = threadIdx.x; r < rows; r += 256) s += (float)dZt[(int64_t)c * rows + r];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) g[c] = sh[0];
}

// Adam (Kingma & Ba) with bias correction; m and v follow P in `adam`.
// omb1 = 1 - beta1 and omb2 = 1 - beta2 come from the host rounded once from
// double (1.0f - 0.999f in float32 would be 5e-5 off 0.001).
__global__ void k_adam(float *__restrict__ P, float *__restrict__ adam, const float *__restrict__ G, int64_t n,
                       float lr, float b1, float b2, float omb1, float omb2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float m = b1 * adam[i] + omb1 * g;
    const float v = b2 * adam[n + i] + omb2 * (g * g);
    adam[i] = m;
    adam[n + i] = v;
    P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Deterministic initialisation: uniform(-a, a) with a = sqrt(6 / (fan_in + fan_out))
// for weights (24 bits of a 64-bit finaliser of seed and parameter index:
// MurmurHash3's fmix64), zero biases.
__device__ __forceinline__ uint32_t mix32(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return (uint32_t)x;
}
__global__ void k_mlp_init(float *__restrict__ P, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpParams) return;
    float fan_in = 0, fan_out = 0;
    bool weight = true;
    if (i < kOffB1) { fan_in = kMlpIn; fan_out = kMlpH; }
    else if (i < kOffW2) weight = false;
    else if (i < kOffB2) { fan_in = kMlpH; fan_out = kMlpH; }
    else if (i < kOffW3) weight = false;
    else if (i < kOffB3) { fan_in = kMlpH; fan_out = kMlpH; }
    else if (i < kOffW4) weight = false;
    else if (i < kOffB4) { fan_in = kMlpH; fan_out = 1; }
    else weight = false;
    if (!weight) {
        P[i] = 0.0f;
        return;
    }
    const float a = sqrtf(6.0f / (fan_in + fan_out));
    const float u = (float)(mix32(seed * 0x9E3779B97F4A7C15ull + (uint64_t)i) >> 8) * (1.0f / 16777216.0f);
    P[i] = (2.0f * u - 1.0f) * a;
}

// ---------------------------------------------------------------------------
// Training scratch for `rows` rows with elements of `esz` bytes (2: BF16,
// 4: FP32); the largest of the two is what the host reserves.
static size_t mlp_scratch_bytes_e(int64_t rows, size_t esz) {
    const size_t h = (size_t)rows * kMlpH;
    size_t b = 0;
    b += (2 * (size_t)kMlpH * kMlpIn + 4 * (size_t)kMlpH * kMlpH) * esz;   // weights and transposes
    b += (size_t)rows * kMlpIn * 2 * esz;                                  // X0, X0t
    b += 3 * h * 4;                                                        // Z1..Z3
    b += 4 * h * esz;                                                      // H1..H3, transposed H
    b += (size_t)rows * 4;                                                 // yhat
    b += 2 * h * esz + h * 4;                                              // dZ, dZt, dH
    b += (size_t)kMlpParams * 4;                                           // gradient buffer
    b += (size_t)kMaxSplits * kMlpH * kMlpH * 4;                           // split-K partial products
    b += (size_t)(rows / 64 + 1) * kHeadCols * 4;                          // head partials per block
    return b + 64 * 256;
}
size_t mlp_scratch_bytes(int64_t rows) { return mlp_scratch_bytes_e(rows, 4); }

template <typename T>
struct MlpBufs {
    T *W1, *W1t, *W2, *W3, *W2t, *W3t, *X0, *X0t, *H1, *H2, *H3, *Ht, *dZ, *dZt;
    float *Z1, *Z2, *Z3, *yhat, *dH, *G, *Gpart, *Hpart;
};

template <typename T>
static MlpBufs<T> carve_mlp(void *base, int64_t rows) {
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        void *r = p + off;
        off += bytes;
        return r;
    };
    const size_t h = (size_t)rows * kMlpH;
    const size_t e = sizeof(T);
    MlpBufs<T> m;
    m.W1 = (T *)take((size_t)kMlpH * kMlpIn * e);
    m.W1t = (T *)take((size_t)kMlpH * kMlpIn * e);
    m.W2 = (T *)take((size_t)kMlpH * kMlpH * e);
    m.W3 = (T *)take((size_t)kMlpH * kMlpH * e);
    m.W2t = (T *)take((size_t)kMlpH * kMlpH * e);
    m.W3t = (T *)take((size_t)kMlpH * kMlpH * e);
    m.X0 = (T *)take((size_t)rows * kMlpIn * e);
    m.X0t = (T *)take((size_t)rows * kMlpIn * e);
    m.Z1 = (float *)take(h * 4);
    m.Z2 = (float *)take(h * 4);
    m.Z3 = (float *)take(h * 4);
    m.H1 = (T *)take(h * e);
    m.H2 = (T *)take(h * e);
    m.H3 = (T *)take(h * e);
    m.Ht = (T *)take(h * e);
    m.yhat = (float *)take((size_t)rows * 4);
    m.dZ = (T *)take(h * e);
    m.dZt = (T *)take(h * e);
    m.dH = (float *)take(h * 4);
    m.G = (float *)take((size_t)kMlpParams * 4);
    m.Gpart = (float *)take((size_t)kMaxSplits * kMlpH * kMlpH * 4);
    m.Hpart = (float *)take((size_t)(rows / 64 + 1) * kHeadCols * 4);
    return m;
}

static inline unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

template <typename T>
static void mlp_forward_rows(const float *P, const MlpBufs<T> &m, int64_t rows, hipStream_t st) {
    const int H = kMlpH;
    gemm_nt<T>(1, m.X0, kMlpIn, m.W1, kMlpIn, rows, H, kMlpIn, m.Z1, H, P + kOffB1, m.H1, H, st);
    gemm_nt<T>(1, m.H1, H, m.W2, H, rows, H, H, m.Z2, H, P + kOffB2, m.H2, H, st);
    gemm_nt<T>(1, m.H2, H, m.W3, H, rows, H, H, m.Z3, H, P + kOffB3, m.H3, H, st);
}

// Fused inference: one block of 4 waves per 128 rows runs the whole network
// with the activations in LDS and the bf16 weights read straight from global
// memory (L2): wave w computes output columns [64 w, 64 w + 64) of every
// layer for the block's 128 rows, with the k order of k_gemm_nt.
// One row-major bf16 buffer (padded row stride, so the 16 rows a fragment
// load reads fall on different banks) holds the input, then each layer's
// output in place: a layer's products are finished in registers, the block
// meets at a barrier, and only then are they written over its input.  128
// rows per block halve the weight reads from L2 against 64 (each block reads
// all 295 KB of bf16 weights once); the 68 KiB of LDS per block leaves room
// for two blocks per CU.  The head sums bf16(SiLU(z3)) w4 over each wave's
// columns (DPP over the 16 lanes of a fragment row), then over the waves.
constexpr int kFuseTiles = 8;                 // 16-row fragment tiles per block
constexpr int kFuseRows = 16 * kFuseTiles;
constexpr int kFusePitch = kMlpH + 8;   // bf16 per LDS row

// The products are taken transposed (the weights as the first MFMA operand,
// the activations as the second): lane l of a 16x16 output tile then holds
// four consecutive output columns 4 (l / 16) .. + 3 of row l % 16, which go to
// LDS as one 8-byte store and are the layout the next layer reads.
template <int kK>
__device__ __forceinline__ void fused_layer(const __bf16 (*In)[kFusePitch], const __bf16 *__restrict__ W,
                                            const float *__restrict__ bias, int w, int lane,
                                            f32x4 (&acc)[kFuseTiles][4]) {
    const int fr = lane & 15, fk = (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < kFuseTiles; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the next k step's weight fragments are loaded while this one multiplies
    bf16x8 b[4], bn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(W + (int64_t)(64 * w + 16 * j + fr) * kK + fk);
    for (int k0 = 0; k0 < kK; k0 += 32) {
        if (k0 + 32 < kK) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bn[j] = *reinterpret_cast<const bf16x8 *>(W + (int64_t)(64 * w + 16 * j + fr) * kK + k0 + 32 + fk);
        }
#pragma unroll
        for (int i = 0; i < kFuseTiles; ++i) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&In[16 * i + fr][k0 + fk]);
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a, acc[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = bn[j];
    }
    const int g4 = (lane >> 4) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float bj[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) bj[r] = bias[64 * w + 16 * j + g4 + r];
#pragma unroll
        for (int i = 0; i < kFuseTiles; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = silu(acc[i][j][r] + bj[r]);
    }
}

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void fused_store(__bf16 (*Out)[kFusePitch], int w, int lane,
                                            const f32x4 (&acc)[kFuseTiles][4]) {
    const int fr = lane & 15, g4 = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < kFuseTiles; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bf16x4 v = {(__bf16)acc[i][j][0], (__bf16)acc[i][j][1], (__bf16)acc[i][j][2], (__bf16)acc[i][j][3]};
            *reinterpret_cast<bf16x4 *>(&Out[16 * i + fr][64 * w + 16 * j + g4]) = v;
        }
}

__global__ __launch_bounds__(256, 2) void k_mlp_fused(const float *__restrict__ feat, const float *__restrict__ norm,
                                                   int64_t n, const __bf16 *__restrict__ W1,
                                                   const __bf16 *__restrict__ W2, const __bf16 *__restrict__ W3,
                                                   const float *__restrict__ P, float *__restrict__ y) {
    __shared__ __attribute__((aligned(16))) __bf16 H[kFuseRows][kFusePitch];
    __shared__ float ypart[4][kFuseRows];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kFuseRows;
    // standardised inputs, rows past n are zero (as k_standardize)
    for (int i = threadIdx.x; i < kFuseRows * kMlpIn; i += 256) {
        const int r = i / kMlpIn, c = i % kMlpIn;
        const int64_t row = r0 + r;
        const float x = row < n ? (feat[row * kMlpIn + c] - norm[c]) * norm[kMlpIn + c] : 0.0f;
        H[r][c] = (__bf16)x;
    }
    __syncthreads();
    f32x4 acc[kFuseTiles][4];
    fused_layer<kMlpIn>(H, W1, P + kOffB1, w, lane, acc);
    __syncthreads();            // every wave has read the inputs
    fused_store(H, w, lane, acc);
    __syncthreads();
    fused_layer<kMlpH>(H, W2, P + kOffB2, w, lane, acc);
    __syncthreads();
    fused_store(H, w, lane, acc);
    __syncthreads();
    fused_layer<kMlpH>(H, W3, P + kOffB3, w, lane, acc);
    // head: this wave's columns of each row (lane l holds columns
    // 16 j + 4 (l / 16) .. + 3 of row l % 16), then over the four lanes of the row
    const int fr = lane & 15, g4 = (lane >> 4) * 4;
    float w4[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) w4[j][r] = (float)(__bf16)P[kOffW4 + 64 * w + 16 * j + g4 + r];
#pragma unroll
    for (int i = 0; i < kFuseTiles; ++i) {
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) s += (float)(__bf16)acc[i][j][r] * w4[j][r];
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        if (lane < 16) ypart[w][16 * i + fr] = s;
    }
    __syncthreads();
    if (threadIdx.x < kFuseRows && r0 + threadIdx.x < n) {
        const int t = threadIdx.x;
        y[r0 + t] = ((ypart[0][t] + ypart[1][t]) + (ypart[2][t] + ypart[3][t])) + P[kOffB4];
    }
}

void mlp_init(float *params, uint64_t seed, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_init, dim3(blocks_for(kMlpParams)), dim3(256), 0, st, params, seed);
}

// Predictions for n rows of raw features: the bf16 weights, then one fused
// launch over every row (the scratch holds only the weights).
void mlp_forward(const float *P, const float *feat, const float *norm, int64_t n, float *y, void *scratch,
                 int64_t rows, hipStream_t st) {
    const MlpBufs<__bf16> m = carve_mlp<__bf16>(scratch, rows);
    hipLaunchKernelGGL(k_weights_cast<__bf16>, dim3(blocks_for(kMlpH * kMlpH)), dim3(256), 0, st, P, m.W1, m.W2, m.W3,
                       m.W2t, m.W3t, m.W1t);
    hipLaunchKernelGGL(k_mlp_fused, dim3((unsigned)((n + kFuseRows - 1) / kFuseRows)), dim3(256), 0, st, feat, norm, n,
                       m.W1, m.W2, m.W3, P, y);
}

// Loss and gradient on one batch of n <= rows rows with elements T; if
// adam != nullptr also applies one Adam step (step >= 1).  grad_out
// (optional) receives the gradient.  Every sum has a fixed order, so two
// calls on the same inputs give the same bits.
template <typename T>
static void train_step_t(float *P, float *adam, int64_t step, float lr, const float *feat, const float *norm,
                         const float *y, int64_t n, float *loss, float *grad_out, void *scratch, int64_t rows,
                         hipStream_t st) {
    const MlpBufs<T> m = carve_mlp<T>(scratch, rows);
    const int H = kMlpH;
    const int64_t R = (n + 63) / 64 * 64;
    hipLaunchKernelGGL(k_weights_cast<T>, dim3(blocks_for(kMlpH * kMlpH)), dim3(256), 0, st, P, m.W1, m.W2, m.W3,
                       m.W2t, m.W3t, m.W1t);
    hipLaunchKernelGGL(k_standardize<T>, dim3(blocks_for(R * kMlpIn)), dim3(256), 0, st, feat, norm, n, R, m.X0);
    mlp_forward_rows<T>(P, m, R, st);
    hipLaunchKernelGGL(k_head<T>, dim3((unsigned)((R + 3) / 4)), dim3(256), 0, st, m.H3, P, R, m.yhat);
    hipLaunchKernelGGL(k_head_backward<T>, dim3((unsigned)(R / 64)), dim3(256), 0, st, m.yhat, y, n, R, m.Z3, m.H3, P,
                       m.dZ, m.dZt, m.Hpart);
    hipLaunchKernelGGL(k_head_sums, dim3((kHeadCols + 63) / 64), dim3(256), 0, st, m.Hpart, (int)(R / 64), m.G, loss);
    // layer 3: grad W3 = dZ3^T H2, grad b3, dH2 = dZ3 W3
    hipLaunchKernelGGL(k_transpose<T>, dim3(blocks_for(R * H)), dim3(256), 0, st, m.H2, R, H, m.Ht);
    gemm_nt_splitk<T>(m.dZt, (int)R, m.Ht, (int)R, H, H, (int)R, m.Gpart, m.G + kOffW3, st);
    hipLaunchKernelGGL(k_bias_grad<T>, dim3(H), dim3(256), 0, st, m.dZt, R, m.G + kOffB3);
    gemm_nt<T>(0, m.dZ, H, m.W3t, H, R, H, H, m.dH, H, nullptr, nullptr, 0, st);
    hipLaunchKernelGGL(k_act_backward<T>, dim3(blocks_for(R * H)), dim3(256), 0, st, m.dH, m.Z2, n, R, m.dZ, m.dZt);
    // layer 2
    hipLaunchKernelGGL(k_transpose<T>, dim3(blocks_for(R * H)), dim3(256), 0, st, m.H1, R, H, m.Ht);
    gemm_nt_splitk<T>(m.dZt, (int)R, m.Ht, (int)R, H, H, (int)R, m.Gpart, m.G + kOffW2, st);
    hipLaunchKernelGGL(k_bias_grad<T>, dim3(H), dim3(256), 0, st, m.dZt, R, m.G + kOffB2);
    gemm_nt<T>(0, m.dZ, H, m.W2t, H, R, H, H, m.dH, H, nullptr, nullptr, 0, st);
    hipLaunchKernelGGL(k_act_backward<T>, dim3(blocks_for(R * H)), dim3(256), 0, st, m.dH, m.Z1, n, R, m.dZ, m.dZt);
    // layer 1: grad W1 = dZ1^T X0
    hipLaunchKernelGGL(k_transpose<T>, dim3(blocks_for(R * kMlpIn)), dim3(256), 0, st, m.X0, R, kMlpIn, m.X0t);
    gemm_nt_splitk<T>(m.dZt, (int)R, m.X0t, (int)R, H, kMlpIn, (int)R, m.Gpart, m.G + kOffW1, st);
    hipLaunchKernelGGL(k_bias_grad<T>, dim3(H), dim3(256), 0, st, m.dZt, R, m.G + kOffB1);
    if (grad_out) hipMemcpyAsync(grad_out, m.G, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, st);
    if (adam) {
        const double b1 = 0.9, b2 = 0.999;
        const float c1 = (float)(1.0 - std::pow(b1, (double)step)), c2 = (float)(1.0 - std::pow(b2, (double)step));
        hipLaunchKernelGGL(k_adam, dim3(blocks_for(kMlpParams)), dim3(256), 0, st, P, adam, m.G, (int64_t)kMlpParams,
                           lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2);
    }
}

void mlp_train_step(float *P, float *adam, int64_t step, float lr, const float *feat, const float *norm,
                    const float *y, int64_t n, float *loss, float *grad_out, void *scratch, int64_t rows,
                    hipStream_t st, bool fp32) {
    if (fp32)
        train_step_t<float>(P, adam, step, lr, feat, norm, y, n, loss, grad_out, scratch, rows, st);
    else
        train_step_t<__bf16>(P, adam, step, lr, feat, norm, y, n, loss, grad_out, scratch, rows, st);
}

}  // namespace gs

namespace gs {

// ---------------------------------------------------------------------------
// Proposal mixture and training targets.
//
// p_i = (1 - f) e_i / sum_j e_j + f / n with e_i = exp(y_i - max_j y_j): the
// network's predicted ln s normalised into a distribution and mixed with a
// uniform floor f, so every Gaussian keeps p_i >= f / n (sensitivity sampling
// stays unbiased for any such proposal, proof of Theorem 2).  The maximum is
// an order-free integer atomic on ordered float bits and the sum is a
// fixed-order FP64 reduction, so the result is deterministic.

__device__ __forceinline__ uint32_t ordered_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_ordered(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

__global__ __launch_bounds__(256) void k_max_ordered(const float *__restrict__ y, int64_t n,
                                                     uint32_t *__restrict__ out) {
    uint32_t m = 0u;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = max(m, ordered_bits(y[i]));
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

__global__ __launch_bounds__(256) void k_exp_shift(const float *__restrict__ y, int64_t n,
                                                   const uint32_t *__restrict__ ymax, float *__restrict__ e) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) e[i] = (float)exp((double)y[i] - (double)from_ordered(*ymax));
}

__global__ __launch_bounds__(256) void k_mix(float *__restrict__ p, int64_t n, const double *__restrict__ esum,
                                             float floor) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = (float)((1.0 - (double)floor) * (double)p[i] / *esum + (double)floor / (double)n);
}

// ln(max(s, floor)): regression targets from exact sensitivities.
__global__ __launch_bounds__(256) void k_log_floor(const float *__restrict__ s, int64_t n, float floor,
                                                   float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (float)log((double)fmaxf(s[i], floor));
}

size_t mixture_scratch_bytes(int64_t n) { return sizeof(double) * ((size_t)(n + 4095) / 4096 + 2) + 256; }

void proposal_mixture(const float *y, int64_t n, float floor, float *p, void *scratch, hipStream_t st) {
    uint32_t *ymax = (uint32_t *)scratch;
    double *esum = (double *)((char *)scratch + 64);
    double *tmp = esum + 1;
    launch_fill_u32(ymax, 0u, 1, st);
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_max_ordered, dim3(blocks), dim3(256), 0, st, y, n, ymax);
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_exp_shift, dim3(g), dim3(256), 0, st, y, n, ymax, p);
    launch_sum_f32_to_f64(p, n, esum, tmp, st);
    hipLaunchKernelGGL(k_mix, dim3(g), dim3(256), 0, st, p, n, esum, floor);
}

void log_targets(const float *s, int64_t n, float floor, float *out, hipStream_t st) {
    hipLaunchKernelGGL(k_log_floor, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, n, floor, out);
}

}  // namespace gs
