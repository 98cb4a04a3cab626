// Per-Gaussian features of the learned proposal: 59 attributes plus five
// features of the k = 16 nearest neighbours of each mean (exact kNN on a
// uniform grid; neighbours ordered by (squared distance, index), self
// excluded).
//
// Feature vector (64 float32 per Gaussian):
//   0-2 mean, 3-5 log-scale, 6-9 normalised quaternion with w >= 0,
//   10 logit(alpha), 11-58 SH coefficients (zero beyond the scene's degree),
//   59 log mean neighbour distance, 60 log distance to the 16th neighbour,
//   61 mean neighbour alpha, 62 max neighbour alpha,
//   63 log(sum of neighbour alphas / volume of the 16th-neighbour ball).
//
// Grid: cell edge = cube root of (bounding-box volume / n), so one point per
// cell on average; points are counting-sorted by cell.  A query visits rings
// of cells at Chebyshev distance r = 0, 1, 2, ... and stops once it holds 16
// neighbours and the 16th is closer than r cell edges (every unvisited point
// is at least that far away).
#include "gs_internal.hpp"

#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>
#include <cstring>

namespace gs {

constexpr int kK = 16;

__device__ __forceinline__ float kload(const void *base, int64_t idx, int fmt, bool half_ieee) {
    if (fmt == 0) return static_cast<const float *>(base)[idx];
    const uint16_t b = static_cast<const uint16_t *>(base)[idx];
    if (half_ieee) return __half2float(__ushort_as_half(b));
    return __uint_as_float((uint32_t)b << 16);
}

__device__ __forceinline__ uint32_t ord_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// box[0..2] = min (ordered bits), box[3..5] = max
// Bounding box of the means (order-preserving bits, so min / max are integer
// operations): a fixed grid strides over the points, each block folds its
// waves in LDS and adds one atomic per bound (atomics on one address
// serialise, so one per wave would cost about a millisecond at 10^6 points).
constexpr int kBoxBlocks = 256;
__global__ __launch_bounds__(256) void k_bbox(SceneDev sc, uint32_t *box) {
    __shared__ uint32_t red[4][6];
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < sc.n; i += (int64_t)gridDim.x * blockDim.x)
        for (int c = 0; c < 3; ++c) {
            const uint32_t b = ord_bits(kload(sc.mean, c * sc.n + i, sc.format, false));
            lo[c] = min(lo[c], b);
            hi[c] = max(hi[c], b);
        }
    for (int c = 0; c < 3; ++c)
        for (int off = 32; off > 0; off >>= 1) {
            lo[c] = min(lo[c], (uint32_t)__shfl_xor((int)lo[c], off));
            hi[c] = max(hi[c], (uint32_t)__shfl_xor((int)hi[c], off));
        }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < 3; ++c) {
            red[w][c] = lo[c];
            red[w][3 + c] = hi[c];
        }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int c = threadIdx.x;
        atomicMin(&box[c], min(min(red[0][c], red[1][c]), min(red[2][c], red[3][c])));
        atomicMax(&box[3 + c], max(max(red[0][3 + c], red[1][3 + c]), max(red[2][3 + c], red[3][3 + c])));
    }
}

struct Grid {
    float lo[3];
    float cell, inv_cell;
    int dim[3];
};

__device__ __forceinline__ int cell_coord(float x, float lo, float inv_cell, int dim) {
    int c = (int)floorf((x - lo) * inv_cell);
    return c < 0 ? 0 : (c >= dim ? dim - 1 : c);
}

__global__ void k_cell_count(SceneDev sc, Grid G, uint32_t *__restrict__ cell_of, uint32_t *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc.n) return;
    int c3[3];
    for (int c = 0; c < 3; ++c)
        c3[c] = cell_coord(kload(sc.mean, c * sc.n + i, sc.format, false), G.lo[c], G.inv_cell, G.dim[c]);
    const uint32_t id = (uint32_t)((c3[2] * G.dim[1] + c3[1]) * G.dim[0] + c3[0]);
    cell_of[i] = id;
    atomicAdd(&count[id], 1u);
}

__global__ void k_cell_scatter(int64_t n, const uint32_t *__restrict__ cell_of, const uint64_t *__restrict__ off,
                               uint32_t *__restrict__ fill, uint32_t *__restrict__ order, float4 *__restrict__ pts,
                               SceneDev sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = cell_of[i];
    const uint64_t p = off[c] + atomicAdd(&fill[c], 1u);
    order[p] = (uint32_t)i;
    const float x = kload(sc.mean, i, sc.format, false), y = kload(sc.mean, sc.n + i, sc.format, false);
    const float z = kload(sc.mean, 2 * sc.n + i, sc.format, false);
    const float a = kload(sc.opacity, i, sc.format, true);
    pts[p] = make_float4(x, y, z, a);
}

__device__ __forceinline__ bool knn_less(float da, uint32_t ia, float db, uint32_t ib) {
    return da < db || (da == db && ia < ib);
}

// kNeighbours: write the neighbour lists (indices and float32 squared
// distances, ordered by (distance, index)) instead of the features.
template <bool kNeighbours>
__global__ __launch_bounds__(256) void k_knn_features(SceneDev sc, Grid G, const uint64_t *__restrict__ off,
                                                      const uint32_t *__restrict__ order,
                                                      const float4 *__restrict__ pts, float *__restrict__ feat,
                                                      uint32_t *__restrict__ nidx, float *__restrict__ nd2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= sc.n) return;
    const uint32_t q = order[t];     // queries in cell order: neighbouring lanes share cells
    const float4 me = pts[t];
    int c3[3];
    c3[0] = cell_coord(me.x, G.lo[0], G.inv_cell, G.dim[0]);
    c3[1] = cell_coord(me.y, G.lo[1], G.inv_cell, G.dim[1]);
    c3[2] = cell_coord(me.z, G.lo[2], G.inv_cell, G.dim[2]);
    float bd[kK];
    uint32_t bi[kK];
    float ba[kK];
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        bd[k] = INFINITY;
        bi[k] = 0xFFFFFFFFu;
        ba[k] = 0.0f;
    }
    const int rmax = max(G.dim[0], max(G.dim[1], G.dim[2]));
    for (int r = 0; r <= rmax; ++r) {
        for (int dz = -r; dz <= r; ++dz) {
            const int z = c3[2] + dz;
            if (z < 0 || z >= G.dim[2]) continue;
            for (int dy = -r; dy <= r; ++dy) {
                const int y = c3[1] + dy;
                if (y < 0 || y >= G.dim[1]) continue;
                const bool face = (dz == -r || dz == r || dy == -r || dy == r);
                const int step = face ? 1 : 2 * r;
                for (int dx = -r; dx <= r; dx += (step > 0 ? step : 1)) {
                    const int x = c3[0] + dx;
                    if (x < 0 || x >= G.dim[0]) continue;
                    const uint32_t id = (uint32_t)((z * G.dim[1] + y) * G.dim[0] + x);
                    const uint64_t lo = off[id], hi = off[id + 1];
                    // candidates four at a time, their loads issued together
                    // (slots past the cell's end repeat the query and are skipped)
                    for (uint64_t p0 = lo; p0 < hi; p0 += 4) {
                        uint32_t jj[4];
                        float4 oo[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const bool ok = p0 + u < hi;
                            jj[u] = ok ? order[p0 + u] : q;
                            oo[u] = ok ? pts[p0 + u] : me;
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const uint32_t j = jj[u];
                            if (j == q) continue;
                            const float4 o = oo[u];
                            const float ex = o.x - me.x, ey = o.y - me.y, ez = o.z - me.z;
                            const float d2 = ex * ex + ey * ey + ez * ez;
                            if (!knn_less(d2, j, bd[kK - 1], bi[kK - 1])) continue;
                            bool placed = false;
#pragma unroll
                            for (int k = kK - 1; k >= 0; --k) {
                                if (placed) continue;
                                const bool move = k > 0 && knn_less(d2, j, bd[k - 1], bi[k - 1]);
                                if (move) {
                                    bd[k] = bd[k - 1];
                                    bi[k] = bi[k - 1];
                                    ba[k] = ba[k - 1];
                                } else {
                                    bd[k] = d2;
                                    bi[k] = j;
                                    ba[k] = o.w;
                                    placed = true;
                                }
                            }
                        }
                    }
                }
            }
        }
        // every point outside the searched cube of cells is at least `reach`
        // away: the distance to the cube's nearest face that has cells beyond
        // it (less a margin for the rounding of the cell assignment)
        float reach = INFINITY;
        const float pc[3] = {me.x, me.y, me.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (c3[a] - r > 0) reach = fminf(reach, pc[a] - (G.lo[a] + (float)(c3[a] - r) * G.cell));
            if (c3[a] + r < G.dim[a] - 1) reach = fminf(reach, (G.lo[a] + (float)(c3[a] + r + 1) * G.cell) - pc[a]);
        }
        reach -= 1e-4f * G.cell;
        if (bi[kK - 1] != 0xFFFFFFFFu && (reach == INFINITY || (reach > 0.0f && bd[kK - 1] < reach * reach))) break;
    }
    if (kNeighbours) {
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            nidx[(int64_t)q * kK + k] = bi[k];
            nd2[(int64_t)q * kK + k] = bd[k];
        }
        return;
    }
    // features, assembled in registers and stored as 16 float4 (one row of
    // 256 bytes per point)
    const int64_t n = sc.n;
    float f[kMlpIn];
    f[0] = kload(sc.mean, q, sc.format, false);
    f[1] = kload(sc.mean, n + q, sc.format, false);
    f[2] = kload(sc.mean, 2 * n + q, sc.format, false);
#pragma unroll
    for (int c = 0; c < 3; ++c) f[3 + c] = kload(sc.log_scale, c * n + q, sc.format, false);
    float qq[4], qn = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        qq[c] = kload(sc.quat, c * n + q, sc.format, true);
        qn += qq[c] * qq[c];
    }
    const float qs = (qq[0] < 0.0f ? -1.0f : 1.0f) * rsqrtf(fmaxf(qn, 1e-30f));
#pragma unroll
    for (int c = 0; c < 4; ++c) f[6 + c] = qq[c] * qs;
    const float al = fminf(fmaxf(me.w, 1e-6f), 1.0f - 1e-6f);
    f[10] = logf(al / (1.0f - al));
    const int K = (sc.sh_degree + 1) * (sc.sh_degree + 1);
#pragma unroll
    for (int k = 0; k < 48; ++k) f[11 + k] = k < 3 * K ? kload(sc.sh, (int64_t)k * n + q, sc.format, false) : 0.0f;
    int cnt = 0;
    float sd = 0.0f, sa = 0.0f, ma = 0.0f;
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        if (bi[k] == 0xFFFFFFFFu) continue;
        ++cnt;
        sd += sqrtf(bd[k]);
        sa += ba[k];
        ma = fmaxf(ma, ba[k]);
    }
    const float d16 = cnt ? sqrtf(bd[cnt - 1]) : 1.0f;
    const float tiny = 1e-12f;
    f[59] = logf(fmaxf(cnt ? sd / cnt : 1.0f, tiny));
    f[60] = logf(fmaxf(d16, tiny));
    f[61] = cnt ? sa / cnt : 0.0f;
    f[62] = ma;
    f[63] = logf(fmaxf(sa, tiny) / fmaxf(4.18879020f * d16 * d16 * d16, tiny));
    float4 *row = reinterpret_cast<float4 *>(feat + (int64_t)q * kMlpIn);
#pragma unroll
    for (int k = 0; k < kMlpIn / 4; ++k) row[k] = make_float4(f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]);
}

// Column means and 1/std (population) of an n x 64 float32 matrix, in FP64.
__global__ __launch_bounds__(256) void k_feature_stats(const float *__restrict__ feat, int64_t n,
                                                       float *__restrict__ norm) {
    __shared__ double s1[256], s2[256];
    const int c = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += 256) {
        const double x = feat[r * kMlpIn + c];
        a += x;
        b += x * x;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = s1[0] / (double)n;
        const double var = fmax(s2[0] / (double)n - mean * mean, 0.0);
        norm[c] = (float)mean;
        norm[kMlpIn + c] = var > 1e-20 ? (float)(1.0 / sqrt(var)) : 1.0f;
    }
}

void feature_stats(const float *feat, int64_t n, float *norm, hipStream_t st) {
    hipLaunchKernelGGL(k_feature_stats, dim3(kMlpIn), dim3(256), 0, st, feat, n, norm);
}

size_t knn_scratch_bytes(int64_t n) {
    // cells <= 8n; per point: cell id, order, point record; per cell: count, fill, offset
    const size_t cells = (size_t)8 * n + 8;
    return (size_t)n * (4 + 4 + 16) + cells * (4 + 4 + 8) + sizeof(uint64_t) * ((cells + 2047) / 2048 + 8) +
           64 * 256;
}

hipError_t knn_features(const SceneDev &sc, float *feat, void *scratch, hipStream_t st, uint32_t *nidx,
                        float *nd2) {
    const int64_t n = sc.n;
    char *p = (char *)scratch;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        o = (o + 255) & ~(size_t)255;
        void *r = p + o;
        o += bytes;
        return r;
    };
    uint32_t *box = (uint32_t *)take(64);
    uint32_t init[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
    hipError_t e = hipMemcpyAsync(box, init, sizeof init, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bbox, dim3(kBoxBlocks), dim3(256), 0, st, sc, box);
    uint32_t hb[6];
    e = hipMemcpyAsync(hb, box, sizeof hb, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    Grid G;
    float ext[3];
    double vol = 1.0;
    auto unord = [](uint32_t u) {
        const uint32_t b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
        float f;
        memcpy(&f, &b, sizeof f);
        return f;
    };
    for (int c = 0; c < 3; ++c) {
        G.lo[c] = unord(hb[c]);
        const float h = unord(hb[3 + c]);
        ext[c] = std::max(h - G.lo[c], 1e-6f);
        vol *= ext[c];
    }
    // about four points per cell of the bounding box (measured on clustered
    // scenes: one per cell scans more cells, sixteen more candidates)
    double cell = cbrt(4.0 * vol / (double)n);
    int64_t cells = 0;
    for (;;) {
        cells = 1;
        for (int c = 0; c < 3; ++c) {
            G.dim[c] = (int)std::min<double>(1024.0, std::max(1.0, std::ceil(ext[c] / cell)));
            cells *= G.dim[c];
        }
        if (cells <= 8 * n + 8) break;
        cell *= 1.25;
    }
    G.cell = (float)cell;
    G.inv_cell = (float)(1.0 / cell);
    uint32_t *cell_of = (uint32_t *)take((size_t)n * 4);
    uint32_t *order = (uint32_t *)take((size_t)n * 4);
    float4 *pts = (float4 *)take((size_t)n * 16);
    uint32_t *count = (uint32_t *)take((size_t)cells * 4);
    uint32_t *fill = (uint32_t *)take((size_t)cells * 4);
    uint64_t *offs = (uint64_t *)take((size_t)(cells + 1) * 8);
    uint64_t *tmp = (uint64_t *)take(sizeof(uint64_t) * scan_tmp_elems(cells + 1));
    launch_fill_u32(count, 0u, cells, st);
    launch_fill_u32(fill, 0u, cells, st);
    hipLaunchKernelGGL(k_cell_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sc, G, cell_of, count);
    scan_u32_to_u64_exclusive(count, offs, cells, tmp, st);
    hipLaunchKernelGGL(k_cell_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, cell_of, offs, fill,
                       order, pts, sc);
    if (nidx)
        hipLaunchKernelGGL(k_knn_features<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sc, G, offs,
                           order, pts, nullptr, nidx, nd2);
    else
        hipLaunchKernelGGL(k_knn_features<false>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sc, G, offs,
                           order, pts, feat, nullptr, nullptr);
    return hipGetLastError();
}

}  // namespace gs
