// Tile binning: per-tile front-to-back lists of Gaussians.
//
// Input: per view, the visible Gaussians in depth order (position p of the
// radix-sorted (depth key, index) sequence; ties by index because the sort is
// stable and starts from index order).  A list entry is keyed by
// (tile, p).  The lists are built by a two-level counting sort on that key:
//   1. count:   entries per (tile, chunk of 2^15 positions)  [LDS histogram]
//   2. scan:    exclusive prefix sum -> segment offsets (tile-major, chunk-minor)
//   3. scatter: each entry lands in its (tile, chunk) segment, in any order
//   4. order:   each segment is re-ordered by p with an LDS bitmap over the
//               chunk's 2^15 positions, which is a counting sort on the low
//               15 bits of p.
// The resulting entry is g | quadrant-mask << 28, where bit q says whether
// the Gaussian's pixel range touches 8x8 quadrant q of the 16x16 tile.
#include "gs_internal.hpp"

namespace gs {

constexpr int kBinThreads = 256;
constexpr int kSegBits = kChunkBits;
constexpr int kSegSize = 1 << kSegBits;          // positions per chunk
constexpr int kSegWords = kSegSize / 32;        // bitmap words (1024)

static_assert(kSegSize % kBinPositions == 0, "a binning block stays inside one chunk");

__device__ __forceinline__ void unpack_range(float f, int &lo, int &hi) {
    const uint32_t u = __float_as_uint(f);
    lo = (int)(int16_t)(u & 0xFFFFu);
    hi = (int)(int16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t quad_mask(int tx, int ty, int xl, int xh, int yl, int yh) {
    uint32_t m = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x0 = tx * kTile + (q & 1) * kQuad, y0 = ty * kTile + (q >> 1) * kQuad;
        const bool hit = xl <= x0 + kQuad - 1 && xh >= x0 && yl <= y0 + kQuad - 1 && yh >= y0;
        m |= hit ? (1u << q) : 0u;
    }
    return m;
}

template <bool kScatter>
__global__ __launch_bounds__(kBinThreads) void k_bin(const ViewDev *__restrict__ views, int64_t N, int nchunks,
                                                     const uint32_t *__restrict__ nvis,
                                                     const uint32_t *__restrict__ sorted_g,
                                                     const float4 *__restrict__ R2, uint32_t *__restrict__ bin_count,
                                                     const uint64_t *__restrict__ bin_off,
                                                     uint32_t *__restrict__ bin_fill, uint32_t *__restrict__ lists) {
    extern __shared__ uint32_t lds[];
    uint32_t *cnt = lds;                              // [tiles]
    uint32_t *base = lds + kMaxTilesPerView;          // [tiles] (scatter only)
    const int v = blockIdx.y;
    const ViewDev &V = views[v];
    const int64_t nv = nvis[v];
    const int64_t lo = (int64_t)blockIdx.x * kBinPositions;
    if (lo >= nv) return;
    const int64_t hi = min(lo + (int64_t)kBinPositions, nv);
    const int chunk = (int)(lo >> kSegBits);
    const int ntiles = V.tiles_x * V.tiles_y;
    for (int t = threadIdx.x; t < ntiles; t += kBinThreads) cnt[t] = 0;
    __syncthreads();
    for (int64_t p = lo + threadIdx.x; p < hi; p += kBinThreads) {
        const uint32_t g = sorted_g[(int64_t)v * N + p];
        const float4 r2 = R2[(int64_t)v * N + g];
        int xl, xh, yl, yh;
        unpack_range(r2.y, xl, xh);
        unpack_range(r2.z, yl, yh);
        for (int ty = yl >> 4; ty <= (yh >> 4); ++ty)
            for (int tx = xl >> 4; tx <= (xh >> 4); ++tx) atomicAdd(&cnt[ty * V.tiles_x + tx], 1u);
    }
    __syncthreads();
    if (!kScatter) {
        for (int t = threadIdx.x; t < ntiles; t += kBinThreads) {
            const uint32_t c = cnt[t];
            if (c) atomicAdd(&bin_count[(int64_t)(V.tile_base + t) * nchunks + chunk], c);
        }
        return;
    }
    for (int t = threadIdx.x; t < ntiles; t += kBinThreads) {
        const uint32_t c = cnt[t];
        base[t] = c ? atomicAdd(&bin_fill[(int64_t)(V.tile_base + t) * nchunks + chunk], c) : 0u;
        cnt[t] = 0;
    }
    __syncthreads();
    for (int64_t p = lo + threadIdx.x; p < hi; p += kBinThreads) {
        const uint32_t g = sorted_g[(int64_t)v * N + p];
        const float4 r2 = R2[(int64_t)v * N + g];
        int xl, xh, yl, yh;
        unpack_range(r2.y, xl, xh);
        unpack_range(r2.z, yl, yh);
        for (int ty = yl >> 4; ty <= (yh >> 4); ++ty)
            for (int tx = xl >> 4; tx <= (xh >> 4); ++tx) {
                const int t = ty * V.tiles_x + tx;
                const uint32_t slot = atomicAdd(&cnt[t], 1u);
                const int64_t idx = (int64_t)(V.tile_base + t) * nchunks + chunk;
                lists[bin_off[idx] + base[t] + slot] = (uint32_t)p | (quad_mask(tx, ty, xl, xh, yl, yh) << 28);
            }
    }
}

void launch_bin_count(const ViewDev *views_dev, int Vc, int64_t N, int nchunks, const ChunkBufs &b,
                      const uint32_t *sorted_g, int max_tiles_per_view, hipStream_t st) {
    (void)max_tiles_per_view;
    const int nb = (int)((N + kBinPositions - 1) / kBinPositions);
    hipLaunchKernelGGL(k_bin<false>, dim3(nb, Vc), dim3(kBinThreads), kMaxTilesPerView * sizeof(uint32_t), st,
                       views_dev, N, nchunks, b.nvis, sorted_g, b.R2, b.bin_count, b.bin_off, b.bin_fill, b.lists);
}

void launch_bin_scatter(const ViewDev *views_dev, int Vc, int64_t N, int nchunks, const ChunkBufs &b,
                        const uint32_t *sorted_g, int max_tiles_per_view, hipStream_t st) {
    (void)max_tiles_per_view;
    const int nb = (int)((N + kBinPositions - 1) / kBinPositions);
    hipLaunchKernelGGL(k_bin<true>, dim3(nb, Vc), dim3(kBinThreads), 2 * kMaxTilesPerView * sizeof(uint32_t), st,
                       views_dev, N, nchunks, b.nvis, sorted_g, b.R2, b.bin_count, b.bin_off, b.bin_fill, b.lists);
}

// 256-thread exclusive scan of one u32 per thread.
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t x, uint32_t *wsum, uint32_t *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t wb = 0;
    for (int k = 0; k < w; ++k) wb += wsum[k];
    *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return wb + incl - x;
}

// One block per tile: re-order every (tile, chunk) segment by depth position
// and convert entries to g | quadrant mask << 28.
__global__ __launch_bounds__(kBinThreads) void k_segment_sort(int nchunks, const uint64_t *__restrict__ bin_off,
                                                              uint32_t *__restrict__ lists,
                                                              const uint32_t *__restrict__ sorted_g,
                                                              const int32_t *__restrict__ tile_view, int64_t N) {
    __shared__ uint32_t bits[kSegWords];
    __shared__ uint8_t qm[kSegSize];
    __shared__ uint32_t wsum[4];
    const int gt = blockIdx.x;
    const int v = tile_view[gt];
    constexpr int kWordsPerThread = kSegWords / kBinThreads;  // 4
    for (int c = 0; c < nchunks; ++c) {
        const int64_t idx = (int64_t)gt * nchunks + c;
        const uint64_t lo = bin_off[idx], hi = bin_off[idx + 1];
        if (hi == lo) continue;  // uniform across the block
#pragma unroll
        for (int k = 0; k < kWordsPerThread; ++k) bits[threadIdx.x * kWordsPerThread + k] = 0u;
        __syncthreads();
        const uint32_t cbase = (uint32_t)c << kSegBits;
        for (uint64_t e = lo + threadIdx.x; e < hi; e += kBinThreads) {
            const uint32_t raw = lists[e];
            const uint32_t local = (raw & kIndexMask) - cbase;
            atomicOr(&bits[local >> 5], 1u << (local & 31));
            qm[local] = (uint8_t)(raw >> 28);
        }
        __syncthreads();
        uint32_t w[kWordsPerThread];
        uint32_t pc = 0;
#pragma unroll
        for (int k = 0; k < kWordsPerThread; ++k) {
            w[k] = bits[threadIdx.x * kWordsPerThread + k];
            pc += __popc(w[k]);
        }
        uint32_t total;
        uint32_t pos = block_excl_scan_256(pc, wsum, &total);
#pragma unroll
        for (int k = 0; k < kWordsPerThread; ++k) {
            uint32_t m = w[k];
            while (m) {
                const int bit = __ffs(m) - 1;
                m &= m - 1;
                const uint32_t local = (uint32_t)((threadIdx.x * kWordsPerThread + k) * 32 + bit);
                const uint32_t g = sorted_g[(int64_t)v * N + cbase + local];
                lists[lo + pos] = g | ((uint32_t)qm[local] << 28);
                ++pos;
            }
        }
        __syncthreads();
    }
}

void launch_segment_sort(int total_tiles, int nchunks, const ChunkBufs &b, const uint32_t *sorted_g,
                         const int32_t *tile_view, int64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_segment_sort, dim3(total_tiles), dim3(kBinThreads), 0, st, nchunks, b.bin_off, b.lists,
                       sorted_g, tile_view, N);
}

}  // namespace gs
