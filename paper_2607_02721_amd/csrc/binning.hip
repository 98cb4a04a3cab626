// Tile binning: per-tile front-to-back lists of Gaussians.
//
// Input: per view, the visible Gaussians in depth order (position p of the
// radix-sorted (depth key, index) sequence; ties by index because the sort is
// stable and starts from index order).  A list entry is keyed by (tile, p)
// and the lists are built by a counting sort on that key:
//   1. count:   one block per chunk of 2^11 consecutive positions counts its
//               entries per tile in LDS and stores them at (tile, chunk);
//   2. scan:    exclusive prefix sum -> segment offsets (tile-major, chunk-minor);
//   3. scatter: the same block writes its entries into its own (tile, chunk)
//               segments (any order inside a segment);
//   4. order:   one wave per tile sorts the entries of every segment by p,
//               on slices made of whole segments (a 64-lane bitonic network
//               in registers; an LDS bitonic sort for a segment of more than
//               64 entries), and converts them to g | quadrant mask << 28.
// Bit q of the mask says whether the Gaussian's pixel range touches 8x8
// quadrant q of the 16x16 tile.
#include "gs_internal.hpp"

namespace gs {

constexpr int kBinThreads = 256;
constexpr int kSegBits = kChunkBits;
constexpr int kSegSize = 1 << kSegBits;          // positions per chunk

static_assert(kSegSize == kBinPositions, "one binning block per chunk");

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
        // this block is the only writer of (tile, chunk) for every tile of the view
        for (int t = threadIdx.x; t < ntiles; t += kBinThreads)
            bin_count[(int64_t)(V.tile_base + t) * nchunks + chunk] = cnt[t];
        return;
    }
    // Start of this block's segment of each tile, relative to the view's first
    // list entry (a view holds fewer than 2^32 entries), so that the entry loop
    // below reads only LDS.
    const uint64_t vlist = bin_off[(int64_t)V.tile_base * nchunks];
    for (int t = threadIdx.x; t < ntiles; t += kBinThreads) {
        if (cnt[t]) base[t] = (uint32_t)(bin_off[(int64_t)(V.tile_base + t) * nchunks + chunk] - vlist);
        cnt[t] = 0;
    }
    __syncthreads();
    uint32_t *vl = lists + vlist;
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
                vl[base[t] + slot] = (uint32_t)p | (quad_mask(tx, ty, xl, xh, yl, yh) << 28);
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

// One wave per tile: sort every (tile, chunk) segment by depth position.
// A slice is the longest run of whole segments that holds at most 64
// entries; boundaries come from the segment offsets (a ballot over 64 of
// them finds the last one within reach).  Keys are p << 4 | mask (p < 2^28),
// so padding with 0xFFFFFFFF sorts last.
constexpr int kSortWave = 64;

__device__ __forceinline__ uint32_t bitonic64(uint32_t key, int lane) {
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t o = __shfl_xor(key, j);
            const bool up = (lane & k) == 0;
            const bool lower = (lane & j) == 0;
            key = (lower == up) ? min(key, o) : max(key, o);
        }
    }
    return key;
}

__device__ __forceinline__ uint32_t entry_key(uint32_t raw) { return ((raw & kIndexMask) << 4) | (raw >> 28); }

__global__ __launch_bounds__(kSortWave) void k_segment_sort(int nchunks, const uint64_t *__restrict__ bin_off,
                                                            uint32_t *__restrict__ lists,
                                                            const uint32_t *__restrict__ sorted_g,
                                                            const int32_t *__restrict__ tile_view, int64_t N) {
    __shared__ uint32_t big[kSegSize];
    const int gt = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t *gv = sorted_g + (int64_t)tile_view[gt] * N;
    const uint64_t *bo = bin_off + (int64_t)gt * nchunks;  // bo[nchunks] = end of this tile's list
    const uint64_t e_end = bo[nchunks];
    uint64_t e0 = bo[0];
    int si = 0;  // e0 == bo[si]
    while (e0 < e_end) {
        const int s = si + 1 + lane;
        const uint64_t b = s <= nchunks ? bo[s] : ~0ull;
        const uint64_t fit = __ballot(b <= e0 + kSortWave);
        const int nseg = __popcll(fit);
        if (nseg > 0) {
            const uint64_t slice_end = __shfl(b, nseg - 1);
            const int n = (int)(slice_end - e0);
            if (n > 0) {
                uint32_t key = lane < n ? entry_key(lists[e0 + lane]) : 0xFFFFFFFFu;
                key = bitonic64(key, lane);
                if (lane < n) lists[e0 + lane] = gv[key >> 4] | ((key & 15u) << 28);
            }
            e0 = slice_end;
            si += nseg;
        } else {
            // segment si alone holds more than 64 (and at most 2^11) entries
            const uint64_t seg_end = bo[si + 1];
            const int n = (int)(seg_end - e0);
            int pad = 128;
            while (pad < n) pad <<= 1;
            for (int i = lane; i < pad; i += kSortWave) big[i] = i < n ? entry_key(lists[e0 + i]) : 0xFFFFFFFFu;
            __syncthreads();
            for (int k = 2; k <= pad; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int i = lane; i < pad; i += kSortWave) {
                        const int ixj = i ^ j;
                        if (ixj > i) {
                            const uint32_t x = big[i], y = big[ixj];
                            const bool up = (i & k) == 0;
                            if ((x > y) == up) {
                                big[i] = y;
                                big[ixj] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            for (int i = lane; i < n; i += kSortWave) {
                const uint32_t key = big[i];
                lists[e0 + i] = gv[key >> 4] | ((key & 15u) << 28);
            }
            __syncthreads();
            e0 = seg_end;
            si += 1;
        }
    }
}

void launch_segment_sort(int total_tiles, int nchunks, const ChunkBufs &b, const uint32_t *sorted_g,
                         const int32_t *tile_view, int64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_segment_sort, dim3(total_tiles), dim3(kSortWave), 0, st, nchunks, b.bin_off, b.lists,
                       sorted_g, tile_view, N);
}

}  // namespace gs
