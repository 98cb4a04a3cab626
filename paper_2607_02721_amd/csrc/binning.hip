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
                                                     const uint32_t *__restrict__ xr_in,
                                                     const uint32_t *__restrict__ yr_in,
                                                     uint32_t *__restrict__ bin_count,
                                                     const uint64_t *__restrict__ bin_off,
                                                     uint32_t *__restrict__ lists,
                                                     const uint8_t *__restrict__ active, uint64_t cap) {
    extern __shared__ uint32_t lds[];
    uint32_t *cnt = lds;                              // [tiles]
    uint32_t *base = lds + kMaxTilesPerView;          // [tiles] (scatter only)
    // Bit 31 of cnt[t] marks a tile without any selected ray (no entries);
    // the counts themselves stay below 2^31.
    constexpr uint32_t kOff = 0x80000000u;
    const int v = blockIdx.y;
    const ViewDev &V = views[v];
    const int64_t nv = nvis[v];
    const int64_t lo = (int64_t)blockIdx.x * kBinPositions;
    if (lo >= nv) return;
    const int64_t hi = min(lo + (int64_t)kBinPositions, nv);
    const int chunk = (int)(lo >> kSegBits);
    const int ntiles = V.tiles_x * V.tiles_y;
    for (int t = threadIdx.x; t < ntiles; t += kBinThreads)
        cnt[t] = (active && !active[V.tile_base + t]) ? kOff : 0u;
    __syncthreads();
    for (int64_t p = lo + threadIdx.x; p < hi; p += kBinThreads) {
        int xl, xh, yl, yh;
        unpack_range(__uint_as_float(xr_in[(int64_t)v * N + p]), xl, xh);
        unpack_range(__uint_as_float(yr_in[(int64_t)v * N + p]), yl, yh);
        for (int ty = yl >> 4; ty <= (yh >> 4); ++ty)
            for (int tx = xl >> 4; tx <= (xh >> 4); ++tx) {
                const int t = ty * V.tiles_x + tx;
                if (cnt[t] & kOff) continue;
                atomicAdd(&cnt[t], 1u);
            }
    }
    __syncthreads();
    if (!kScatter) {
        // this block is the only writer of (tile, chunk) for every tile of the view
        for (int t = threadIdx.x; t < ntiles; t += kBinThreads)
            bin_count[(int64_t)(V.tile_base + t) * nchunks + chunk] = cnt[t] & ~kOff;
        return;
    }
    // Start of this block's segment of each tile, relative to the view's first
    // list entry (a view holds fewer than 2^32 entries), so that the entry loop
    // below reads only LDS.
    const uint64_t vlist = bin_off[(int64_t)V.tile_base * nchunks];
    for (int t = threadIdx.x; t < ntiles; t += kBinThreads) {
        const uint32_t c = cnt[t];
        if (c & ~kOff) base[t] = (uint32_t)(bin_off[(int64_t)(V.tile_base + t) * nchunks + chunk] - vlist);
        cnt[t] = c & kOff;
    }
    __syncthreads();
    uint32_t *vl = lists + vlist;
    for (int64_t p = lo + threadIdx.x; p < hi; p += kBinThreads) {
        int xl, xh, yl, yh;
        unpack_range(__uint_as_float(xr_in[(int64_t)v * N + p]), xl, xh);
        unpack_range(__uint_as_float(yr_in[(int64_t)v * N + p]), yl, yh);
        for (int ty = yl >> 4; ty <= (yh >> 4); ++ty)
            for (int tx = xl >> 4; tx <= (xh >> 4); ++tx) {
                const int t = ty * V.tiles_x + tx;
                if (cnt[t] & kOff) continue;
                const uint32_t slot = atomicAdd(&cnt[t], 1u);
                const uint64_t at = vlist + base[t] + slot;
                if (at < cap) vl[base[t] + slot] = (uint32_t)p | (quad_mask(tx, ty, xl, xh, yl, yh) << 28);
            }
    }
}

void launch_bin_count(const ViewDev *views_dev, int Vc, int64_t N, int nchunks, const ChunkBufs &b,
                      const uint32_t *xr, const uint32_t *yr, hipStream_t st) {
    const int nb = (int)((N + kBinPositions - 1) / kBinPositions);
    hipLaunchKernelGGL(k_bin<false>, dim3(nb, Vc), dim3(kBinThreads), kMaxTilesPerView * sizeof(uint32_t), st,
                       views_dev, N, nchunks, b.nvis, xr, yr, b.bin_count, b.bin_off, b.lists, b.tile_active,
                       (uint64_t)0);
}

void launch_bin_scatter(const ViewDev *views_dev, int Vc, int64_t N, int nchunks, const ChunkBufs &b,
                        const uint32_t *xr, const uint32_t *yr, uint64_t cap, hipStream_t st) {
    const int nb = (int)((N + kBinPositions - 1) / kBinPositions);
    hipLaunchKernelGGL(k_bin<true>, dim3(nb, Vc), dim3(kBinThreads), 2 * kMaxTilesPerView * sizeof(uint32_t), st,
                       views_dev, N, nchunks, b.nvis, xr, yr, b.bin_count, b.bin_off, b.lists, b.tile_active, cap);
}

// Capacity guard for lists sized in advance (plans): if the counted entries
// exceed the capacity, flag it and empty every list of the scene so that no
// later kernel reads past the buffer.
__global__ void k_guard_check(const uint64_t *__restrict__ bin_off, int64_t nbins, uint64_t cap,
                              uint32_t *__restrict__ over, uint32_t *__restrict__ flag) {
    const bool o = bin_off[nbins] > cap;
    *over = o ? 1u : 0u;
    if (o) atomicOr(flag, 1u);
}
__global__ void k_guard_apply(uint64_t *__restrict__ bin_off, int64_t nbins, const uint32_t *__restrict__ over) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (*over && i <= nbins) bin_off[i] = 0;
}
void launch_list_guard(uint64_t *bin_off, int64_t nbins, uint64_t cap, uint32_t *over, uint32_t *flag,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_guard_check, dim3(1), dim3(1), 0, st, bin_off, nbins, cap, over, flag);
    hipLaunchKernelGGL(k_guard_apply, dim3((unsigned)((nbins + 256) / 256)), dim3(256), 0, st, bin_off, nbins, over);
}

// A tile is active when at least one of its rays is selected by the ray mask;
// inactive tiles get empty lists.  One wave per tile, 4 rays per lane.
__global__ __launch_bounds__(64) void k_tile_active(const ViewDev *__restrict__ views,
                                                    const int32_t *__restrict__ tile_view,
                                                    const uint32_t *__restrict__ mask, uint8_t *__restrict__ active) {
    const int gt = blockIdx.x;
    const ViewDev &V = views[tile_view[gt]];
    const int tl = gt - V.tile_base;
    const int tx = tl % V.tiles_x, ty = tl / V.tiles_x;
    bool any = false;
    for (int k = 0; k < 4; ++k) {
        const int r = threadIdx.x * 4 + k;             // 0..255 inside the tile
        const int px = tx * kTile + (r & 15), py = ty * kTile + (r >> 4);
        if (px < V.W && py < V.H) {
            const int64_t ray = V.ray_base + (int64_t)py * V.W + px;
            any = any || ((mask[ray >> 5] >> (ray & 31)) & 1u);
        }
    }
    const bool a = __any(any);
    if (threadIdx.x == 0) active[gt] = a ? 1 : 0;
}

void launch_tile_active(const ViewDev *views_dev, const int32_t *tile_view, int total_tiles, const uint32_t *mask,
                        uint8_t *active, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_active, dim3(total_tiles), dim3(64), 0, st, views_dev, tile_view, mask, active);
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

// Append the first nbig lanes' queued segments to the work list.
__device__ __forceinline__ void flush_big(uint64_t *big, int64_t big_cap, uint64_t start, uint64_t meta, int nbig,
                                          int lane) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd((unsigned long long *)&big[0], (unsigned long long)nbig);
    base = __shfl(base, 0);
    const int64_t k = (int64_t)base + lane;
    if (lane < nbig && k < big_cap) {
        big[1 + 2 * k] = start;
        big[2 + 2 * k] = meta;
    }
}

__global__ __launch_bounds__(kSortWave) void k_segment_sort(int nchunks, const uint64_t *__restrict__ bin_off,
                                                            uint32_t *__restrict__ lists,
                                                            const uint32_t *__restrict__ sorted_g,
                                                            const int32_t *__restrict__ tile_view, int64_t N,
                                                            uint64_t *__restrict__ big, int64_t big_cap) {
    const int gt = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t *gv = sorted_g + (int64_t)tile_view[gt] * N;
    const uint64_t *bo = bin_off + (int64_t)gt * nchunks;  // bo[nchunks] = end of this tile's list
    const uint64_t e_end = bo[nchunks];
    uint64_t e0 = bo[0];
    int si = 0;  // e0 == bo[si]
    uint64_t b = (1 <= nchunks - lane) ? bo[1 + lane] : ~0ull;   // boundaries bo[si+1 ..]
    // software pipeline: the previous slice's gathered entries are stored one
    // iteration late, so its gather overlaps the next slice's loads
    uint64_t pend_at = 0;
    uint32_t pend_val = 0;
    bool pend = false;
    int nbig = 0;
    uint64_t my_start = 0, my_meta = 0;
    while (e0 < e_end) {
        const uint64_t fit = __ballot(b <= e0 + kSortWave);
        const int nseg = __popcll(fit);
        if (nseg > 0) {
            const uint64_t slice_end = __shfl(b, nseg - 1);
            const int n = (int)(slice_end - e0);
            const uint32_t raw = lane < n ? lists[e0 + lane] : 0u;
            const int s = si + nseg + 1 + lane;
            const uint64_t bn = s <= nchunks ? bo[s] : ~0ull;
            if (pend) lists[pend_at] = pend_val;
            pend = false;
            if (n > 0) {
                uint32_t key = lane < n ? entry_key(raw) : 0xFFFFFFFFu;
                key = bitonic64(key, lane);
                if (lane < n) {
                    pend_at = e0 + lane;
                    pend_val = gv[key >> 4] | ((key & 15u) << 28);
                    pend = true;
                }
            }
            e0 = slice_end;
            si += nseg;
            b = bn;
        } else {
            // segment si alone holds more than 64 (and at most 2^11) entries:
            // queue it for the LDS sorter (lane nbig of this wave keeps it;
            // the wave appends 64 at a time with one atomic)
            const uint64_t seg_end = __shfl(b, 0);
            if (lane == nbig) {
                my_start = e0;
                my_meta = (uint64_t)(seg_end - e0) | ((uint64_t)gt << 32);
            }
            if (++nbig == kSortWave) {
                flush_big(big, big_cap, my_start, my_meta, nbig, lane);
                nbig = 0;
            }
            e0 = seg_end;
            si += 1;
            const int s = si + 1 + lane;
            b = s <= nchunks ? bo[s] : ~0ull;
        }
    }
    if (nbig) flush_big(big, big_cap, my_start, my_meta, nbig, lane);
    if (pend) lists[pend_at] = pend_val;
}

// Segments of more than 64 entries: one wave per segment (the waves loop
// over the work list), bitonic sort in LDS.
__global__ __launch_bounds__(kSortWave) void k_big_segment_sort(uint32_t *__restrict__ lists,
                                                                const uint32_t *__restrict__ sorted_g,
                                                                const int32_t *__restrict__ tile_view, int64_t N,
                                                                const uint64_t *__restrict__ big, int64_t big_cap) {
    __shared__ uint32_t keys[kSegSize];
    const int64_t count = min((int64_t)big[0], big_cap);
    const int lane = threadIdx.x;
    for (int64_t w = blockIdx.x; w < count; w += gridDim.x) {
        const uint64_t e0 = big[1 + 2 * w];
        const uint64_t meta = big[2 + 2 * w];
        const int n = (int)(meta & 0xFFFFFFFFull);
        const int gt = (int)(meta >> 32);
        const uint32_t *gv = sorted_g + (int64_t)tile_view[gt] * N;
        int pad = 128;
        while (pad < n) pad <<= 1;
        for (int i = lane; i < pad; i += kSortWave) keys[i] = i < n ? entry_key(lists[e0 + i]) : 0xFFFFFFFFu;
        __syncthreads();
        for (int k = 2; k <= pad; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = lane; i < pad; i += kSortWave) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const uint32_t x = keys[i], y = keys[ixj];
                        const bool up = (i & k) == 0;
                        if ((x > y) == up) {
                            keys[i] = y;
                            keys[ixj] = x;
                        }
                    }
                }
                __syncthreads();
            }
        for (int i = lane; i < n; i += kSortWave) {
            const uint32_t key = keys[i];
            lists[e0 + i] = gv[key >> 4] | ((key & 15u) << 28);
        }
        __syncthreads();
    }
}

void launch_segment_sort(int total_tiles, int nchunks, const ChunkBufs &b, const uint32_t *sorted_g,
                         const int32_t *tile_view, int64_t N, uint64_t *big, int64_t big_cap, hipStream_t st) {
    launch_fill_u64(big, 0ull, 1, st);
    hipLaunchKernelGGL(k_segment_sort, dim3(total_tiles), dim3(kSortWave), 0, st, nchunks, b.bin_off, b.lists,
                       sorted_g, tile_view, N, big, big_cap);
    hipLaunchKernelGGL(k_big_segment_sort, dim3(8192), dim3(kSortWave), 0, st, b.lists, sorted_g, tile_view, N,
                       big, big_cap);
}

}  // namespace gs
