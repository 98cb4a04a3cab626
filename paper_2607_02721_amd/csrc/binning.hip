// Tile binning: per-tile front-to-back lists of Gaussians.
//
// Input: per view, the visible Gaussians in depth order (position p of the
// radix-sorted (depth key, index) sequence; ties by index because the sort is
// stable and starts from index order).  A list entry is keyed by (tile, p)
// and the lists are built by a counting sort on that key:
//   1. count: one block per chunk of 2^11 consecutive positions counts its
//             entries per tile in LDS and stores them, one row per chunk;
//   2. scan:  per tile, the exclusive prefix over chunks (in place) and the
//             tile's total; a scan of the totals gives each tile's list start,
//             so a tile's list is its chunks' segments in order;
//   3. emit:  one wave per (chunk, group of tile rows) expands the chunk's
//             positions that meet its rows, in order, into (position, tile)
//             items packed 64 to a batch; every tile's next slot comes from a
//             wave-private LDS cursor (atomic add, executed in issue order),
//             so each (tile, chunk) segment is written already sorted by p,
//             as g | quadrant mask << 28.
// Bit q of the mask says whether the Gaussian's pixel range touches 8x8
// quadrant q of the 16x16 tile.
#include "gs_internal.hpp"

namespace gs {

constexpr int kBinThreads = 256;
constexpr int kCountGroup = 32;        // chunks per XCD run (multiples of the 16 counts in a 64-byte line)
constexpr int kEmitGroupChunks = 16;   // chunks (times the row groups) per XCD run
constexpr int kSegBits = kChunkBits;
constexpr int kSegSize = 1 << kSegBits;          // positions per chunk

static_assert(kSegSize == kBinPositions, "one binning block per chunk");

__device__ __forceinline__ void unpack_range(float f, int &lo, int &hi) {
    const uint32_t u = __float_as_uint(f);
    lo = (int)(int16_t)(u & 0xFFFFu);
    hi = (int)(int16_t)(u >> 16);
}

// Workgroups are dealt to the 8 XCDs round-robin.  Renumbering hands out
// logical blocks in runs of `group` per XCD (run k to XCD k mod 8), so
// neighbouring chunks (which write neighbouring words of the same lines) and
// the row groups of one chunk (which read the same positions) share one L2,
// while all XCDs stay on nearby chunks of one view.  The grid size must be a
// multiple of 8 * group.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t group) {
    const int64_t xcd = b & 7, slot = b >> 3;
    return ((slot / group) * 8 + xcd) * group + slot % group;
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

__global__ __launch_bounds__(kBinThreads) void k_bin_count(const ViewDev *__restrict__ views, int n_views,
                                                           int64_t N, int nchunks,
                                                           const uint32_t *__restrict__ nvis,
                                                           const uint32_t *__restrict__ xr_in,
                                                           const uint32_t *__restrict__ yr_in,
                                                           uint32_t *__restrict__ bin_count,
                                                           const uint8_t *__restrict__ active) {
    extern __shared__ uint32_t cnt[];                 // [tiles]
    // Bit 31 of cnt[t] marks a tile without any selected ray (no entries);
    // the counts themselves stay below 2^31.
    constexpr uint32_t kOff = 0x80000000u;
    const int64_t lb = xcd_block(blockIdx.x, kCountGroup);   // logical block: chunk + nchunks * view
    const int v = (int)(lb / nchunks);
    if (v >= n_views) return;
    const ViewDev &V = views[v];
    const int64_t nv = nvis[v];
    const int64_t lo = (lb - (int64_t)v * nchunks) * kBinPositions;
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
    // this block is the only writer of (tile, chunk) for every tile of the view
    uint32_t *row = bin_count + (int64_t)V.tile_base * nchunks + (int64_t)chunk * ntiles;
    for (int t = threadIdx.x; t < ntiles; t += kBinThreads) row[t] = cnt[t] & ~kOff;
}

// Column pass over one view's [chunk][tile] counts: each thread owns one tile
// and replaces its counts, chunk by chunk, with their exclusive prefix (the
// tile's segment offsets inside its list); the tile's total goes to tile_tot.
__global__ __launch_bounds__(kBinThreads) void k_chunk_prefix(const ViewDev *__restrict__ views, int nchunks,
                                                              uint32_t *__restrict__ bin_count,
                                                              uint32_t *__restrict__ tile_tot) {
    const ViewDev &V = views[blockIdx.y];
    const int ntiles = V.tiles_x * V.tiles_y;
    const int t = blockIdx.x * kBinThreads + threadIdx.x;
    if (t >= ntiles) return;
    uint32_t *col = bin_count + (int64_t)V.tile_base * nchunks + t;
    uint32_t run = 0;
    int c = 0;
    for (; c + 8 <= nchunks; c += 8) {
        uint32_t x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = col[(int64_t)(c + k) * ntiles];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            col[(int64_t)(c + k) * ntiles] = run;
            run += x[k];
        }
    }
    for (; c < nchunks; ++c) {
        const uint32_t x = col[(int64_t)c * ntiles];
        col[(int64_t)c * ntiles] = run;
        run += x;
    }
    tile_tot[V.tile_base + t] = run;
}

// Ordered emission.  One wave per (group of kEmitRows tile rows, chunk,
// view).  The wave first compacts, in order, the chunk's positions whose
// rectangle meets its rows (an LDS queue), then takes them 64 at a time and
// expands them into (position, tile) items in position order: a wave prefix
// sum of the per-position item counts numbers the items, and each 64-item
// batch finds every item's owner with one LDS write of run heads and a
// max-scan.  A tile's slot comes from an LDS atomic add on its cursor.  Items
// of one batch that hit distinct tiles are independent; when two of them hit
// the same tile (an LDS claim byte per tile detects it) the batch takes its
// owners one at a time in order.  A wave's LDS operations execute in issue
// order, so later positions always receive later slots and every (tile,
// chunk) segment is filled in increasing p.  Splitting a chunk by rows keeps
// the wave's cursors small (high occupancy) and the list lines being written
// at any moment few, so partial lines merge in the caches before they reach
// HBM.
constexpr int kEmitWave = 64;
constexpr int kEmitRows = 4;

__device__ __forceinline__ uint64_t lanemask_lt64_bin() {
    const unsigned lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Wave-wide inclusive scans over the 64 lanes with DPP: shifts by 1, 2, 4, 8
// inside each row of 16 lanes, then row_bcast:15 (row r-1's last lane into
// rows 1 and 3) and row_bcast:31 (lane 31 into rows 2 and 3).  Lanes without
// a source take the identity.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_src(int identity, int x) {
    return __builtin_amdgcn_update_dpp(identity, x, kCtrl, kRowMask, 0xF, false);
}

__device__ __forceinline__ int wave_scan_add(int v) {
    v += dpp_src<0x111, 0xF>(0, v);
    v += dpp_src<0x112, 0xF>(0, v);
    v += dpp_src<0x114, 0xF>(0, v);
    v += dpp_src<0x118, 0xF>(0, v);
    v += dpp_src<0x142, 0xA>(0, v);
    v += dpp_src<0x143, 0xC>(0, v);
    return v;
}

__device__ __forceinline__ int wave_scan_max(int v) {  // identity -1
    v = max(v, dpp_src<0x111, 0xF>(-1, v));
    v = max(v, dpp_src<0x112, 0xF>(-1, v));
    v = max(v, dpp_src<0x114, 0xF>(-1, v));
    v = max(v, dpp_src<0x118, 0xF>(-1, v));
    v = max(v, dpp_src<0x142, 0xA>(-1, v));
    v = max(v, dpp_src<0x143, 0xC>(-1, v));
    return v;
}

template <bool kMasked>
__device__ __forceinline__ bool tile_on(const uint32_t *act, int t) {
    return !kMasked || ((act[t >> 5] >> (t & 31)) & 1u);
}

template <bool kMasked>
__global__ __launch_bounds__(kEmitWave) void k_bin_emit(const ViewDev *__restrict__ views, int n_views, int64_t N,
                                                        int nchunks, int row_groups,
                                                        const uint32_t *__restrict__ nvis,
                                                        const uint32_t *__restrict__ xr_in,
                                                        const uint32_t *__restrict__ yr_in,
                                                        const uint32_t *__restrict__ sorted_g,
                                                        const uint32_t *__restrict__ bin_count,
                                                        const uint64_t *__restrict__ tile_off,
                                                        uint32_t *__restrict__ lists,
                                                        const uint8_t *__restrict__ active, uint64_t cap,
                                                        int group_tiles) {
    extern __shared__ uint32_t lds[];
    uint32_t *cur = lds;                                  // [group tiles] next slot, relative to the view's first entry
    int32_t *head = (int32_t *)(cur + group_tiles);        // [64] lane owning the item that starts a run
    uint32_t *rx = (uint32_t *)head + kEmitWave;           // [64] the round's pixel ranges and indices
    uint32_t *ry = rx + kEmitWave;
    uint32_t *rg = ry + kEmitWave;
    uint16_t *queue = (uint16_t *)(rg + kEmitWave);       // [2048] chunk-local positions meeting the rows
    uint8_t *claim = (uint8_t *)(queue + kBinPositions);  // [group tiles] lane that last claimed the tile
    uint32_t *act = (uint32_t *)(claim + ((group_tiles + 3) & ~3));  // [group tiles / 32] (masked form only)
    // logical block: row group + row_groups * (chunk + nchunks * view)
    const int64_t lb = xcd_block(blockIdx.x, (int64_t)kEmitGroupChunks * row_groups);
    const int64_t per_view = (int64_t)row_groups * nchunks;
    const int v = (int)(lb / per_view);
    if (v >= n_views) return;
    const int grp = (int)(lb % row_groups);
    const int chunk = (int)((lb - (int64_t)v * per_view) / row_groups);
    const int lane = threadIdx.x;
    const ViewDev &V = views[v];
    const int64_t nv = nvis[v];
    const int64_t lo = (int64_t)chunk * kBinPositions;
    const int r0 = grp * kEmitRows;
    if (lo >= nv || r0 >= V.tiles_y) return;
    const int r1 = min(r0 + kEmitRows, V.tiles_y);    // rows [r0, r1)
    const int hi = (int)(min(lo + (int64_t)kBinPositions, nv) - lo);
    const int tiles_x = V.tiles_x;
    const int ntiles = (r1 - r0) * tiles_x;           // this wave's tiles: t = tile_base + r0 * tiles_x + local
    const int64_t t0 = (int64_t)V.tile_base + (int64_t)r0 * tiles_x;
    const uint64_t vlist = tile_off[V.tile_base];
    // segment start of each of the wave's tiles for this chunk, relative to
    // the view's first entry: the tile's list start plus the tile's prefix
    const uint32_t *pre = bin_count + (int64_t)V.tile_base * nchunks + (int64_t)chunk * (V.tiles_x * V.tiles_y) +
                          (int64_t)r0 * tiles_x;
    for (int t = lane; t < ntiles; t += kEmitWave) cur[t] = (uint32_t)(tile_off[t0 + t] - vlist) + pre[t];
    if (kMasked) {
        for (int w = lane; w < (ntiles + 31) / 32; w += kEmitWave) {
            uint32_t bits = 0;
            for (int b = 0; b < 32; ++b) {
                const int t = 32 * w + b;
                bits |= (t < ntiles && active[t0 + t]) ? (1u << b) : 0u;
            }
            act[w] = bits;
        }
    }
    // entries at or past `room` would fall outside the list buffer
    const uint64_t room = cap > vlist ? cap - vlist : 0ull;
    uint32_t *__restrict__ vl = lists + vlist;
    const int64_t o = (int64_t)v * N + lo;
    // 1. positions whose rows meet [r0, r1), in order
    int nq = 0;
    for (int base = 0; base < hi; base += kEmitWave) {
        const int p = base + lane;
        bool meets = false;
        if (p < hi) {
            int yl, yh;
            unpack_range(__uint_as_float(yr_in[o + p]), yl, yh);
            meets = (yl >> 4) < r1 && (yh >> 4) >= r0;
        }
        const uint64_t bal = __ballot(meets);
        if (meets) queue[nq + __popcll(bal & lanemask_lt64_bin())] = (uint16_t)p;
        nq += __popcll(bal);
    }
    __syncthreads();
    // 2. expansion of the queued positions against this wave's tiles
    for (int base = 0; base < nq; base += kEmitWave) {
        const int qi = base + lane;
        uint32_t ux = 0, uy = 0, ug = 0;
        int k = 0;
        if (qi < nq) {
            const int p = queue[qi];
            ux = xr_in[o + p];
            uy = yr_in[o + p];
            ug = sorted_g[o + p];
            int xl, xh, yl, yh;
            unpack_range(__uint_as_float(ux), xl, xh);
            unpack_range(__uint_as_float(uy), yl, yh);
            k = ((xh >> 4) - (xl >> 4) + 1) * (min(yh >> 4, r1 - 1) - max(yl >> 4, r0) + 1);
        }
        const int incl = wave_scan_add(k);
        const int K = __builtin_amdgcn_readlane(incl, kEmitWave - 1);
        const int excl = incl - k;   // first item of this lane's position
        rx[lane] = ux;
        ry[lane] = uy;
        rg[lane] = ug;
        __syncthreads();
        for (int i0 = 0; i0 < K; i0 += kEmitWave) {
            const int i = i0 + lane;
            const bool item = i < K;
            // owner of item i: the last position lane whose first item is <= i.
            // Item i0's owner is the highest lane with excl <= i0; a lane whose
            // run starts inside the batch marks its first item, and a max-scan
            // over the marks carries each owner forward.
            const uint64_t started = __ballot(excl <= i0);
            const int carry = 63 - __builtin_clzll(started);
            head[lane] = -1;
            if (k > 0 && excl > i0 && excl < i0 + kEmitWave) head[excl - i0] = lane;
            __syncthreads();
            const int L = max(carry, wave_scan_max(head[lane]));
            const int j = i - __shfl(excl, L);
            int xl, xh, yl, yh;
            unpack_range(__uint_as_float(rx[L]), xl, xh);
            unpack_range(__uint_as_float(ry[L]), yl, yh);
            const uint32_t g = rg[L];
            const int tx0 = xl >> 4, ty0 = max(yl >> 4, r0);
            const int nx = (xh >> 4) - tx0 + 1;
            // j / nx as floor((j + 1/2) r) with r within one ulp of 1/nx:
            // exact for nx * ny <= 8160 (checked exhaustively on the host)
            const int dy = (int)(((float)j + 0.5f) * __builtin_amdgcn_rcpf((float)nx));
            const int tx = tx0 + (j - dy * nx), ty = ty0 + dy;
            const int tc = (ty - r0) * tiles_x + tx;
            const bool in = item && (unsigned)tc < (unsigned)ntiles;
            const int t = in ? tc : 0;
            const bool on = in && tile_on<kMasked>(act, t);
            if (on) claim[t] = (uint8_t)lane;
            __syncthreads();
            const bool clash = on && claim[t] != (uint8_t)lane;
            uint32_t c = 0;
            if (__ballot(clash) == 0ull) {
                if (on) c = atomicAdd(&cur[t], 1u);
            } else {
                // owners in increasing order; one owner's tiles are distinct
                uint64_t rem = __ballot(on);
                while (rem) {
                    const int first = __ffsll((long long)rem) - 1;
                    const int owner = __shfl(L, first);
                    const bool mine = on && L == owner;
                    if (mine) c = atomicAdd(&cur[t], 1u);
                    rem &= ~__ballot(mine);
                }
            }
            if (on && (uint64_t)c < room) vl[c] = g | (quad_mask(tx, ty, xl, xh, yl, yh) << 28);
            __syncthreads();
        }
    }
}

void launch_bin_count(const ViewDev *views_dev, int Vc, int64_t N, int nchunks, const ChunkBufs &b,
                      const uint32_t *xr, const uint32_t *yr, int max_tiles, hipStream_t st) {
    const int64_t run = 8 * kCountGroup;
    const int64_t blocks = ((int64_t)nchunks * Vc + run - 1) / run * run;
    hipLaunchKernelGGL(k_bin_count, dim3((unsigned)blocks), dim3(kBinThreads), (size_t)max_tiles * sizeof(uint32_t),
                       st, views_dev, Vc, N, nchunks, b.nvis, xr, yr, b.bin_count, b.tile_active);
}

void launch_chunk_prefix(const ViewDev *views_dev, int Vc, int nchunks, const ChunkBufs &b, int max_tiles,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_chunk_prefix, dim3((unsigned)((max_tiles + kBinThreads - 1) / kBinThreads), (unsigned)Vc),
                       dim3(kBinThreads), 0, st, views_dev, nchunks, b.bin_count, b.tile_tot);
}

void launch_bin_emit(const ViewDev *views_dev, int Vc, int64_t N, int nchunks, const ChunkBufs &b,
                     const uint32_t *xr, const uint32_t *yr, const uint32_t *sorted_g, int max_tiles_x,
                     int max_tiles_y, uint64_t cap, hipStream_t st) {
    const int row_groups = (max_tiles_y + kEmitRows - 1) / kEmitRows;
    const int64_t run = 8 * (int64_t)kEmitGroupChunks * row_groups;
    const int64_t blocks = ((int64_t)row_groups * nchunks * Vc + run - 1) / run * run;
    const int group_tiles = kEmitRows * max_tiles_x;
    // cursors, run heads, three round arrays, queue, claim bytes, tile bitmap
    const size_t lds = sizeof(uint32_t) * ((size_t)group_tiles + kEmitWave + 3 * kEmitWave) +
                       sizeof(uint16_t) * kBinPositions + (((size_t)group_tiles + 3) & ~(size_t)3) +
                       (b.tile_active ? sizeof(uint32_t) * ((size_t)group_tiles + 31) / 32 : 0);
    const dim3 grid((unsigned)blocks);
    if (b.tile_active)
        hipLaunchKernelGGL(k_bin_emit<true>, grid, dim3(kEmitWave), lds, st, views_dev, Vc, N, nchunks, row_groups,
                           b.nvis, xr, yr, sorted_g, b.bin_count, b.tile_off, b.lists, b.tile_active, cap,
                           group_tiles);
    else
        hipLaunchKernelGGL(k_bin_emit<false>, grid, dim3(kEmitWave), lds, st, views_dev, Vc, N, nchunks, row_groups,
                           b.nvis, xr, yr, sorted_g, b.bin_count, b.tile_off, b.lists, b.tile_active, cap,
                           group_tiles);
}

// Capacity guard for lists sized in advance (plans): if the counted entries
// exceed the capacity, flag it and empty every list of the scene so that no
// later kernel reads past the buffer.
__global__ void k_guard_check(const uint64_t *__restrict__ tile_off, int64_t ntiles, uint64_t cap,
                              uint32_t *__restrict__ over, uint32_t *__restrict__ flag) {
    const bool o = tile_off[ntiles] > cap;
    *over = o ? 1u : 0u;
    if (o) atomicOr(flag, 1u);
}
__global__ void k_guard_apply(uint64_t *__restrict__ tile_off, int64_t ntiles, const uint32_t *__restrict__ over) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (*over && i <= ntiles) tile_off[i] = 0;
}
void launch_list_guard(uint64_t *tile_off, int64_t ntiles, uint64_t cap, uint32_t *over, uint32_t *flag,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_guard_check, dim3(1), dim3(1), 0, st, tile_off, ntiles, cap, over, flag);
    hipLaunchKernelGGL(k_guard_apply, dim3((unsigned)((ntiles + 256) / 256)), dim3(256), 0, st, tile_off, ntiles,
                       over);
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

}  // namespace gs
