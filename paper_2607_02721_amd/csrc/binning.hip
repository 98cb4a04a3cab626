// Tile binning: per-tile front-to-back lists of Gaussians.
//
// Input: per view, the visible Gaussians in depth order (position p of the
// radix-sorted (depth key, index) sequence; ties by index because the sort is
// stable and starts from index order).  A list entry is keyed by (tile, p)
// and the lists are built by a counting sort on that key:
//   1. count: one block per chunk of 2^14 consecutive positions counts its
//             entries per tile in LDS and stores them, one row per chunk;
//   2. scan:  per tile, the exclusive prefix over chunks (in place) and the
//             tile's total; a scan of the totals gives each tile's list start,
//             so a tile's list is its chunks' segments in order;
//   3. emit:  one wave per (chunk, group of tile rows) expands the chunk's
//             positions that meet its rows, in order and 2^10 at a time, into
//             (position, tile) items packed 64 to a batch; every tile's next
//             slot comes from a wave-private LDS cursor (atomic add, executed
//             in issue order), so each (tile, chunk) segment is written
//             already sorted by p, as g | quadrant mask << 28.
// Chunks are long so that a tile's segment in a chunk spans whole cache
// lines: list entries are 4 bytes, and segments of a few entries each end in
// partial lines that cost a full write each.
// Bit q of the mask says whether the Gaussian's pixel range touches 8x8
// quadrant q of the 16x16 tile.
#include "gs_internal.hpp"

#include <algorithm>

namespace gs {

constexpr int kBinThreads = 256;
constexpr int kCountGroup = 32;        // chunks per XCD run (multiples of the 16 counts in a 64-byte line)
constexpr int kEmitGroupChunks = 4;    // chunks (times the row groups) per XCD run
constexpr int kSegBits = kChunkBits;
constexpr int kSegSize = 1 << kSegBits;          // positions per chunk

static_assert(kSegSize == kBinPositions, "one binning block per chunk");
static_assert(kBinPositions <= 65536, "queued positions are 16-bit chunk offsets");

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

// Sub-rectangles (halves in x and y) of tile (tx, ty) met by the pixel
// rectangle [xl, xh] x [yl, yh], which meets the tile: it meets the left
// (top) half iff it starts before the middle, and the right (bottom) half
// iff it ends after it.
__device__ __forceinline__ uint32_t quad_mask(int tx, int ty, int xl, int xh, int yl, int yh, int tsx, int tsy) {
    const int mx = (tx << tsx) + (1 << (tsx - 1)), my = (ty << tsy) + (1 << (tsy - 1));
    const uint32_t l = xl < mx ? 1u : 0u, r = xh >= mx ? 2u : 0u;
    const uint32_t top = yl < my ? (l | r) : 0u, bottom = yh >= my ? (l | r) << 2 : 0u;
    return top | bottom;
}

__global__ __launch_bounds__(kBinThreads) void k_bin_count(const ViewDev *__restrict__ views, int n_views,
                                                           int64_t N, int nchunks,
                                                           const uint32_t *__restrict__ nvis,
                                                           const uint32_t *__restrict__ xr_in,
                                                           const uint32_t *__restrict__ yr_in,
                                                           uint32_t *__restrict__ bin_count,
                                                           const uint16_t *__restrict__ active,
                                                           uint64_t *__restrict__ rowbits, int rows_stride) {
    // A position adds 1 to every tile of its tile rectangle: +1 / -1 at the
    // rectangle's corners of a 2D difference array, whose prefix sums along
    // x and then y are the counts (four LDS atomics per position, whatever
    // its size).
    extern __shared__ int32_t dif[];                  // [tiles_y + 1][tiles_x + 1]
    __shared__ uint64_t rowword[kBinThreads / 64][128];   // per wave: row words on their way to the lanes
    const int64_t lb = xcd_block(blockIdx.x, kCountGroup);   // logical block: chunk + nchunks * view
    const int v = (int)(lb / nchunks);
    if (v >= n_views) return;
    const ViewDev &V = views[v];
    const int64_t nv = nvis[v];
    const int64_t lo = (lb - (int64_t)v * nchunks) * kBinPositions;
    if (lo >= nv) return;
    const int64_t hi = min(lo + (int64_t)kBinPositions, nv);
    const int chunk = (int)(lo >> kSegBits);
    const int tx_n = V.tiles_x, ty_n = V.tiles_y, ntiles = tx_n * ty_n;
    const int stride = tx_n + 1, cells = stride * (ty_n + 1);
    for (int i = threadIdx.x; i < cells; i += kBinThreads) dif[i] = 0;
    __syncthreads();
    // the view's row bitmaps for this chunk: word w of row r at
    // rb + r * row_pitch + w
    constexpr int kWords = kBinPositions / 64;
    const int64_t row_pitch = (int64_t)nchunks * kWords;
    uint64_t *rb = rowbits + (int64_t)v * rows_stride * row_pitch + (int64_t)chunk * kWords;
    // every lane of a wave runs each step (positions past the chunk's end
    // are invalid), so the row words gathered into the lanes can be stored
    // by the whole wave
    const int lane = threadIdx.x & 63;
    uint64_t *sw = rowword[threadIdx.x >> 6];
    for (int64_t p0 = lo + (threadIdx.x & ~63); p0 < hi; p0 += kBinThreads) {
        const int64_t p = p0 + lane;
        const bool valid = p < hi;
        // rows [ty0, ty0 + span]; invalid positions meet none (r - ty0 wraps
        // to a large unsigned value for every row r)
        int ty0 = 0x40000000;
        uint32_t span = 0u;
        if (valid) {
            int xl, xh, yl, yh;
            unpack_range(__uint_as_float(xr_in[(int64_t)v * N + p]), xl, xh);
            unpack_range(__uint_as_float(yr_in[(int64_t)v * N + p]), yl, yh);
            const int x0 = xl >> V.tsx, x1 = (xh >> V.tsx) + 1;
            ty0 = yl >> V.tsy;
            const int ty1 = yh >> V.tsy;
            span = (uint32_t)(ty1 - ty0);
            const int y0 = ty0 * stride, y1 = (ty1 + 1) * stride;
            atomicAdd(&dif[y0 + x0], 1);
            atomicAdd(&dif[y0 + x1], -1);
            atomicAdd(&dif[y1 + x0], -1);
            atomicAdd(&dif[y1 + x1], 1);
        }
        // the wave's 64 positions form one bitmap word per tile row: one
        // ballot per row, written to LDS by lane 0 (128 rows at a time) and
        // read back by the lane that stores the row's word
        const int w = (int)((p0 - lo) >> 6);
        for (int rb0 = 0; rb0 < ty_n; rb0 += 128) {
            const int rn = __builtin_amdgcn_readfirstlane(min(128, ty_n - rb0));
            const uint32_t rel = (uint32_t)(rb0 - ty0);
#pragma unroll 8
            for (int k = 0; k < rn; ++k) {
                const uint64_t bits = __ballot(rel + (uint32_t)k <= span);
                if (lane == 0) sw[k] = bits;
            }
            wave_sync();
            if (lane < rn) rb[(int64_t)(rb0 + lane) * row_pitch + w] = sw[lane];
            if (lane + 64 < rn) rb[(int64_t)(rb0 + lane + 64) * row_pitch + w] = sw[lane + 64];
            wave_sync();   // the words are read before the next rows overwrite them
        }
    }
    __syncthreads();
    for (int ty = threadIdx.x; ty < ty_n; ty += kBinThreads) {       // along x, one row per thread
        int run = 0;
        for (int tx = 0; tx < tx_n; ++tx) {
            run += dif[ty * stride + tx];
            dif[ty * stride + tx] = run;
        }
    }
    __syncthreads();
    for (int tx = threadIdx.x; tx < tx_n; tx += kBinThreads) {       // along y, one column per thread
        int run = 0;
        for (int ty = 0; ty < ty_n; ++ty) {
            run += dif[ty * stride + tx];
            dif[ty * stride + tx] = run;
        }
    }
    __syncthreads();
    // this block is the only writer of (tile, chunk) for every tile of the
    // view; tiles without a selected ray get no entries
    uint32_t *row = bin_count + (int64_t)V.tile_base * nchunks + (int64_t)chunk * ntiles;
    for (int t = threadIdx.x; t < ntiles; t += kBinThreads) {
        const bool off = active && !active[V.tile_base + t];
        row[t] = off ? 0u : (uint32_t)dif[(t / tx_n) * stride + t % tx_n];
    }
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

// Ordered emission.  One wave per (group of kEmitRows tile rows and at most
// kEmitCols tile columns, chunk, view).  For each batch of kEmitBatch
// positions of its chunk, the wave first compacts, in order, the positions
// whose rectangle meets its rows (an LDS queue), then takes them 64 at a
// time and expands them into (position,
// tile) items in position order: a wave prefix sum of the per-position item
// counts numbers the items, and each 64-item batch finds every item's owner
// with one LDS write of run heads and a max-scan.  A tile's slot comes from
// an LDS atomic add on its cursor.  Items of one batch that hit the same tile
// must take their slots in position (= lane) order: a per-tile LDS lane mask
// gives each item the lanes that share its tile, the lowest of them takes the
// whole run from the cursor and each item adds its rank.  A
// wave's LDS operations execute in issue order, so later positions always
// receive later slots and every (tile, chunk) segment is filled in
// increasing p.
//
// Entries are not stored one by one: each tile keeps the block ("line") of
// its list that it is filling in LDS (slot = absolute entry index mod the
// line length), and a line goes out as one store of consecutive lanes once
// its last slot is filled.  Only the first and last line of a segment
// (shared with the neighbouring chunks' segments) are written partially.
// Scattered 4-byte stores leave the L2 as several partial-line writes per
// line (about 24 GB of writes for 4.3 GB of entries at 1M Gaussians x 100
// views with 16x16 tiles, against 6.6 GB with 32-byte lines).  Lines are 8
// entries (32 bytes) for tiles 8 or 16 pixels wide, which keeps the wave's
// LDS small, and 16 entries (64 bytes, streamed past the L2) for tiles 32
// pixels wide, whose segments per chunk are long enough to fill them.
constexpr int kEmitWave = 64;
constexpr int kEmitRows = 1;
constexpr int kEmitCols = 128;     // tile columns per wave (2048 pixels)

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

__device__ __forceinline__ int wave_scan_max(int v) {
    constexpr int lo = -2147483647 - 1;   // identity of max
    v = max(v, dpp_src<0x111, 0xF>(lo, v));
    v = max(v, dpp_src<0x112, 0xF>(lo, v));
    v = max(v, dpp_src<0x114, 0xF>(lo, v));
    v = max(v, dpp_src<0x118, 0xF>(lo, v));
    v = max(v, dpp_src<0x142, 0xA>(lo, v));
    v = max(v, dpp_src<0x143, 0xC>(lo, v));
    return v;
}

// Bits >= s of a 64-bit word (s may be negative or past 63).
__device__ __forceinline__ uint64_t bits_from(int s) {
    return s >= 64 ? 0ull : (s <= 0 ? ~0ull : (~0ull << s));
}

// Whether the 128-bit set (lo, hi) holds any of the bits a..b (0 <= a <= b < 128).
__device__ __forceinline__ bool range_hits(uint64_t lo, uint64_t hi, int a, int b) {
    const uint64_t mlo = bits_from(a) & ~bits_from(b + 1);
    const uint64_t mhi = bits_from(a - 64) & ~bits_from(b + 1 - 64);
    return ((lo & mlo) | (hi & mhi)) != 0ull;
}

template <bool kMasked>
__device__ __forceinline__ bool tile_on(const uint32_t *act, int t) {
    return !kMasked || ((act[t >> 5] >> (t & 31)) & 1u);
}

// A list entry's store: 64-byte lines bypass the L2 (they are whole write
// requests, and the lists are read only by a later launch); 32-byte lines
// go through it, where the halves of a request that two chunks' segments
// share are merged.
template <int kLine>
__device__ __forceinline__ void store_entry(uint32_t v, uint32_t *dst) {
    if (kLine >= 16)
        __builtin_nontemporal_store(v, dst);
    else
        *dst = v;
}

// LDS layout of one emission wave (32-bit words unless noted).
struct EmitLds {
    uint64_t *lanes;    // [tiles] lanes of the current item batch on the tile
    uint32_t *line;     // [tiles][2^kLineLog] the line each tile is filling
    uint32_t *cur;      // [tiles] next entry, relative to the view's first entry
    uint32_t *seg0;     // [tiles] first entry of the tile's segment in this chunk
    int32_t *head;      // [64] lane owning the item that starts a run
    uint32_t *rx, *ry, *rg;   // [64] the round's pixel ranges and indices
    uint32_t *ft, *fc;  // [64] lines to store: tile, and the entry in its last slot
    uint16_t *queue;    // [kEmitBatch] chunk-local positions meeting the rows
    uint32_t *act;      // [tiles / 32] (masked form only)
};

__host__ __device__ constexpr size_t emit_lds_bytes(int tiles, bool masked, int line_log) {
    return sizeof(uint32_t) * ((size_t)tiles * ((1 << line_log) + 4) + 6 * kEmitWave) + sizeof(uint16_t) * kEmitBatch +
           (masked ? sizeof(uint32_t) * (((size_t)tiles + 31) / 32) : 0);
}

template <int kLine>
__device__ __forceinline__ EmitLds emit_lds(uint32_t *base, int tiles) {
    EmitLds L;
    L.lanes = (uint64_t *)base;
    L.line = base + 2 * (size_t)tiles;
    L.cur = L.line + (size_t)tiles * kLine;
    L.seg0 = L.cur + tiles;
    L.head = (int32_t *)(L.seg0 + tiles);
    L.rx = (uint32_t *)L.head + kEmitWave;
    L.ry = L.rx + kEmitWave;
    L.rg = L.ry + kEmitWave;
    L.ft = L.rg + kEmitWave;
    L.fc = L.ft + kEmitWave;
    L.queue = (uint16_t *)(L.fc + kEmitWave);
    L.act = (uint32_t *)(L.queue + kEmitBatch);
    return L;
}

// Stores the staged blocks ("lines") listed in L.ft / L.fc (n of them), 64 / kLine per step
// with kLine lanes each; entries before the tile's segment (another chunk's) and at or
// past `room` are left alone.
template <int kLine>
__device__ __forceinline__ void store_lines(const EmitLds &L, int n, uint32_t align, uint32_t *__restrict__ vl,
                                            uint64_t room) {
    const int lane = threadIdx.x;
    for (int f0 = 0; f0 < n; f0 += kEmitWave / kLine) {
        const int f = f0 + lane / kLine, k = lane % kLine;
        if (f < n) {
            const int t = (int)L.ft[f];
            const uint32_t last = L.fc[f];                           // entry in the line's last slot
            const int64_t e = (int64_t)last - (int64_t)((align + last) & (kLine - 1u)) + k;
            if (e >= (int64_t)L.seg0[t] && (uint64_t)e < room && e <= (int64_t)last)
                store_entry<kLine>(L.line[t * kLine + k], &vl[e]);
        }
    }
}

template <bool kMasked, int kLineLog>
__global__ __launch_bounds__(kEmitWave) void k_bin_emit(const ViewDev *__restrict__ views, int n_views, int64_t N,
                                                        int nchunks, int row_groups, int col_groups,
                                                        const uint32_t *__restrict__ nvis,
                                                        const uint32_t *__restrict__ xr_in,
                                                        const uint32_t *__restrict__ yr_in,
                                                        const uint32_t *__restrict__ sorted_g,
                                                        const uint32_t *__restrict__ bin_count,
                                                        const uint64_t *__restrict__ tile_off,
                                                        uint32_t *__restrict__ lists,
                                                        const uint16_t *__restrict__ active, uint64_t cap,
                                                        int group_tiles, const uint64_t *__restrict__ rowbits,
                                                        int rows_stride) {
    extern __shared__ uint32_t lds[];
    constexpr int kLine = 1 << kLineLog;
    const EmitLds L = emit_lds<kLine>(lds, group_tiles);
    // logical block: group + groups * (chunk + nchunks * view), with group =
    // row group + row_groups * column group
    const int groups = row_groups * col_groups;
    const int64_t lb = xcd_block(blockIdx.x, (int64_t)kEmitGroupChunks * groups);
    const int64_t per_view = (int64_t)groups * nchunks;
    const int v = (int)(lb / per_view);
    if (v >= n_views) return;
    const int grp = (int)(lb % groups);
    const int chunk = (int)((lb - (int64_t)v * per_view) / groups);
    const int lane = threadIdx.x;
    const ViewDev &V = views[v];
    const int sx = V.tsx, sy = V.tsy;
    const int64_t nv = nvis[v];
    const int64_t lo = (int64_t)chunk * kBinPositions;
    const int r0 = (grp % row_groups) * kEmitRows, c0 = (grp / row_groups) * kEmitCols;
    if (lo >= nv || r0 >= V.tiles_y || c0 >= V.tiles_x) return;
    const int r1 = min(r0 + kEmitRows, V.tiles_y);    // rows [r0, r1)
    const int c1 = min(c0 + kEmitCols, V.tiles_x);    // columns [c0, c1)
    const int hi = (int)(min(lo + (int64_t)kBinPositions, nv) - lo);
    const int tiles_x = V.tiles_x, ncols = c1 - c0;
    const int ntiles = (r1 - r0) * ncols;             // local tile (ty - r0) * ncols + (tx - c0)
    const uint64_t vlist = tile_off[V.tile_base];
    const uint32_t align = (uint32_t)(vlist & (kLine - 1u));   // slot of the view's first entry in its line
    // segment start of each of the wave's tiles for this chunk, relative to
    // the view's first entry: the tile's list start plus the tile's prefix
    const uint32_t *pre = bin_count + (int64_t)V.tile_base * nchunks + (int64_t)chunk * (V.tiles_x * V.tiles_y);
    for (int t = lane; t < ntiles; t += kEmitWave) {
        const int vt = (r0 + t / ncols) * tiles_x + c0 + t % ncols;   // tile within the view
        const uint32_t s0 = (uint32_t)(tile_off[V.tile_base + vt] - vlist) + pre[vt];
        L.cur[t] = s0;
        L.seg0[t] = s0;
    }
    if (kMasked) {
        for (int w = lane; w < (ntiles + 31) / 32; w += kEmitWave) {
            uint32_t bits = 0;
            for (int b = 0; b < 32; ++b) {
                const int t = 32 * w + b;
                const int vt = (r0 + t / ncols) * tiles_x + c0 + t % ncols;
                bits |= (t < ntiles && active[V.tile_base + vt]) ? (1u << b) : 0u;
            }
            L.act[w] = bits;
        }
    }
    wave_sync();
    // masked form: the wave's active tiles as a 128-bit set (one tile row);
    // a wave with none has nothing to emit
    static_assert(!kMasked || (kEmitRows == 1 && kEmitCols <= 128), "one row of at most 128 tiles");
    uint64_t act_lo = 0ull, act_hi = 0ull;
    if (kMasked) {
        const int nw = (ntiles + 31) / 32;
        act_lo = (uint64_t)L.act[0] | (nw > 1 ? (uint64_t)L.act[1] << 32 : 0ull);
        act_hi = (nw > 2 ? (uint64_t)L.act[2] : 0ull) | (nw > 3 ? (uint64_t)L.act[3] << 32 : 0ull);
        if ((act_lo | act_hi) == 0ull) return;
    }
    // entries at or past `room` would fall outside the list buffer
    const uint64_t room = cap > vlist ? cap - vlist : 0ull;
    uint32_t *__restrict__ vl = lists + vlist;
    const int64_t o = (int64_t)v * N + lo;
    // this wave's row bitmap in the chunk (one word per 64 positions)
    static_assert(kEmitRows == 1, "the row bitmaps select one tile row");
    constexpr int kWords = kBinPositions / 64;
    const uint64_t *rbits =
        rowbits + ((int64_t)v * rows_stride + r0) * ((int64_t)nchunks * kWords) + (int64_t)chunk * kWords;
    static_assert(kEmitBatch % 64 == 0 && kEmitBatch <= 64 * kEmitWave, "one row-bitmap word per lane");
    for (int b0 = 0; b0 < hi; b0 += kEmitBatch) {
        const int b1 = min(b0 + kEmitBatch, hi);
        // 1. positions of the batch that meet row r0, in order: lane l < 16
        // takes the bitmap word of positions b0 + 64 l ... + 63 (bits past the
        // chunk's visible positions are clear), a wave prefix sum of the
        // popcounts places each lane's positions in the queue
        const int nw = (b1 - b0 + 63) >> 6;
        uint64_t word = lane < nw ? __builtin_nontemporal_load(&rbits[(b0 >> 6) + lane]) : 0ull;
        const int cnt = __popcll(word);
        const int incl = wave_scan_add(cnt);
        const int nq = __builtin_amdgcn_readlane(incl, kEmitWave - 1);
        int slot = incl - cnt;
        while (word) {
            const int bit = __ffsll((long long)word) - 1;
            L.queue[slot++] = (uint16_t)(b0 + 64 * lane + bit);
            word &= word - 1ull;
        }
        wave_sync();
        // 2. expansion of the queued positions against this wave's tiles; the
        // next round's ranges and indices are loaded while this one expands
        uint32_t nx_ = 0, ny_ = 0, ng_ = 0;
        if (lane < nq) {
            const int p = L.queue[lane];
            nx_ = xr_in[o + p];
            ny_ = yr_in[o + p];
            ng_ = sorted_g[o + p];
        }
        for (int base = 0; base < nq; base += kEmitWave) {
            const int qi = base + lane;
            const uint32_t ux = nx_, uy = ny_, ug = ng_;
            if (qi + kEmitWave < nq) {
                const int p = L.queue[qi + kEmitWave];
                nx_ = xr_in[o + p];
                ny_ = yr_in[o + p];
                ng_ = sorted_g[o + p];
            }
            int k = 0;
            if (qi < nq) {
                int xl, xh, yl, yh;
                unpack_range(__uint_as_float(ux), xl, xh);
                unpack_range(__uint_as_float(uy), yl, yh);
                // the tiles of its rectangle inside this wave's rows and columns
                // (masked form: none unless one of them is active)
                const int kx = min(xh >> sx, c1 - 1) - max(xl >> sx, c0) + 1;
                k = kx > 0 ? kx * (min(yh >> sy, r1 - 1) - max(yl >> sy, r0) + 1) : 0;
                if (kMasked && k > 0 &&
                    !range_hits(act_lo, act_hi, max(xl >> sx, c0) - c0, min(xh >> sx, c1 - 1) - c0))
                    k = 0;
            }
            const int incl = wave_scan_add(k);
            const int K = __builtin_amdgcn_readlane(incl, kEmitWave - 1);
            const int excl = incl - k;   // first item of this lane's position
            L.rx[lane] = ux;
            L.ry[lane] = uy;
            L.rg[lane] = ug;
            wave_sync();
            for (int i0 = 0; i0 < K; i0 += kEmitWave) {
                const int i = i0 + lane;
                const bool item = i < K;
                // owner of item i: the last position lane whose first item is <= i.
                // Item i0's owner is the highest lane with excl <= i0; a lane whose
                // run starts inside the batch marks its first item, and a max-scan
                // over the marks carries each owner forward.
                const uint64_t started = __ballot(excl <= i0);
                const int carry = 63 - __builtin_clzll(started);
                L.head[lane] = -1;
                if (k > 0 && excl > i0 && excl < i0 + kEmitWave) L.head[excl - i0] = lane;
                wave_sync();
                const int own = max(carry, wave_scan_max(L.head[lane]));
                const int j = i - __shfl(excl, own);
                int xl, xh, yl, yh;
                unpack_range(__uint_as_float(L.rx[own]), xl, xh);
                unpack_range(__uint_as_float(L.ry[own]), yl, yh);
                const uint32_t g = L.rg[own];
                const int tx0 = max(xl >> sx, c0), ty0 = max(yl >> sy, r0);
                const int nx = min(xh >> sx, c1 - 1) - tx0 + 1;
                // j / nx as floor((j + 1/2) r) with r within one ulp of 1/nx:
                // exact for nx * ny <= 8160 (checked exhaustively on the host;
                // only groups of several tile rows divide)
                const int dy = kEmitRows == 1 ? 0 : (int)(((float)j + 0.5f) * __builtin_amdgcn_rcpf((float)nx));
                const int tx = tx0 + (j - dy * nx), ty = kEmitRows == 1 ? r0 : ty0 + dy;
                const int tc = kEmitRows == 1 ? tx - c0 : (ty - r0) * ncols + (tx - c0);
                const bool in = item && (unsigned)tc < (unsigned)ntiles;
                const int t = in ? tc : 0;
                const bool on = in && tile_on<kMasked>(L.act, t);
                const uint32_t val = g | (quad_mask(tx, ty, xl, xh, yl, yh, sx, sy) << 28);
                // Lanes on the same tile: each lane ORs its bit into its tile's
                // 64-bit LDS mask (cleared just before), then reads it back.
                // A lane's rank among them (lanes are in position order) is its
                // offset in the tile's run of entries; the lowest lane takes the
                // run from the tile's cursor.
                if (on) L.lanes[t] = 0ull;
                wave_sync();
                if (on) atomicOr((unsigned long long *)&L.lanes[t], 1ull << lane);
                wave_sync();
                const uint64_t same = on ? L.lanes[t] : 0ull;
                const int rank = __popcll(same & lanemask_lt64_bin());
                uint32_t base = 0;
                if (on && rank == 0) base = atomicAdd(&L.cur[t], (uint32_t)__popcll(same));
                const int lead = on ? __ffsll((long long)same) - 1 : lane;
                const uint32_t c = (uint32_t)__shfl((int)base, lead) + (uint32_t)rank;
                // The entries go into their tiles' lines one line at a time: in
                // step s every tile writes only within the s-th line its run
                // touches, and the lines whose last slot was filled are stored
                // before the next step reuses their slots.
                const uint32_t slot = (align + c) & (kLine - 1u);
                const int step = on ? (int)(((align + c - (uint32_t)rank) & (kLine - 1u)) + (uint32_t)rank) / kLine : -1;
                for (int s = 0; __ballot(step >= s) != 0ull; ++s) {
                    const bool now = step == s;
                    if (now) L.line[t * kLine + slot] = val;
                    const bool full = now && slot == kLine - 1u;
                    const uint64_t need = __ballot(full);
                    if (need) {
                        if (full) {
                            const int r = __popcll(need & lanemask_lt64_bin());
                            L.ft[r] = (uint32_t)t;
                            L.fc[r] = c;
                        }
                        wave_sync();
                        store_lines<kLine>(L, __popcll(need), align, vl, room);
                        wave_sync();
                    }
                }
                wave_sync();
            }
        }
        wave_sync();   // the queue is refilled by the next batch
    }
    // 3. the last, partly filled line of every tile whose segment ends inside one
    for (int t4 = 0; t4 < ntiles; t4 += kEmitWave) {
        const int t = t4 + lane;
        bool part = false;
        uint32_t c = 0;
        if (t < ntiles) {
            c = L.cur[t];
            part = c > L.seg0[t] && ((align + c) & (kLine - 1u)) != 0u;
        }
        const uint64_t need = __ballot(part);
        if (part) {
            const int r = __popcll(need & lanemask_lt64_bin());
            L.ft[r] = (uint32_t)t;
            L.fc[r] = c - 1u;       // the last entry; slots after it are not stored
        }
        wave_sync();
        const int n = __popcll(need);
        for (int f0 = 0; f0 < n; f0 += kEmitWave / kLine) {
            const int f = f0 + lane / kLine, k = lane % kLine;
            if (f < n) {
                const int tt = (int)L.ft[f];
                const uint32_t last = L.fc[f];
                const int64_t e = (int64_t)last - (int64_t)((align + last) & (kLine - 1u)) + k;
                if (e >= (int64_t)L.seg0[tt] && (uint64_t)e < room && e <= (int64_t)last)
                    store_entry<kLine>(L.line[tt * kLine + k], &vl[e]);
            }
        }
        wave_sync();
    }
}

void launch_bin_count(const ViewDev *views_dev, int Vc, int64_t N, int nchunks, const ChunkBufs &b,
                      const uint32_t *xr, const uint32_t *yr, int max_cells, hipStream_t st) {
    const int64_t run = 8 * kCountGroup;
    const int64_t blocks = ((int64_t)nchunks * Vc + run - 1) / run * run;
    static const bool lds_ok = [] {
        // views up to kMaxCellsPerView cells take more than 64 KiB of LDS
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_bin_count),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 kMaxCellsPerView * (int)sizeof(int32_t));
        if (e != hipSuccess) (void)hipGetLastError();
        return e == hipSuccess;
    }();
    (void)lds_ok;
    hipLaunchKernelGGL(k_bin_count, dim3((unsigned)blocks), dim3(kBinThreads), (size_t)max_cells * sizeof(int32_t),
                       st, views_dev, Vc, N, nchunks, b.nvis, xr, yr, b.bin_count, b.tile_active, b.rowbits,
                       b.rows_stride);
}

void launch_chunk_prefix(const ViewDev *views_dev, int Vc, int nchunks, const ChunkBufs &b, int max_tiles,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_chunk_prefix, dim3((unsigned)((max_tiles + kBinThreads - 1) / kBinThreads), (unsigned)Vc),
                       dim3(kBinThreads), 0, st, views_dev, nchunks, b.bin_count, b.tile_tot);
}

void launch_bin_emit(const ViewDev *views_dev, int Vc, int64_t N, int nchunks, const ChunkBufs &b,
                     const uint32_t *xr, const uint32_t *yr, const uint32_t *sorted_g, int max_tiles_x,
                     int max_tiles_y, uint64_t cap, int tile_shift_x, hipStream_t st) {
    const int row_groups = (max_tiles_y + kEmitRows - 1) / kEmitRows;
    const int col_groups = (max_tiles_x + kEmitCols - 1) / kEmitCols;
    const int64_t run = 8 * (int64_t)kEmitGroupChunks * row_groups * col_groups;
    const int64_t blocks = ((int64_t)row_groups * col_groups * nchunks * Vc + run - 1) / run * run;
    const int group_tiles = kEmitRows * std::min(max_tiles_x, kEmitCols);
    const int line_log = tile_shift_x >= 5 ? 4 : 3;
    const size_t lds = emit_lds_bytes(group_tiles, b.tile_active != nullptr, line_log);
    const dim3 grid((unsigned)blocks);
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, dim3(kEmitWave), lds, st, views_dev, Vc, N, nchunks, row_groups, col_groups,
                           b.nvis, xr, yr, sorted_g, b.bin_count, b.tile_off, b.lists, b.tile_active, cap,
                           group_tiles, b.rowbits, b.rows_stride);
    };
    if (b.tile_active)
        line_log == 4 ? go(k_bin_emit<true, 4>) : go(k_bin_emit<true, 3>);
    else
        line_log == 4 ? go(k_bin_emit<false, 4>) : go(k_bin_emit<false, 3>);
}

// Capacity guard for lists sized in advance (plans): if the counted entries
// exceed the capacity, flag it and empty every list of the scene so that no
// later kernel reads past the buffer.
// Plan guards.  A scene whose lists outgrow their capacity, or (with the
// three-pass depth sort) whose view's depth keys span 2^24 or more, gets
// empty lists this run (its output is zero) and raises the sticky flag.
__global__ void k_span_check(const uint32_t *__restrict__ kmin, int Vc, uint32_t *__restrict__ over,
                             uint32_t *__restrict__ flag) {
    bool bad = false;
    for (int v = threadIdx.x; v < Vc; v += blockDim.x)
        bad = bad || (kmin[Vc + v] >= kmin[v] && kmin[Vc + v] - kmin[v] >= 0xFFFFFFu);
    bad = __any(bad);
    if (threadIdx.x == 0) {
        *over = bad ? 1u : 0u;
        if (bad) atomicOr(flag, kGuardSpan);
    }
}
__global__ void k_guard_check(const uint64_t *__restrict__ tile_off, int64_t ntiles, uint64_t cap,
                              uint32_t *__restrict__ over, uint32_t *__restrict__ flag, int keep) {
    const bool o = tile_off[ntiles] > cap;
    *over = (o || (keep && *over)) ? 1u : 0u;
    if (o) atomicOr(flag, kGuardList);
}
__global__ void k_guard_apply(uint64_t *__restrict__ tile_off, int64_t ntiles, const uint32_t *__restrict__ over) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (*over && i <= ntiles) tile_off[i] = 0;
}
void launch_span_check(const uint32_t *kmin, int Vc, uint32_t *over, uint32_t *flag, hipStream_t st) {
    hipLaunchKernelGGL(k_span_check, dim3(1), dim3(64), 0, st, kmin, Vc, over, flag);
}
void launch_list_guard(uint64_t *tile_off, int64_t ntiles, uint64_t cap, uint32_t *over, uint32_t *flag, bool keep,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_guard_check, dim3(1), dim3(1), 0, st, tile_off, ntiles, cap, over, flag, keep ? 1 : 0);
    hipLaunchKernelGGL(k_guard_apply, dim3((unsigned)((ntiles + 256) / 256)), dim3(256), 0, st, tile_off, ntiles,
                       over);
}

// A tile is active when at least one of its rays is selected by the ray mask;
// inactive tiles get empty lists.  active[t] holds one bit per 8x8 quadrant
// (bit q: quadrant q, row-major inside the tile, holds a selected ray).  One
// wave per tile: lane L takes the pixels L, L + 64, ... of the tile (row-major),
// and the bits are OR-ed over the wave with a ballot per quadrant.
__global__ __launch_bounds__(64) void k_tile_active(const ViewDev *__restrict__ views,
                                                    const int32_t *__restrict__ tile_view,
                                                    const uint32_t *__restrict__ mask, uint16_t *__restrict__ active) {
    const int gt = blockIdx.x;
    const ViewDev &V = views[tile_view[gt]];
    const int tl = gt - V.tile_base;
    const int tx = tl % V.tiles_x, ty = tl / V.tiles_x;
    const int tw = 1 << V.tsx, area = tw << V.tsy, qlx = V.tsx - 3;
    uint32_t mine = 0u;    // quadrants of this lane's pixels that hold a selected ray
    for (int k = threadIdx.x; k < area; k += 64) {
        const int lx = k & (tw - 1), ly = k >> V.tsx;
        const int px = (tx << V.tsx) + lx, py = (ty << V.tsy) + ly;
        if (px < V.W && py < V.H) {
            const int64_t ray = V.ray_base + (int64_t)py * V.W + px;
            if ((mask[ray >> 5] >> (ray & 31)) & 1u) mine |= 1u << ((lx >> 3) + ((ly >> 3) << qlx));
        }
    }
    const int nq = 1 << (V.tsx + V.tsy - 6);
    uint32_t bits = 0u;
    for (int q = 0; q < nq; ++q) bits |= __any((mine >> q) & 1u) ? (1u << q) : 0u;
    if (threadIdx.x == 0) active[gt] = (uint16_t)bits;
}

void launch_tile_active(const ViewDev *views_dev, const int32_t *tile_view, int total_tiles, const uint32_t *mask,
                        uint16_t *active, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_active, dim3(total_tiles), dim3(64), 0, st, views_dev, tile_view, mask, active);
}

// Row y + 1 of view v's table: running counts of active tiles along tile row
// y; row 0 is all zeros (written by the thread of row 0).
__global__ __launch_bounds__(64) void k_tile_sat_rows(const ViewDev *__restrict__ views,
                                                      const uint16_t *__restrict__ active, uint32_t *__restrict__ sat) {
    const ViewDev &V = views[blockIdx.y];
    const int ty = blockIdx.x * 64 + threadIdx.x;
    if (ty >= V.tiles_y) return;
    const int stride = V.tiles_x + 1;
    uint32_t *S = sat + V.sat_base;
    if (ty == 0)
        for (int x = 0; x < stride; ++x) S[x] = 0u;
    uint32_t *row = S + (int64_t)(ty + 1) * stride;
    const uint16_t *a = active + V.tile_base + (int64_t)ty * V.tiles_x;
    uint32_t run = 0;
    row[0] = 0u;
    for (int x = 0; x < V.tiles_x; ++x) {
        run += a[x] ? 1u : 0u;
        row[x + 1] = run;
    }
}

// Column x of view v's table: running sums down the rows.
__global__ __launch_bounds__(64) void k_tile_sat_cols(const ViewDev *__restrict__ views, uint32_t *__restrict__ sat) {
    const ViewDev &V = views[blockIdx.y];
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int stride = V.tiles_x + 1;
    if (x >= stride) return;
    uint32_t *S = sat + V.sat_base;
    uint32_t run = 0;
    for (int y = 1; y <= V.tiles_y; ++y) {
        run += S[(int64_t)y * stride + x];
        S[(int64_t)y * stride + x] = run;
    }
}

__global__ __launch_bounds__(256) void k_quad_count(const uint16_t *__restrict__ active, int n,
                                                    uint32_t *__restrict__ qcnt) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < n) qcnt[t] = (uint32_t)__popc((unsigned)active[t]);
}

__global__ __launch_bounds__(256) void k_quad_write(const uint16_t *__restrict__ active, int n, int quad_log,
                                                    const uint64_t *__restrict__ qoff, uint32_t *__restrict__ qlist) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    const unsigned bits = active[t];
    uint64_t o = qoff[t];
    for (int q = 0; q < (1 << quad_log); ++q)
        if ((bits >> q) & 1u) qlist[o++] = (uint32_t)(((uint32_t)t << quad_log) + q);
}

void launch_quad_list(const uint16_t *active, int total_tiles, int quad_log, uint32_t *qcnt, uint64_t *qoff,
                      uint64_t *scan_tmp, uint32_t *qlist, hipStream_t st) {
    const unsigned blocks = (unsigned)((total_tiles + 255) / 256);
    hipLaunchKernelGGL(k_quad_count, dim3(blocks), dim3(256), 0, st, active, total_tiles, qcnt);
    scan_u32_to_u64_exclusive(qcnt, qoff, total_tiles, scan_tmp, st);
    hipLaunchKernelGGL(k_quad_write, dim3(blocks), dim3(256), 0, st, active, total_tiles, quad_log, qoff, qlist);
}

void launch_tile_sat(const ViewDev *views_dev, int Vc, int max_tx, int max_ty, const uint16_t *active, uint32_t *sat,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_tile_sat_rows, dim3((unsigned)((max_ty + 63) / 64), (unsigned)Vc), dim3(64), 0, st,
                       views_dev, active, sat);
    hipLaunchKernelGGL(k_tile_sat_cols, dim3((unsigned)((max_tx + 1 + 63) / 64), (unsigned)Vc), dim3(64), 0, st,
                       views_dev, sat);
}

}  // namespace gs
