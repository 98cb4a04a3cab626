// Host side of the C ABI declared in include/gs_coreset.h: argument checks,
// view chunking, scratch arenas and kernel sequencing.
#include "../../include/gs_coreset.h"
#include "gs_internal.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace gs;

namespace {

thread_local std::string g_last_error;
std::mutex g_lock;

gs_status fail(gs_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
gs_status fail(gs_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(GS_ERR_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                          \
    } while (0)

// Device memory of the library: hipMalloc / hipFree unless the caller
// registered an allocator (gs_set_allocator).  Each block remembers the
// allocator that produced it, so a change of allocator never frees a block
// with the wrong one.
struct Allocator {
    gs_alloc_fn alloc = nullptr;   // null: hipMalloc / hipFree
    gs_free_fn release = nullptr;
    void *ctx = nullptr;
};
Allocator g_allocator;

hipError_t dev_alloc(const Allocator &A, void **p, size_t bytes, hipStream_t st) {
    if (!A.alloc) return hipMalloc(p, bytes);
    *p = A.alloc(A.ctx, bytes, (void *)st);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
void dev_free(const Allocator &A, void *p, hipStream_t st) {
    if (!p) return;
    if (A.alloc)
        A.release(A.ctx, p, (void *)st);
    else
        (void)hipFree(p);
}

// Grow-only device arena, one per device and purpose.
struct Arena {
    void *base = nullptr;
    size_t cap = 0;
    int device = -1;
    Allocator from;                // allocator of base
};
constexpr int kMaxDevices = 16;
Arena g_work[kMaxDevices], g_lists[kMaxDevices], g_agg[kMaxDevices], g_compact[kMaxDevices];
// Device statistics of a call, at one address for all of its view chunks
// (the work arena is carved differently per chunk and may be reallocated).
Arena g_cnt[kMaxDevices];
// Recorded at the end of every call on the call's stream; the next call waits
// for it on its own stream, so the shared arenas are never used by two
// streams at once.
hipEvent_t g_done[kMaxDevices];

hipError_t order_after_previous(int dev, hipStream_t st) {
    if (!g_done[dev]) {
        hipError_t e = hipEventCreateWithFlags(&g_done[dev], hipEventDisableTiming);
        if (e != hipSuccess) return e;
        return hipSuccess;
    }
    return hipStreamWaitEvent(st, g_done[dev], 0);
}
hipError_t mark_done(int dev, hipStream_t st) { return hipEventRecord(g_done[dev], st); }

// Blocks are taken on the null stream: the arenas serve every stream, and a
// block is only released after the device has finished with it.
hipError_t arena_reserve(Arena &a, size_t bytes) {
    if (a.base && a.cap >= bytes) return hipSuccess;
    if (a.base) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        dev_free(a.from, a.base, nullptr);
        a.base = nullptr;
        a.cap = 0;
    }
    a.from = g_allocator;
    size_t want = std::max(bytes + bytes / 8, (size_t)1 << 20);
    hipError_t e = dev_alloc(a.from, &a.base, want, nullptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        e = dev_alloc(a.from, &a.base, bytes, nullptr);
        if (e != hipSuccess) {
            a.base = nullptr;
            return e;
        }
        want = bytes;
    }
    a.cap = want;
    return hipSuccess;
}

// Bump allocator over an arena (256-byte aligned sub-buffers).
struct Carve {
    char *p;
    size_t off = 0;
    explicit Carve(void *base) : p((char *)base) {}
    template <typename T>
    T *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T *r = (T *)(p + off);
        off += count * sizeof(T);
        return r;
    }
};

struct ChunkPlan {
    int v0, vc;                 // first view, views in chunk
    int64_t rays;               // rays in chunk
    int total_tiles;
};

struct Setup {
    int64_t N;
    int nchunks;
    int agg = GS_AGG_RAY;       // query granularity of the sensitivity pass
    int nq = 1;                 // queries per ray (3 for per-channel queries)
    bool compact = false;       // pass 1 leaves compacted quadrant lists for pass 2
    int tsx = kTileShiftDefault, tsy = kTileShiftDefault;   // binning tile 2^tsx x 2^tsy pixels
    int quad_log = 2 * kTileShiftDefault - 6;               // log2 of the 8x8 quadrants per tile
    std::vector<int> tiles_x, tiles_y;
    std::vector<int64_t> ray_base;
};

// Compaction ranges are cut at every ceil(tiles / kRangeSamples)-th tile.
constexpr int64_t kRangeSamples = 4096;

int chunk_max_rows(const Setup &S, const ChunkPlan &c) {
    int m = 1;
    for (int k = 0; k < c.vc; ++k) m = std::max(m, S.tiles_y[c.v0 + k]);
    return m;
}

size_t chunk_scratch_bytes(const Setup &S, const ChunkPlan &c) {
    const int64_t N = S.N;
    const int64_t nbins = (int64_t)c.total_tiles * S.nchunks;
    size_t b = 0;
    auto add = [&](size_t x) { b += ((x + 255) & ~(size_t)255); };
    add(sizeof(GeoRec) * (size_t)c.vc * N);          // records
    add(sizeof(float) * (size_t)c.vc * N);
    add(sizeof(uint2) * (size_t)c.vc * N);
    if (S.nq > 1) add(sizeof(float4) * (size_t)c.vc * N);   // channel colours
    for (int k = 0; k < 4; ++k) add(sizeof(uint32_t) * (size_t)c.vc * N);
    add(sizeof(uint32_t) * (size_t)radix_sort_scratch_words(N, c.vc));
    add(4 * sizeof(uint32_t) * (size_t)c.vc);
    add(4 * sizeof(uint32_t) * (size_t)c.vc * proj_blocks(N));
    add(sizeof(uint32_t) * nbins);
    add(sizeof(uint64_t) * (size_t)rowbits_words(c.vc, chunk_max_rows(S, c), S.nchunks));
    add(sizeof(uint32_t) * c.total_tiles);
    add(sizeof(uint64_t) * (c.total_tiles + 1));
    add(sizeof(uint64_t) * scan_tmp_elems(c.total_tiles + 1));
    add(sizeof(float) * (size_t)c.rays * S.nq);
    add(sizeof(uint64_t) * CNT_WORDS);
    add(sizeof(ViewDev) * c.vc);
    add(sizeof(int32_t) * c.total_tiles);
    const size_t quads = (size_t)c.total_tiles << S.quad_log;
    add(sizeof(uint16_t) * c.total_tiles);                  // tile activity
    add(sizeof(uint32_t) * 4 * (size_t)c.total_tiles);      // active-tile tables ((tx+1)(ty+1) <= 4 tx ty)
    add(sizeof(uint32_t) * (size_t)c.total_tiles);          // listed quadrants: per-tile counts,
    add(sizeof(uint64_t) * ((size_t)c.total_tiles + 1));    // their scan,
    add(sizeof(uint64_t) * scan_tmp_elems(c.total_tiles + 1));
    add(sizeof(uint32_t) * quads);                          // and the list
    add(sizeof(uint64_t) * (kRangeSamples + 2));            // sampled tile offsets (compaction ranges)
    add(sizeof(int32_t) * c.total_tiles);                   // tile -> scene slot
    add(sizeof(SceneSlot) + 256);                           // slot + work counter
    add(sizeof(double) * ((N + 4095) / 4096 + 2));
    add(sizeof(double) * 3 * quads);                        // objective partials
    add(sizeof(double) * (3 * (size_t)c.vc + 1));
    add(sizeof(uint32_t) * quads);                          // compacted entries per quadrant
    add(sizeof(double) * quads);                            // per-region A(Q)
    add(sizeof(double) * ((size_t)c.vc + 1));               // per-view A(Q), launch total
    if (S.agg == GS_AGG_IMAGE) add(sizeof(uint64_t) * (size_t)c.vc * N);   // per (view, Gaussian) shares
    if (S.agg == GS_AGG_SCENE) add(sizeof(uint64_t) * (size_t)N);          // per Gaussian shares
    return b + (64 << 10);  // slack for the per-buffer alignment
}

gs_status check_scene(const gs_scene *s) {
    if (!s) return fail(GS_ERR_INVALID_ARGUMENT, "scene is NULL");
    if (s->n < 1) return fail(GS_ERR_INVALID_ARGUMENT, "scene->n must be >= 1 (got %lld)", (long long)s->n);
    if (s->n >= (int64_t)kIndexMask)
        return fail(GS_ERR_UNSUPPORTED, "scene->n must be < 2^28 (got %lld)", (long long)s->n);
    if (s->sh_degree < 0 || s->sh_degree > 3)
        return fail(GS_ERR_INVALID_ARGUMENT, "sh_degree must be in 0..3 (got %d)", s->sh_degree);
    if (s->format != GS_ATTR_F32 && s->format != GS_ATTR_MIXED16)
        return fail(GS_ERR_INVALID_ARGUMENT, "unknown attribute format %d", s->format);
    if (!s->mean || !s->log_scale || !s->quat || !s->opacity || !s->sh)
        return fail(GS_ERR_INVALID_ARGUMENT, "scene attribute pointer is NULL");
    return GS_OK;
}

gs_status check_views(const gs_views *v, Setup &S) {
    if (!v) return fail(GS_ERR_INVALID_ARGUMENT, "views is NULL");
    if (v->n_views < 1) return fail(GS_ERR_INVALID_ARGUMENT, "n_views must be >= 1");
    if (!v->world_to_cam || !v->intrinsics || !v->size)
        return fail(GS_ERR_INVALID_ARGUMENT, "views array pointer is NULL");
    S.tiles_x.resize(v->n_views);
    S.tiles_y.resize(v->n_views);
    S.ray_base.resize(v->n_views + 1);
    S.ray_base[0] = 0;
    for (int i = 0; i < v->n_views; ++i) {
        const int W = v->size[2 * i], H = v->size[2 * i + 1];
        if (W < 1 || H < 1 || W > 16384 || H > 16384)
            return fail(GS_ERR_INVALID_ARGUMENT, "view %d: size %dx%d outside 1..16384", i, W, H);
        const double *in = v->intrinsics + 4 * i;
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(in[k])) return fail(GS_ERR_INVALID_ARGUMENT, "view %d: non-finite intrinsics", i);
        if (in[0] <= 0 || in[1] <= 0) return fail(GS_ERR_INVALID_ARGUMENT, "view %d: focal lengths must be > 0", i);
        for (int k = 0; k < 12; ++k)
            if (!std::isfinite(v->world_to_cam[12 * i + k]))
                return fail(GS_ERR_INVALID_ARGUMENT, "view %d: non-finite extrinsics", i);
        S.tiles_x[i] = (W + (1 << S.tsx) - 1) >> S.tsx;
        S.tiles_y[i] = (H + (1 << S.tsy) - 1) >> S.tsy;
        if ((int64_t)(S.tiles_x[i] + 1) * (S.tiles_y[i] + 1) > kMaxCellsPerView)
            return fail(GS_ERR_UNSUPPORTED,
                        "view %d: %dx%d needs more than %d cells ((tiles_x + 1)(tiles_y + 1)) with tiles of %dx%d",
                        i, W, H, kMaxCellsPerView, 1 << S.tsx, 1 << S.tsy);
        S.ray_base[i + 1] = S.ray_base[i] + (int64_t)W * H;
    }
    return GS_OK;
}

// Whether every view (already checked) stays within kMaxCellsPerView with
// tiles of 2^tsx x 2^tsy.
bool tiles_fit(const gs_views *v, int tsx, int tsy) {
    for (int i = 0; i < v->n_views; ++i) {
        const int64_t tx = (v->size[2 * i] + (1 << tsx) - 1) >> tsx, ty = (v->size[2 * i + 1] + (1 << tsy) - 1) >> tsy;
        if ((tx + 1) * (ty + 1) > kMaxCellsPerView) return false;
    }
    return true;
}

// log2 of a tile side (0 stands for 16), -1 for a side the kernels do not take.
int tile_shift(int side) {
    switch (side) {
        case 0: return kTileShiftDefault;
        case 8: return 3;
        case 16: return 4;
        case 32: return 5;
        default: return -1;
    }
}

gs_status check_params(const gs_params *p) {
    if (!p) return fail(GS_ERR_INVALID_ARGUMENT, "params is NULL");
    if (!(p->footprint_sigma > 0.0f) || !std::isfinite(p->footprint_sigma))
        return fail(GS_ERR_INVALID_ARGUMENT, "footprint_sigma must be > 0");
    if (!(p->dilation >= 0.0f) || !std::isfinite(p->dilation))
        return fail(GS_ERR_INVALID_ARGUMENT, "dilation must be >= 0");
    if (!(p->z_near > 0.0f) || !std::isfinite(p->z_near))
        return fail(GS_ERR_INVALID_ARGUMENT, "z_near must be finite and > 0");
    if (!(p->share_floor >= 0.0f) || !std::isfinite(p->share_floor))
        return fail(GS_ERR_INVALID_ARGUMENT, "share_floor must be >= 0");
    if (p->query_mode < GS_QUERY_RGBSUM || p->query_mode > GS_QUERY_CHANNEL)
        return fail(GS_ERR_INVALID_ARGUMENT, "unknown query_mode %d", p->query_mode);
    if (p->max_views_per_chunk < 0) return fail(GS_ERR_INVALID_ARGUMENT, "max_views_per_chunk must be >= 0");
    if (p->flags & ~GS_FLAG_COUNT_PAIRS) return fail(GS_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", p->flags);
    if (p->aggregate < GS_AGG_RAY || p->aggregate > GS_AGG_SCENE)
        return fail(GS_ERR_INVALID_ARGUMENT, "unknown aggregate %d", p->aggregate);
    if (p->aggregate != GS_AGG_RAY && (p->flags & GS_FLAG_COUNT_PAIRS))
        return fail(GS_ERR_UNSUPPORTED, "pair counting needs per-ray queries");
    if (p->ambiguous_rays && !(p->flags & GS_FLAG_COUNT_PAIRS))
        return fail(GS_ERR_INVALID_ARGUMENT, "ambiguous_rays needs GS_FLAG_COUNT_PAIRS");
    if (p->aggregate != GS_AGG_RAY && p->query_mode == GS_QUERY_CHANNEL)
        return fail(GS_ERR_UNSUPPORTED, "per-channel queries have no aggregated form (an aggregated query sums "
                                        "its channels: use GS_QUERY_RGBSUM)");
    const int tw = tile_shift(p->tile_w), th = tile_shift(p->tile_h);
    if (tw < 0 || th < 0)
        return fail(GS_ERR_INVALID_ARGUMENT, "tile %dx%d: each side must be 8, 16 or 32 (or 0 for 16)", p->tile_w,
                    p->tile_h);
    if (p->aggregate == GS_AGG_TILE && (tw < 4 || th < 4))
        return fail(GS_ERR_UNSUPPORTED,
                    "tile queries are 16x16 pixel tiles: they need binning tiles of 16 or 32 pixels per side");
    return GS_OK;
}

// Tile shapes gs_tune_tile chose, by size class: (log2 of the largest
// view's pixel count, log2 of N) -> (tsx, tsy).  Guarded by g_tile_lock.
std::mutex g_tile_lock;
std::map<std::pair<int, int>, std::pair<int, int>> g_tile_cache;

int log2_floor(int64_t x) {
    int k = 0;
    while (x > 1) {
        x >>= 1;
        ++k;
    }
    return k;
}

std::pair<int, int> size_class(const gs_views *v, int64_t n) {
    int64_t px = 1;
    if (v && v->size)
        for (int i = 0; i < v->n_views; ++i)
            px = std::max(px, (int64_t)std::max(v->size[2 * i], 1) * std::max(v->size[2 * i + 1], 1));
    return {log2_floor(px), log2_floor(std::max<int64_t>(n, 1))};
}

// The binning tile of a call, from checked parameters: tile_w = tile_h = 0
// takes the shape the tuner chose for this size class; if it has not run for
// it, 16 x 16, or 16 x 32 and then 32 x 32 for views whose 16 x 16 tiles
// would exceed the per-view limit (tile queries always take 16 x 16); a
// single 0 side stands for 16.
void setup_tiles(const gs_params *p, Setup &S, const gs_views *v = nullptr, int64_t n = 0) {
    S.tsx = tile_shift(p->tile_w);
    S.tsy = tile_shift(p->tile_h);
    if (p->tile_w == 0 && p->tile_h == 0) {
        std::lock_guard<std::mutex> lk(g_tile_lock);
        const auto it = g_tile_cache.find(size_class(v, n));
        if (it != g_tile_cache.end()) {
            S.tsx = it->second.first;
            S.tsy = it->second.second;
        } else if (v && v->size && v->n_views > 0) {
            static const int shapes[3][2] = {{4, 4}, {4, 5}, {5, 5}};
            for (const auto &sh : shapes)
                if (tiles_fit(v, sh[0], sh[1])) {
                    S.tsx = sh[0];
                    S.tsy = sh[1];
                    break;
                }
        }
        // (per-tile queries need sides of 16 or 32 pixels)
        if (p->aggregate == GS_AGG_TILE) {
            S.tsx = std::max(S.tsx, 4);
            S.tsy = std::max(S.tsy, 4);
        }
    }
    S.quad_log = S.tsx + S.tsy - 6;
}

// A size in GiB from the environment: false (and *bytes untouched) when the
// variable is unset, not a number, negative or not finite.
bool env_gib(const char *name, size_t *bytes) {
    const char *e = getenv(name);
    if (!e) return false;
    char *end = nullptr;
    const double g = strtod(e, &end);
    if (end == e || !std::isfinite(g) || g < 0.0 || g > 1.0e6) return false;
    *bytes = (size_t)(g * (double)(1ull << 30));
    return true;
}

size_t scratch_budget() {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = (size_t)16 << 30;
    }
    size_t budget = (size_t)(0.45 * (double)free_b);
    env_gib("GS_SCRATCH_GB", &budget);
    return std::max(budget, (size_t)256 << 20);
}

std::vector<ChunkPlan> plan_chunks(const gs_views *v, const Setup &S, const gs_params *p, size_t budget) {
    std::vector<ChunkPlan> out;
    int v0 = 0;
    while (v0 < v->n_views) {
        ChunkPlan c{v0, 0, 0, 0};
        while (v0 + c.vc < v->n_views) {
            const int i = v0 + c.vc;
            ChunkPlan t = c;
            t.vc += 1;
            t.rays += S.ray_base[i + 1] - S.ray_base[i];
            t.total_tiles += S.tiles_x[i] * S.tiles_y[i];
            if (c.vc > 0 && chunk_scratch_bytes(S, t) > budget) break;
            if (p->max_views_per_chunk > 0 && t.vc > p->max_views_per_chunk) break;
            if (t.vc > 65535) break;
            c = t;
        }
        out.push_back(c);
        v0 += c.vc;
    }
    return out;
}

struct Timer {
    hipEvent_t ev[8];
    bool on;
    explicit Timer(bool enable) : on(enable) {
        if (on)
            for (auto &e : ev) hipEventCreate(&e);
    }
    ~Timer() {
        if (on)
            for (auto &e : ev) hipEventDestroy(e);
    }
    void mark(int i, hipStream_t st) {
        if (on) hipEventRecord(ev[i], st);
    }
    float ms(int a, int b) {
        float t = 0;
        if (on) hipEventElapsedTime(&t, ev[a], ev[b]);
        return t;
    }
};

// Projection + sort + binning of one chunk.  Leaves the tile lists ready for
// the compositing kernels.  Synchronises once (to size the lists).
struct ChunkRun {
    ChunkBufs b{};
    SceneSlot host_slot{};
    SceneSlot *slot_dev = nullptr;
    int32_t *tile_scene = nullptr;
    uint32_t *work = nullptr;
    ViewDev *views_dev = nullptr;
    int32_t *tile_view = nullptr;
    uint32_t *sorted_g = nullptr;
    uint64_t *scan_tmp = nullptr;
    double *sum_tmp = nullptr;
    double *tile_sums = nullptr;
    double *view_sums = nullptr;
    double *tile_A = nullptr;      // aggregated queries: A(Q) per tile, per view (+ the launch total)
    double *view_A = nullptr;
    uint64_t *acc = nullptr;       // aggregated shares (fixed point); per list entry for tiles
    uint32_t *ccount = nullptr;    // entries pass 1 compacted per quadrant
    uint32_t *quad_list = nullptr; // ray-masked runs: the quadrants holding a selected ray
    int32_t n_listed = 0;
    int64_t n_entries = 0;
    int32_t passes = 4;            // 8-bit passes of the depth sort
    // Compositing launches: tiles [t0, t1) whose compacted lists start at
    // list entry `first` (their pool offsets are 4 (entry - first)).  One
    // range over every tile unless the compacted lists only fit in pieces.
    struct Range {
        int t0, t1;
        uint64_t first;
    };
    std::vector<Range> ranges;
};

gs_status run_front(const gs_scene *scene, const gs_views *views, const gs_params *p, const Setup &S,
                    const ChunkPlan &c, hipStream_t st, int dev, std::vector<ViewDev> &hv,
                    std::vector<int32_t> &htv, ChunkRun &r, Timer &tm, double *ms_acc, bool zero_counters,
                    uint32_t *sens_bits) {
    const int64_t N = S.N;
    const int64_t nbins = (int64_t)c.total_tiles * S.nchunks;
    size_t need = chunk_scratch_bytes(S, c);
    HIP_TRY(arena_reserve(g_work[dev], need));
    Carve cv(g_work[dev].base);
    ChunkBufs &b = r.b;
    b.R = cv.take<GeoRec>((size_t)c.vc * N);
    b.CB = cv.take<float>((size_t)c.vc * N);
    b.XY = cv.take<uint2>((size_t)c.vc * N);
    b.R3 = S.nq > 1 ? cv.take<float4>((size_t)c.vc * N) : nullptr;
    b.key0 = cv.take<uint32_t>((size_t)c.vc * N);
    b.val0 = cv.take<uint32_t>((size_t)c.vc * N);
    b.key1 = cv.take<uint32_t>((size_t)c.vc * N);
    b.val1 = cv.take<uint32_t>((size_t)c.vc * N);
    b.hist = cv.take<uint32_t>((size_t)radix_sort_scratch_words(N, c.vc));
    b.nvis = cv.take<uint32_t>(4 * (size_t)c.vc);
    b.cmax = b.nvis + c.vc;
    b.kmin = b.nvis + 2 * c.vc;
    b.proj_part = cv.take<uint32_t>(4 * (size_t)c.vc * proj_blocks(N));
    b.bin_count = cv.take<uint32_t>(nbins);
    b.rows_stride = chunk_max_rows(S, c);
    b.rowbits = cv.take<uint64_t>((size_t)rowbits_words(c.vc, b.rows_stride, S.nchunks));
    b.tile_tot = cv.take<uint32_t>(c.total_tiles);
    b.tile_off = cv.take<uint64_t>(c.total_tiles + 1);
    r.scan_tmp = cv.take<uint64_t>(scan_tmp_elems(c.total_tiles + 1));
    b.ray_A = cv.take<float>((size_t)c.rays * S.nq);
    HIP_TRY(arena_reserve(g_cnt[dev], sizeof(uint64_t) * CNT_WORDS));
    b.counters = (uint64_t *)g_cnt[dev].base;
    r.views_dev = cv.take<ViewDev>(c.vc);
    r.tile_view = cv.take<int32_t>(c.total_tiles);
    b.tile_active = p->ray_mask ? cv.take<uint16_t>(c.total_tiles) : nullptr;
    b.tile_sat = p->ray_mask ? cv.take<uint32_t>(4 * (size_t)c.total_tiles) : nullptr;
    uint32_t *qcnt = nullptr;
    uint64_t *qoff = nullptr, *qtmp = nullptr;
    r.quad_list = nullptr;
    r.n_listed = 0;
    if (p->ray_mask) {
        qcnt = cv.take<uint32_t>(c.total_tiles);
        qoff = cv.take<uint64_t>((size_t)c.total_tiles + 1);
        qtmp = cv.take<uint64_t>(scan_tmp_elems(c.total_tiles + 1));
        r.quad_list = cv.take<uint32_t>((size_t)c.total_tiles << S.quad_log);
    }
    uint64_t *off_samples = cv.take<uint64_t>(kRangeSamples + 2);
    r.tile_scene = cv.take<int32_t>(c.total_tiles);
    r.slot_dev = cv.take<SceneSlot>(1);
    r.work = cv.take<uint32_t>(64);
    r.sum_tmp = cv.take<double>((N + 4095) / 4096 + 2);
    r.tile_sums = cv.take<double>(3 * ((size_t)c.total_tiles << S.quad_log));
    r.view_sums = cv.take<double>(3 * (size_t)c.vc + 1);
    r.ccount = cv.take<uint32_t>((size_t)c.total_tiles << S.quad_log);
    r.tile_A = cv.take<double>((size_t)c.total_tiles << S.quad_log);
    r.view_A = cv.take<double>((size_t)c.vc + 1);
    r.acc = nullptr;
    if (S.agg == GS_AGG_IMAGE) r.acc = cv.take<uint64_t>((size_t)c.vc * N);
    if (S.agg == GS_AGG_SCENE) r.acc = cv.take<uint64_t>((size_t)N);

    hv.assign(c.vc, ViewDev{});
    htv.assign(c.total_tiles, 0);
    int tb = 0, sb = 0;
    for (int k = 0; k < c.vc; ++k) {
        const int i = c.v0 + k;
        ViewDev &V = hv[k];
        const double *P = views->world_to_cam + 12 * i;
        for (int a = 0; a < 3; ++a) {
            for (int bb = 0; bb < 3; ++bb) V.R[3 * a + bb] = P[4 * a + bb];
            V.t[a] = P[4 * a + 3];
        }
        for (int a = 0; a < 3; ++a) V.cam[a] = -(V.R[a] * V.t[0] + V.R[3 + a] * V.t[1] + V.R[6 + a] * V.t[2]);
        V.fx = views->intrinsics[4 * i];
        V.fy = views->intrinsics[4 * i + 1];
        V.cx = views->intrinsics[4 * i + 2];
        V.cy = views->intrinsics[4 * i + 3];
        V.W = views->size[2 * i];
        V.H = views->size[2 * i + 1];
        V.tiles_x = S.tiles_x[i];
        V.tiles_y = S.tiles_y[i];
        V.tsx = S.tsx;
        V.tsy = S.tsy;
        V.ray_base = S.ray_base[i];
        V.ray_local = S.ray_base[i] - S.ray_base[c.v0];
        V.tile_base = tb;
        V.sat_base = sb;
        for (int t = 0; t < V.tiles_x * V.tiles_y; ++t) htv[tb + t] = k;
        tb += V.tiles_x * V.tiles_y;
        sb += (V.tiles_x + 1) * (V.tiles_y + 1);
    }
    int max_tiles = 1, max_tx = 1, max_ty = 1, max_cells = 1;
    for (const ViewDev &V : hv) {
        max_tiles = std::max(max_tiles, V.tiles_x * V.tiles_y);
        max_cells = std::max(max_cells, (V.tiles_x + 1) * (V.tiles_y + 1));
        max_tx = std::max(max_tx, V.tiles_x);
        max_ty = std::max(max_ty, V.tiles_y);
    }
    HIP_TRY(hipMemcpyAsync(r.views_dev, hv.data(), sizeof(ViewDev) * c.vc, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(r.tile_view, htv.data(), sizeof(int32_t) * c.total_tiles, hipMemcpyHostToDevice, st));
    launch_fill_u32(b.nvis, 0u, 2 * (int64_t)c.vc, st);
    launch_fill_u32(b.bin_count, 0u, nbins, st);
    // every chunk projects every Gaussian, so the invalid count restarts per chunk
    if (zero_counters)
        launch_fill_u64(b.counters, 0ull, CNT_WORDS, st);
    else
        launch_fill_u64(b.counters + CNT_INVALID, 0ull, 1, st);

    SceneDev sd{scene->n, scene->sh_degree, scene->format, scene->mean, scene->log_scale,
                scene->quat, scene->opacity, scene->sh};
    ProjParams pp{p->footprint_sigma, p->dilation, p->z_near, p->query_mode};
    // ray-masked runs: which tiles hold a selected ray, as per-view tables
    // that projection uses to drop Gaussians meeting none of them
    if (b.tile_active) {
        launch_tile_active(r.views_dev, r.tile_view, c.total_tiles, p->ray_mask, b.tile_active, st);
        launch_tile_sat(r.views_dev, c.vc, max_tx, max_ty, b.tile_active, b.tile_sat, st);
        launch_quad_list(b.tile_active, c.total_tiles, S.quad_log, qcnt, qoff, qtmp, r.quad_list, st);
    }
    tm.mark(0, st);
    launch_project(sd, r.views_dev, c.vc, pp, b, st);
    HIP_TRY(hipGetLastError());
    tm.mark(1, st);
    // Three 8-bit passes suffice when every view's visible depth keys, less
    // the view's smallest, stay below 2^24 - 1 (depths within about a factor
    // of four: the float bits of a positive depth grow by 2^23 per octave).
    std::vector<uint32_t> kr(2 * (size_t)c.vc), nv(c.vc);
    HIP_TRY(hipMemcpyAsync(kr.data(), b.kmin, sizeof(uint32_t) * 2 * c.vc, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(nv.data(), b.nvis, sizeof(uint32_t) * c.vc, hipMemcpyDeviceToHost, st));
    uint64_t n_listed = 0;
    if (qoff)
        HIP_TRY(hipMemcpyAsync(&n_listed, qoff + c.total_tiles, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    r.n_listed = (int32_t)n_listed;
    uint32_t span = 0;
    for (int k = 0; k < c.vc; ++k)
        if (kr[c.vc + k] >= kr[k]) span = std::max(span, kr[c.vc + k] - kr[k]);
    const int passes = span < 0xFFFFFFu ? 3 : 4;
    r.passes = passes;
    uint32_t *skeys = nullptr;
    // When a quarter or more of the (view, Gaussian) pairs are dropped (ray
    // masks, views that see little of the scene) the kept keys are moved to
    // the front of each view's segment first and only they are sorted.
    uint64_t kept = 0;
    for (uint32_t x : nv) kept += x;
    if (4 * kept <= 3 * (uint64_t)N * (uint64_t)c.vc) {
        launch_key_compact(b, c.vc, N, b.key1, b.val1, st);
        HIP_TRY(radix_sort_segments(b.key1, b.val1, b.key0, b.val0, b.hist, N, c.vc, false, passes,
                                    passes == 3 ? b.kmin : nullptr, b.nvis, &skeys, &r.sorted_g, st));
    } else {
        HIP_TRY(radix_sort_segments(b.key0, b.val0, b.key1, b.val1, b.hist, N, c.vc, true, passes,
                                    passes == 3 ? b.kmin : nullptr, nullptr, &skeys, &r.sorted_g, st));
    }
    tm.mark(2, st);
    // the pair of sort buffers that does not hold the sorted output is free
    const bool out_in_0 = r.sorted_g == b.val0;
    uint32_t *xr = out_in_0 ? b.key1 : b.key0, *yr = out_in_0 ? b.val1 : b.val0;
    launch_ranges_in_order(r.sorted_g, b, c.vc, N, xr, yr, st);
    launch_bin_count(r.views_dev, c.vc, N, S.nchunks, b, xr, yr, max_cells, st);
    launch_chunk_prefix(r.views_dev, c.vc, S.nchunks, b, max_tiles, st);
    scan_u32_to_u64_exclusive(b.tile_tot, b.tile_off, c.total_tiles, r.scan_tmp, st);
    HIP_TRY(hipGetLastError());
    uint64_t total = 0;
    HIP_TRY(hipMemcpyAsync(&total, b.tile_off + c.total_tiles, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    r.n_entries = (int64_t)total;
    const size_t list_bytes = ((std::max<size_t>(total, 1) * sizeof(uint32_t) + 255) & ~(size_t)255);
    // per-tile queries keep one accumulator per list entry, after the lists
    const size_t acc_bytes = S.agg == GS_AGG_TILE ? std::max<size_t>(total, 1) * sizeof(uint64_t) : 0;
    HIP_TRY(arena_reserve(g_lists[dev], list_bytes + acc_bytes));
    b.lists = (uint32_t *)g_lists[dev].base;
    if (S.agg == GS_AGG_TILE) r.acc = (uint64_t *)((char *)g_lists[dev].base + list_bytes);
    // room for the quadrants' compacted lists (4 x the lists), if it fits in
    // half of the free memory; without it pass 2 filters the tile lists again
    // (when only part fits, the tiles are cut into ranges whose compacted
    // lists fit, composited one range after another through the same room)
    uint32_t *clist = nullptr;
    r.ranges.assign(1, ChunkRun::Range{0, c.total_tiles, 0});
    if (S.compact) {
        // each quadrant of a tile gets a region of the tile's list length
        const size_t cbytes = ((size_t)std::max<uint64_t>(total, 1) << S.quad_log) * sizeof(uint32_t);
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            free_b = 0;
        }
        const size_t held = g_compact[dev].cap;
        size_t avail = std::max(held, (free_b + held) / 2);
        env_gib("GS_COMPACT_POOL_GB", &avail);
        if (avail == 0) {
            // no room: pass 2 filters the tile lists itself
        } else if (cbytes <= avail) {
            if (arena_reserve(g_compact[dev], cbytes) == hipSuccess)
                clist = (uint32_t *)g_compact[dev].base;
            else
                (void)hipGetLastError();
        } else if (!r.quad_list && S.agg == GS_AGG_RAY) {
            // list offsets at every G-th tile: ranges are cut there
            const int64_t T = c.total_tiles;
            const int64_t G = (T + kRangeSamples - 1) / kRangeSamples;
            const int64_t K = (T + G - 1) / G;                      // blocks of G tiles
            std::vector<uint64_t> off((size_t)K + 1);
            launch_gather_u64(off_samples, b.tile_off, T, G, st);
            HIP_TRY(hipMemcpyAsync(off.data(), off_samples, sizeof(uint64_t) * off.size(), hipMemcpyDeviceToHost,
                                   st));
            HIP_TRY(hipStreamSynchronize(st));
            const uint64_t room = avail / (sizeof(uint32_t) << S.quad_log);   // list entries whose compacted lists fit
            uint64_t longest = 0;
            for (int64_t k = 0; k < K; ++k) longest = std::max(longest, off[k + 1] - off[k]);
            if (longest <= room && arena_reserve(g_compact[dev], avail) == hipSuccess) {
                clist = (uint32_t *)g_compact[dev].base;
                r.ranges.clear();
                int64_t k0 = 0;
                for (int64_t k = 0; k < K; ++k)
                    if (off[k + 1] - off[k0] > room) {
                        r.ranges.push_back(ChunkRun::Range{(int)(k0 * G), (int)(k * G), off[k0]});
                        k0 = k;
                    }
                r.ranges.push_back(ChunkRun::Range{(int)(k0 * G), (int)T, off[k0]});
            } else {
                (void)hipGetLastError();
            }
        }
    }
    tm.mark(6, st);
    launch_bin_emit(r.views_dev, c.vc, N, S.nchunks, b, xr, yr, r.sorted_g, max_tx, max_ty, (uint64_t)total, S.tsx,
                    st);
    HIP_TRY(hipGetLastError());
    tm.mark(7, st);

    // the compositing launch sees this chunk as a single scene slot
    r.host_slot = SceneSlot{b.R, b.CB, b.lists, b.tile_off, b.cmax, b.ray_A, sens_bits, p->ray_mask,
                            N, 0, 0, b.R3, c.rays, clist};
    HIP_TRY(hipMemcpyAsync(r.slot_dev, &r.host_slot, sizeof(SceneSlot), hipMemcpyHostToDevice, st));
    launch_fill_u32((uint32_t *)r.tile_scene, 0u, c.total_tiles, st);
    tm.mark(3, st);
    if (tm.on) {
        HIP_TRY(hipEventSynchronize(tm.ev[3]));
        ms_acc[0] += tm.ms(0, 1);
        ms_acc[1] += tm.ms(1, 2);
        ms_acc[2] += tm.ms(2, 6) + tm.ms(7, 3);   // binning around the emission, which has its own slot
        ms_acc[5] += tm.ms(6, 7);
    }
    return GS_OK;
}

CompositeArgs composite_args(const ChunkRun &r, int total_tiles, const gs_params *p, float share_floor,
                             const Setup &S) {
    CompositeArgs a{};
    a.quad_log = S.quad_log;
    a.clist_pos = S.agg == GS_AGG_TILE ? 1 : 0;
    a.region_log = region_log_of(S.tsx, S.tsy);
    a.views = r.views_dev;
    a.tile_view = r.tile_view;
    a.tile_scene = r.tile_scene;
    a.slots = r.slot_dev;
    a.total_tiles = total_tiles;
    a.query_mode = p->query_mode;
    a.r2_log2 = -0.5f * 1.4426950408889634f * p->footprint_sigma * p->footprint_sigma;
    a.share_floor = share_floor;
    a.work = nullptr;
    a.xcd_remap = 1;
    a.report_floor = share_floor > 0.0f ? std::nextafter(share_floor, 0.0f) : 0.0f;
    a.amb_rays = p->ambiguous_rays;
    return a;
}

struct DoneGuard {
    int dev;
    hipStream_t st;
    ~DoneGuard() {
        if (dev >= 0) (void)mark_done(dev, st);
    }
};

int current_device(gs_status *st) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *st = fail(GS_ERR_DEVICE, "no usable HIP device (device %d)", dev);
        return -1;
    }
    *st = GS_OK;
    return dev;
}

// Sampling without allocation: the inclusive CDF of the quanta lives in a
// file-scope device array instead of the scratch arena (the weights kernel
// recomputes each q_i from s_i).  Every GPU the library runs on holds its own
// copy for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress returns on that device.
constexpr int64_t kNoAllocMaxN = (int64_t)1 << 23;
constexpr int64_t kNoAllocTmp = (kNoAllocMaxN + 2047) / 2048 + 1;       // scan block partials
constexpr size_t kNoAllocBytes = sizeof(uint64_t) * (size_t)(kNoAllocMaxN + kNoAllocTmp) + 256;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];
void *g_noalloc_ptr[kMaxDevices];

// The calling device's copy of `scratch`, looked up once per device (with
// that device current).
gs_status noalloc_scratch(int dev, void **out) {
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GS_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return GS_OK;
}

}  // namespace

extern "C" {

void gs_default_params(gs_params *p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->footprint_sigma = 3.0f;
    p->dilation = 0.3f;
    p->z_near = 0.2f;
    p->share_floor = 1e-12f;
    p->query_mode = GS_QUERY_RGBSUM;
    p->max_views_per_chunk = 0;
    p->flags = 0;
    p->ray_mask = nullptr;
    p->aggregate = GS_AGG_RAY;
    p->tile_w = 16;
    p->tile_h = 16;
}

const char *gs_last_error(void) { return g_last_error.c_str(); }

const char *gs_status_string(gs_status s) {
    switch (s) {
        case GS_OK: return "ok";
        case GS_ERR_INVALID_ARGUMENT: return "invalid argument";
        case GS_ERR_UNSUPPORTED: return "unsupported";
        case GS_ERR_OUT_OF_MEMORY: return "out of memory";
        case GS_ERR_NO_POSITIVE_SENSITIVITY: return "no positive sensitivity";
        case GS_ERR_INVALID_DATA: return "invalid data";
        case GS_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

gs_status gs_release_workspace(void) {
    std::lock_guard<std::mutex> lk(g_lock);
    gs_status s;
    const int dev = current_device(&s);
    if (dev < 0) return s;
    HIP_TRY(hipDeviceSynchronize());
    for (Arena *a : {&g_work[dev], &g_lists[dev], &g_agg[dev], &g_compact[dev], &g_cnt[dev]}) {
        dev_free(a->from, a->base, nullptr);
        a->base = nullptr;
        a->cap = 0;
    }
    return GS_OK;
}

gs_status gs_set_allocator(gs_alloc_fn alloc, gs_free_fn release, void *ctx) {
    g_last_error.clear();
    if ((alloc == nullptr) != (release == nullptr))
        return fail(GS_ERR_INVALID_ARGUMENT, "give both an allocation and a release function, or neither");
    std::lock_guard<std::mutex> lk(g_lock);
    // every arena goes back to the allocator it came from (on its device)
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    for (int dev = 0; dev < kMaxDevices; ++dev) {
        Arena *arenas[] = {&g_work[dev], &g_lists[dev], &g_agg[dev], &g_compact[dev], &g_cnt[dev]};
        bool any = false;
        for (Arena *a : arenas) any = any || a->base;
        if (!any) continue;
        HIP_TRY(hipSetDevice(dev));
        HIP_TRY(hipDeviceSynchronize());
        for (Arena *a : arenas) {
            dev_free(a->from, a->base, nullptr);
            a->base = nullptr;
            a->cap = 0;
        }
    }
    HIP_TRY(hipSetDevice(cur));
    g_allocator = Allocator{alloc, release, ctx};
    return GS_OK;
}

gs_status gs_sensitivity(const gs_scene *scene, const gs_views *views, const gs_params *params, float *sens,
                         gs_stats *stats, void *stream) {
    g_last_error.clear();
    gs_status s;
    if ((s = check_scene(scene)) != GS_OK) return s;
    Setup S;
    if ((s = check_params(params)) != GS_OK) return s;
    setup_tiles(params, S, views, scene->n);
    if ((s = check_views(views, S)) != GS_OK) return s;
    if (!sens) return fail(GS_ERR_INVALID_ARGUMENT, "sens is NULL");
    std::lock_guard<std::mutex> lk(g_lock);
    const int dev = current_device(&s);
    if (dev < 0) return s;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(order_after_previous(dev, st));
    DoneGuard done_guard{dev, st};
    S.N = scene->n;
    S.nchunks = (int)((S.N + (1 << kChunkBits) - 1) >> kChunkBits);
    S.agg = params->aggregate;
    S.nq = params->query_mode == GS_QUERY_CHANNEL ? 3 : 1;
    // every granularity composites on compacted lists (per-tile queries keep
    // list positions in them: their accumulators are indexed by position)
    S.compact = true;
    const auto chunks = plan_chunks(views, S, params, scratch_budget());
    launch_fill_u32((uint32_t *)sens, 0u, S.N, st);
    // per-scene queries: the absolute contributions and A summed over chunks
    double *agg_num = nullptr, *agg_den = nullptr;
    if (S.agg == GS_AGG_SCENE) {
        const size_t nb = ((size_t)S.N * sizeof(double) + 255) & ~(size_t)255;
        HIP_TRY(arena_reserve(g_agg[dev], nb + 256));
        agg_num = (double *)g_agg[dev].base;
        agg_den = (double *)((char *)g_agg[dev].base + nb);
        launch_fill_u64((uint64_t *)agg_num, 0ull, S.N, st);
        launch_fill_u64((uint64_t *)agg_den, 0ull, 1, st);
    }
    HIP_TRY(hipGetLastError());
    Timer tm(stats != nullptr);
    double ms[6] = {0, 0, 0, 0, 0, 0};
    int64_t n_bins = 0;
    std::vector<ViewDev> hv;
    std::vector<int32_t> htv;
    int64_t entries = 0, projected = 0;
    int32_t sort_passes = 0;
    ChunkRun r;
    const float log2e = 1.4426950408889634f;
    for (size_t ci = 0; ci < chunks.size(); ++ci) {
        const ChunkPlan &c = chunks[ci];
        if ((s = run_front(scene, views, params, S, c, st, dev, hv, htv, r, tm, ms, ci == 0, (uint32_t *)sens)) !=
            GS_OK)
            return s;
        entries += r.n_entries;
        n_bins += (int64_t)c.total_tiles * S.nchunks;
        sort_passes = std::max(sort_passes, r.passes);
        CompositeArgs a = composite_args(r, c.total_tiles, params, params->share_floor, S);
        a.ccount = r.host_slot.clist ? r.ccount : nullptr;
        // (per-tile queries keep the quadrant lists only at 16x16 tiles: their
        // per-entry accumulators would mix a larger tile's four queries)
        if (r.quad_list && 4 * (int64_t)r.n_listed <= ((int64_t)c.total_tiles << S.quad_log) &&
            !(S.agg == GS_AGG_TILE && region_log_of(S.tsx, S.tsy) > 0)) {
            // a sparse mask (a quarter of the quadrants or fewer hold a
            // selected ray): only the listed quadrants are composited, one wave
            // each, and the other rays read A = 0; denser masks take the flat
            // launches, whose waves leave at once where no ray is selected
            launch_fill_u32((uint32_t *)r.b.ray_A, 0u, (int64_t)c.rays * S.nq, st);
            a.quad_list = r.quad_list;
            a.n_listed = r.n_listed;
        }
        // per-tile queries composited by regions (every region one whole
        // 16x16 query): the region lists hold Gaussians and pass 2 takes each
        // share's maximum itself, with no per-entry accumulators
        const bool tile_direct = S.agg == GS_AGG_TILE && a.ccount && !a.quad_list && !a.work;
        if (tile_direct) a.clist_pos = 0;
        if (S.agg == GS_AGG_TILE && !tile_direct && region_log_of(S.tsx, S.tsy) > 0)
            return fail(GS_ERR_UNSUPPORTED, "tile queries on binning tiles above 16x16 need the region form");
        if (r.ranges.size() > 1) {
            // per-ray queries through a compaction room that holds part of
            // the chunk's lists: pass 1 and pass 2 of one tile range after
            // another (each pass 2 reads what its pass 1 left in the room)
            std::vector<hipEvent_t> ev(tm.on ? 3 * r.ranges.size() : 0);
            for (hipEvent_t &e : ev) HIP_TRY(hipEventCreate(&e));
            for (size_t k = 0; k < r.ranges.size(); ++k) {
                const ChunkRun::Range &g = r.ranges[k];
                CompositeArgs ar = a;
                ar.tile_first = g.t0;
                ar.total_tiles = g.t1 - g.t0;
                ar.ccount = r.ccount + ((size_t)g.t0 << S.quad_log);
                ar.clist_shift = g.first << S.quad_log;
                if (tm.on) HIP_TRY(hipEventRecord(ev[3 * k], st));
                launch_composite_pass1(ar, st);
                if (tm.on) HIP_TRY(hipEventRecord(ev[3 * k + 1], st));
                launch_composite_pass2(ar, (params->flags & GS_FLAG_COUNT_PAIRS) != 0, r.b.counters, st);
                if (tm.on) HIP_TRY(hipEventRecord(ev[3 * k + 2], st));
                HIP_TRY(hipGetLastError());
            }
            if (tm.on) {
                HIP_TRY(hipEventSynchronize(ev.back()));
                for (size_t k = 0; k < r.ranges.size(); ++k) {
                    float t1 = 0.0f, t2 = 0.0f;
                    hipEventElapsedTime(&t1, ev[3 * k], ev[3 * k + 1]);
                    hipEventElapsedTime(&t2, ev[3 * k + 1], ev[3 * k + 2]);
                    ms[3] += t1;
                    ms[4] += t2;
                }
            }
            for (hipEvent_t &e : ev) hipEventDestroy(e);
            if (stats) {
                std::vector<uint32_t> nv(c.vc);
                HIP_TRY(hipMemcpyAsync(nv.data(), r.b.nvis, sizeof(uint32_t) * c.vc, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                for (uint32_t x : nv) projected += x;
            }
            continue;
        }
        tm.mark(3, st);
        launch_composite_pass1(a, st);
        HIP_TRY(hipGetLastError());
        tm.mark(4, st);
        if (S.agg != GS_AGG_RAY) {
            double *total = r.view_A + c.vc;
            launch_query_sums(a, c.vc, r.tile_A, r.view_A, S.agg == GS_AGG_SCENE ? total : nullptr, st);
            a.agg = S.agg;
            a.query_A = S.agg == GS_AGG_TILE ? r.tile_A : (S.agg == GS_AGG_IMAGE ? r.view_A : total);
            a.acc = r.acc;
            const int64_t n_acc = S.agg == GS_AGG_TILE ? std::max<int64_t>(r.n_entries, 1)
                                                       : (S.agg == GS_AGG_IMAGE ? (int64_t)c.vc * S.N : S.N);
            if (!tile_direct) launch_fill_u64(r.acc, 0ull, n_acc, st);
        }
        launch_composite_pass2(a, (params->flags & GS_FLAG_COUNT_PAIRS) != 0, r.b.counters, st);
        HIP_TRY(hipGetLastError());
        if (S.agg != GS_AGG_RAY && !tile_direct) {
            launch_agg_finalize(S.agg, r.acc, r.b.lists, (uint64_t)r.n_entries, S.N, c.vc, (uint32_t *)sens,
                                agg_num, agg_den, r.view_A + c.vc, st);
            HIP_TRY(hipGetLastError());
        }
        tm.mark(5, st);
        if (stats) {
            std::vector<uint32_t> nv(c.vc);
            HIP_TRY(hipMemcpyAsync(nv.data(), r.b.nvis, sizeof(uint32_t) * c.vc, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            for (uint32_t x : nv) projected += x;
            ms[3] += tm.ms(3, 4);
            ms[4] += tm.ms(4, 5);
        }
    }
    if (S.agg == GS_AGG_SCENE) {
        launch_div_f64_to_f32(agg_num, agg_den, S.N, sens, st);
        HIP_TRY(hipGetLastError());
    }
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        double S_total = 0.0;
        uint64_t cnt[CNT_WORDS];
        launch_sum_f32_to_f64(sens, S.N, r.sum_tmp + (S.N + 4095) / 4096, r.sum_tmp, st);
        HIP_TRY(hipMemcpyAsync(&S_total, r.sum_tmp + (S.N + 4095) / 4096, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(cnt, r.b.counters, sizeof(cnt), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        stats->n_projected = projected;
        stats->n_entries = entries;
        uint64_t spread[kCntSpreadKinds] = {};
        for (int k = 0; k < kCntSpreadKinds; ++k)
            for (int i = 0; i < kCntSpread; ++i) spread[k] += cnt[CNT_SLOTS + k * kCntSpread + i];
        stats->n_pairs = (int64_t)spread[0];
        stats->n_live_pairs = (int64_t)spread[1];
        stats->n_rays_positive = (int64_t)spread[2];
        stats->n_lane_pairs = (int64_t)spread[3];
        stats->n_invalid_gaussians = (int64_t)cnt[CNT_INVALID];
        stats->total_sensitivity = S_total;
        stats->ms_project = ms[0];
        stats->ms_sort = ms[1];
        stats->ms_bin = ms[2];
        stats->ms_pass1 = ms[3];
        stats->ms_pass2 = ms[4];
        stats->ms_emit = ms[5];
        stats->n_bins = n_bins;
        stats->sort_passes = sort_passes;
        stats->n_ambiguous_keys = (int64_t)cnt[CNT_AMB_KEYS];
        stats->n_ambiguous_pairs = (int64_t)spread[4];
        if (cnt[CNT_INVALID]) return fail(GS_ERR_INVALID_DATA, "%llu Gaussians have non-finite attributes",
                                          (unsigned long long)cnt[CNT_INVALID]);
    }
    return GS_OK;
}

gs_status gs_render_objective(const gs_scene *scene, const gs_views *views, const gs_params *params,
                              const double *weights, int32_t objective, float *per_ray, double *per_view,
                              gs_render_diag *diag, void *stream) {
    g_last_error.clear();
    gs_status s;
    if ((s = check_scene(scene)) != GS_OK) return s;
    Setup S;
    if ((s = check_params(params)) != GS_OK) return s;
    setup_tiles(params, S, views, scene->n);
    if ((s = check_views(views, S)) != GS_OK) return s;
    if (objective != GS_OBJ_FULL && objective != GS_OBJ_FIXED && objective != GS_OBJ_TRUE)
        return fail(GS_ERR_INVALID_ARGUMENT, "unknown objective %d", objective);
    if (objective != GS_OBJ_FULL && !weights)
        return fail(GS_ERR_INVALID_ARGUMENT, "weights are required for the fixed and true objectives");
    if (params->query_mode == GS_QUERY_CHANNEL)
        return fail(GS_ERR_UNSUPPORTED, "the objectives hold one query per ray (no per-channel queries)");
    if (params->ambiguous_rays) return fail(GS_ERR_INVALID_ARGUMENT, "ambiguous_rays is for gs_sensitivity");
    std::lock_guard<std::mutex> lk(g_lock);
    const int dev = current_device(&s);
    if (dev < 0) return s;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(order_after_previous(dev, st));
    DoneGuard done_guard{dev, st};
    S.N = scene->n;
    S.nchunks = (int)((S.N + (1 << kChunkBits) - 1) >> kChunkBits);
    const auto chunks = plan_chunks(views, S, params, scratch_budget());
    Timer tm(false);
    double ms[6] = {0, 0, 0, 0, 0, 0};
    std::vector<ViewDev> hv;
    std::vector<int32_t> htv;
    ChunkRun r;
    const float log2e = 1.4426950408889634f;
    uint64_t inv_total = 0;
    uint32_t gamma_bits = 0;
    for (size_t ci = 0; ci < chunks.size(); ++ci) {
        const ChunkPlan &c = chunks[ci];
        if ((s = run_front(scene, views, params, S, c, st, dev, hv, htv, r, tm, ms, true, nullptr)) != GS_OK)
            return s;
        CompositeArgs a = composite_args(r, c.total_tiles, params, 0.0f, S);
        ObjectiveArgs o{weights, objective, per_ray, r.tile_sums, nullptr, 1e-9f};
        if (r.quad_list) {
            // only the listed quadrants are rendered: the chunk's other rays read 0
            if (per_ray) launch_fill_u32((uint32_t *)(per_ray + S.ray_base[c.v0]), 0u, (int64_t)c.rays, st);
            a.quad_list = r.quad_list;
            a.n_listed = r.n_listed;
        }
        if (objective != GS_OBJ_TRUE) {
            // w_max (1 without weights) bounds every later fixed-objective term
            uint64_t *wmax = (uint64_t *)(r.view_sums + 3 * (size_t)c.vc);
            if (weights) {
                launch_max_f64(weights, S.N, wmax, st);
            } else {
                const double one = 1.0;
                uint64_t bits;
                memcpy(&bits, &one, sizeof bits);
                launch_fill_u64(wmax, bits, 1, st);
            }
            o.wmax_bits = wmax;
        }
        launch_fill_u64((uint64_t *)r.tile_sums, 0ull, 3 * ((int64_t)c.total_tiles << S.quad_log), st);
        launch_objective(a, o, r.b.counters, st);
        HIP_TRY(hipGetLastError());
        if (per_view) {
            launch_view_sums(r.tile_sums, r.views_dev, c.vc, S.quad_log, per_view + 3 * (int64_t)c.v0, st);
            HIP_TRY(hipGetLastError());
        }
        if (diag) {
            uint64_t cnt[CNT_SLOTS];
            HIP_TRY(hipMemcpyAsync(cnt, r.b.counters, sizeof(cnt), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            inv_total += cnt[CNT_INVALID_PAIRS];
            gamma_bits = std::max(gamma_bits, (uint32_t)cnt[CNT_GAMMA_BITS]);
        }
    }
    if (diag) {
        diag->n_invalid_pairs = (int64_t)inv_total;
        float g;
        memcpy(&g, &gamma_bits, sizeof g);
        diag->gamma_max = g;
    }
    return GS_OK;
}

gs_status gs_sample_coreset(const float *sens, int64_t n, int64_t m, uint64_t seed, uint32_t *counts,
                            double *weights, int64_t *support, void *stream) {
    g_last_error.clear();
    if (!sens || !counts || !weights || !support) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n < 1) return fail(GS_ERR_INVALID_ARGUMENT, "n must be >= 1");
    if (n > kSampleMaxN) return fail(GS_ERR_UNSUPPORTED, "n must be <= 2^24 - 2^16 so that Q fits 64 bits");
    if (m < 1) return fail(GS_ERR_INVALID_ARGUMENT, "m must be >= 1");
    if (m >= ((int64_t)1 << 31)) return fail(GS_ERR_UNSUPPORTED, "m must be < 2^31");
    std::lock_guard<std::mutex> lk(g_lock);
    gs_status s;
    const int dev = current_device(&s);
    if (dev < 0) return s;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(order_after_previous(dev, st));
    DoneGuard done_guard{dev, st};
    const size_t need = 2 * sizeof(uint64_t) * (size_t)n + sizeof(uint64_t) * (scan_tmp_elems(n) + 2) + 2048;
    HIP_TRY(arena_reserve(g_work[dev], need));
    Carve cv(g_work[dev].base);
    uint64_t *q = cv.take<uint64_t>(n);
    uint64_t *C = cv.take<uint64_t>(n);
    uint64_t *tmp = cv.take<uint64_t>(scan_tmp_elems(n) + 2);
    uint32_t *bad = cv.take<uint32_t>(64);
    launch_fill_u32(bad, 0u, 1, st);
    launch_quantize(sens, n, q, bad, st);
    scan_u64_inclusive(q, C, n, tmp, st);
    launch_fill_u32(counts, 0u, n, st);
    launch_fill_u64((uint64_t *)weights, 0ull, n, st);
    launch_fill_u64((uint64_t *)support, 0ull, 1, st);
    HIP_TRY(hipGetLastError());
    uint64_t Q = 0;
    uint32_t hbad = 0;
    HIP_TRY(hipMemcpyAsync(&Q, C + n - 1, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hbad) return fail(GS_ERR_INVALID_DATA, "a sensitivity is outside [0, 1 + 2^-10] or NaN");
    if (Q == 0) return fail(GS_ERR_NO_POSITIVE_SENSITIVITY, "every sensitivity is 0");
    launch_draws(C, n, m, seed, counts, st);
    launch_weights(counts, q, sens, C, n, m, weights, support, st);
    HIP_TRY(hipGetLastError());
    return GS_OK;
}

// ---------------------------------------------------------------------------
// Learned proposal.
constexpr int64_t kMlpRows = 65536;

gs_status gs_sample_coreset_noalloc(const float *sens, int64_t n, int64_t m, uint64_t seed, uint32_t *counts,
                                    double *weights, int64_t *support, void *stream) {
    g_last_error.clear();
    if (!sens || !counts || !weights || !support) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n < 1) return fail(GS_ERR_INVALID_ARGUMENT, "n must be >= 1");
    if (n > kNoAllocMaxN)
        return fail(GS_ERR_UNSUPPORTED, "n = %lld exceeds the %lld Gaussians the allocation-free sampler's fixed "
                                        "scratch holds (use gs_sample_coreset)",
                    (long long)n, (long long)kNoAllocMaxN);
    if (m < 1) return fail(GS_ERR_INVALID_ARGUMENT, "m must be >= 1");
    if (m >= ((int64_t)1 << 31)) return fail(GS_ERR_UNSUPPORTED, "m must be < 2^31");
    std::lock_guard<std::mutex> lk(g_lock);
    gs_status s;
    const int dev = current_device(&s);
    if (dev < 0) return s;
    void *base = nullptr;
    if ((s = noalloc_scratch(dev, &base)) != GS_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    uint64_t *C = (uint64_t *)base;
    uint64_t *tmp = C + kNoAllocMaxN;
    uint32_t *bad = (uint32_t *)(tmp + kNoAllocTmp);
    // the array keeps the previous call's contents: the flag starts at zero,
    // and every C entry used is written (quanta, then their prefix sums)
    // before it is read
    launch_fill_u32(bad, 0u, 1, st);
    launch_quantize(sens, n, C, bad, st);
    scan_u64_inclusive_inplace(C, n, tmp, st);
    launch_fill_u32(counts, 0u, n, st);
    launch_fill_u64((uint64_t *)weights, 0ull, n, st);
    launch_fill_u64((uint64_t *)support, 0ull, 1, st);
    HIP_TRY(hipGetLastError());
    uint64_t Q = 0;
    uint32_t hbad = 0;
    HIP_TRY(hipMemcpyAsync(&Q, C + n - 1, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hbad) return fail(GS_ERR_INVALID_DATA, "a sensitivity is outside [0, 1 + 2^-10] or NaN");
    if (Q == 0) return fail(GS_ERR_NO_POSITIVE_SENSITIVITY, "every sensitivity is 0");
    launch_draws(C, n, m, seed, counts, st);
    launch_weights(counts, nullptr, sens, C, n, m, weights, support, st);
    HIP_TRY(hipGetLastError());
    return GS_OK;
}

int64_t gs_mlp_param_count(void) { return kMlpParams; }

static gs_status begin_call(int *dev_out, hipStream_t st) {
    gs_status s;
    const int dev = current_device(&s);
    if (dev < 0) return s;
    HIP_TRY(order_after_previous(dev, st));
    *dev_out = dev;
    return GS_OK;
}

gs_status gs_mlp_init(float *params, uint64_t seed, void *stream) {
    g_last_error.clear();
    if (!params) return fail(GS_ERR_INVALID_ARGUMENT, "params is NULL");
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    gs_status s = begin_call(&dev, st);
    if (s != GS_OK) return s;
    DoneGuard done_guard{dev, st};
    mlp_init(params, seed, st);
    HIP_TRY(hipGetLastError());
    return GS_OK;
}

gs_status gs_features(const gs_scene *scene, float *features, void *stream) {
    g_last_error.clear();
    gs_status s;
    if ((s = check_scene(scene)) != GS_OK) return s;
    if (!features) return fail(GS_ERR_INVALID_ARGUMENT, "features is NULL");
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    if ((s = begin_call(&dev, st)) != GS_OK) return s;
    DoneGuard done_guard{dev, st};
    HIP_TRY(arena_reserve(g_work[dev], knn_scratch_bytes(scene->n)));
    SceneDev sd{scene->n, scene->sh_degree, scene->format, scene->mean, scene->log_scale,
                scene->quat, scene->opacity, scene->sh};
    HIP_TRY(knn_features(sd, features, g_work[dev].base, st));
    return GS_OK;
}

gs_status gs_coreset_error(const double *per_view, int32_t n_views, double *out, void *stream) {
    g_last_error.clear();
    if (!per_view || !out) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n_views < 1) return fail(GS_ERR_INVALID_ARGUMENT, "n_views must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    launch_coreset_error(per_view, n_views, out, st);
    HIP_TRY(hipGetLastError());
    return GS_OK;
}

// Compact-region extension: host-side pose metric and greedy rho-net.
static void pose_centre(const double *M, double c[3]) {
    for (int a = 0; a < 3; ++a) c[a] = -(M[a] * M[3] + M[4 + a] * M[7] + M[8 + a] * M[11]);
}
// Angle of Ra Rb^T from its skew part (sine) and trace (cosine).
static double pose_angle(const double *Ma, const double *Mb) {
    double R[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) R[r][c] = Ma[4 * r] * Mb[4 * c] + Ma[4 * r + 1] * Mb[4 * c + 1] + Ma[4 * r + 2] * Mb[4 * c + 2];
    const double sx = R[2][1] - R[1][2], sy = R[0][2] - R[2][0], sz = R[1][0] - R[0][1];
    const double sn = 0.5 * std::sqrt(sx * sx + sy * sy + sz * sz);
    const double cs = 0.5 * (R[0][0] + R[1][1] + R[2][2] - 1.0);
    return std::atan2(sn, cs);
}

gs_status gs_region_bound(const double *world_to_cam, int32_t n_poses, double lambda, double rho_target,
                          const float *A, const float *A_w, int64_t n_pixels, float a_floor, int32_t *is_net,
                          gs_region_report *report, void *stream) {
    g_last_error.clear();
    if (!world_to_cam || !A || !A_w || !is_net || !report) return fail(GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (n_poses < 2 || n_poses > 4096) return fail(GS_ERR_INVALID_ARGUMENT, "n_poses must be in 2..4096");
    if (n_pixels < 1) return fail(GS_ERR_INVALID_ARGUMENT, "n_pixels must be >= 1");
    if (!(lambda >= 0.0) || !(rho_target >= 0.0) || !std::isfinite(lambda) || !std::isfinite(rho_target))
        return fail(GS_ERR_INVALID_ARGUMENT, "lambda and rho_target must be finite and >= 0");
    if (!(a_floor >= 0.0f)) return fail(GS_ERR_INVALID_ARGUMENT, "a_floor must be >= 0");
    for (int64_t i = 0; i < 12 * (int64_t)n_poses; ++i)
        if (!std::isfinite(world_to_cam[i])) return fail(GS_ERR_INVALID_ARGUMENT, "non-finite pose");
    const int K = n_poses;
    // pose distances and the greedy net (first pose, then the farthest one)
    std::vector<double> D((size_t)K * K, 0.0), cen((size_t)3 * K);
    for (int i = 0; i < K; ++i) pose_centre(world_to_cam + 12 * i, &cen[3 * i]);
    for (int i = 0; i < K; ++i)
        for (int j = i + 1; j < K; ++j) {
            const double dx = cen[3 * i] - cen[3 * j], dy = cen[3 * i + 1] - cen[3 * j + 1];
            const double dz = cen[3 * i + 2] - cen[3 * j + 2];
            const double d = std::sqrt(dx * dx + dy * dy + dz * dz) +
                             lambda * pose_angle(world_to_cam + 12 * i, world_to_cam + 12 * j);
            D[(size_t)i * K + j] = D[(size_t)j * K + i] = d;
        }
    std::vector<double> near(D.begin(), D.begin() + K);
    std::fill(is_net, is_net + K, 0);
    is_net[0] = 1;
    int n_net = 1;
    for (;;) {
        int far = 0;
        for (int k = 1; k < K; ++k)
            if (near[k] > near[far]) far = k;
        if (near[far] <= rho_target) break;
        is_net[far] = 1;
        ++n_net;
        for (int k = 0; k < K; ++k) near[k] = std::min(near[k], D[(size_t)far * K + k]);
    }
    double rho = 0.0;
    for (int k = 0; k < K; ++k) rho = std::max(rho, near[k]);
    std::vector<int32_t> pi, pj;
    for (int i = 0; i < K; ++i)
        for (int j = i + 1; j < K; ++j) {
            pi.push_back(i);
            pj.push_back(j);
        }
    const int npairs = (int)pi.size();
    std::lock_guard<std::mutex> lk(g_lock);
    gs_status s;
    const int dev = current_device(&s);
    if (dev < 0) return s;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(order_after_previous(dev, st));
    DoneGuard done_guard{dev, st};
    const size_t need = (size_t)n_pixels + 4 * sizeof(int32_t) * (size_t)(K + 2 * npairs) +
                        2 * sizeof(float) * (size_t)npairs + 8192;
    HIP_TRY(arena_reserve(g_work[dev], need));
    Carve cv(g_work[dev].base);
    uint8_t *keep = cv.take<uint8_t>((size_t)n_pixels);
    int32_t *net_d = cv.take<int32_t>(K);
    int32_t *pi_d = cv.take<int32_t>(npairs);
    int32_t *pj_d = cv.take<int32_t>(npairs);
    float *diff = cv.take<float>(2 * (size_t)npairs);
    uint32_t *bits = cv.take<uint32_t>(64);
    HIP_TRY(hipMemcpyAsync(net_d, is_net, sizeof(int32_t) * K, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pi_d, pi.data(), sizeof(int32_t) * npairs, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pj_d, pj.data(), sizeof(int32_t) * npairs, hipMemcpyHostToDevice, st));
    launch_fill_u32(bits, 0x7F800000u, 1, st);     // +inf
    launch_fill_u32(bits + 1, 0u, 3, st);
    launch_region_pixels(A, A_w, K, n_pixels, a_floor, net_d, keep, bits, st);
    launch_region_pairs(A, A_w, K, n_pixels, keep, pi_d, pj_d, npairs, diff, st);
    HIP_TRY(hipGetLastError());
    std::vector<float> hd(2 * (size_t)npairs);
    uint32_t hb[4];
    HIP_TRY(hipMemcpyAsync(hd.data(), diff, sizeof(float) * hd.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hb, bits, sizeof hb, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    gs_region_report R{};
    R.n_pixels = hb[3];
    R.n_net = n_net;
    R.rho = rho;
    for (int q = 0; q < npairs; ++q) {
        const double d = D[(size_t)pi[q] * K + pj[q]];
        if (d > 0.0) {
            R.L_full = std::max(R.L_full, (double)hd[2 * q] / d);
            R.L_w = std::max(R.L_w, (double)hd[2 * q + 1] / d);
        }
    }
    float f;
    memcpy(&f, &hb[0], 4);
    R.A_min = hb[3] ? (double)f : 0.0;
    memcpy(&f, &hb[1], 4);
    R.eps_0 = f;
    memcpy(&f, &hb[2], 4);
    R.max_err = f;
    R.eps_reg = R.A_min > 0.0 ? R.eps_0 + ((1.0 + R.eps_0) * R.L_full + R.L_w) * R.rho / R.A_min : INFINITY;
    *report = R;
    if (!hb[3]) return fail(GS_ERR_NO_POSITIVE_SENSITIVITY, "no pixel has A above the floor at every pose");
    return GS_OK;
}

gs_status gs_knn(const gs_scene *scene, uint32_t *neighbours, float *sq_dist, void *stream) {
    g_last_error.clear();
    gs_status s;
    if ((s = check_scene(scene)) != GS_OK) return s;
    if (!neighbours || !sq_dist) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    if ((s = begin_call(&dev, st)) != GS_OK) return s;
    DoneGuard done_guard{dev, st};
    HIP_TRY(arena_reserve(g_work[dev], knn_scratch_bytes(scene->n)));
    SceneDev sd{scene->n, scene->sh_degree, scene->format, scene->mean, scene->log_scale,
                scene->quat, scene->opacity, scene->sh};
    HIP_TRY(knn_features(sd, nullptr, g_work[dev].base, st, neighbours, sq_dist));
    return GS_OK;
}

gs_status gs_feature_stats(const float *features, int64_t n, float *norm, void *stream) {
    g_last_error.clear();
    if (!features || !norm) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n < 1) return fail(GS_ERR_INVALID_ARGUMENT, "n must be >= 1");
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    gs_status s = begin_call(&dev, st);
    if (s != GS_OK) return s;
    DoneGuard done_guard{dev, st};
    feature_stats(features, n, norm, st);
    HIP_TRY(hipGetLastError());
    return GS_OK;
}

gs_status gs_proposal_mixture(const float *log_s, int64_t n, float floor, float *p, void *stream) {
    g_last_error.clear();
    if (!log_s || !p) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n < 1) return fail(GS_ERR_INVALID_ARGUMENT, "n must be >= 1");
    if (!(floor > 0.0f && floor <= 1.0f)) return fail(GS_ERR_INVALID_ARGUMENT, "floor must be in (0, 1]");
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    gs_status s = begin_call(&dev, st);
    if (s != GS_OK) return s;
    DoneGuard done_guard{dev, st};
    HIP_TRY(arena_reserve(g_work[dev], mixture_scratch_bytes(n)));
    proposal_mixture(log_s, n, floor, p, g_work[dev].base, st);
    HIP_TRY(hipGetLastError());
    return GS_OK;
}

gs_status gs_log_targets(const float *sens, int64_t n, float floor, float *out, void *stream) {
    g_last_error.clear();
    if (!sens || !out) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n < 1) return fail(GS_ERR_INVALID_ARGUMENT, "n must be >= 1");
    if (!(floor > 0.0f) || !std::isfinite(floor)) return fail(GS_ERR_INVALID_ARGUMENT, "floor must be > 0");
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    gs_status s = begin_call(&dev, st);
    if (s != GS_OK) return s;
    DoneGuard done_guard{dev, st};
    log_targets(sens, n, floor, out, st);
    HIP_TRY(hipGetLastError());
    return GS_OK;
}

gs_status gs_measure_peaks(gs_peaks *out, void *stream) {
    g_last_error.clear();
    if (!out) return fail(GS_ERR_INVALID_ARGUMENT, "out is NULL");
    memset(out, 0, sizeof(*out));
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    gs_status s = begin_call(&dev, st);
    if (s != GS_OK) return s;
    DoneGuard done_guard{dev, st};
    const size_t bytes = (size_t)2 << 30;   // 1 GiB copied into another 1 GiB
    HIP_TRY(arena_reserve(g_work[dev], bytes));
    HIP_TRY(measure_peaks(&out->copy_bytes_per_s, &out->fma_per_s, &out->exp_per_s, &out->mfma_bf16_flop_per_s,
                          g_work[dev].base, bytes, st));
    HIP_TRY(hipGetLastError());
    return GS_OK;
}

gs_status gs_mlp_forward(const float *params, const float *features, const float *norm, int64_t n, float *out,
                         void *stream) {
    g_last_error.clear();
    if (!params || !features || !norm || !out) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n < 1) return fail(GS_ERR_INVALID_ARGUMENT, "n must be >= 1");
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    gs_status s = begin_call(&dev, st);
    if (s != GS_OK) return s;
    DoneGuard done_guard{dev, st};
    const int64_t rows = 64;   // the fused forward needs only the bf16 weights from the scratch
    HIP_TRY(arena_reserve(g_work[dev], mlp_scratch_bytes(rows)));
    mlp_forward(params, features, norm, n, out, g_work[dev].base, rows, st);
    HIP_TRY(hipGetLastError());
    return GS_OK;
}

gs_status gs_mlp_train_step(float *params, float *adam, int64_t step, float lr, const float *features,
                            const float *norm, const float *targets, int64_t n, float *loss, float *grad,
                            void *stream) {
    g_last_error.clear();
    if (!params || !features || !norm || !targets || !loss)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n < 1 || n > kMlpRows) return fail(GS_ERR_INVALID_ARGUMENT, "batch rows must be in 1..65536");
    if (adam && step < 1) return fail(GS_ERR_INVALID_ARGUMENT, "step must be >= 1");
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(GS_ERR_INVALID_ARGUMENT, "lr must be >= 0");
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    gs_status s = begin_call(&dev, st);
    if (s != GS_OK) return s;
    DoneGuard done_guard{dev, st};
    const int64_t rows = (n + 63) / 64 * 64;
    HIP_TRY(arena_reserve(g_work[dev], mlp_scratch_bytes(rows)));
    mlp_train_step(params, adam, step, lr, features, norm, targets, n, loss, grad, g_work[dev].base, rows, st);
    HIP_TRY(hipGetLastError());
    return GS_OK;
}

gs_status gs_mlp_gradient(const float *params, const float *features, const float *norm, const float *targets,
                          int64_t n, int32_t precision, float *loss, float *grad, void *stream) {
    g_last_error.clear();
    if (!params || !features || !norm || !targets || !loss || !grad)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n < 1 || n > kMlpRows) return fail(GS_ERR_INVALID_ARGUMENT, "batch rows must be in 1..65536");
    if (precision != GS_MLP_BF16 && precision != GS_MLP_FP32)
        return fail(GS_ERR_INVALID_ARGUMENT, "unknown precision %d", precision);
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    gs_status s = begin_call(&dev, st);
    if (s != GS_OK) return s;
    DoneGuard done_guard{dev, st};
    const int64_t rows = (n + 63) / 64 * 64;
    HIP_TRY(arena_reserve(g_work[dev], mlp_scratch_bytes(rows)));
    mlp_train_step(const_cast<float *>(params), nullptr, 0, 0.0f, features, norm, targets, n, loss, grad,
                   g_work[dev].base, rows, st, precision == GS_MLP_FP32);
    HIP_TRY(hipGetLastError());
    return GS_OK;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Batched plans: several scenes (each with its own views) in one sequence
// with capacities fixed at creation, so that the whole sequence has no host
// synchronisation and can be captured into a hipGraph.  Scenes are packed
// into groups that fit the scratch budget; in each group every scene is
// projected, sorted and binned, then one compositing launch per pass covers
// the tiles of all the group's scenes.
struct PlanScene {
    gs_scene sc{};
    Setup S;
    ChunkPlan c{};
    std::vector<ViewDev> hv;
    std::vector<int32_t> htv;     // tile -> scene-local view
    ChunkBufs b{};
    ViewDev *views_dev = nullptr; // slice of the group's view table
    uint32_t *sorted_g = nullptr, *xr = nullptr, *yr = nullptr;
    uint64_t *scan_tmp = nullptr;
    uint32_t *over = nullptr;
    int64_t nbins = 0;
    int max_tiles = 1, max_tx = 1, max_ty = 1, max_cells = 1;
    uint64_t cap = 0;
    int group = 0, view0 = 0, tile0 = 0;
    uint32_t *clist = nullptr;    // the scene's compacted quadrant lists in the plan's pool (null: none)
    int passes = 4;               // depth sort passes (3 when the keys span well under 2^24 at creation)
};

// One pass-1 + pass-2 launch over consecutive scenes of a group (tiles
// [t0, t1) of the group's tile table).  Compacting launches share the plan's
// pool: each scene owns 4 x its list capacity there, so no run can write past
// its region (the list guard empties lists that outgrow the capacity).
struct CompositeBatch {
    int t0 = 0, t1 = 0;
    bool compact = false;
};

struct PlanGroup {
    std::vector<int> scenes;
    void *buf = nullptr, *lists = nullptr;
    ViewDev *views = nullptr;
    int32_t *tile_view = nullptr, *tile_scene = nullptr;
    SceneSlot *slots = nullptr;
    uint32_t *work = nullptr;
    uint32_t *ccount = nullptr;   // [total_tiles << quad_log] entries pass 1 compacted per quadrant
    std::vector<CompositeBatch> batches;
    int total_tiles = 0, total_views = 0;
    size_t bytes = 0, list_bytes = 0;
};

}  // namespace

struct gs_plan {
    int dev = -1;
    Allocator from;              // allocator of every block the plan owns
    gs_params p{};
    std::vector<PlanScene> scenes;
    std::vector<PlanGroup> groups;
    uint32_t *flag = nullptr;   // device: 1 if some list capacity was exceeded
    void *pool = nullptr;       // compacted quadrant lists, shared by the compacting launches
    size_t pool_bytes = 0;
    gs_plan_config cfg{0, 1};
    int quad_log = 2 * kTileShiftDefault - 6;   // 8x8 quadrants per tile, log2
    int region_log = 0;                          // pass-1 regions per tile, log2
    hipStream_t cap = nullptr;  // stream the sequence is captured on (the null stream cannot capture)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<float *> bound;  // output pointers baked into the graph
    int use_graph = 1;
    int graph_ok = 0;
};

namespace {

size_t scene_buffer_bytes(const PlanScene &ps) {
    const int64_t N = ps.S.N;
    size_t b = 0;
    auto add = [&](size_t x) { b += ((x + 255) & ~(size_t)255); };
    add(sizeof(GeoRec) * (size_t)ps.c.vc * N);
    add(sizeof(float) * (size_t)ps.c.vc * N);
    add(sizeof(uint2) * (size_t)ps.c.vc * N);
    for (int k = 0; k < 4; ++k) add(sizeof(uint32_t) * (size_t)ps.c.vc * N);
    add(sizeof(uint32_t) * (size_t)radix_sort_scratch_words(N, ps.c.vc));
    add(4 * sizeof(uint32_t) * (size_t)ps.c.vc);
    add(4 * sizeof(uint32_t) * (size_t)ps.c.vc * proj_blocks(N));
    add(sizeof(uint32_t) * ps.nbins);
    add(sizeof(uint64_t) * (size_t)rowbits_words(ps.c.vc, chunk_max_rows(ps.S, ps.c), ps.S.nchunks));
    add(sizeof(uint32_t) * ps.c.total_tiles);
    add(sizeof(uint64_t) * (ps.c.total_tiles + 1));
    add(sizeof(uint64_t) * scan_tmp_elems(ps.c.total_tiles + 1));
    add(sizeof(float) * (size_t)ps.c.rays);
    add(sizeof(uint64_t) * CNT_WORDS);
    add(256);
    return b;
}

void carve_scene(PlanScene &ps, Carve &cv) {
    const int64_t N = ps.S.N;
    ChunkBufs &b = ps.b;
    b.R = cv.take<GeoRec>((size_t)ps.c.vc * N);
    b.CB = cv.take<float>((size_t)ps.c.vc * N);
    b.XY = cv.take<uint2>((size_t)ps.c.vc * N);
    b.key0 = cv.take<uint32_t>((size_t)ps.c.vc * N);
    b.val0 = cv.take<uint32_t>((size_t)ps.c.vc * N);
    b.key1 = cv.take<uint32_t>((size_t)ps.c.vc * N);
    b.val1 = cv.take<uint32_t>((size_t)ps.c.vc * N);
    b.hist = cv.take<uint32_t>((size_t)radix_sort_scratch_words(N, ps.c.vc));
    b.nvis = cv.take<uint32_t>(4 * (size_t)ps.c.vc);
    b.cmax = b.nvis + ps.c.vc;
    b.kmin = b.nvis + 2 * ps.c.vc;
    b.proj_part = cv.take<uint32_t>(4 * (size_t)ps.c.vc * proj_blocks(N));
    b.bin_count = cv.take<uint32_t>(ps.nbins);
    b.rows_stride = chunk_max_rows(ps.S, ps.c);
    b.rowbits = cv.take<uint64_t>((size_t)rowbits_words(ps.c.vc, b.rows_stride, ps.S.nchunks));
    b.tile_tot = cv.take<uint32_t>(ps.c.total_tiles);
    b.tile_off = cv.take<uint64_t>(ps.c.total_tiles + 1);
    ps.scan_tmp = cv.take<uint64_t>(scan_tmp_elems(ps.c.total_tiles + 1));
    b.ray_A = cv.take<float>(ps.c.rays);
    b.counters = cv.take<uint64_t>(CNT_WORDS);
    ps.over = cv.take<uint32_t>(64);
    b.tile_active = nullptr;
    b.tile_sat = nullptr;
}

// Projection, depth sort and the count of the lists of one plan scene.
void enqueue_front(const gs_plan *P, PlanScene &ps, hipStream_t st) {
    const int64_t N = ps.S.N;
    ChunkBufs &b = ps.b;
    launch_fill_u32(b.nvis, 0u, 2 * (int64_t)ps.c.vc, st);
    launch_fill_u32(b.bin_count, 0u, ps.nbins, st);
    launch_fill_u64(b.counters, 0ull, CNT_WORDS, st);
    SceneDev sd{ps.sc.n, ps.sc.sh_degree, ps.sc.format, ps.sc.mean, ps.sc.log_scale,
                ps.sc.quat, ps.sc.opacity, ps.sc.sh};
    ProjParams pp{P->p.footprint_sigma, P->p.dilation, P->p.z_near, P->p.query_mode};
    launch_project(sd, ps.views_dev, ps.c.vc, pp, b, st);
    uint32_t *skeys = nullptr;
    radix_sort_segments(b.key0, b.val0, b.key1, b.val1, b.hist, N, ps.c.vc, true, ps.passes,
                        ps.passes == 3 ? b.kmin : nullptr, nullptr, &skeys, &ps.sorted_g, st);
    // the pair of sort buffers that does not hold the sorted output
    const bool out_in_0 = ps.sorted_g == b.val0;
    ps.xr = out_in_0 ? b.key1 : b.key0;
    ps.yr = out_in_0 ? b.val1 : b.val0;
    launch_ranges_in_order(ps.sorted_g, b, ps.c.vc, N, ps.xr, ps.yr, st);
    launch_bin_count(ps.views_dev, ps.c.vc, N, ps.S.nchunks, b, ps.xr, ps.yr, ps.max_cells, st);
    launch_chunk_prefix(ps.views_dev, ps.c.vc, ps.S.nchunks, b, ps.max_tiles, st);
    scan_u32_to_u64_exclusive(b.tile_tot, b.tile_off, ps.c.total_tiles, ps.scan_tmp, st);
}

void enqueue_plan(gs_plan *P, hipStream_t st, float *const *sens) {
    const float log2e = 1.4426950408889634f;
    for (PlanGroup &G : P->groups) {
        for (int si : G.scenes) {
            PlanScene &ps = P->scenes[si];
            enqueue_front(P, ps, st);
            if (ps.passes == 3) launch_span_check(ps.b.kmin, ps.c.vc, ps.over, P->flag, st);
            launch_list_guard(ps.b.tile_off, ps.c.total_tiles, ps.cap, ps.over, P->flag, ps.passes == 3, st);
            launch_bin_emit(ps.views_dev, ps.c.vc, ps.S.N, ps.S.nchunks, ps.b, ps.xr, ps.yr, ps.sorted_g,
                            ps.max_tx, ps.max_ty, ps.cap, ps.S.tsx, st);
            launch_fill_u32((uint32_t *)sens[si], 0u, ps.S.N, st);
        }
        for (const CompositeBatch &cb : G.batches) {
            CompositeArgs a{};
            a.views = G.views;
            a.tile_view = G.tile_view;
            a.tile_scene = G.tile_scene;
            a.slots = G.slots;
            a.total_tiles = cb.t1 - cb.t0;
            a.tile_first = cb.t0;
            a.query_mode = P->p.query_mode;
            a.r2_log2 = -0.5f * log2e * P->p.footprint_sigma * P->p.footprint_sigma;
            a.share_floor = P->p.share_floor;
            a.work = P->cfg.persistent ? G.work : nullptr;
            a.xcd_remap = P->cfg.xcd_remap;
            a.quad_log = P->quad_log;
            a.region_log = P->region_log;
            a.ccount = cb.compact ? G.ccount + ((size_t)cb.t0 << P->quad_log) : nullptr;
            a.report_floor = P->p.share_floor > 0.0f ? std::nextafter(P->p.share_floor, 0.0f) : 0.0f;
            launch_composite_pass1(a, st);
            launch_composite_pass2(a, false, nullptr, st);
        }
    }
}

void plan_free(gs_plan *P) {
    if (P->exec) hipGraphExecDestroy(P->exec);
    if (P->graph) hipGraphDestroy(P->graph);
    for (PlanGroup &G : P->groups) {
        dev_free(P->from, G.buf, nullptr);
        dev_free(P->from, G.lists, nullptr);
    }
    dev_free(P->from, P->flag, nullptr);
    dev_free(P->from, P->pool, nullptr);
    if (P->cap) hipStreamDestroy(P->cap);
    delete P;
}


// Compositing launches of each group.  Pass 2 walks compacted lists when
// they fit: scenes are taken in order into launches whose regions (4 x each
// scene's list capacity) fit a pool of half the scratch budget left after the
// plan's other buffers; a scene whose region alone exceeds it gets a launch
// of its own without compaction, and so does every scene if the pool cannot
// be allocated.  GS_COMPACT_POOL_GB replaces the pool's budget.  All forms
// give the same sensitivities.
void plan_batches(gs_plan *P) {
    size_t pool_budget = scratch_budget() / 2;
    env_gib("GS_COMPACT_POOL_GB", &pool_budget);
    const int ql = P->quad_log;
    auto region = [ql](const PlanScene &ps) { return ((ps.cap << ql) * sizeof(uint32_t) + 255) & ~(size_t)255; };
    std::vector<size_t> off(P->scenes.size(), 0);
    size_t pool = 0;
    for (PlanGroup &G : P->groups) {
        G.batches.clear();
        size_t used = 0;
        for (int si : G.scenes) {
            const PlanScene &ps = P->scenes[si];
            const int t0 = ps.tile0, t1 = ps.tile0 + ps.c.total_tiles;
            const size_t need = region(ps);
            if (need > pool_budget) {
                G.batches.push_back(CompositeBatch{t0, t1, false});
                used = 0;
                continue;
            }
            if (G.batches.empty() || !G.batches.back().compact || used + need > pool_budget) {
                G.batches.push_back(CompositeBatch{t0, t1, true});
                used = 0;
            }
            G.batches.back().t1 = t1;
            off[si] = used;
            used += need;
            pool = std::max(pool, used);
        }
    }
    if (pool > 0 && dev_alloc(P->from, &P->pool, pool, nullptr) != hipSuccess) {
        (void)hipGetLastError();
        P->pool = nullptr;
        for (PlanGroup &G : P->groups) {
            G.batches.clear();
            if (G.total_tiles > 0) G.batches.push_back(CompositeBatch{0, G.total_tiles, false});
        }
        return;
    }
    P->pool_bytes = P->pool ? pool : 0;
    for (PlanGroup &G : P->groups)
        for (const CompositeBatch &cb : G.batches)
            for (int si : G.scenes) {
                PlanScene &ps = P->scenes[si];
                if (cb.compact && ps.tile0 >= cb.t0 && ps.tile0 + ps.c.total_tiles <= cb.t1 && ps.c.total_tiles > 0)
                    ps.clist = (uint32_t *)((char *)P->pool + off[si]);
            }
}

// Groups, buffers, tables and list capacities of a new plan.
gs_status plan_allocate(gs_plan *P, hipStream_t st) {
    const int n_scenes = (int)P->scenes.size();
    // pack scenes into groups under half the scratch budget (the rest is for lists)
    const size_t budget = scratch_budget() / 2;
    for (int i = 0; i < n_scenes; ++i) {
        const size_t need = scene_buffer_bytes(P->scenes[i]);
        if (need > budget) {
            return fail(GS_ERR_UNSUPPORTED, "scene %d needs %zu bytes of scratch, more than the %zu budget", i,
                        need, budget);
        }
        if (P->groups.empty() || P->groups.back().bytes + need > budget) P->groups.push_back(PlanGroup{});
        PlanGroup &G = P->groups.back();
        G.scenes.push_back(i);
        G.bytes += need;
        P->scenes[i].group = (int)P->groups.size() - 1;
    }
    if (dev_alloc(P->from, (void **)&P->flag, 256, nullptr) != hipSuccess) {
        return fail(GS_ERR_OUT_OF_MEMORY, "plan flag");
    }
    launch_fill_u32(P->flag, 0u, 1, st);
    std::vector<std::vector<ViewDev>> group_views(P->groups.size());
    std::vector<std::vector<int32_t>> group_tv(P->groups.size()), group_ts(P->groups.size());
    for (size_t gi = 0; gi < P->groups.size(); ++gi) {
        PlanGroup &G = P->groups[gi];
        for (int si : G.scenes) {
            PlanScene &ps = P->scenes[si];
            ps.view0 = G.total_views;
            ps.tile0 = G.total_tiles;
            G.total_views += ps.c.vc;
            G.total_tiles += ps.c.total_tiles;
        }
        const size_t table_bytes = sizeof(ViewDev) * G.total_views + 2 * sizeof(int32_t) * G.total_tiles +
                                   (sizeof(uint32_t) << P->quad_log) * G.total_tiles + sizeof(SceneSlot) * G.scenes.size() +
                                   8192;
        if (dev_alloc(P->from, &G.buf, G.bytes + table_bytes + 65536, nullptr) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GS_ERR_OUT_OF_MEMORY, "plan group %zu: %zu bytes", gi, G.bytes + table_bytes);
        }
        Carve cv(G.buf);
        for (int si : G.scenes) carve_scene(P->scenes[si], cv);
        G.views = cv.take<ViewDev>(G.total_views);
        G.tile_view = cv.take<int32_t>(G.total_tiles);
        G.tile_scene = cv.take<int32_t>(G.total_tiles);
        G.slots = cv.take<SceneSlot>(G.scenes.size());
        G.work = cv.take<uint32_t>(64);
        G.ccount = cv.take<uint32_t>((size_t)G.total_tiles << P->quad_log);
        auto &gv = group_views[gi];
        auto &gtv = group_tv[gi];
        auto &gts = group_ts[gi];
        for (size_t k = 0; k < G.scenes.size(); ++k) {
            PlanScene &ps = P->scenes[G.scenes[k]];
            ps.views_dev = G.views + ps.view0;
            gv.insert(gv.end(), ps.hv.begin(), ps.hv.end());
            for (int t = 0; t < ps.c.total_tiles; ++t) {
                gtv.push_back(ps.view0 + ps.htv[t]);
                gts.push_back((int32_t)k);
            }
        }
        HIP_TRY(hipMemcpyAsync(G.views, gv.data(), sizeof(ViewDev) * gv.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(G.tile_view, gtv.data(), sizeof(int32_t) * gtv.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(G.tile_scene, gts.data(), sizeof(int32_t) * gts.size(), hipMemcpyHostToDevice, st));
        // count pre-pass: list sizes of every scene of the group
        std::vector<uint64_t> totals(G.scenes.size());
        std::vector<std::vector<uint32_t>> kr(G.scenes.size());
        for (size_t k = 0; k < G.scenes.size(); ++k) {
            PlanScene &ps = P->scenes[G.scenes[k]];
            enqueue_front(P, ps, st);
            HIP_TRY(hipMemcpyAsync(&totals[k], ps.b.tile_off + ps.c.total_tiles, sizeof(uint64_t),
                                   hipMemcpyDeviceToHost, st));
            kr[k].resize(2 * (size_t)ps.c.vc);
            HIP_TRY(hipMemcpyAsync(kr[k].data(), ps.b.kmin, sizeof(uint32_t) * kr[k].size(), hipMemcpyDeviceToHost,
                                   st));
        }
        HIP_TRY(hipStreamSynchronize(st));
        size_t lb = 0;
        for (size_t k = 0; k < G.scenes.size(); ++k) {
            PlanScene &ps = P->scenes[G.scenes[k]];
            // three sort passes when every view's depth keys span under 2^24
            // - 1 at creation, as in gs_sensitivity (attributes that change in
            // place can cross it: the span check guards every run)
            uint32_t span = 0;
            for (int v = 0; v < ps.c.vc; ++v)
                if (kr[k][ps.c.vc + v] >= kr[k][v]) span = std::max(span, kr[k][ps.c.vc + v] - kr[k][v]);
            ps.passes = span < 0xFFFFFFu ? 3 : 4;
            ps.cap = totals[k] + totals[k] / 64 + 1024;
            lb += ((ps.cap * sizeof(uint32_t) + 255) & ~(size_t)255);
        }
        if (dev_alloc(P->from, &G.lists, lb + 4096, nullptr) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GS_ERR_OUT_OF_MEMORY, "plan group %zu lists: %zu bytes", gi, lb);
        }
        G.list_bytes = lb;
        Carve lc(G.lists);
        for (int si : G.scenes) {
            PlanScene &ps = P->scenes[si];
            ps.b.lists = lc.take<uint32_t>(ps.cap);
        }

    }
    plan_batches(P);
    HIP_TRY(hipStreamSynchronize(st));
    return GS_OK;
}
}  // namespace

extern "C" {

gs_status gs_plan_create(const gs_scene *scenes, const gs_views *views, int32_t n_scenes, const gs_params *params,
                         gs_plan **out, void *stream) {
    g_last_error.clear();
    if (!out) return fail(GS_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    if (!scenes || !views || n_scenes < 1) return fail(GS_ERR_INVALID_ARGUMENT, "need n_scenes >= 1 scenes and views");
    gs_status s;
    if ((s = check_params(params)) != GS_OK) return s;
    if (params->ray_mask) return fail(GS_ERR_UNSUPPORTED, "plans do not take a ray mask");
    if (params->aggregate != GS_AGG_RAY) return fail(GS_ERR_UNSUPPORTED, "plans compute per-ray sensitivities");
    if (params->query_mode == GS_QUERY_CHANNEL)
        return fail(GS_ERR_UNSUPPORTED, "plans compute one query per ray (no per-channel queries)");
    if (params->flags) return fail(GS_ERR_UNSUPPORTED, "plans do not count pairs");
    gs_plan *P = new gs_plan();
    {
        std::lock_guard<std::mutex> lk(g_lock);
        P->from = g_allocator;
    }
    P->p = *params;
    // one binning tile for the whole plan (with tile_w = tile_h = 0, the
    // tuner's choice for the plan's largest view and scene)
    Setup T;
    {
        int64_t nmax = 1;
        int big = 0;
        int64_t pmax = 0;
        for (int i = 0; i < n_scenes; ++i) {
            nmax = std::max(nmax, scenes[i].n);
            const auto c = size_class(&views[i], 1);
            if (c.first >= pmax) {
                pmax = c.first;
                big = i;
            }
        }
        setup_tiles(params, T, &views[big], nmax);
    }
    P->p.tile_w = 1 << T.tsx;
    P->p.tile_h = 1 << T.tsy;
    P->quad_log = T.quad_log;
    P->region_log = region_log_of(T.tsx, T.tsy);
    P->scenes.resize(n_scenes);
    for (int i = 0; i < n_scenes; ++i) {
        PlanScene &ps = P->scenes[i];
        setup_tiles(&P->p, ps.S);
        if ((s = check_scene(&scenes[i])) != GS_OK || (s = check_views(&views[i], ps.S)) != GS_OK) {
            delete P;
            return s;
        }
        ps.sc = scenes[i];
        ps.S.N = scenes[i].n;
        ps.S.nchunks = (int)((ps.S.N + (1 << kChunkBits) - 1) >> kChunkBits);
        ps.c = ChunkPlan{0, views[i].n_views, ps.S.ray_base[views[i].n_views], 0};
        for (int v = 0; v < views[i].n_views; ++v) ps.c.total_tiles += ps.S.tiles_x[v] * ps.S.tiles_y[v];
        if (views[i].n_views > 65535) {
            delete P;
            return fail(GS_ERR_UNSUPPORTED, "scene %d: more than 65535 views", i);
        }
        ps.nbins = (int64_t)ps.c.total_tiles * ps.S.nchunks;
        // host view table (tile_base and ray numbering local to the scene)
        ps.hv.assign(ps.c.vc, ViewDev{});
        ps.htv.assign(ps.c.total_tiles, 0);
        int tb = 0;
        for (int k = 0; k < ps.c.vc; ++k) {
            ViewDev &V = ps.hv[k];
            const double *Pm = views[i].world_to_cam + 12 * k;
            for (int a = 0; a < 3; ++a) {
                for (int bb = 0; bb < 3; ++bb) V.R[3 * a + bb] = Pm[4 * a + bb];
                V.t[a] = Pm[4 * a + 3];
            }
            for (int a = 0; a < 3; ++a) V.cam[a] = -(V.R[a] * V.t[0] + V.R[3 + a] * V.t[1] + V.R[6 + a] * V.t[2]);
            V.fx = views[i].intrinsics[4 * k];
            V.fy = views[i].intrinsics[4 * k + 1];
            V.cx = views[i].intrinsics[4 * k + 2];
            V.cy = views[i].intrinsics[4 * k + 3];
            V.W = views[i].size[2 * k];
            V.H = views[i].size[2 * k + 1];
            V.tiles_x = ps.S.tiles_x[k];
            V.tiles_y = ps.S.tiles_y[k];
            V.tsx = ps.S.tsx;
            V.tsy = ps.S.tsy;
            V.ray_base = ps.S.ray_base[k];
            V.ray_local = ps.S.ray_base[k];
            V.tile_base = tb;
            ps.max_tiles = std::max(ps.max_tiles, V.tiles_x * V.tiles_y);
            ps.max_cells = std::max(ps.max_cells, (V.tiles_x + 1) * (V.tiles_y + 1));
            ps.max_tx = std::max(ps.max_tx, V.tiles_x);
            ps.max_ty = std::max(ps.max_ty, V.tiles_y);
            for (int t = 0; t < V.tiles_x * V.tiles_y; ++t) ps.htv[tb + t] = k;
            tb += V.tiles_x * V.tiles_y;
        }
    }
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    if ((s = begin_call(&dev, st)) != GS_OK) {
        delete P;
        return s;
    }
    DoneGuard done_guard{dev, st};
    P->dev = dev;
    s = plan_allocate(P, st);
    if (s != GS_OK) {
        plan_free(P);
        return s;
    }
    *out = P;
    return GS_OK;
}

gs_status gs_plan_set_config(gs_plan *plan, const gs_plan_config *cfg) {
    g_last_error.clear();
    if (!plan || !cfg) return fail(GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if ((cfg->persistent != 0 && cfg->persistent != 1) || (cfg->xcd_remap != 0 && cfg->xcd_remap != 1))
        return fail(GS_ERR_INVALID_ARGUMENT, "config fields are 0 or 1");
    std::lock_guard<std::mutex> lk(g_lock);
    if (plan->cfg.persistent != cfg->persistent || plan->cfg.xcd_remap != cfg->xcd_remap) {
        plan->cfg = *cfg;
        plan->bound.clear();  // forces a new capture
    }
    return GS_OK;
}

gs_status gs_plan_get_info(const gs_plan *plan, gs_plan_info *info) {
    g_last_error.clear();
    if (!plan || !info) return fail(GS_ERR_INVALID_ARGUMENT, "NULL argument");
    memset(info, 0, sizeof(*info));
    info->n_scenes = (int32_t)plan->scenes.size();
    info->n_groups = (int32_t)plan->groups.size();
    info->config = plan->cfg;
    info->graph_captured = plan->graph_ok;
    for (const PlanGroup &G : plan->groups) {
        info->device_bytes += (int64_t)(G.bytes + G.list_bytes);
        info->n_launches += (int32_t)G.batches.size();
        for (const CompositeBatch &cb : G.batches) info->n_compact_launches += cb.compact ? 1 : 0;
    }
    info->device_bytes += (int64_t)plan->pool_bytes;
    info->compact_bytes = (int64_t)plan->pool_bytes;
    for (const PlanScene &ps : plan->scenes) {
        info->list_capacity += (int64_t)ps.cap;
        info->n_sort3_scenes += ps.passes == 3 ? 1 : 0;
    }
    return GS_OK;
}

gs_status gs_plan_sensitivity(gs_plan *plan, float *const *sens, void *stream) {
    g_last_error.clear();
    if (!plan || !sens) return fail(GS_ERR_INVALID_ARGUMENT, "NULL argument");
    for (size_t i = 0; i < plan->scenes.size(); ++i)
        if (!sens[i]) return fail(GS_ERR_INVALID_ARGUMENT, "sens[%zu] is NULL", i);
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = -1;
    gs_status s = begin_call(&dev, st);
    if (s != GS_OK) return s;
    DoneGuard done_guard{dev, st};
    if (dev != plan->dev) return fail(GS_ERR_INVALID_ARGUMENT, "plan was created on device %d", plan->dev);
    const std::vector<float *> want(sens, sens + plan->scenes.size());
    if (want != plan->bound) {
        // (re)bind the outputs: slot tables, then a fresh capture
        for (PlanGroup &G : plan->groups) {
            std::vector<SceneSlot> hs;
            for (int si : G.scenes) {
                PlanScene &ps = plan->scenes[si];
                hs.push_back(SceneSlot{ps.b.R, ps.b.CB, ps.b.lists, ps.b.tile_off, ps.b.cmax, ps.b.ray_A,
                                       (uint32_t *)sens[si], nullptr, ps.S.N, ps.view0, ps.tile0, nullptr, 0,
                                       ps.clist});
            }
            HIP_TRY(hipMemcpyAsync(G.slots, hs.data(), sizeof(SceneSlot) * hs.size(), hipMemcpyHostToDevice, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        if (plan->exec) hipGraphExecDestroy(plan->exec);
        if (plan->graph) hipGraphDestroy(plan->graph);
        plan->exec = nullptr;
        plan->graph = nullptr;
        plan->graph_ok = 0;
        if (plan->use_graph) {
            hipError_t e = hipSuccess;
            if (!plan->cap) e = hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                enqueue_plan(plan, plan->cap, sens);
                e = hipStreamEndCapture(plan->cap, &plan->graph);
                if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
            }
            if (e != hipSuccess) {
                (void)hipGetLastError();
                plan->use_graph = 0;
                if (plan->graph) hipGraphDestroy(plan->graph);
                plan->graph = nullptr;
                plan->exec = nullptr;
            } else {
                plan->graph_ok = 1;
            }
        }
        plan->bound = want;
    }
    if (plan->graph_ok) {
        HIP_TRY(hipGraphLaunch(plan->exec, st));
    } else {
        enqueue_plan(plan, st, sens);
        HIP_TRY(hipGetLastError());
    }
    return GS_OK;
}

gs_status gs_tune_tile(const gs_scene *scene, const gs_views *views, const gs_params *params, int32_t reps,
                       float *sens, int32_t *best_w, int32_t *best_h, float *ms, void *stream) {
    g_last_error.clear();
    if (!params || !sens || !best_w || !best_h) return fail(GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (reps < 1) return fail(GS_ERR_INVALID_ARGUMENT, "reps must be >= 1");
    gs_status s;
    if ((s = check_params(params)) != GS_OK) return s;
    if (params->ambiguous_rays) return fail(GS_ERR_INVALID_ARGUMENT, "the tuner takes no ambiguous_rays");
    {
        Setup S;   // the views' own checks, at the widest shape
        S.tsx = S.tsy = 5;
        if ((s = check_views(views, S)) != GS_OK) return s;
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(GS_ERR_DEVICE, "hipEventCreate failed");
    }
    const int sides[3] = {8, 16, 32};
    float t[9];
    int best = -1;
    s = GS_OK;
    for (int k = 0; k < 9 && s == GS_OK; ++k) {
        t[k] = -1.0f;
        gs_params p = *params;
        p.tile_w = sides[k / 3];
        p.tile_h = sides[k % 3];
        if (p.aggregate == GS_AGG_TILE && (p.tile_w < 16 || p.tile_h < 16)) continue;
        if (!tiles_fit(views, tile_shift(p.tile_w), tile_shift(p.tile_h))) continue;
        if ((s = gs_sensitivity(scene, views, &p, sens, nullptr, stream)) != GS_OK) break;   // warm-up
        if (hipEventRecord(e0, st) != hipSuccess) s = fail(GS_ERR_DEVICE, "hipEventRecord failed");
        for (int r = 0; r < reps && s == GS_OK; ++r) s = gs_sensitivity(scene, views, &p, sens, nullptr, stream);
        if (s == GS_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&t[k], e0, e1) != hipSuccess))
            s = fail(GS_ERR_DEVICE, "timing the sensitivity pass failed");
        t[k] /= (float)reps;
        if (s == GS_OK && (best < 0 || t[k] < t[best])) best = k;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (s != GS_OK) return s;
    if (best < 0) return fail(GS_ERR_UNSUPPORTED, "no tile shape fits these views");
    *best_w = sides[best / 3];
    *best_h = sides[best % 3];
    if (params->aggregate != GS_AGG_TILE) {
        std::lock_guard<std::mutex> lk(g_tile_lock);
        g_tile_cache[size_class(views, scene->n)] = {tile_shift(*best_w), tile_shift(*best_h)};
    }
    if (ms)
        for (int k = 0; k < 9; ++k) ms[k] = t[k];
    return GS_OK;
}

gs_status gs_plan_tune(gs_plan *plan, float *const *sens, int32_t reps, gs_plan_config *best, float *ms,
                       void *stream) {
    g_last_error.clear();
    if (!plan || !sens) return fail(GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (reps < 1) return fail(GS_ERR_INVALID_ARGUMENT, "reps must be >= 1");
    const gs_plan_config cand[3] = {{0, 1}, {0, 0}, {1, 0}};
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(GS_ERR_DEVICE, "hipEventCreate failed");
    }
    float t[3] = {0, 0, 0};
    gs_status s = GS_OK;
    for (int k = 0; k < 3 && s == GS_OK; ++k) {
        if ((s = gs_plan_set_config(plan, &cand[k])) != GS_OK) break;
        if ((s = gs_plan_sensitivity(plan, sens, stream)) != GS_OK) break;  // capture + warm-up
        if (hipEventRecord(e0, st) != hipSuccess) s = fail(GS_ERR_DEVICE, "hipEventRecord failed");
        for (int r = 0; r < reps && s == GS_OK; ++r) s = gs_plan_sensitivity(plan, sens, stream);
        if (s == GS_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&t[k], e0, e1) != hipSuccess))
            s = fail(GS_ERR_DEVICE, "timing the plan failed");
        t[k] /= (float)reps;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (s != GS_OK) return s;
    int b = 0;
    for (int k = 1; k < 3; ++k)
        if (t[k] < t[b]) b = k;
    if ((s = gs_plan_set_config(plan, &cand[b])) != GS_OK) return s;
    if (best) *best = cand[b];
    if (ms)
        for (int k = 0; k < 3; ++k) ms[k] = t[k];
    return GS_OK;
}

gs_status gs_plan_status(gs_plan *plan, void *stream) {
    g_last_error.clear();
    if (!plan) return fail(GS_ERR_INVALID_ARGUMENT, "plan is NULL");
    uint32_t f = 0;
    HIP_TRY(hipMemcpyAsync(&f, plan->flag, sizeof f, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    if (f & kGuardSpan && f & kGuardList)
        return fail(GS_ERR_INVALID_DATA, "a scene's depth keys spanned 2^24 or more in a view (its plan sorts with "
                                         "three passes) and a scene produced more tile-list entries than at plan "
                                         "creation; their lists were emptied (recreate the plan)");
    if (f & kGuardSpan)
        return fail(GS_ERR_INVALID_DATA, "a scene's depth keys spanned 2^24 or more in a view, which the plan's "
                                         "three-pass depth sort cannot order; its lists were emptied (recreate "
                                         "the plan)");
    if (f)
        return fail(GS_ERR_INVALID_DATA, "a scene produced more tile-list entries than at plan creation; "
                                         "its lists were emptied (recreate the plan)");
    return GS_OK;
}

void gs_plan_destroy(gs_plan *plan) {
    if (!plan) return;
    std::lock_guard<std::mutex> lk(g_lock);
    (void)hipDeviceSynchronize();
    plan_free(plan);
}

}  // extern "C"
