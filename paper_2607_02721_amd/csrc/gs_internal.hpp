// Internal declarations shared by the HIP kernels and the host-side C ABI.
// Not part of the public interface (that is include/gs_coreset.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

// Binning tiles are 2^tsx x 2^tsy pixels with tsx, tsy in {3, 4, 5} (8, 16
// or 32); 16 x 16 unless the caller or the tuner picks another shape.
constexpr int kTileShiftDefault = 4;
constexpr int kQuad = 8;           // compositing quadrant edge: one wave per 8x8 quadrant
constexpr int kChunkBits = 14;     // depth ranks are binned in chunks of 2^14 (one list segment per tile)
// The counting kernel keeps a view's 2D difference array of
// (tiles_x + 1)(tiles_y + 1) int32 cells in LDS beside its 4 KiB of row
// words: 38 912 cells (152 KiB) fit the 160 KiB a workgroup may take on CDNA4.
constexpr int kMaxCellsPerView = 38912;
constexpr int kSortTile = 4096;    // radix sort: keys per block (4 waves x 16 rounds x 64 lanes)
constexpr int kBinPositions = 1 << kChunkBits;  // binning: depth-sorted positions per chunk (count block)
constexpr int kEmitBatch = 2048;   // emission: positions a wave queues at a time (2048 measured best of 512-4096)
constexpr uint32_t kInvisibleKey = 0xFFFFFFFFu;
constexpr uint32_t kIndexMask = 0x0FFFFFFFu; // list entry = gaussian | quadrant mask << 28

// MLP proposal: 64 -> 256 -> 256 -> 256 -> 1; offsets into the FP32 parameter vector.
constexpr int kMlpIn = 64, kMlpH = 256;
constexpr int64_t kOffW1 = 0, kOffB1 = 16384, kOffW2 = 16640, kOffB2 = 82176, kOffW3 = 82432, kOffB3 = 147968,
                  kOffW4 = 148224, kOffB4 = 148480, kMlpParams = 148481;

// One camera of the current chunk, as the kernels see it.
struct ViewDev {
    double R[9];     // world-to-camera rotation, row-major
    double t[3];
    double cam[3];   // camera centre in world coordinates (-R^T t)
    double fx, fy, cx, cy;
    int32_t W, H, tiles_x, tiles_y;
    int64_t ray_base;   // global index of the view's first ray
    int64_t ray_local;  // index of the view's first ray inside this chunk's ray buffers
    int32_t tile_base;  // first tile of this view inside the chunk
    int32_t sat_base;   // first entry of this view's active-tile table (ray-masked runs)
    int32_t tsx, tsy;   // tile width 2^tsx, height 2^tsy pixels
};

// A tile of 2^tsx x 2^tsy pixels holds 2^(tsx-3) x 2^(tsy-3) quadrants of
// 8 x 8.  A list entry carries 4 bits (<< 28): the 2 x 2 sub-rectangles of
// the tile (halves in x and y) that the Gaussian's pixel range meets.  The
// bits of quadrant q (row-major inside the tile) are the sub-rectangles it
// overlaps: one for tiles of 16 or 32 pixels per side, both halves along a
// side of 8 pixels.
// Pass 1 walks each tile list once per region of up to 2 x 2 quadrants (16 x
// 16 pixels; one quadrant column or row for tiles 8 pixels wide or tall):
// log2 of the regions per tile.
__host__ __device__ inline int region_log_of(int tsx, int tsy) {
    return (tsx > 4 ? tsx - 4 : 0) + (tsy > 4 ? tsy - 4 : 0);
}

__host__ __device__ inline uint32_t quad_subrect_bits(int q, int tsx, int tsy) {
    const int qlx = tsx - 3, qly = tsy - 3;
    const int qx = q & ((1 << qlx) - 1), qy = q >> qlx;
    const uint32_t xm = qlx == 0 ? 3u : (qx >= (1 << (qlx - 1)) ? 2u : 1u);
    const uint32_t ym = qly == 0 ? 3u : (qy >= (1 << (qly - 1)) ? 2u : 1u);
    return ((ym & 1u) ? xm : 0u) | ((ym & 2u) ? xm << 2 : 0u);
}

struct SceneDev {
    int64_t n;
    int32_t sh_degree;
    int32_t format;     // 0 = f32, 1 = mixed16 (bf16 mean/log_scale/sh, f16 quat/opacity)
    const void *mean, *log_scale, *quat, *opacity, *sh;
};

struct ProjParams {
    float footprint_sigma, dilation, z_near;
    int32_t query_mode;
};

// Per-chunk device pointers produced by projection and binning.
// The geometry record of a (view, Gaussian) pair: both halves in one
// 32-byte-aligned record, so that a gather by Gaussian index touches one
// cache line.
struct __align__(32) GeoRec {
    float4 m;            // mean2d hi.x, hi.y, lo.x, lo.y
    float4 q;            // beta, a', g', alpha   (d^2 form, see project.hip)
};

struct ChunkBufs {
    GeoRec *R;           // [Vc*N] geometry records
    float *CB;           // [Vc*N] cbar, the query colour factor
    uint2 *XY;           // [Vc*N] x-range, y-range (int16 pairs as bits)
    float4 *R3;          // [Vc*N] per-channel queries only: c_R, c_G, c_B, 0 (else null)
    uint32_t *key0, *val0, *key1, *val1;  // [Vc*N] sort ping-pong
    uint32_t *hist;      // radix histograms [Vc][256][nb]
    uint32_t *nvis;      // [Vc] visible Gaussians per view
    uint32_t *cmax;      // [Vc] largest query colour per view (float bits)
    uint32_t *kmin;      // [Vc] smallest visible depth key per view; kmax = kmin + Vc the largest
    uint32_t *proj_part; // [Vc][projection blocks][4] per-block kept count (then its exclusive offset), colour maximum, key minimum, maximum
    // per (tile, chunk) entry counts, chunk-major inside each view (view v at
    // tile_base(v) * nchunks, then [chunk][tile of v]); turned in place into
    // each tile's exclusive prefix over chunks
    uint32_t *bin_count;
    // Per (view, tile row, chunk): bit i of word w is set when depth position
    // chunk * 2^14 + 64 w + i meets the tile row ([Vc][rows_stride][nchunks][256]
    // u64, written by the counting kernel, read by the emission).
    uint64_t *rowbits;
    int32_t rows_stride; // largest tile-row count of the chunk's views
    uint32_t *tile_tot;  // [tiles in chunk] entries per tile
    uint64_t *tile_off;  // exclusive scan of tile_tot (+1 trailing total): the tile's list
    uint32_t *lists;     // [D] entries
    float *ray_A;        // [queries per ray][rays in chunk] pass-1 render
    uint16_t *tile_active; // [tiles in chunk] bit q set: quadrant q of the tile holds a selected ray (null: all)
    // Ray-masked runs: per view, (tiles_y + 1) x (tiles_x + 1) counts, entry
    // (y, x) = active tiles with row < y and column < x, from sat_base on
    // (null: no ray mask).  Projection drops (view, Gaussian) pairs whose tile
    // rectangle holds no active tile: they can meet no selected ray.
    uint32_t *tile_sat;
    uint64_t *counters;  // device statistics
};

// counters[] slots
enum : int {
    CNT_PAIRS = 0, CNT_LANE_PAIRS = 1, CNT_RAYS_POS = 2, CNT_INVALID = 3, CNT_INVALID_PAIRS = 4,
    CNT_GAMMA_BITS = 5, CNT_LIVE = 6, CNT_AMB_KEYS = 7, CNT_SLOTS = 8
};
// The pass-2 pair counters (pairs, live pairs, positive rays, lane
// evaluations, pairs within the cutoff's ambiguity band) are each spread over
// kCntSpread words after the CNT_SLOTS words (word CNT_SLOTS + k * kCntSpread
// + (block mod kCntSpread)), so that the per-wave additions do not all meet on
// one address; the host sums them.
constexpr int kCntSpread = 64;
constexpr int kCntSpreadKinds = 5;
constexpr int CNT_WORDS = CNT_SLOTS + kCntSpreadKinds * kCntSpread;
// A pair is ambiguous when |d^2 - r^2| <= kAmbiguityBeta r^2: float32 and
// float64 arithmetic may put it on different sides of the cutoff.
constexpr float kAmbiguityBeta = 1e-5f;

// Blocks of the projection launch (256 threads, one Gaussian per thread).
// The projection runs one wave per block (its per-view folds need no block
// barrier); proj_part holds one entry per wave.
constexpr int kProjThreads = 64;
inline int64_t proj_blocks(int64_t n) { return (n + kProjThreads - 1) / kProjThreads; }

// Ordering of LDS accesses inside a one-wave workgroup.  A wave's LDS
// instructions execute and return in issue order, so a write by one lane is
// seen by a later read of any lane of the same wave; what must not happen is
// the compiler moving an access across the point.  This is a code-motion
// barrier only: unlike __syncthreads() it does not wait for the wave's
// outstanding LDS operations to drain.  Only for kernels launched with one
// wave per workgroup.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- launchers (each enqueues on `st`) -------------------------------------
void launch_project(const SceneDev &sc, const ViewDev *views_dev, int Vc, const ProjParams &pp,
                    const ChunkBufs &b, hipStream_t st);
// `passes` 8-bit LSD passes (3 or 4).  With kbase non-null the first pass
// subtracts kbase[seg] from every key but kInvisibleKey (the result must stay
// below 2^(8 passes) - 1 for the visible keys, so that invisible keys still
// sort last).  seg_len (device, nullable): only the first seg_len[seg] items
// of each segment are sorted (the rest are left alone).  Only the values
// leave the last pass: *key_out is null and *val_out holds them.  hist is
// scratch of radix_sort_scratch_words(n_per_seg, n_segs) words.
hipError_t radix_sort_segments(uint32_t *key0, uint32_t *val0, uint32_t *key1, uint32_t *val1,
                               uint32_t *hist, int64_t n_per_seg, int n_segs, bool vals_are_iota,
                               int passes, const uint32_t *kbase, const uint32_t *seg_len, uint32_t **key_out,
                               uint32_t **val_out, hipStream_t st);
int64_t radix_sort_scratch_words(int64_t n_per_seg, int n_segs);
// The kept depth keys of each view, moved to the front of the view's segment
// of kout in index order with their Gaussian indices in vout (after
// launch_project, whose per-block counts it turns into offsets).
void launch_key_compact(const ChunkBufs &b, int Vc, int64_t N, uint32_t *kout, uint32_t *vout, hipStream_t st);
void launch_ranges_in_order(const uint32_t *sorted_g, const ChunkBufs &b, int Vc, int64_t N, uint32_t *xr,
                            uint32_t *yr, hipStream_t st);
void launch_tile_active(const ViewDev *views_dev, const int32_t *tile_view, int total_tiles, const uint32_t *mask,
                        uint16_t *active, hipStream_t st);
// The quadrants with a selected ray, in order: per-tile counts, their
// exclusive scan (qoff[total_tiles] = the number listed) and the list of
// (tile << quad_log) + quadrant.
void launch_quad_list(const uint16_t *active, int total_tiles, int quad_log, uint32_t *qcnt, uint64_t *qoff,
                      uint64_t *scan_tmp, uint32_t *qlist, hipStream_t st);
// tile_sat from tile_active (two passes: along each tile row, then down each
// column).  max_tx / max_ty: the largest tile grid of the chunk's views.
void launch_tile_sat(const ViewDev *views_dev, int Vc, int max_tx, int max_ty, const uint16_t *active, uint32_t *sat,
                     hipStream_t st);
// u64 words of the row bitmaps of Vc views with at most max_ty tile rows.
inline int64_t rowbits_words(int Vc, int max_ty, int nchunks) {
    return (int64_t)Vc * max_ty * nchunks * (kBinPositions / 64);
}
// max_cells: the largest (tiles_x + 1) (tiles_y + 1) of the views.
void launch_bin_count(const ViewDev *views_dev, int Vc, int64_t N, int nchunks, const ChunkBufs &b,
                      const uint32_t *xr, const uint32_t *yr, int max_cells, hipStream_t st);
// bin_count -> per-tile prefix over chunks (in place) and tile_tot.
void launch_chunk_prefix(const ViewDev *views_dev, int Vc, int nchunks, const ChunkBufs &b, int max_tiles,
                         hipStream_t st);
// Writes every list entry (g | quadrant mask << 28) in its final, sorted
// place; entries at list index >= cap are dropped.
void launch_bin_emit(const ViewDev *views_dev, int Vc, int64_t N, int nchunks, const ChunkBufs &b,
                     const uint32_t *xr, const uint32_t *yr, const uint32_t *sorted_g, int max_tiles_x,
                     int max_tiles_y, uint64_t cap, int tile_shift_x, hipStream_t st);
// Plan guards: *over = 1 (and *flag |= kGuardSpan) when some view's kept
// depth keys span 2^24 or more (a three-pass sort would misorder them); the
// list guard sets *over (and *flag |= kGuardList) when the lists outgrow
// `cap` (keep: *over also stays set when the span guard set it) and then
// empties the lists.
constexpr uint32_t kGuardList = 1u, kGuardSpan = 2u;
void launch_span_check(const uint32_t *kmin, int Vc, uint32_t *over, uint32_t *flag, hipStream_t st);
void launch_list_guard(uint64_t *tile_off, int64_t ntiles, uint64_t cap, uint32_t *over, uint32_t *flag, bool keep,
                       hipStream_t st);
void scan_u32_to_u64_exclusive(const uint32_t *in, uint64_t *out, int64_t n, uint64_t *block_tmp,
                               hipStream_t st);
void scan_u64_inclusive(const uint64_t *in, uint64_t *out, int64_t n, uint64_t *block_tmp, hipStream_t st);
void scan_u64_inclusive_inplace(uint64_t *data, int64_t n, uint64_t *block_tmp, hipStream_t st);
int64_t scan_tmp_elems(int64_t n);

// One scene of a compositing launch (a launch may cover several scenes).
struct SceneSlot {
    const GeoRec *R;              // geometry records [views of the scene][N]
    const float *CB;              // query colour factor [views of the scene][N]
    const uint32_t *lists;        // tile lists; tile_off values index this array
    const uint64_t *tile_off;     // [scene tiles + 1] start of each tile's list
    const uint32_t *cmax;         // [views of the scene] largest query colour (float bits)
    float *ray_A;                 // pass-1 render of the scene's rays (indexed by ViewDev::ray_local)
    uint32_t *sens_bits;          // sensitivities (float bits, atomicMax) [N]
    const uint32_t *ray_mask;     // bitset over the scene's rays (ViewDev::ray_base numbering) or null
    int64_t N;
    int32_t view0;                // first view of the scene in the launch's view table
    int32_t tile0;                // first tile of the scene in the launch's tile table
    const float4 *R3;             // per-channel queries: channel colours [views][N] (else null)
    int64_t ray_stride;           // per-channel queries: distance between the R, G and B planes of ray_A
    // Pass 1 leaves each quadrant's entries that pass its exact test here
    // (the Gaussian indices, in list order, up to where the quadrant's rays
    // stopped): quadrant q of a tile with list [start, end) and Q = 2^quad_log
    // quadrants owns [Q start + q (end - start), Q start + (q + 1)(end - start)).  Pass 2
    // walks these dense lists.  The region form of pass 1 (2 x 2 quadrants
    // per wave) leaves one list per region instead, in the slots of the
    // region's first quadrant: each entry that reaches one of the region's
    // quadrants, as its Gaussian index with those quadrants' bits in the top
    // four bits; the region form of pass 2 walks it.  Null: no compaction
    // (pass 2 filters the tile lists again).  Both give the same sensitivities (pass 2 reports no
    // share below the share floor, and every pair before a ray's stop is
    // walked either way).
    uint32_t *clist;
};

// Compositing arithmetic of a query mode: one L1 query per ray (RGB sum or
// colour 1), one L2 query, or three per-channel L1 queries.
enum : int { kModeL1 = 0, kModeL2 = 1, kModeChannel = 2 };
constexpr int composite_mode(int query_mode) {
    return query_mode == 2 ? kModeL2 : (query_mode == 3 ? kModeChannel : kModeL1);
}

struct CompositeArgs {
    const ViewDev *views;        // view table of the launch (tile_base is scene-local)
    const int32_t *tile_view;    // [total_tiles] view of each tile
    const int32_t *tile_scene;   // [total_tiles] scene slot of each tile
    const SceneSlot *slots;
    int32_t total_tiles;         // tiles of this launch
    int32_t tile_first;          // launch tile t is tile tile_first + t of tile_view / tile_scene
    int32_t quad_log;            // log2 of the 8x8 quadrants per tile (every view of the launch has the same shape)
    int32_t region_log;          // log2 of the pass-1 regions (up to 2x2 quadrants) per tile
    int32_t query_mode;
    float r2_log2;               // -0.5 log2(e) r^2  (cut on the exp2 argument)
    float share_floor;
    uint32_t *work;              // persistent form: work counter (zeroed before the launch); null = one wave per quadrant
    int32_t xcd_remap;           // 1: give each XCD a contiguous range of quadrants
    int32_t agg;                 // query granularity (gs_aggregate) of pass 2
    const double *query_A;       // agg 1: A per tile of the launch; 2: per view; 3: [0] the launch's total
    uint64_t *acc;               // agg 1: per list entry; 2: per (view, Gaussian); 3: per Gaussian (fixed point)
    uint32_t *ccount;            // [quadrants] entries pass 1 compacted per quadrant of the launch (with SceneSlot::clist;
                                 // the region form: per region, at the region's first quadrant)
    uint64_t clist_shift;        // subtracted from every compacted-list offset (launches over a tile range
                                 // whose compacted lists fill a pool from its start)
    int32_t clist_pos;           // 1: the region lists hold each entry's position in its tile's list instead
                                 // of its Gaussian index (per-tile queries index their accumulators by it)
    const uint32_t *quad_list;   // ray-masked runs: the quadrants ((tile << quad_log) + q) holding a selected ray,
    int32_t n_listed;            // in order; only these are composited (null: every quadrant)
    float report_floor;          // pass 2 reports no share below the share floor: the float just below it, or 0
    uint32_t *amb_rays;          // pass 2 with counters: bit of every ray (ViewDev::ray_base numbering) with an
                                 // ambiguous pair is OR-ed in (null: none)
};
// Fixed-point scale of the aggregated shares.  A Gaussian's accumulated share
// of one query is at most 1 (a_i(q) <= A(q) on every ray), so 2^60 leaves a
// factor 16 of headroom in 64 bits; one unit is 8.7e-19 of the query's A.
constexpr double kAggScale = 1152921504606846976.0;   // 2^60
void launch_composite_pass1(const CompositeArgs &a, hipStream_t st);
void launch_composite_pass2(const CompositeArgs &a, bool stats, uint64_t *counters, hipStream_t st);
// Query objectives of the aggregated granularities from pass 1's per-ray A:
// tile_A[t] over each tile's rays and view_A[v] over each view's tiles, FP64
// sums in a fixed order; total[0] = sum of view_A (total may be null).
// Launches with a single scene slot at tile 0 (one call's chunk).
void launch_query_sums(const CompositeArgs &a, int Vc, double *tile_A, double *view_A, double *total,
                       hipStream_t st);
// Folds one launch's accumulators into the result.  agg 1: every list entry's
// share raises its Gaussian's sens_bits (float-bit maximum); agg 2: the maximum
// over the launch's views raises sens_bits; agg 3: num[g] += acc[g] 2^-60
// launch_A[0] (the launch's absolute contributions) and den[0] += launch_A[0].
void launch_agg_finalize(int agg, const uint64_t *acc, const uint32_t *lists, uint64_t n_entries, int64_t N,
                         int Vc, uint32_t *sens_bits, double *num, double *den, const double *launch_A,
                         hipStream_t st);
// out[i] = den[0] > 0 ? num[i] / den[0] : 0, rounded to float.
void launch_div_f64_to_f32(const double *num, const double *den, int64_t n, float *out, hipStream_t st);

struct ObjectiveArgs {
    const double *weights;
    int objective;
    float *per_ray;             // global, nullable
    double *tile_sums;          // [quadrants][3] per-wave partial sums
    const uint64_t *wmax_bits;  // largest weight (double bits); null = no early stop
    float stop_rel;             // stop a ray once T c_max w_max < stop_rel A
};
void launch_max_f64(const double *x, int64_t n, uint64_t *out_bits, hipStream_t st);
void launch_objective(const CompositeArgs &a, const ObjectiveArgs &o, uint64_t *counters, hipStream_t st);
void launch_view_sums(const double *tile_sums, const ViewDev *views_dev, int Vc, int quad_log, double *per_view_out,
                      hipStream_t st);
// out[0] = max over views with A > 0 of |A^th_w - A| / A, out[1] with A_w.
void launch_coreset_error(const double *per_view, int n_views, double *out, hipStream_t st);

// Sampler
// q_i = ceil(s_i 2^40); *bad |= 1 if some s_i is outside [0, 1 + 2^-10] or
// NaN (*bad must be zeroed first).
constexpr int64_t kSampleMaxN = ((int64_t)1 << 24) - ((int64_t)1 << 16);
void launch_quantize(const float *sens, int64_t n, uint64_t *q, uint32_t *bad, hipStream_t st);
void launch_draws(const uint64_t *C, int64_t n, int64_t m, uint64_t seed, uint32_t *counts, hipStream_t st);
// q: the quanta of k_quantize, or null to recompute them from sens.
void launch_weights(const uint32_t *counts, const uint64_t *q, const float *sens, const uint64_t *C, int64_t n,
                    int64_t m, double *weights, int64_t *support, hipStream_t st);

// MLP proposal and features
size_t mlp_scratch_bytes(int64_t rows);
void mlp_init(float *params, uint64_t seed, hipStream_t st);
void mlp_forward(const float *P, const float *feat, const float *norm, int64_t n, float *y, void *scratch,
                 int64_t rows, hipStream_t st);
// fp32: products in FP32 (v_mfma_f32_16x16x4_f32) with FP32 activations
// instead of BF16 (a precision mode of the same kernels).
void mlp_train_step(float *P, float *adam, int64_t step, float lr, const float *feat, const float *norm,
                    const float *y, int64_t n, float *loss, float *grad_out, void *scratch, int64_t rows,
                    hipStream_t st, bool fp32 = false);
size_t knn_scratch_bytes(int64_t n);
// Features [n][64], or with nidx non-null the 16 neighbours of every point
// instead (nidx [n][16] indices, nd2 [n][16] float32 squared distances).
hipError_t knn_features(const SceneDev &sc, float *feat, void *scratch, hipStream_t st, uint32_t *nidx = nullptr,
                        float *nd2 = nullptr);
void feature_stats(const float *feat, int64_t n, float *norm, hipStream_t st);
size_t mixture_scratch_bytes(int64_t n);
void proposal_mixture(const float *y, int64_t n, float floor, float *p, void *scratch, hipStream_t st);
void log_targets(const float *s, int64_t n, float floor, float *out, hipStream_t st);
hipError_t measure_peaks(double *copy_bytes_per_s, double *fma_per_s, double *exp_per_s, double *mfma_flop_per_s,
                         void *scratch, size_t scratch_bytes, hipStream_t st);

// Compact-region bound: kept pixels and min A / max errors (out_bits: min A,
// max error over the representatives, over all poses, kept count; the first
// must start at +inf bits, the others at 0), and per pose pair the largest
// differences of A and A_w over the kept pixels.
void launch_region_pixels(const float *A, const float *Aw, int K, int64_t P, float floor_, const int32_t *is_net,
                          uint8_t *keep, uint32_t *out_bits, hipStream_t st);
void launch_region_pairs(const float *A, const float *Aw, int K, int64_t P, const uint8_t *keep, const int32_t *pi,
                         const int32_t *pj, int n_pairs, float *diff, hipStream_t st);

// Small utilities
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
void launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t st);
// dst[k] = src[min(k stride, n)] for k = 0 .. ceil(n / stride) (dst holds that many + 1).
void launch_gather_u64(uint64_t *dst, const uint64_t *src, int64_t n, int64_t stride, hipStream_t st);
void launch_copy_u64(uint64_t *dst, const uint64_t *src, int64_t n, hipStream_t st);
void launch_sum_f32_to_f64(const float *x, int64_t n, double *out, double *block_tmp, hipStream_t st);

}  // namespace gs
