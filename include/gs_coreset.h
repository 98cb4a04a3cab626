/*
 * gs_coreset.h - C ABI of the MI355X (gfx950) sensitivity pass and
 * sensitivity sampler for coreset pruning of 3D Gaussian Splatting scenes
 * (Mousa & Maalouf, "Provable Pruning for Efficient 3D Gaussian Splatting via
 * Coresets").
 *
 * Plain C: fixed-width integers, plain pointers, no C++ or HIP types.  A
 * stream argument is a hipStream_t passed as void* (NULL = the null stream).
 *
 * Memory: every array argument documented "device" must be device memory on
 * the current HIP device; "host" arrays are read during the call only.  The
 * caller owns all of them; the library never frees caller memory.  The
 * library keeps a grow-only scratch arena per device (released by
 * gs_release_workspace or at process exit).  Calls are serialised by a
 * library-wide lock, so two host threads never share scratch at once.
 *
 * Errors: every call returns a gs_status.  Argument errors are detected on the
 * host before any work is queued.  HIP failures return GS_ERR_DEVICE; the text
 * of the last error of the calling thread is in gs_last_error().
 *
 * Query set and conventions (the paper leaves these open; this library fixes
 * them): a query is one ray = (view, pixel); pixel (px, py) has its centre at
 * (px + 1/2, py + 1/2); camera axes are x right, y down, z forward; the
 * projected kernel is the local-affine (EWA) projection of Sigma, dilated by
 * `dilation` px^2, truncated to the Mahalanobis ellipse d^2 <= r^2 (boundary
 * included); Gaussians with camera depth z <= z_near are absent; the
 * front-to-back order is ascending float32-rounded camera depth with ties
 * broken by index; colour is real SH of degree <= 3 at the direction from the
 * camera centre to the mean, plus 1/2, clamped at 0.
 */
#ifndef GS_CORESET_H
#define GS_CORESET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID_ARGUMENT = 1,      /* bad size, null pointer, unknown enum, ... */
    GS_ERR_UNSUPPORTED = 2,           /* valid but outside what this build handles */
    GS_ERR_OUT_OF_MEMORY = 3,         /* scratch could not be allocated */
    GS_ERR_NO_POSITIVE_SENSITIVITY = 4, /* sampler: every sensitivity is 0 */
    GS_ERR_INVALID_DATA = 5,          /* non-finite attributes or zero quaternion */
    GS_ERR_DEVICE = 6                 /* a HIP runtime call failed */
} gs_status;

typedef enum { GS_ATTR_F32 = 0, GS_ATTR_MIXED16 = 1 } gs_attr_format;
/* What a query measures (Section 3.5, score variants; Algorithm 1's channel
 * queries).  With rho the attenuation of a pair and T the transmittance in
 * front of it, a Gaussian's contribution to a query of its ray is
 *   GS_QUERY_RGBSUM:  (c_R + c_G + c_B) rho T   (one query per ray: the L1
 *                     score with the channels summed)
 *   GS_QUERY_NOCOLOR: rho T                     (the "nocolor" variant)
 *   GS_QUERY_L2:      (c_R^2 + c_G^2 + c_B^2) rho^2 T^2  (the L2 variant,
 *                     its three channel terms summed into one pixel query)
 *   GS_QUERY_CHANNEL: c_k rho T for k = R, G, B (three queries per ray)
 * and a query's objective A is the sum of the contributions over its ray.
 * GS_QUERY_CHANNEL has no aggregated form (an aggregated query sums its
 * channels: use GS_QUERY_RGBSUM) and no gs_render_objective form (which
 * reports one value per ray); plans take every mode but GS_QUERY_CHANNEL. */
typedef enum {
    GS_QUERY_RGBSUM = 0,
    GS_QUERY_NOCOLOR = 1,
    GS_QUERY_L2 = 2,
    GS_QUERY_CHANNEL = 3
} gs_query_mode;
typedef enum { GS_OBJ_FULL = 0, GS_OBJ_FIXED = 1, GS_OBJ_TRUE = 2 } gs_objective;
/* GS_FLAG_COUNT_PAIRS: gs_sensitivity fills the pair counters of gs_stats
 * (a pass-2 variant that counts; without it those counters read 0). */
typedef enum { GS_FLAG_COUNT_PAIRS = 1 } gs_flag;
/* Query granularity of the sensitivity (Section 3.5, practical extensions):
 * a query is one ray (GS_AGG_RAY, Eq. sen), the rays of one 16x16 pixel tile
 * of a view (ragged at the right and bottom edges), the rays of one view, or
 * every ray (the per-scene variant).  For an aggregated query Q,
 * a_i(Q) = sum over its rays of a_i(q), A(Q) = sum of A(q), and
 * s_i = max over queries with A(Q) > 0 of a_i(Q) / A(Q); only rays selected
 * by the ray mask belong to queries. */
typedef enum { GS_AGG_RAY = 0, GS_AGG_TILE = 1, GS_AGG_IMAGE = 2, GS_AGG_SCENE = 3 } gs_aggregate;

/* Scene G = {(mu_i, Sigma_i, alpha_i, c_i)} (Section 3, "3DGS scene"), as
 * structure-of-arrays planes in device memory, n Gaussians.
 *   GS_ATTR_F32:     every plane float32.
 *   GS_ATTR_MIXED16: mean, log_scale and sh bfloat16; quat and opacity
 *                    float16 (IEEE binary16).
 * Planes: mean [3][n] (x, y, z); log_scale [3][n] (Sigma = R(q) diag(exp(2 l))
 * R(q)^T); quat [4][n] (w, x, y, z, normalised internally); opacity [n]
 * (alpha in [0, 1]); sh [(sh_degree+1)^2][3][n] (coefficient-major, then
 * R, G, B). */
typedef struct {
    int64_t n;
    int32_t sh_degree; /* 0..3 */
    int32_t format;    /* gs_attr_format */
    const void *mean;
    const void *log_scale;
    const void *quat;
    const void *opacity;
    const void *sh;
} gs_scene;

/* The finite query set's cameras (Section 3.2, "finite query set"), host
 * arrays.  world_to_cam [n_views][12] row-major [R | t] with p_cam = R p + t
 * and R in SO(3); intrinsics [n_views][4] = fx, fy, cx, cy in pixels;
 * size [n_views][2] = width, height.  Rays are numbered view-major, then
 * row-major inside a view. */
typedef struct {
    int32_t n_views;
    const double *world_to_cam;
    const double *intrinsics;
    const int32_t *size;
} gs_views;

typedef struct {
    float footprint_sigma;    /* r of the truncated footprint; default 3 */
    float dilation;           /* delta added to the 2D covariance, px^2; default 0.3 */
    float z_near;             /* > 0; default 0.2 */
    float share_floor;        /* a ray stops once T * c_max < floor * A; 0 = never; default 1e-12 */
    int32_t query_mode;       /* gs_query_mode */
    int32_t max_views_per_chunk; /* 0 = as many as the scratch budget allows */
    int32_t flags;            /* GS_FLAG_* bits */
    const uint32_t *ray_mask; /* device bitset over all rays (bit r%32 of word r/32), NULL = all */
    int32_t aggregate;        /* gs_aggregate: query granularity of gs_sensitivity; default GS_AGG_RAY */
    /* gs_sensitivity with GS_FLAG_COUNT_PAIRS (per-ray queries): device bitset
     * over all rays (as ray_mask) into which the bit of every scored ray that
     * holds an ambiguous pair (|d^2 - r^2| <= 1e-5 r^2: float32 and float64
     * may put it on different sides of the cutoff) is OR-ed; the caller
     * clears it.  NULL = not reported.  Must be NULL for other calls. */
    uint32_t *ambiguous_rays;
    /* Binning tile of the pipeline, pixels: 8, 16 or 32 each.  Any shape
     * gives the same sensitivities (the tile only decides which lists a
     * Gaussian enters, never which pairs count); wider tiles mean fewer list
     * entries per Gaussian and more rays per list.  A view may take at most
     * 38912 cells, (tiles_x + 1)(tiles_y + 1): 3840 x 2160 at 16 x 16, 7680 x
     * 4320 at 32 x 32; larger views are GS_ERR_UNSUPPORTED.  tile_w = tile_h = 0: the shape
     * gs_tune_tile last chose in this process for the same size class (the
     * largest view's pixel count and n, each rounded down to a power of two;
     * for a plan, its largest view and scene), else 16 x 16, or the first of
     * 16 x 32 and 32 x 32 that keeps every view within that limit; a single 0
     * side stands for 16.  GS_AGG_TILE queries need sides of 16 or 32
     * (GS_ERR_UNSUPPORTED for 8; with 0 a side of 8 becomes 16); their
     * results do not depend on which. */
    int32_t tile_w, tile_h;
} gs_params;

/* Filled only when a non-NULL pointer is passed (the call then synchronises
 * the stream once at its end and times each stage with HIP events on the
 * call's stream).  The pair counters need GS_FLAG_COUNT_PAIRS. */
typedef struct {
    int64_t n_projected;      /* (view, Gaussian) pairs in front of the camera and on screen (with a
                                 ray mask: and meeting a 16x16 tile that holds a selected ray) */
    int64_t n_entries;        /* (tile, Gaussian) list entries */
    int64_t n_pairs;          /* pass-2 ray-Gaussian pairs inside the footprint on scored rays */
    int64_t n_live_pairs;     /* ... of which the ray still needed (T c_max >= floor A before the pair) */
    int64_t n_lane_pairs;     /* pass-2 (pixel, entry) evaluations by the lanes, inside or not */
    int64_t n_rays_positive;  /* scored rays with A > 0 */
    int64_t n_invalid_gaussians; /* non-finite attributes or zero quaternion (treated as absent) */
    double total_sensitivity; /* S = sum_i s_i, fixed-order reduction */
    double ms_project, ms_sort, ms_bin, ms_pass1, ms_pass2; /* device time per stage, summed over chunks */
    double ms_emit;           /* the tile-list emission kernel (not part of ms_bin) */
    int64_t n_bins;           /* (tile, chunk) segments: tiles x chunks of 16384 depth positions */
    int32_t sort_passes;      /* most 8-bit passes a view chunk's depth sort took: 3 when every view's
                                 depth keys span under 2^24 - 1, else 4 */
    int32_t pad0;
    int64_t n_ambiguous_keys; /* (view, Gaussian) pairs in front of the camera whose FP64 depth lies within
                                 2^-40 of a midpoint between float32 values (its key could round either way) */
    int64_t n_ambiguous_pairs; /* pass-2 pairs on scored rays with |d^2 - r^2| <= 1e-5 r^2 (needs
                                  GS_FLAG_COUNT_PAIRS) */
} gs_stats;

typedef struct {
    int64_t n_invalid_pairs;  /* pairs with w_i rho_i >= 1 (Definition 2 violated) */
    double gamma_max;         /* max |log T - log T_w| over contributing retained pairs on valid rays */
} gs_render_diag;

/* Sensitivity pass (Algorithm 1, steps 1-3; Section 3.2, Eq. sen):
 *   s_i = max over rays q with A(q) > 0 of a(G, g_i, q) / A(G, q),
 * with a = c rho T and A = sum a (Section 3, scalar rendering function).
 * sens: device float[n], written (0 for Gaussians that never contribute).
 * Rays outside params->ray_mask are not scored.  Rays stop once the largest
 * possible remaining share is below params->share_floor, so every s_i below
 * that floor may read 0.  Synchronises the stream once per view chunk (to
 * size the tile lists).  stats may be NULL.  params->aggregate selects the
 * query granularity (gs_aggregate); aggregated sums are accumulated in exact
 * 64-bit fixed point, so every granularity is deterministic.  The pair
 * counters (GS_FLAG_COUNT_PAIRS) need GS_AGG_RAY.  Per-ray queries: pass 1
 * leaves each 8x8 quadrant's culled list for pass 2 in a device room of up
 * to 4 x the list bytes, at most half of the free memory (the environment
 * variable GS_COMPACT_POOL_GB, in GiB, replaces that bound; 0 turns the room
 * off; a value that is not a number of GiB >= 0 is ignored); when the room
 * holds only part of the lists, the tiles are composited in ranges that fit.
 * The results do not depend on the room. */
gs_status gs_sensitivity(const gs_scene *scene, const gs_views *views, const gs_params *params,
                         float *sens, gs_stats *stats, void *stream);

/* Sensitivity sampling (Algorithm 1, steps 3-5; proof of Theorem 2):
 * p_i is realised exactly as q_i / Q with q_i = ceil(s_i 2^40) (0 iff s_i = 0)
 * and Q = sum_i q_i; draw t in [0, m) takes the Philox4x32-10 block of
 * key (seed low, seed high) and counter (t low, t high, 0, 0) as a 128-bit u
 * (word 0 least significant), and picks the first i whose inclusive prefix
 * sum exceeds floor(u Q / 2^128).  counts[i] = number of draws of i;
 * weights[i] = counts[i] Q / (m q_i) in IEEE double (0 if not drawn);
 * support[0] = number of distinct drawn i.
 * sens: device float[n], every value in [0, 1 + 2^-10] (a sensitivity is a
 * largest share, Eq. sen, at most 1 up to the float32 rounding of the share;
 * a normalised proposal also qualifies), n <= 2^24 - 2^16, which keeps Q
 * below 2^64.  counts: device uint32[n]; weights: device double[n];
 * support: device int64[1]; 1 <= m < 2^31.
 * Returns GS_ERR_INVALID_DATA if some sens[i] is outside [0, 1 + 2^-10] or
 * NaN (detected on the device) and GS_ERR_NO_POSITIVE_SENSITIVITY if Q = 0;
 * in both cases the outputs are zeroed and nothing is drawn.
 * Synchronises the stream once (to read Q and the range check). */
gs_status gs_sample_coreset(const float *sens, int64_t n, int64_t m, uint64_t seed,
                            uint32_t *counts, double *weights, int64_t *support, void *stream);

/* gs_sample_coreset for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, checks and results, bit for bit, but the
 * library allocates nothing.  Its scratch (the u64 CDF and the scan's block
 * partials) is a file-scope device array sized for n <= 2^23 = 8,388,608
 * Gaussians (64 MiB plus 32 KiB per GPU, held until the process ends); larger
 * n returns GS_ERR_UNSUPPORTED.  Every call on a GPU uses that GPU's one
 * array, so calls that overlap on one GPU (different streams, or threads
 * that do not wait for each other's streams) race; the array keeps the last
 * call's contents, and each call rewrites what it reads.  Synchronises the
 * stream once (to read Q and the range check), like gs_sample_coreset. */
gs_status gs_sample_coreset_noalloc(const float *sens, int64_t n, int64_t m, uint64_t seed,
                                    uint32_t *counts, double *weights, int64_t *support, void *stream);

/* Objectives of a weighted pruned scene (Section 3: A, the fixed relaxation
 * A^th_w = sum_i w_i a(G, g_i, q), and the true reduced render
 * A_w = sum_i w_i c_i rho_i T_w with T_w = prod_{j before i} (1 - w_j rho_j)).
 * weights: device double[n] (NULL only for GS_OBJ_FULL).
 * per_ray: device float[rays] (nullable): the chosen objective, 0 on rays
 *   that are masked or have A = 0.
 * per_view: device double[n_views][3] (nullable): sums over scored rays of
 *   A, A^th_w and A_w (the last two 0 when weights is NULL).
 * diag (nullable, host): validity violations and the log-transmittance gap
 *   (Definition 2, Assumption 1); the call synchronises the stream when set.
 * For GS_OBJ_FULL and GS_OBJ_FIXED a ray stops once T c_max w_max < 1e-9 A
 * (no later term can move A or A^th_w by more than 1e-9 A), and the reduced
 * render is not computed: the A_w column of per_view is 0 and the
 * diagnostics count nothing.  GS_OBJ_TRUE walks every ray to its end and
 * fills all three columns and the diagnostics. */
gs_status gs_render_objective(const gs_scene *scene, const gs_views *views, const gs_params *params,
                              const double *weights, int32_t objective, float *per_ray,
                              double *per_view, gs_render_diag *diag, void *stream);

/* Coreset-objective error of a weighted draw at per-image resolution
 * (Definition 1 applied to objectives aggregated over each view's scored
 * rays, Section 3.5): from the per-view sums of gs_render_objective,
 *   out[0] = max over views with sum A > 0 of |sum A^th_w - sum A| / sum A,
 *   out[1] = the same with the reduced render sum A_w (column 2; 0 when
 *            that column was not computed),
 * in FP64 (the maximum is order-free, so the result is deterministic).
 * per_view: device double[n_views][3]; out: device double[2].  Queued on
 * the stream; no synchronisation. */
gs_status gs_coreset_error(const double *per_view, int32_t n_views, double *out, void *stream);

/* ---- Compact-region extension (Section 3.4: Assumption 2, the rho-net
 * definition, Theorem 4) -------------------------------------------------
 * A query region: sampled camera poses around a representative one (same
 * intrinsics and pixels), with the pose distance
 *   d(q, q') = |c - c'| + lambda * angle(R R'^T)
 * (camera centres c = -R^T t; lambda in length units per radian).  From the
 * per-ray full and reduced renders at every sampled pose (gs_render_objective
 * per_ray with GS_OBJ_FULL and GS_OBJ_TRUE, or GS_OBJ_FIXED for the fixed
 * relaxation), the call
 *   - picks representatives greedily (the first pose, then repeatedly the
 *     pose farthest from those chosen) until every sampled pose is within
 *     rho_target of one: is_net (host int32[n_poses]) = 1 for them, and
 *     rho = the covering radius reached;
 *   - keeps the pixels with A > a_floor at every pose (Assumption 2 (iv));
 *   - estimates L_full and L_w as the largest |A(q) - A(q')| / d(q, q') and
 *     |A_w(q) - A_w(q')| / d(q, q') over pairs of poses and kept pixels;
 *   - A_min = smallest A there; eps_0 = largest |A - A_w| / A over the
 *     representatives; max_err = the same over every pose;
 *   - eps_reg = eps_0 + ((1 + eps_0) L_full + L_w) rho / A_min (Theorem 4).
 * The constants are estimates from the samples (lower bounds of the true
 * ones), so the bound holds at every sampled query by construction of the
 * estimates; max_err shows how tight it is.
 * world_to_cam: host double[n_poses][12]; A, A_w: device float
 * [n_poses][n_pixels] (pose-major); 2 <= n_poses <= 4096.  Synchronises the
 * stream.  GS_ERR_NO_POSITIVE_SENSITIVITY if no pixel is kept. */
typedef struct {
    double L_full, L_w, A_min, eps_0, rho, eps_reg, max_err;
    int64_t n_pixels;     /* pixels kept */
    int32_t n_net;        /* representatives */
    int32_t pad;
} gs_region_report;
gs_status gs_region_bound(const double *world_to_cam, int32_t n_poses, double lambda, double rho_target,
                          const float *A, const float *A_w, int64_t n_pixels, float a_floor, int32_t *is_net,
                          gs_region_report *report, void *stream);

/* ---- Batched plans -------------------------------------------------------
 * A plan runs the sensitivity pass (Algorithm 1, steps 1-3) of several
 * scenes, each with its own views, as one sequence with no host
 * synchronisation: list capacities are fixed when the plan is created (a
 * counting pass over the current attributes, plus 1/64 + 1024 entries of
 * slack per scene), every buffer is owned by the plan, and the sequence is
 * captured into a HIP graph that later calls replay.  Scenes are packed into
 * groups that fit the scratch budget; in each group one compositing launch
 * per pass covers the tiles of consecutive scenes whose compacted quadrant
 * lists (4 x the list capacity) fit a shared pool sized at creation, usually
 * all of the group's scenes; a scene too large for the pool composites alone
 * on its plain tile lists.  Each scene's output equals that of
 * gs_sensitivity with the same params and no ray mask.
 * Memory: the scratch budget is 45% of the device's free memory (the
 * environment variable GS_SCRATCH_GB, in GiB >= 0, replaces it; other
 * values are ignored, and the budget is never below 256 MiB); groups take
 * half of it, the compaction pool at most half of what is left after the
 * plan's other buffers (GS_COMPACT_POOL_GB replaces that bound; 0 turns
 * compaction off). */
typedef struct gs_plan gs_plan;

/* Launch shape of the compositing kernels.  persistent = 1: a fixed grid of
 * 4096 one-wave workgroups takes 8x8 quadrants from an atomic counter;
 * persistent = 0: one workgroup per quadrant, and xcd_remap = 1 renumbers
 * workgroups so that consecutive quadrants of a tile row land on one XCD
 * (shared L2).  Default {0, 1}. */
typedef struct {
    int32_t persistent;
    int32_t xcd_remap;
} gs_plan_config;

typedef struct {
    int32_t n_scenes, n_groups;
    gs_plan_config config;
    int32_t graph_captured;   /* 1 once the sequence runs as a HIP graph */
    int64_t device_bytes;     /* plan-owned device memory */
    int64_t list_capacity;    /* tile-list entries reserved over all scenes */
    int64_t compact_bytes;    /* pool of compacted quadrant lists (0: none) */
    int32_t n_launches;       /* pass-1 + pass-2 launch pairs per run */
    int32_t n_compact_launches; /* of which pass 2 walks compacted lists */
    int32_t n_sort3_scenes;   /* scenes whose depth sort takes three 8-bit passes (every view's keys
                                 spanned under 2^24 - 1 at creation; a run where a view's keys span
                                 more empties that scene's lists and reports GS_ERR_INVALID_DATA
                                 through gs_plan_status) */
    int32_t pad;
} gs_plan_info;

/* scenes, views: host arrays of n_scenes (the attribute arrays they point to
 * are device memory and must stay valid, at the same addresses, for the
 * plan's life; their values may change between runs).  params: ray_mask must
 * be NULL and flags 0.  Synchronises the stream.  *out = NULL on error. */
gs_status gs_plan_create(const gs_scene *scenes, const gs_views *views, int32_t n_scenes,
                         const gs_params *params, gs_plan **out, void *stream);

/* Changes the compositing launch shape (the next run re-captures). */
gs_status gs_plan_set_config(gs_plan *plan, const gs_plan_config *config);

/* Binning-tile tuner for gs_sensitivity: times one call per shape (after an
 * untimed one) for each of the nine shapes {8, 16, 32} x {8, 16, 32}, in the
 * order w = 8, 16, 32 outer, h = 8, 16, 32 inner, with `params` otherwise as
 * given, writing into sens (device float[n], the caller's).  ms (host
 * float[9], nullable) receives the mean time per call of each shape, or -1
 * for a shape the views cannot take (too many tiles per view) or the
 * parameters exclude (GS_AGG_TILE: 16 x 16 only); *best_w, *best_h the
 * fastest, which is also kept for the size class of these views and this
 * scene (see gs_params.tile_w).  A calibration subset of the views may be
 * passed: the class is that of the views given.  The shape changes the speed
 * only: every shape gives the same sensitivities.  Synchronises the stream. */
gs_status gs_tune_tile(const gs_scene *scene, const gs_views *views, const gs_params *params, int32_t reps,
                       float *sens, int32_t *best_w, int32_t *best_h, float *ms, void *stream);

/* Times each launch shape ({0,1}, {0,0}, {1,0}) over `reps` >= 1 runs into
 * sens and keeps the fastest; ms (host float[3], nullable) receives the mean
 * time per run of each.  Synchronises the stream. */
gs_status gs_plan_tune(gs_plan *plan, float *const *sens, int32_t reps, gs_plan_config *best, float *ms,
                       void *stream);

gs_status gs_plan_get_info(const gs_plan *plan, gs_plan_info *info);

/* sens: host array of n_scenes device float pointers, sens[i] of length
 * scenes[i].n.  Queues the whole pass; no host synchronisation.  A new set
 * of output pointers re-captures the graph (and synchronises once). */
gs_status gs_plan_sensitivity(gs_plan *plan, float *const *sens, void *stream);

/* Synchronises the stream and returns GS_ERR_INVALID_DATA if, in any run
 * since creation, a scene needed more tile-list entries than its capacity,
 * or a view of a scene planned for the three-pass depth sort had depth keys
 * spanning 2^24 or more (that scene's output of that run is then all zeros);
 * gs_last_error() names which guard fired. */
gs_status gs_plan_status(gs_plan *plan, void *stream);

/* Waits for the device and frees the plan (NULL is ignored). */
void gs_plan_destroy(gs_plan *plan);

/* ---- Learned sampling proposal ------------------------------------------
 * A proposal distribution for sensitivity sampling: the sampler's
 * unbiasedness (proof of Theorem 2) holds for any p with p_i > 0 wherever
 * a_i can be > 0, so a cheap predictor of s, mixed with a uniform floor, can
 * replace the exact pass; the fixed objective then judges the draw.
 * MLP 64 -> 256 -> 256 -> 256 -> 1 with SiLU; the Python layer trains it to
 * predict ln(max(s, 1e-6)).
 * Parameters are float32 in PyTorch Linear layout, concatenated:
 *   W1[256][64] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] w4[256] b4
 * (gs_mlp_param_count() floats).  Products run in BF16 on the matrix cores
 * with FP32 accumulation; hidden activations are stored in BF16. */
int64_t gs_mlp_param_count(void);

/* Uniform(-a, a) weights with a = sqrt(6 / (fan_in + fan_out)) from `seed`,
 * zero biases.  params: device float[gs_mlp_param_count()]. */
gs_status gs_mlp_init(float *params, uint64_t seed, void *stream);

/* Per-Gaussian features, device float[n][64]: mean (3), log-scale (3),
 * quaternion normalised with w >= 0 (4), logit(alpha) (1), SH coefficients
 * padded to 48, then over the 16 nearest other means (exact, ties by
 * index): log mean distance, log 16th distance, mean and max neighbour
 * alpha, log(sum of alphas / volume of the 16th-neighbour ball).
 * Synchronises the stream once (grid sizing). */
gs_status gs_features(const gs_scene *scene, float *features, void *stream);

/* The 16 nearest other means of every Gaussian, the neighbourhood the
 * features above are built from: neighbours device uint32[n][16] (indices;
 * 0xFFFFFFFF where fewer than 16 others exist), sq_dist device float[n][16]
 * (squared distances as float32 (dx dx + dy dy) + dz dz, +inf where missing),
 * ordered by (squared distance, index).  Synchronises the stream once. */
gs_status gs_knn(const gs_scene *scene, uint32_t *neighbours, float *sq_dist, void *stream);

/* Column means and 1/std of device float[n][64] into device float[2][64]. */
gs_status gs_feature_stats(const float *features, int64_t n, float *norm, void *stream);

/* Predicted ln s for n rows of raw features (standardised with `norm`):
 * out device float[n]. */
gs_status gs_mlp_forward(const float *params, const float *features, const float *norm, int64_t n,
                         float *out, void *stream);

/* One batch (1 <= n <= 65536 rows): loss = mean((yhat - targets)^2) into
 * device float[1]; gradient of the loss into `grad` (device float[P],
 * nullable); if `adam` (device float[2][P]: first then second moments) is
 * non-NULL, one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected
 * with `step` >= 1) updates `params` in place.  Weight gradients sum the
 * batch in up to 32 row ranges whose partial products are added in order,
 * and no sum uses float atomics, so the result is deterministic. */
gs_status gs_mlp_train_step(float *params, float *adam, int64_t step, float lr, const float *features,
                            const float *norm, const float *targets, int64_t n, float *loss, float *grad,
                            void *stream);

/* Precision of gs_mlp_gradient: BF16 operands (the training path of
 * gs_mlp_train_step), or FP32 operands and activations through the same
 * kernels (v_mfma_f32_16x16x4_f32), to check the gradient's arithmetic. */
typedef enum { GS_MLP_BF16 = 0, GS_MLP_FP32 = 1 } gs_mlp_precision;

/* Loss and gradient of one batch (as gs_mlp_train_step without the update)
 * in the given precision: loss device float[1], grad device float[P]; the
 * parameters are not changed.  Every sum has a fixed order (deterministic). */
gs_status gs_mlp_gradient(const float *params, const float *features, const float *norm, const float *targets,
                          int64_t n, int32_t precision, float *loss, float *grad, void *stream);

/* Learned proposal for sensitivity sampling: p_i = (1 - floor) e_i / sum e +
 * floor / n with e_i = exp(log_s[i] - max log_s), from predicted ln s
 * (0 < floor <= 1; every p_i >= floor / n, so the sampler stays unbiased,
 * proof of Theorem 2).  log_s, p: device float[n] (p may alias nothing else);
 * deterministic (order-free maximum, fixed-order FP64 sum). */
gs_status gs_proposal_mixture(const float *log_s, int64_t n, float floor, float *p, void *stream);

/* Regression targets ln(max(s_i, floor)) from exact sensitivities (floor > 0):
 * device float[n] in and out. */
gs_status gs_log_targets(const float *sens, int64_t n, float floor, float *out, void *stream);

/* Measured rates of the calling device, the denominators of the rooflines:
 * a 1 GiB device copy (bytes read + written per second), FP32 FMAs (non-packed,
 * one per lane-instruction), v_exp_f32 and dense BF16 MFMA (16x16x32,
 * flops).  Synchronises the stream; uses 2 GiB of the scratch arena. */
typedef struct {
    double copy_bytes_per_s;
    double fma_per_s;
    double exp_per_s;
    double mfma_bf16_flop_per_s;
} gs_peaks;
gs_status gs_measure_peaks(gs_peaks *out, void *stream);

/* Defaults for gs_params (r = 3, delta = 0.3, z_near = 0.2, floor 1e-12, RGB sum,
 * per-ray queries, 16 x 16 tiles). */
void gs_default_params(gs_params *params);

/* Frees the calling device's scratch arena (waits for the device first). */
gs_status gs_release_workspace(void);

/* Where the library's device memory comes from (its scratch arenas and
 * the buffers of plans created afterwards): hipMalloc / hipFree by default,
 * or a caller's allocator, e.g. a framework's caching allocator (the Python
 * binding can register torch's).  alloc(ctx, bytes, stream) returns device
 * memory on the current device, or NULL when it cannot (the call that asked
 * then fails with GS_ERR_DEVICE); release(ctx, ptr, stream) takes back a
 * block alloc returned.  The library passes the null stream and releases a
 * block only after the device has finished with it.  Both functions, or
 * neither (NULL, NULL: back to hipMalloc / hipFree).  Process-wide; the
 * call waits for every device that holds arenas and returns each arena to
 * the allocator it came from (plans keep their allocator until destroyed).
 * The functions must not call into this library. */
typedef void *(*gs_alloc_fn)(void *ctx, size_t bytes, void *stream);
typedef void (*gs_free_fn)(void *ctx, void *ptr, void *stream);
gs_status gs_set_allocator(gs_alloc_fn alloc, gs_free_fn release, void *ctx);

/* Text of the last error on the calling thread ("" if none). */
const char *gs_last_error(void);
const char *gs_status_string(gs_status status);

#ifdef __cplusplus
}
#endif
#endif /* GS_CORESET_H */
