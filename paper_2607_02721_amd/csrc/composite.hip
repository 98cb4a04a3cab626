// Front-to-back compositing along every ray (Section 3, scalar rendering
// function: rho = alpha k, T = prod (1 - rho) over earlier Gaussians,
// a = c rho T, A = sum a) and the per-Gaussian maximum share
// (Section 3.2, Eq. sen: s_i = max_q a_i(q) / A(q), rays with A = 0 skipped).
//
// Work decomposition: one wave (64 lanes) per 8x8 quadrant of a 16x16 bin
// tile, one lane per pixel.  Waves are independent: each walks its tile's
// front-to-back list in slices of 64 entries, keeps the entries whose pixel
// range touches its quadrant (bit 28+q of the entry), stages their records
// in wave-private LDS and then composites them from LDS broadcasts.  A ray
// stops once T * c_max < floor * A (no later Gaussian can reach a share of
// `floor`); a wave stops when all of its rays have stopped.
//
// Pass 1 writes A per ray.  Pass 2 repeats the walk with the same arithmetic,
// forms shares a / A, reduces each entry's share over the wave's 64 pixels
// with a transposed butterfly (32 entries at a time; lane L ends with the
// maximum of entry L/2), and raises s with an atomic maximum on the float
// bits (order-free, so the result is deterministic).
//
// A launch may cover several scenes (batched plans): each tile of the launch
// names its scene slot (records, lists, outputs) and its view.  In the
// persistent form a fixed grid of waves takes quadrants from an atomic work
// counter until none are left.
#include "gs_internal.hpp"

#include <algorithm>

namespace gs {

constexpr int kWave = 64;
constexpr int kBlock = 4;   // pairs per unguarded step of the pass-2 loop

__device__ __forceinline__ uint64_t lanemask_lt64() {
    const unsigned lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// range of quadrants so that neighbouring quadrants (which share list entries
// and records) meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nblk_padded) {
    const int per = nblk_padded >> 3;
    return (b & 7) * per + (b >> 3);
}

struct WaveSetup {
    int v, gt, quad, px, py;
    bool inside;
    float xl, yl, qx0, qy0;
    int64_t ray_local, ray_global;
    uint64_t start, end;
    uint32_t qbit;
    int W;
    int64_t vbase;
    // the scene slot's fields, read once per quadrant
    const GeoRec *R;
    const float *CB;
    const uint32_t *lists;
    uint32_t *sens_bits;
    const uint32_t *ray_mask;
    float *ray_A;
    float cmax;
    const float4 *R3;       // per-channel queries: channel colours
    int64_t ray_stride;     // per-channel queries: ray_A plane stride
    uint32_t *clist;        // compacted entries of the scene's quadrants (null: none)
    uint64_t cbase;         // this quadrant's compacted slots start at clist + cbase
    float sfloor;           // staged sensitivities are raised to this (pass 2)
};

__device__ __forceinline__ int quad_count(const CompositeArgs &a) { return a.total_tiles << a.quad_log; }

// Quadrant `logical` of the launch -> this wave's pixels, list range and scene.
__device__ __forceinline__ bool setup_quad(const CompositeArgs &a, int logical, WaveSetup &w) {
    w.gt = a.tile_first + (logical >> a.quad_log);
    w.quad = logical & ((1 << a.quad_log) - 1);
    w.v = a.tile_view[w.gt];
    const SceneSlot &S = a.slots[a.tile_scene[w.gt]];
    const ViewDev &V = a.views[w.v];
    const int tl = w.gt - S.tile0 - V.tile_base;
    const int tx = tl % V.tiles_x, ty = tl / V.tiles_x;
    const int qlx = V.tsx - 3;
    const int qx0 = (tx << V.tsx) + (w.quad & ((1 << qlx) - 1)) * kQuad;
    const int qy0 = (ty << V.tsy) + (w.quad >> qlx) * kQuad;
    if (qx0 >= V.W || qy0 >= V.H) return false;
    const int lane = threadIdx.x;
    w.px = qx0 + (lane & 7);
    w.py = qy0 + (lane >> 3);
    w.inside = w.px < V.W && w.py < V.H;
    w.xl = (float)(lane & 7) + 0.5f;
    w.yl = (float)(lane >> 3) + 0.5f;
    w.qx0 = (float)qx0;
    w.qy0 = (float)qy0;
    w.W = V.W;
    w.ray_local = V.ray_local + (int64_t)w.py * V.W + w.px;
    w.ray_global = V.ray_base + (int64_t)w.py * V.W + w.px;
    w.start = S.tile_off[w.gt - S.tile0];
    w.end = S.tile_off[w.gt - S.tile0 + 1];
    w.qbit = quad_subrect_bits(w.quad, V.tsx, V.tsy) << 28;
    w.vbase = (int64_t)(w.v - S.view0) * S.N;
    w.R = S.R;
    w.CB = S.CB;
    w.lists = S.lists;
    w.sens_bits = S.sens_bits;
    w.ray_mask = S.ray_mask;
    w.ray_A = S.ray_A;
    w.cmax = __uint_as_float(S.cmax[w.v - S.view0]);
    w.R3 = S.R3;
    w.ray_stride = S.ray_stride;
    w.clist = S.clist;
    w.cbase = (w.start << a.quad_log) + (uint64_t)w.quad * (w.end - w.start) - a.clist_shift;
    w.sfloor = a.report_floor;
    return true;
}

// Next quadrant for this wave: the block's own (remapped) index in the flat
// form, or the next item of the work counter in the persistent form.  The
// form is a template parameter so that the flat kernels keep every
// per-quadrant value in scalar registers without a loop around them.
template <bool kPersistent>
__device__ __forceinline__ int next_quad(const CompositeArgs &a, int &iter) {
    const int nq = quad_count(a);
    if (!kPersistent) {
        if (iter++) return nq;
        if (a.quad_list) return (int)blockIdx.x < a.n_listed ? (int)a.quad_list[blockIdx.x] : nq;
        if (!a.xcd_remap) return blockIdx.x;
        const int padded = (nq + 7) & ~7;
        return xcd_remap(blockIdx.x, padded);
    }
    int q = 0;
    if (threadIdx.x == 0) q = (int)atomicAdd(a.work, 1u);
    // lane 0's value, as a wave-uniform (scalar) quantity
    q = __builtin_amdgcn_readfirstlane(q);
    if (a.quad_list) return q < a.n_listed ? (int)a.quad_list[q] : nq;
    return q;
}

__device__ __forceinline__ bool ray_selected(const uint32_t *mask, int64_t ray) {
    return mask == nullptr || ((mask[ray >> 5] >> (ray & 31)) & 1u);
}

// Can a pixel centre of the quadrant pass the footprint test P >= cut?
// P = a' u^2 + g' dy^2 (a', g' < 0), u = dx + beta dy, with (dx, dy) the
// centre minus the mean and centres at 0.5 ... 7.5 in quadrant coordinates.
// The minimum of -P over the continuous square [0.5, 7.5]^2 bounds the
// centres' values from below; it sits at the mean if the mean is inside,
// else on an edge (a one-dimensional quadratic, clamped).  An entry is
// dropped only when that minimum exceeds -cut by more than `err`, a bound
// (with a wide safety factor) on the float32 rounding of this test and of
// the per-pixel one, so a dropped entry contributes exactly nothing anyway:
// pass 1, pass 2 and the objectives give bit-identical results either way.
__device__ __forceinline__ bool quad_hit(float mx, float my, float beta, float ap, float gp, float cut) {
    const float A = -ap, G = -gp, C = -cut;
    const float x0 = 0.5f - mx, x1 = 7.5f - mx, y0 = 0.5f - my, y1 = 7.5f - my;
    if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) return true;
    auto q = [&](float dx, float dy) {
        const float u = fmaf(beta, dy, dx);
        return (A * u) * u + (G * dy) * dy;
    };
    // edges dy = y0, y1: best dx = -beta dy, clamped to [x0, x1] (x0 < x1: a
    // median of three is the clamp)
    float best = fminf(q(__builtin_amdgcn_fmed3f(-beta * y0, x0, x1), y0),
                       q(__builtin_amdgcn_fmed3f(-beta * y1, x0, x1), y1));
    // edges dx = x0, x1: best dy = -A beta dx / (A beta^2 + G)
    const float k = -(A * beta) * __builtin_amdgcn_rcpf(fmaf(A * beta, beta, G));
    best = fminf(best, q(x0, __builtin_amdgcn_fmed3f(k * x0, y0, y1)));
    best = fminf(best, q(x1, __builtin_amdgcn_fmed3f(k * x1, y0, y1)));
    const float S = fabsf(mx) + fabsf(my) + 16.0f;
    // (v_sqrt_f32, within about an ulp, is ample for a bound this loose)
    const float err = 3.814697265625e-6f /* 2^-18 */ * S *
                          ((1.0f + fabsf(beta)) * __builtin_amdgcn_sqrtf(A * C) + __builtin_amdgcn_sqrtf(G * C)) +
                      1e-4f * C;
    return best <= C + err;
}

// The staged geometry of an entry: with u = dx + beta dy and the exponent's
// coefficient a' < 0, the exponent a' u^2 + t equals t - (s u)^2 for
// s = sqrt(-a'), and s u = (s x - s mean_x) + (s beta) dy.  Staged as
// (-s mean_x, mean_y, s beta, s), a pixel's exponent then takes one FMA for
// s dx, one for s u and one for t - (s u)^2 (instead of a product and an FMA
// for a' u u).  Every form of both passes and the objectives stage through
// here, so they form the same exponents.
__device__ __forceinline__ float4 scaled_geo(float mx, float my, float beta, float a2) {
    const float sc = __builtin_amdgcn_sqrtf(-a2);
    return make_float4(-sc * mx, my, sc * beta, sc);
}

// Stage the slice's entries whose footprint reaches this quadrant (pixel
// range bit, then the exact test above); returns how many.  With kPad > 1
// the slots up to the next multiple of kPad hold null entries, so a loop can
// run in unguarded blocks of kPad pairs.
// geo = scaled_geo(mean_x, mean_y relative to the quadrant origin, beta, a'),
// col = (g', alpha, cbar, extra), or with kChannel (g', alpha, c_R, c_G) and
// c_B in cblue.  With kLog (no extra value, one query per ray) col = (g',
// log2 alpha, cbar, cut + log2 alpha) for pair_rho_log2; null entries then
// carry an infinite bar.
// stage_raw: the same for one list entry per lane (raw = 0: none), at list
// position e (read only for kExtra 3).
template <int kExtra, int kPad = 1, bool kChannel = false, bool kLog = false>  // kExtra 0: none, 1: s_old + index, 2: weight, 3: index + list position
__device__ __forceinline__ int stage_raw(const WaveSetup &w, uint32_t raw, uint64_t e, float cut, float4 *geo,
                                         float4 *col, uint32_t *sid, float *sold, const double *__restrict__ weights,
                                         float *cblue = nullptr, uint32_t *cout = nullptr) {
    static_assert(!(kChannel && kExtra == 2), "per-channel queries have no weighted objective");
    static_assert(!(kLog && (kChannel || kExtra == 2)), "the log form has no room for an extra value");
    const int lane = threadIdx.x;
    const GeoRec *__restrict__ R = w.R;
    const float *__restrict__ CB = w.CB;
    const int64_t vbase = w.vbase;
    bool touch = (raw & w.qbit) != 0u;
    const uint32_t g = raw & kIndexMask;
    const int64_t o = vbase + g;
    float4 r1 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float mx = 0.0f, my = 0.0f;
    if (touch) {
        const float4 r0 = R[o].m;
        r1 = R[o].q;
        mx = (r0.x - w.qx0) + r0.z;
        my = (r0.y - w.qy0) + r0.w;
        touch = quad_hit(mx, my, r1.x, r1.y, r1.z, cut);
    }
    const uint64_t bal = __ballot(touch);
    const int n = __popcll(bal);
    if (kPad > 1 && !touch) {
        // null entries (alpha = 0: rho = 0, so A, T and every share are
        // unchanged) fill the slots up to a multiple of kPad
        const int slot = n + __popcll(~bal & lanemask_lt64());
        if (slot < ((n + kPad - 1) & ~(kPad - 1))) {
            geo[slot] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            col[slot] = make_float4(0.0f, 0.0f, 0.0f, kLog ? __builtin_inff() : 0.0f);
            if (kChannel) cblue[slot] = 0.0f;
        }
    }
    if (touch) {
        const int slot = __popcll(bal & lanemask_lt64());
        // pass 1 keeps the quadrant's entries in order (streamed past L2: pass 2
        // reads them in a later launch)
        if (cout) __builtin_nontemporal_store(g, &cout[slot]);
        float cb = 0.0f, cg = 0.0f;
        if (kChannel) {
            const float4 c3 = w.R3[o];
            cb = c3.x;
            cg = c3.y;
            cblue[slot] = c3.z;
        } else {
            cb = CB[o];
        }
        geo[slot] = scaled_geo(mx, my, r1.x, r1.y);
        float extra = 0.0f;
        if (kExtra == 1) {
            sid[slot] = g;
            sold[slot] = fmaxf(__uint_as_float(w.sens_bits[g]), w.sfloor);
        }
        if (kExtra == 3) {   // aggregated pass 2: index and position in the tile's list
            sid[slot] = g;
            sold[slot] = __uint_as_float((uint32_t)(e - w.start));
        }
        if (kExtra == 2) extra = (float)weights[g];
        if (kChannel) extra = cg;
        if (kLog) {
            const float la = __builtin_amdgcn_logf(r1.w);
            col[slot] = make_float4(r1.z, la, cb, cut + la);
        } else {
            col[slot] = make_float4(r1.z, r1.w, cb, extra);
        }
    }
    return n;
}

template <int kExtra, int kPad = 1, bool kChannel = false, bool kLog = false>
__device__ __forceinline__ int stage_slice(const WaveSetup &w, uint64_t e0, float cut, float4 *geo, float4 *col,
                                           uint32_t *sid, float *sold, const double *__restrict__ weights,
                                           float *cblue = nullptr, uint32_t *cout = nullptr) {
    const uint64_t e = e0 + threadIdx.x;
    const uint32_t raw = e < w.end ? w.lists[e] : 0u;
    return stage_raw<kExtra, kPad, kChannel, kLog>(w, raw, e, cut, geo, col, sid, sold, weights, cblue, cout);
}

// Stage up to 64 entries of a quadrant's compacted list (every one passed
// the quadrant's exact test in pass 1): the same slots as stage_slice would
// fill for them, padded with null entries to a multiple of kPad.
template <int kPad, bool kChannel, bool kLog = false>
__device__ __forceinline__ int stage_compact(const WaveSetup &w, const uint32_t *__restrict__ cl, uint32_t left,
                                             float cut, float4 *geo, float4 *col, uint32_t *sid, float *sold,
                                             float *cblue) {
    static_assert(!(kLog && kChannel), "the log form holds one query per ray");
    const int lane = threadIdx.x;
    const int n = (int)min(left, (uint32_t)kWave);
    if (lane < n) {
        const uint32_t g = cl[lane];
        const int64_t o = w.vbase + g;
        const float4 r0 = w.R[o].m;
        const float4 r1 = w.R[o].q;
        float cb = 0.0f, cg = 0.0f;
        if (kChannel) {
            const float4 c3 = w.R3[o];
            cb = c3.x;
            cg = c3.y;
            cblue[lane] = c3.z;
        } else {
            cb = w.CB[o];
        }
        geo[lane] = scaled_geo((r0.x - w.qx0) + r0.z, (r0.y - w.qy0) + r0.w, r1.x, r1.y);
        if (kLog) {
            const float la = __builtin_amdgcn_logf(r1.w);
            col[lane] = make_float4(r1.z, la, cb, cut + la);
        } else {
            col[lane] = make_float4(r1.z, r1.w, cb, kChannel ? cg : 0.0f);
        }
        sid[lane] = g;
        sold[lane] = fmaxf(__uint_as_float(w.sens_bits[g]), w.sfloor);
    } else if (lane < ((n + kPad - 1) & ~(kPad - 1))) {
        geo[lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        col[lane] = make_float4(0.0f, 0.0f, 0.0f, kLog ? __builtin_inff() : 0.0f);
        if (kChannel) cblue[lane] = 0.0f;
    }
    return n;
}

// exp2 argument of the kernel for this lane's pixel; rho = alpha exp2(P)
// inside the footprint (P >= cut), else 0.
__device__ __forceinline__ float pair_rho(const float4 &G, const float4 &Cc, float xl, float yl, float cut,
                                          bool &in_fp) {
    const float dx = fmaf(G.w, xl, G.x);   // s (x - mean_x)
    const float dy = yl - G.y;
    const float u = fmaf(G.z, dy, dx);      // s u
    const float t = Cc.x * (dy * dy);
    const float P = fmaf(-u, u, t);
    const float E = __builtin_amdgcn_exp2f(P);
    in_fp = P >= cut;
    return in_fp ? Cc.y * E : 0.0f;
}

// The same with alpha folded into the exponent: col = (g', log2 alpha, ., bar)
// with bar = cut + log2 alpha (stage_slice / stage_compact with kLog), so
// rho = exp2(P + log2 alpha) inside the footprint (P + log2 alpha >= bar).
__device__ __forceinline__ float pair_rho_log2(const float4 &G, const float4 &Cc, float xl, float yl, bool &in_fp) {
    const float dx = fmaf(G.w, xl, G.x);
    const float dy = yl - G.y;
    const float u = fmaf(G.z, dy, dx);
    const float t = fmaf(Cc.x, dy * dy, Cc.y);
    const float P = fmaf(-u, u, t);
    const float E = __builtin_amdgcn_exp2f(P);
    in_fp = P >= Cc.w;
    return in_fp ? E : 0.0f;
}

// Pass 1 per query mode (kModeL1: a = c rho T; kModeL2: a = c (rho T)^2;
// kModeChannel: three queries, a_k = c_k rho T).  A ray stops once no later
// Gaussian can add floor times its objective: c_max T (c_max T^2 for L2)
// below floor A, with the smallest of the three objectives per channel.
template <bool kPersistent, int kMode>
__global__ __launch_bounds__(kWave) void k_pass1(CompositeArgs a) {
    __shared__ float4 geo[kWave], col[kWave];
    __shared__ float cblue[kMode == kModeChannel ? kWave : 1];
    constexpr bool kCh = kMode == kModeChannel;
    const int nq = quad_count(a);
    int iter = 0;
    for (int qi = next_quad<kPersistent>(a, iter); qi < nq; qi = next_quad<kPersistent>(a, iter)) {
        WaveSetup w;
        if (!setup_quad(a, qi, w)) continue;
        const bool scored = w.inside && ray_selected(w.ray_mask, w.ray_global);
        const float cmax = w.cmax;
        float T = 1.0f, A = 0.0f, AG = 0.0f, AB = 0.0f;
        bool done = !scored;
        // this quadrant's compacted list (see SceneSlot::clist)
        uint32_t *cl = w.clist ? w.clist + w.cbase : nullptr;
        uint32_t ccnt = 0;
        for (uint64_t e0 = w.start; e0 < w.end; e0 += kWave) {
            if (__all(done)) break;
            const int n = stage_slice<0, 1, kCh, !kCh>(w, e0, a.r2_log2, geo, col, nullptr, nullptr, nullptr, cblue,
                                                 cl ? cl + ccnt : nullptr);
            ccnt += (uint32_t)n;
            wave_sync();
            for (int j = 0; j < n; ++j) {
                const float4 G = geo[j], Cc = col[j];
                bool in_fp;
                const float rho = kCh ? pair_rho(G, Cc, w.xl, w.yl, a.r2_log2, in_fp)
                                      : pair_rho_log2(G, Cc, w.xl, w.yl, in_fp);
                if (kMode == kModeL1) {
                    const float cr = Cc.z * rho;
                    A = fmaf(cr, T, A);
                } else if (kMode == kModeL2) {
                    const float rt = rho * T;
                    A = fmaf(Cc.z * rt, rt, A);
                } else {
                    const float rt = rho * T;
                    A = fmaf(Cc.z, rt, A);
                    AG = fmaf(Cc.w, rt, AG);
                    AB = fmaf(cblue[j], rt, AB);
                }
                T = fmaf(-rho, T, T);
            }
            if (kMode == kModeL1) done = done || (T * cmax < a.share_floor * A);
            if (kMode == kModeL2) done = done || ((T * T) * cmax < a.share_floor * A);
            if (kCh) done = done || (T * cmax < a.share_floor * fminf(A, fminf(AG, AB)));
            wave_sync();
        }
        if (w.inside) {
            w.ray_A[w.ray_local] = scored ? A : 0.0f;
            if (kCh) {
                w.ray_A[w.ray_stride + w.ray_local] = scored ? AG : 0.0f;
                w.ray_A[2 * w.ray_stride + w.ray_local] = scored ? AB : 0.0f;
            }
        }
        if (cl && threadIdx.x == 0) a.ccount[qi] = ccnt;
    }
}

// An entry staged for a region: g = (mean x, y relative to the region's
// first quadrant, beta, a'), c = (g', log2 alpha, colour sum, cut + log2
// alpha), m1 = mean relative to the second quadrant column / row.
// Pass 2 adds the entry's staged sensitivity (raised to the report floor),
// its Gaussian index and the bar below which a pixel's rho T (L1) or
// (rho T)^2 (L2) cannot give a share above the staged sensitivity.
// Per-channel queries stage c = (g', alpha, c_R, c_G) and c_B in cblue.
struct __align__(16) RegionRec {
    float4 g, c;
    float2 m1;
    float sold;
    uint32_t sid;
    float bar, cblue;
    uint32_t hq;   // the entry's quadrant bits
    float pad;
};

// Region `logical` of the launch: its tile, view, scene slot, origin and, per
// quadrant k (column k & 1, row k >> 1), the quadrant's index in the tile,
// its sub-rectangle bit and whether it exists (inside the view and the tile).
struct RegionSetup {
    int gt, v;
    const SceneSlot *S;
    const ViewDev *V;
    int ox, oy;
    int quad[4];
    uint32_t qbit[4];
    uint32_t valid;
};

__device__ __forceinline__ bool setup_region(const CompositeArgs &a, int logical, RegionSetup &r) {
    r.gt = a.tile_first + (logical >> a.region_log);
    const int rg = logical & ((1 << a.region_log) - 1);
    r.v = a.tile_view[r.gt];
    r.S = &a.slots[a.tile_scene[r.gt]];
    r.V = &a.views[r.v];
    const ViewDev &V = *r.V;
    const int tl = r.gt - r.S->tile0 - V.tile_base;
    const int tx = tl % V.tiles_x, ty = tl / V.tiles_x;
    const int qlx = V.tsx - 3, qly = V.tsy - 3;            // log2 quadrant columns, rows per tile
    const int rlx = qlx > 1 ? qlx - 1 : 0;                 // log2 region columns per tile
    const int kxn = qlx > 0 ? 2 : 1, kyn = qly > 0 ? 2 : 1;
    const int qxb = (rg & ((1 << rlx) - 1)) * kxn, qyb = (rg >> rlx) * kyn;
    r.ox = (tx << V.tsx) + kQuad * qxb;
    r.oy = (ty << V.tsy) + kQuad * qyb;
    r.valid = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int kx = k & 1, ky = k >> 1;
        r.quad[k] = (qxb + kx) + ((qyb + ky) << qlx);
        const bool ok = kx < kxn && ky < kyn && r.ox + kQuad * kx < V.W && r.oy + kQuad * ky < V.H;
        r.qbit[k] = ok ? quad_subrect_bits(r.quad[k], V.tsx, V.tsy) << 28 : 0u;
        r.valid |= ok ? (1u << k) : 0u;
    }
    // quadrant 0 exists whenever any does (it holds the region's origin)
    return r.valid != 0u;
}

// Pass 1 over regions of up to 2 x 2 quadrants (one wave per region, region
// r of a tile covering quadrant columns 2 rx + kx and rows 2 ry + ky, k =
// kx + 2 ky): the wave reads the tile list once for its quadrants, gathers
// each candidate's records once, tests it against each of its quadrants with
// quad_hit and composites the four pixels of each lane (one per quadrant, at
// the lane's position inside the quadrant).  Per quadrant everything is
// k_pass1's: the sub-rectangle bit and the exact test on the mean taken
// relative to the quadrant's origin in the same float operations, the
// staged entries in list order, the pixel arithmetic and the stop at the
// same 64-entry slice boundaries (a quadrant whose rays have all stopped
// takes no further entries), so the results are bit-identical; what is
// shared is the list walk and the record loads.  Instead of one compacted
// list per quadrant the wave leaves one per region: the Gaussian index of
// every entry that reaches one of its quadrants, with the quadrant bits in
// the top four bits (per quadrant, exactly the entries of its compacted
// list), for k_pass2_region.
// Every query mode (per-channel queries: the three objectives of
// k_pass1 per pixel), one wave per region, no quadrant list.
template <int kMode>
__global__ __launch_bounds__(kWave) void k_pass1_region(CompositeArgs a) {
    constexpr bool kCh = kMode == kModeChannel;
    __shared__ RegionRec rec[kWave];
    const int lane = threadIdx.x;
    const int nreg = a.total_tiles << a.region_log;
    const int logical = a.xcd_remap ? xcd_remap(blockIdx.x, (nreg + 7) & ~7) : (int)blockIdx.x;
    if (logical >= nreg) return;
    RegionSetup R;
    if (!setup_region(a, logical, R)) return;
    const int gt = R.gt, v = R.v, ox = R.ox, oy = R.oy;
    const uint32_t valid = R.valid;
    const SceneSlot &S = *R.S;
    const ViewDev &V = *R.V;
    const int lx = lane & 7, ly = lane >> 3;
    const float xl = (float)lx + 0.5f, yl = (float)ly + 0.5f;
    const float fx0 = (float)ox, fx1 = (float)(ox + kQuad), fy0 = (float)oy, fy1 = (float)(oy + kQuad);
    bool inside[4], scored[4], done[4];
    int64_t ray_local[4];
    float T[4], A[4], AG[4], AB[4];   // AG, AB: the G and B objectives of per-channel queries
    uint32_t alive = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int px = ox + kQuad * (k & 1) + lx, py = oy + kQuad * (k >> 1) + ly;
        inside[k] = ((valid >> k) & 1u) && px < V.W && py < V.H;
        ray_local[k] = V.ray_local + (int64_t)py * V.W + px;
        scored[k] = inside[k] && ray_selected(S.ray_mask, V.ray_base + (int64_t)py * V.W + px);
        T[k] = 1.0f;
        A[k] = 0.0f;
        AG[k] = 0.0f;
        AB[k] = 0.0f;
        done[k] = !scored[k];
        alive |= (((valid >> k) & 1u) && !__all(done[k])) ? (1u << k) : 0u;
    }
    const uint64_t start = S.tile_off[gt - S.tile0], end = S.tile_off[gt - S.tile0 + 1];
    const int64_t vbase = (int64_t)(v - S.view0) * S.N;
    const float cmax = __uint_as_float(S.cmax[v - S.view0]);
    const float cut = a.r2_log2;
    // the region's list: entries that reach one of its quadrants, each with
    // its quadrant bits (in the slots of quadrant 0's compacted list)
    uint32_t *cl = S.clist ? S.clist + ((start << a.quad_log) + (uint64_t)R.quad[0] * (end - start) - a.clist_shift)
                           : nullptr;
    uint32_t ccnt = 0u;
    const uint64_t lt = lanemask_lt64();
    for (uint64_t e0 = start; e0 < end && alive; e0 += kWave) {
        const uint64_t e = e0 + lane;
        const uint32_t raw = e < end ? S.lists[e] : 0u;
        uint32_t want = 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k) want |= ((alive >> k) & 1u) ? R.qbit[k] : 0u;
        uint32_t h = 0u;
        const uint32_t g = raw & kIndexMask;
        const int64_t o = vbase + g;
        float4 r1 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float mx0 = 0.0f, my0 = 0.0f, mx1 = 0.0f, my1 = 0.0f;
        if (raw & want) {
            const float4 r0 = S.R[o].m;
            r1 = S.R[o].q;
            mx0 = (r0.x - fx0) + r0.z;
            my0 = (r0.y - fy0) + r0.w;
            mx1 = (r0.x - fx1) + r0.z;
            my1 = (r0.y - fy1) + r0.w;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (((alive >> k) & 1u) && (raw & R.qbit[k]) &&
                    quad_hit((k & 1) ? mx1 : mx0, (k >> 1) ? my1 : my0, r1.x, r1.y, r1.z, cut))
                    h |= 1u << k;
        }
        const uint64_t bal = __ballot(h != 0u);
        const int n = __popcll(bal);
        if (h) {
            const int slot = __popcll(bal & lt);
            RegionRec &q = rec[slot];
            const float4 sg = scaled_geo(mx0, my0, r1.x, r1.y);
            q.g = sg;
            q.m1 = make_float2(-sg.w * mx1, my1);
            if (kCh) {
                // as stage_raw with kChannel: (g', alpha, c_R, c_G), c_B
                const float4 c3 = S.R3[o];
                q.c = make_float4(r1.z, r1.w, c3.x, c3.y);
                q.cblue = c3.z;
            } else {
                const float cb = S.CB[o];
                const float la = __builtin_amdgcn_logf(r1.w);
                q.c = make_float4(r1.z, la, cb, cut + la);
            }
        }
        if (cl && h)
            __builtin_nontemporal_store((a.clist_pos ? (uint32_t)(e - start) : g) | (h << 28),
                                        &cl[ccnt + (uint32_t)__popcll(bal & lt)]);
        ccnt += (uint32_t)n;
        uint64_t bq[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) bq[k] = __ballot((h >> k) & 1u);
        wave_sync();
        // Slot j holds the entry of the j-th lane of bal in lane order; its
        // quadrant bits are that lane's bits of bq[k] (scalar work only).  Two
        // slots per iteration share one LDS address; a slot past n has no bits.
        uint64_t rem = bal;
        for (int j = 0; j < n; j += 2) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const uint64_t lowbit = rem & (~rem + 1ull);
                rem ^= lowbit;
                const RegionRec &q = rec[j + u];
                const float4 G = q.g, C = q.c;
                const float2 M1 = q.m1;
                // offsets from the mean per quadrant column and row and the
                // row's part of the exponent, formed once for the quadrants
                // that share them (the operations of pair_rho_log2, or of
                // pair_rho for per-channel queries)
                const float dxq[2] = {fmaf(G.w, xl, G.x), fmaf(G.w, xl, M1.x)};
                const float dy0 = yl - G.y, dy1 = yl - M1.y;
                const float dyq[2] = {dy0, dy1};
                const float tq[2] = {kCh ? C.x * (dy0 * dy0) : fmaf(C.x, dy0 * dy0, C.y),
                                     kCh ? C.x * (dy1 * dy1) : fmaf(C.x, dy1 * dy1, C.y)};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (bq[k] & lowbit) {
                        const float uu = fmaf(G.z, dyq[k >> 1], dxq[k & 1]);
                        const float P = fmaf(-uu, uu, tq[k >> 1]);
                        const float E = __builtin_amdgcn_exp2f(P);
                        const float rho = kCh ? (P >= cut ? C.y * E : 0.0f) : (P >= C.w ? E : 0.0f);
                        if (kMode == kModeL1) {
                            const float cr = C.z * rho;
                            A[k] = fmaf(cr, T[k], A[k]);
                        } else if (kMode == kModeL2) {
                            const float rt = rho * T[k];
                            A[k] = fmaf(C.z * rt, rt, A[k]);
                        } else {
                            const float rt = rho * T[k];
                            A[k] = fmaf(C.z, rt, A[k]);
                            AG[k] = fmaf(C.w, rt, AG[k]);
                            AB[k] = fmaf(q.cblue, rt, AB[k]);
                        }
                        T[k] = fmaf(-rho, T[k], T[k]);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (kMode == kModeL1) done[k] = done[k] || (T[k] * cmax < a.share_floor * A[k]);
            if (kMode == kModeL2) done[k] = done[k] || ((T[k] * T[k]) * cmax < a.share_floor * A[k]);
            if (kCh) done[k] = done[k] || (T[k] * cmax < a.share_floor * fminf(A[k], fminf(AG[k], AB[k])));
            if (((alive >> k) & 1u) && __all(done[k])) alive &= ~(1u << k);
        }
        wave_sync();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (inside[k]) {
            S.ray_A[ray_local[k]] = scored[k] ? A[k] : 0.0f;
            if (kCh) {
                S.ray_A[S.ray_stride + ray_local[k]] = scored[k] ? AG[k] : 0.0f;
                S.ray_A[2 * S.ray_stride + ray_local[k]] = scored[k] ? AB[k] : 0.0f;
            }
        }
    }
    if (cl && lane == 0) a.ccount[((gt - a.tile_first) << a.quad_log) + R.quad[0]] = ccnt;
}

// Transposed butterfly over 64 lanes for 16 values: afterwards lane L holds
// the maximum over all 64 lanes of value (L >> 2) & 15.  Each level pairs
// every lane with a partner on the other side of one lane-index bit; the
// lane keeps one half of its values and sends the other half, which is the
// half its partner keeps:
//   bit 5: v_permlane32_swap (upper 32 lanes of one register <-> lower 32 of another)
//   bit 4: v_permlane16_swap (odd 16-lane rows <-> even rows)
//   bit 3: DPP row_mirror (i <-> 15-i in a row), bit 2: row_half_mirror (i <-> 7-i),
// then two plain reductions over bits 1 and 0 (quad_perm [2,3,0,1], [1,0,3,2]).
// Every index is a compile-time constant, so the values stay in registers.
// The shares are non-negative floats, whose order is that of their bit
// patterns as unsigned integers: the maxima are taken as such (v_max_u32,
// with the DPP move folded in and no NaN canonicalisation).
__device__ __forceinline__ uint32_t umax32(uint32_t a, uint32_t b) { return a > b ? a : b; }

template <int kCtrl>
__device__ __forceinline__ uint32_t dpp_umax(uint32_t keep, uint32_t send) {
    return umax32(keep, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)send, kCtrl, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_transpose_max16(const float (&sh)[16]) {
    const int lane = threadIdx.x & 63;
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(sh[k]), __float_as_uint(sh[k + 8]),
                                                        false, false);
        v[k] = umax32(r[0], r[1]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const auto r = __builtin_amdgcn_permlane16_swap(v[k], v[k + 4], false, false);
        v[k] = umax32(r[0], r[1]);
    }
    const bool s3 = (lane & 8) != 0, s2 = (lane & 4) != 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) v[k] = dpp_umax<0x140>(s3 ? v[k + 2] : v[k], s3 ? v[k] : v[k + 2]);
    v[0] = dpp_umax<0x141>(s2 ? v[1] : v[0], s2 ? v[0] : v[1]);
    v[0] = dpp_umax<0x4E>(v[0], v[0]);
    return __uint_as_float(dpp_umax<0xB1>(v[0], v[0]));
}

template <int kCtrl>
__device__ __forceinline__ float dpp_add(float x) {
    const float y = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xF, 0xF, false));
    return x + y;
}

// The 16-value network with sums instead of maxima: lane L ends with the sum
// over all 64 lanes of value (L >> 2) & 15 (each level pairs disjoint lane
// sets, so every lane's value is counted once).
__device__ __forceinline__ float wave_transpose_sum16(float (&v)[16]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]), __float_as_uint(v[k + 8]),
                                                        false, false);
        v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[k]), __float_as_uint(v[k + 4]),
                                                        false, false);
        v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool s3 = (lane & 8) != 0, s2 = (lane & 4) != 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float m0 = dpp_add<0x140>(v[k]), m1 = dpp_add<0x140>(v[k + 2]);
        v[k] = s3 ? m1 : m0;
    }
    {
        const float m0 = dpp_add<0x141>(v[0]), m1 = dpp_add<0x141>(v[1]);
        v[0] = s2 ? m1 : m0;
    }
    return dpp_add<0xB1>(dpp_add<0x4E>(v[0]));
}

template <bool kStats, bool kPersistent, int kAgg, int kMode, bool kCompact>
__global__ __launch_bounds__(kWave, kPersistent ? 5 : ((kAgg != 0 || kMode == kModeChannel) ? 6 : 7))
void k_pass2(CompositeArgs a, uint64_t *__restrict__ counters) {
    static_assert(!(kAgg != 0 && kMode == kModeChannel), "per-channel queries have no aggregated form");
    static_assert(!(kAgg != 0 && kCompact), "aggregated queries walk the tile lists");
    constexpr bool kCh = kMode == kModeChannel;
    __shared__ float4 geo[kWave], col[kWave];
    __shared__ uint32_t sid[kWave];
    __shared__ float sold[kWave];
    __shared__ float cblue[kCh ? kWave : 1];
    const int lane = threadIdx.x;
    const int nq = quad_count(a);
    int iter = 0;
    uint64_t pin = 0, plive = 0, pos = 0, peval = 0, pamb = 0;
    for (int qi = next_quad<kPersistent>(a, iter); qi < nq; qi = next_quad<kPersistent>(a, iter)) {
        WaveSetup w;
        if (!setup_quad(a, qi, w)) continue;
        const bool scored = w.inside && ray_selected(w.ray_mask, w.ray_global);
        const float Af = scored ? w.ray_A[w.ray_local] : 0.0f;
        const float invA = Af > 0.0f ? 1.0f / Af : 0.0f;
        // per channel: the G and B objectives, and the smallest of the three
        // (the stop bar); a ray counts as positive if one of them is
        float invG = 0.0f, invB = 0.0f, Amin = Af;
        bool positive = invA > 0.0f;
        if (kCh) {
            const float AG = scored ? w.ray_A[w.ray_stride + w.ray_local] : 0.0f;
            const float AB = scored ? w.ray_A[2 * w.ray_stride + w.ray_local] : 0.0f;
            invG = AG > 0.0f ? 1.0f / AG : 0.0f;
            invB = AB > 0.0f ? 1.0f / AB : 0.0f;
            Amin = fminf(Af, fminf(AG, AB));
            positive = positive || invG > 0.0f || invB > 0.0f;
        }
        // the share's denominator: the ray's A, or the A of the lane's query
        float invQ = invA;
        if (kAgg != 0) {
            // (per-tile queries take this form only with 16x16 binning
            // tiles, where a tile is one region and its own query)
            const double qA = kAgg == 1 ? a.query_A[w.gt] : (kAgg == 2 ? a.query_A[w.v] : a.query_A[0]);
            invQ = (invA > 0.0f && qA > 0.0) ? (float)(1.0 / qA) : 0.0f;
        }
        const float cmax = w.cmax;
        uint32_t *sens_bits = w.sens_bits;
        // One query per ray: the running transmittance is kept scaled, by
        // 1/A(Q) for L1 shares (share = c rho T / A(Q) = c rho T') and by
        // 1/sqrt(A(Q)) for L2 shares (c (rho T')^2), and the stop bar with it.
        // Per channel: T itself.
        const float tscale = kCh ? 1.0f : (kMode == kModeL2 ? sqrtf(invQ) : invQ);
        float T = tscale;
        bool done = !positive;
        uint32_t n_in = 0, n_live = 0, n_eval = 0, n_amb = 0;
        const float amb_band = kAmbiguityBeta * fabsf(a.r2_log2);
        const float live_bar = kCh ? a.share_floor * Amin : a.share_floor * (Amin * invQ);
        // the quadrant's entries: its compacted list from pass 1, or its
        // tile's list filtered again
        const uint32_t *cl = kCompact ? w.clist + w.cbase : nullptr;
        const uint64_t lo = kCompact ? 0 : w.start, hi = kCompact ? (uint64_t)a.ccount[qi] : w.end;
        for (uint64_t e0 = lo; e0 < hi; e0 += kWave) {
            if (__all(done)) break;
            int n;
            if (kCompact)
                n = stage_compact<kBlock, kCh, !kCh>(w, cl + e0, (uint32_t)(hi - e0), a.r2_log2, geo, col, sid,
                                                     sold, cblue);
            else
                n = stage_slice<kAgg == 0 ? 1 : 3, kBlock, kCh, !kCh>(w, e0, a.r2_log2, geo, col, sid, sold,
                                                                      nullptr, cblue);
            wave_sync();
            for (int jb = 0; jb < n; jb += 16) {
                float sh[16];
#pragma unroll
                for (int k0 = 0; k0 < 16; k0 += kBlock) {
                    if (jb + k0 < n) {
#pragma unroll
                        for (int q = 0; q < kBlock; ++q) {
                            const int j = jb + k0 + q;
                            const float4 G = geo[j], Cc = col[j];
                            bool in_fp;
                            const float rho = kCh ? pair_rho(G, Cc, w.xl, w.yl, a.r2_log2, in_fp)
                                                  : pair_rho_log2(G, Cc, w.xl, w.yl, in_fp);
                            if (kMode == kModeL1) {
                                sh[k0 + q] = Cc.z * (rho * T);
                            } else if (kMode == kModeL2) {
                                const float rt = rho * T;
                                sh[k0 + q] = Cc.z * (rt * rt);
                            } else {
                                const float rt = rho * T;
                                sh[k0 + q] = rt * fmaxf(Cc.z * invA, fmaxf(Cc.w * invG, cblue[j] * invB));
                            }
                            if (kStats) {
                                const bool real = j < n;
                                const float later = kMode == kModeL2 ? (T * T) * cmax : T * cmax;
                                n_in += (real && in_fp) ? 1u : 0u;
                                n_live += (real && in_fp && later >= live_bar) ? 1u : 0u;
                                // the exponent against the cutoff, as pair_rho(_log2) forms
                                // them: P - bar = -(log2 e / 2)(d^2 - r^2)
                                const float ddx = fmaf(G.w, w.xl, G.x), ddy = w.yl - G.y;
                                const float uu = fmaf(G.z, ddy, ddx);
                                const float tt = kCh ? Cc.x * (ddy * ddy) : fmaf(Cc.x, ddy * ddy, Cc.y);
                                const float PP = fmaf(-uu, uu, tt);
                                const float bar = kCh ? a.r2_log2 : Cc.w;
                                n_amb += (real && positive && fabsf(PP - bar) <= amb_band) ? 1u : 0u;
                            }
                            T = fmaf(-rho, T, T);
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < kBlock; ++q) sh[k0 + q] = 0.0f;
                    }
                }
                if (kStats) n_eval += (uint32_t)min(16, n - jb);
                const int j = jb + (lane >> 2);
                if (kAgg == 0) {
                    // the reduction is needed only if some pixel beats the
                    // staged sensitivity of its entry (padded entries have
                    // share 0, which beats no sensitivity)
                    // (one compare per value, its lane mask OR-ed in scalar registers)
                    uint64_t beat = 0ull;
#pragma unroll
                    for (int k = 0; k < 16; ++k) beat |= __ballot(sh[k] > sold[jb + k]);
                    if (beat != 0ull) {
                        // (a share cannot exceed 1; its rounding can, by an ulp or two)
                        const float m = fminf(wave_transpose_max16(sh), 1.0f);
                        if ((lane & 3) == 0 && j < n && m > sold[j])
                            atomicMax(&sens_bits[sid[j]], __float_as_uint(m));
                    }
                } else {
                    const float m = wave_transpose_sum16(sh);
                    if ((lane & 3) == 0 && j < n && m > 0.0f) {
                        const int64_t idx = kAgg == 1 ? (int64_t)(w.start + __float_as_uint(sold[j]))
                                                      : (kAgg == 2 ? w.vbase + sid[j] : (int64_t)sid[j]);
                        atomicAdd((unsigned long long *)&a.acc[idx], (unsigned long long)fma((double)m, kAggScale, 0.5));
                    }
                }
            }
            const float later = kMode == kModeL2 ? (T * T) * cmax : T * cmax;
            done = done || (later < live_bar);
            wave_sync();
        }
        if (kStats) {
            pin += positive ? n_in : 0u;
            plive += positive ? n_live : 0u;
            pos += positive ? 1u : 0u;
            peval += (uint64_t)n_eval;
            pamb += n_amb;
            if (n_amb && a.amb_rays)
                atomicOr(&a.amb_rays[w.ray_global >> 5], 1u << (uint32_t)(w.ray_global & 31));
        }
    }
    if (kStats) {
        for (int off = 32; off > 0; off >>= 1) {
            pin += __shfl_xor(pin, off);
            plive += __shfl_xor(plive, off);
            pos += __shfl_xor(pos, off);
            pamb += __shfl_xor(pamb, off);
        }
        if (lane == 0) {
            unsigned long long *c = (unsigned long long *)counters + CNT_SLOTS + (blockIdx.x % kCntSpread);
            atomicAdd(c + 0 * kCntSpread, (unsigned long long)pin);
            atomicAdd(c + 1 * kCntSpread, (unsigned long long)plive);
            atomicAdd(c + 2 * kCntSpread, (unsigned long long)pos);
            atomicAdd(c + 3 * kCntSpread, (unsigned long long)peval * 64ull);
            if (pamb) atomicAdd(c + 4 * kCntSpread, (unsigned long long)pamb);
        }
    }
}

// Pass 2 over regions of up to 2 x 2 quadrants, on the region lists that
// k_pass1_region leaves.  Per quadrant the wave takes the entries of its
// compacted list in the same order, with the same pixel arithmetic and the
// same shares as k_pass2; a quadrant whose rays have all stopped (tested at
// 64-entry slices of the region list) takes no further entries, which
// changes nothing that is reported (no share after a ray's stop reaches the
// share floor).  What is shared: each entry's record loads and staging, the
// offsets and row terms of the quadrants' pixels, and the reduction: a
// lane's values of its four pixels are maximised first (integer maxima of
// the bit patterns of non-negative floats), then one transposed butterfly
// and at most one atomic per entry instead of one per (quadrant, entry).
// The value reduced is x = rho T (L1) or (rho T)^2 (L2), of which the share
// is c x: one product per entry instead of one per pair.
// With kAgg (1: per-tile, 2: per-image, 3: per-scene queries) the shares are
// against the query's A and summed instead: per quadrant, the 16 entries'
// shares go through the transposed sum of k_pass2 (the same per-pixel shares
// and the same sums over each quadrant's 64 pixels), each sum becomes u64
// fixed point as there, and the quadrants' integers are added before one
// atomic per entry.  Per-tile queries (16x16 binning tiles: one region per
// tile, so a region is one whole query) take the share's maximum at once when
// the region lists hold Gaussians; with list positions
// (CompositeArgs::clist_pos) they accumulate per list entry instead.
template <bool kStats, int kMode, int kAgg = 0>
__global__ __launch_bounds__(kWave, kStats ? 5 : 7) void k_pass2_region(CompositeArgs a,
                                                                         uint64_t *__restrict__ counters) {
    constexpr bool kCh = kMode == kModeChannel;
    static_assert(!(kCh && kAgg != 0), "per-channel queries have no aggregated form");
    static_assert(kAgg >= 0 && kAgg <= 3, "query granularities 0 (ray) to 3 (scene)");
    static_assert(!(kAgg != 0 && kStats), "aggregated queries count no pairs");
    __shared__ RegionRec rec[kWave];
    const int lane = threadIdx.x;
    const int nreg = a.total_tiles << a.region_log;
    const int logical = a.xcd_remap ? xcd_remap(blockIdx.x, (nreg + 7) & ~7) : (int)blockIdx.x;
    if (logical >= nreg) return;
    RegionSetup R;
    if (!setup_region(a, logical, R)) return;
    const int gt = R.gt, v = R.v, ox = R.ox, oy = R.oy;
    const SceneSlot &S = *R.S;
    const ViewDev &V = *R.V;
    const int lx = lane & 7, ly = lane >> 3;
    const float xl = (float)lx + 0.5f, yl = (float)ly + 0.5f;
    const float fx0 = (float)ox, fx1 = (float)(ox + kQuad), fy0 = (float)oy, fy1 = (float)(oy + kQuad);
    // per quadrant: the running transmittance scaled as in k_pass2 (by 1/A
    // for L1, 1/sqrt(A) for L2), the stop bar and whether the ray counts
    // (per-channel queries: T itself, the three objectives' reciprocals and
    // the smallest objective's bar, as k_pass2)
    float T[4], live_bar[4], invR[4], invG[4], invB[4];
    bool done[4], positive[4];
    int64_t ray_global[4];
    uint32_t alive = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int px = ox + kQuad * (k & 1) + lx, py = oy + kQuad * (k >> 1) + ly;
        const bool inside = ((R.valid >> k) & 1u) && px < V.W && py < V.H;
        ray_global[k] = V.ray_base + (int64_t)py * V.W + px;
        const bool scored = inside && ray_selected(S.ray_mask, ray_global[k]);
        const int64_t rl = V.ray_local + (int64_t)py * V.W + px;
        const float Af = scored ? S.ray_A[rl] : 0.0f;
        const float invA = Af > 0.0f ? 1.0f / Af : 0.0f;
        positive[k] = invA > 0.0f;
        if (kCh) {
            const float AG = scored ? S.ray_A[S.ray_stride + rl] : 0.0f;
            const float AB = scored ? S.ray_A[2 * S.ray_stride + rl] : 0.0f;
            invR[k] = invA;
            invG[k] = AG > 0.0f ? 1.0f / AG : 0.0f;
            invB[k] = AB > 0.0f ? 1.0f / AB : 0.0f;
            positive[k] = positive[k] || invG[k] > 0.0f || invB[k] > 0.0f;
            T[k] = 1.0f;
            live_bar[k] = a.share_floor * fminf(Af, fminf(AG, AB));
            done[k] = !positive[k];
            alive |= (((R.valid >> k) & 1u) && !__all(done[k])) ? (1u << k) : 0u;
            continue;
        }
        // the share's denominator: the ray's A, or the A of the ray's query
        float invQ = invA;
        if (kAgg != 0) {
            // (per-tile queries: the region's own A(Q), entry (tile << region_log) + region)
            const double qA = kAgg == 1 ? a.query_A[((int64_t)gt << a.region_log) + (logical & ((1 << a.region_log) - 1))]
                                        : (kAgg == 2 ? a.query_A[v] : a.query_A[0]);
            invQ = (invA > 0.0f && qA > 0.0) ? (float)(1.0 / qA) : 0.0f;
        }
        T[k] = kMode == kModeL2 ? sqrtf(invQ) : invQ;
        live_bar[k] = a.share_floor * (Af * invQ);
        done[k] = !positive[k];
        alive |= (((R.valid >> k) & 1u) && !__all(done[k])) ? (1u << k) : 0u;
    }
    const uint64_t start = S.tile_off[gt - S.tile0], end = S.tile_off[gt - S.tile0 + 1];
    const uint32_t *__restrict__ cl =
        S.clist + ((start << a.quad_log) + (uint64_t)R.quad[0] * (end - start) - a.clist_shift);
    const uint32_t count = a.ccount[((gt - a.tile_first) << a.quad_log) + R.quad[0]];
    const int64_t vbase = (int64_t)(v - S.view0) * S.N;
    const float cmax = __uint_as_float(S.cmax[v - S.view0]);
    const float cut = a.r2_log2;
    const float amb_band = kAmbiguityBeta * fabsf(a.r2_log2);
    uint32_t *sens_bits = S.sens_bits;
    uint32_t n_in = 0, n_live = 0, n_amb = 0, amb = 0u;   // amb: quadrants whose ray saw an ambiguous pair
    uint64_t n_eval = 0;
    const uint64_t lt = lanemask_lt64();
    for (uint32_t e0 = 0; e0 < count && alive; e0 += kWave) {
        const uint32_t e = e0 + lane;
        const uint32_t raw = e < count ? cl[e] : 0u;
        const uint32_t h = (raw >> 28) & alive;
        const uint64_t bal = __ballot(h != 0u);
        const int n = __popcll(bal);
        if (h) {
            // (per-tile queries: the list holds the entry's position in the
            // tile's list, whose entry gives the Gaussian)
            const uint32_t pos = raw & kIndexMask;
            const uint32_t g = (kAgg == 1 && a.clist_pos) ? S.lists[start + pos] & kIndexMask : pos;
            const int64_t o = vbase + g;
            const float4 r0 = S.R[o].m;
            const float4 r1 = S.R[o].q;
            float cb;
            RegionRec &q = rec[__popcll(bal & lt)];
            const float4 sg = scaled_geo((r0.x - fx0) + r0.z, (r0.y - fy0) + r0.w, r1.x, r1.y);
            q.g = sg;
            if (kCh) {
                const float4 c3 = S.R3[o];
                cb = c3.x;
                q.c = make_float4(r1.z, r1.w, c3.x, c3.y);
                q.cblue = c3.z;
            } else {
                cb = S.CB[o];
                const float la = __builtin_amdgcn_logf(r1.w);
                q.c = make_float4(r1.z, la, cb, cut + la);
            }
            q.m1 = make_float2(-sg.w * ((r0.x - fx1) + r0.z), (r0.y - fy1) + r0.w);
            q.sid = (kAgg == 1 && a.clist_pos) ? pos : g;
            q.hq = h;
            if (kAgg == 0) {
                const float sold = fmaxf(__uint_as_float(sens_bits[g]), a.report_floor);
                q.sold = sold;
                // c x > sold implies x > sold / (c (1 + 2^-24)); the bar sits
                // below that by more than the rounding of v_rcp_f32 and the
                // products (and is 0, which lets every positive x through, for
                // tiny c)
                if (!kCh)
                    q.bar = (sold > 0.0f && cb >= 0x1p-100f) ? (sold * __builtin_amdgcn_rcpf(cb)) * 0.99999905f : 0.0f;
            }
        }
        uint64_t bq[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) bq[k] = __ballot((h >> k) & 1u);
        if (kStats) n_eval += (uint64_t)(__popcll(bq[0]) + __popcll(bq[1]) + __popcll(bq[2]) + __popcll(bq[3]));
        wave_sync();
        if constexpr (kAgg != 0) {
            // per quadrant, its entries as bits in slot order (slot j is the
            // j-th lane of bal): the loops below test one bit per slot
            const uint32_t hs = lane < n ? rec[lane].hq : 0u;
            uint64_t sq[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) sq[k] = __ballot((hs >> k) & 1u);
            for (int jb = 0; jb < n; jb += 16) {
                uint64_t acc = 0ull;   // lane 4 i: entry jb + i's fixed-point sum over the quadrants
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t m16 = ((alive >> k) & 1u) ? (uint32_t)(sq[k] >> jb) & 0xFFFFu : 0u;
                    if (!m16) continue;
                    float sh[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        float share = 0.0f;
                        if ((m16 >> i) & 1u) {
                            const RegionRec &q = rec[jb + i];
                            const float4 G = q.g, C = q.c;
                            const float mx = (k & 1) ? q.m1.x : G.x, my = (k >> 1) ? q.m1.y : G.y;
                            bool in_fp;
                            const float rho = pair_rho_log2(make_float4(mx, my, G.z, G.w), C, xl, yl, in_fp);
                            const float rt = rho * T[k];
                            share = kMode == kModeL1 ? C.z * rt : C.z * (rt * rt);
                            T[k] = fmaf(-rho, T[k], T[k]);
                        }
                        sh[i] = share;
                    }
                    const float m = wave_transpose_sum16(sh);
                    acc += m > 0.0f ? (uint64_t)fma((double)m, kAggScale, 0.5) : 0ull;
                }
                const int j = jb + (lane >> 2);
                if ((lane & 3) == 0 && j < n && acc) {
                    if (kAgg == 1 && !a.clist_pos) {
                        // the region is the whole 16x16 query and the list
                        // holds the Gaussian: the sum is complete, so its share
                        // raises the sensitivity here (the value k_agg_tile_max
                        // takes from an accumulator of the same integers)
                        const float sq_share = (float)((double)acc * (1.0 / kAggScale));
                        if (sq_share > 0.0f) atomicMax(&sens_bits[rec[j].sid], __float_as_uint(sq_share));
                    } else {
                        const int64_t idx = kAgg == 1 ? (int64_t)(start + rec[j].sid)
                                                      : (kAgg == 2 ? vbase + rec[j].sid : (int64_t)rec[j].sid);
                        atomicAdd((unsigned long long *)&a.acc[idx], (unsigned long long)acc);
                    }
                }
            }
        } else {
            // per quadrant, its entries as bits in slot order (slot j is the
            // j-th lane of bal): one bit test per slot and quadrant
            const uint32_t hs = lane < n ? rec[lane].hq : 0u;
            uint64_t sq[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) sq[k] = __ballot((hs >> k) & 1u);
            for (int jb = 0; jb < n; jb += 16) {
                uint32_t mq[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) mq[k] = (uint32_t)(sq[k] >> jb) & 0xFFFFu;
                const uint32_t mall = mq[0] | mq[1] | mq[2] | mq[3];
                float sh[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    uint32_t m = 0u;
                    if ((mall >> i) & 1u) {
                        const RegionRec &q = rec[jb + i];
                        const float4 G = q.g, C = q.c;
                        const float2 M1 = q.m1;
                        const float dxq[2] = {fmaf(G.w, xl, G.x), fmaf(G.w, xl, M1.x)};
                        const float dy0 = yl - G.y, dy1 = yl - M1.y;
                        const float dyq[2] = {dy0, dy1};
                        const float tq[2] = {kCh ? C.x * (dy0 * dy0) : fmaf(C.x, dy0 * dy0, C.y),
                                             kCh ? C.x * (dy1 * dy1) : fmaf(C.x, dy1 * dy1, C.y)};
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            if ((mq[k] >> i) & 1u) {
                                const float uu = fmaf(G.z, dyq[k >> 1], dxq[k & 1]);
                                const float P = fmaf(-uu, uu, tq[k >> 1]);
                                const float E = __builtin_amdgcn_exp2f(P);
                                const float bar = kCh ? cut : C.w;
                                const bool in_fp = P >= bar;
                                const float rho = in_fp ? (kCh ? C.y * E : E) : 0.0f;
                                const float rt = rho * T[k];
                                float x;
                                if (kCh) {
                                    // the share itself, as k_pass2 forms it
                                    x = rt * fmaxf(C.z * invR[k], fmaxf(C.w * invG[k], q.cblue * invB[k]));
                                } else {
                                    // the share is c x, and c x is monotone in
                                    // x: the entry's largest share is c times
                                    // its largest x (rounding is monotone too)
                                    x = kMode == kModeL1 ? rt : rt * rt;
                                }
                                m = umax32(m, __float_as_uint(x));
                                if (kStats) {
                                    const float later = kMode == kModeL2 ? (T[k] * T[k]) * cmax : T[k] * cmax;
                                    n_in += (positive[k] && in_fp) ? 1u : 0u;
                                    n_live += (positive[k] && in_fp && later >= live_bar[k]) ? 1u : 0u;
                                    const bool am = positive[k] && fabsf(P - bar) <= amb_band;
                                    n_amb += am ? 1u : 0u;
                                    amb |= am ? (1u << k) : 0u;
                                }
                                T[k] = fmaf(-rho, T[k], T[k]);
                            }
                        }
                    }
                    sh[i] = __uint_as_float(m);
                }
                // the reduction only if some pixel beats its entry's staged
                // sensitivity (slots past n hold share 0, which beats none)
                uint64_t beat = 0ull;
#pragma unroll
                for (int i = 0; i < 16; ++i) beat |= __ballot(sh[i] > (kCh ? rec[jb + i].sold : rec[jb + i].bar));
                if (beat != 0ull) {
                    const float mx = wave_transpose_max16(sh);
                    const int j = jb + (lane >> 2);
                    if ((lane & 3) == 0 && j < n) {
                        // (a share cannot exceed 1; its rounding can, by an ulp or two)
                        const float share = fminf(kCh ? mx : rec[j].c.z * mx, 1.0f);
                        if (share > rec[j].sold) atomicMax(&sens_bits[rec[j].sid], __float_as_uint(share));
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float later = kMode == kModeL2 ? (T[k] * T[k]) * cmax : T[k] * cmax;
            done[k] = done[k] || (later < live_bar[k]);
            if (((alive >> k) & 1u) && __all(done[k])) alive &= ~(1u << k);
        }
        wave_sync();
    }
    if (kStats) {
        uint64_t pin = n_in, plive = n_live, pos = 0, pamb = n_amb;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            pos += positive[k] ? 1u : 0u;
            if (((amb >> k) & 1u) && a.amb_rays)
                atomicOr(&a.amb_rays[ray_global[k] >> 5], 1u << (uint32_t)(ray_global[k] & 31));
        }
        for (int off = 32; off > 0; off >>= 1) {
            pin += __shfl_xor(pin, off);
            plive += __shfl_xor(plive, off);
            pos += __shfl_xor(pos, off);
            pamb += __shfl_xor(pamb, off);
        }
        if (lane == 0) {
            unsigned long long *c = (unsigned long long *)counters + CNT_SLOTS + (blockIdx.x % kCntSpread);
            atomicAdd(c + 0 * kCntSpread, (unsigned long long)pin);
            atomicAdd(c + 1 * kCntSpread, (unsigned long long)plive);
            atomicAdd(c + 2 * kCntSpread, (unsigned long long)pos);
            atomicAdd(c + 3 * kCntSpread, (unsigned long long)n_eval * 64ull);
            if (pamb) atomicAdd(c + 4 * kCntSpread, (unsigned long long)pamb);
        }
    }
}

// Flat form: one wave per quadrant (rounded up to a multiple of 8 for the XCD
// remap).  Persistent form: as many waves as the chip holds at once for the
// kernel (its occupancy times the CU count), taking quadrants from a counter.
template <typename K>
static unsigned resident_waves(K kernel) {
    int dev = 0, cus = 256, per_cu = 8;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave, 0) != hipSuccess) {
        (void)hipGetLastError();
        cus = 256;
        per_cu = 8;
    }
    return (unsigned)std::max(1, cus) * (unsigned)std::max(1, per_cu);
}

static inline unsigned flat_grid(const CompositeArgs &a) {
    if (a.quad_list) return (unsigned)std::max(a.n_listed, 1);
    return (unsigned)(((a.total_tiles << a.quad_log) + 7) & ~7);
}

// The flat form over every quadrant runs by regions (k_pass1_region,
// bit-identical, every query mode); runs over a quadrant list (sparse ray
// masks) and the persistent form run by quadrants.
template <int kMode>
static void pass1_mode(const CompositeArgs &a, hipStream_t st) {
    if constexpr (kMode != kModeChannel) {
        if (a.work) {
            static const unsigned grid = resident_waves(k_pass1<true, kMode>);
            launch_fill_u32(a.work, 0u, 1, st);
            hipLaunchKernelGGL((k_pass1<true, kMode>), dim3(grid), dim3(kWave), 0, st, a);
            return;
        }
    }
    if (!a.quad_list) {
        const unsigned grid = (unsigned)(((a.total_tiles << a.region_log) + 7) & ~7);
        hipLaunchKernelGGL((k_pass1_region<kMode>), dim3(grid), dim3(kWave), 0, st, a);
        return;
    }
    hipLaunchKernelGGL((k_pass1<false, kMode>), dim3(flat_grid(a)), dim3(kWave), 0, st, a);
}

// The persistent form exists for the one-query modes (per-channel launches
// are always flat).
void launch_composite_pass1(const CompositeArgs &a, hipStream_t st) {
    switch (composite_mode(a.query_mode)) {
        case kModeL2: pass1_mode<kModeL2>(a, st); break;
        case kModeChannel: pass1_mode<kModeChannel>(a, st); break;
        default: pass1_mode<kModeL1>(a, st); break;
    }
}

template <int kMode>
static void pass2_agg(const CompositeArgs &a, uint64_t *counters, hipStream_t st) {
    if (a.agg == 1)
        hipLaunchKernelGGL((k_pass2<false, false, 1, kMode, false>), dim3(flat_grid(a)), dim3(kWave), 0, st, a,
                           counters);
    else if (a.agg == 2)
        hipLaunchKernelGGL((k_pass2<false, false, 2, kMode, false>), dim3(flat_grid(a)), dim3(kWave), 0, st, a,
                           counters);
    else
        hipLaunchKernelGGL((k_pass2<false, false, 3, kMode, false>), dim3(flat_grid(a)), dim3(kWave), 0, st, a,
                           counters);
}

template <int kMode, bool kPersistentForm, bool kCompact>
static void pass2_ray(const CompositeArgs &a, bool stats, uint64_t *counters, hipStream_t st) {
    if constexpr (kPersistentForm) {
        if (a.work) {
            launch_fill_u32(a.work, 0u, 1, st);
            if (stats) {
                static const unsigned grid = resident_waves(k_pass2<true, true, 0, kMode, kCompact>);
                hipLaunchKernelGGL((k_pass2<true, true, 0, kMode, kCompact>), dim3(grid), dim3(kWave), 0, st, a,
                                   counters);
            } else {
                static const unsigned grid = resident_waves(k_pass2<false, true, 0, kMode, kCompact>);
                hipLaunchKernelGGL((k_pass2<false, true, 0, kMode, kCompact>), dim3(grid), dim3(kWave), 0, st, a,
                                   counters);
            }
            return;
        }
    }
    if (stats) {
        hipLaunchKernelGGL((k_pass2<true, false, 0, kMode, kCompact>), dim3(flat_grid(a)), dim3(kWave), 0, st, a,
                           counters);
    } else {
        hipLaunchKernelGGL((k_pass2<false, false, 0, kMode, kCompact>), dim3(flat_grid(a)), dim3(kWave), 0, st, a,
                           counters);
    }
}

// With compaction, pass 2 takes the form pass 1 took: the region form (flat
// launches with no quadrant list) reads the region lists, the others the
// quadrant lists.
template <int kMode, bool kPersistentForm>
static void pass2_ray_any(const CompositeArgs &a, bool stats, uint64_t *counters, hipStream_t st) {
    if (a.ccount && !a.work && !a.quad_list) {
        const unsigned grid = (unsigned)(((a.total_tiles << a.region_log) + 7) & ~7);
        if (stats)
            hipLaunchKernelGGL((k_pass2_region<true, kMode>), dim3(grid), dim3(kWave), 0, st, a, counters);
        else
            hipLaunchKernelGGL((k_pass2_region<false, kMode>), dim3(grid), dim3(kWave), 0, st, a, counters);
        return;
    }
    if (a.ccount)
        pass2_ray<kMode, kPersistentForm, true>(a, stats, counters, st);
    else
        pass2_ray<kMode, kPersistentForm, false>(a, stats, counters, st);
}

// Aggregated queries run the flat form without pair counters (by regions on
// the region lists when pass 1 left them);
// per-channel queries have no aggregated or persistent form (the host
// rejects the first).
template <int kMode>
static bool pass2_agg_region(const CompositeArgs &a, hipStream_t st) {
    if (!(a.ccount && !a.work && !a.quad_list && a.agg >= 1 && a.agg <= 3)) return false;
    const unsigned grid = (unsigned)(((a.total_tiles << a.region_log) + 7) & ~7);
    if (a.agg == 1)
        hipLaunchKernelGGL((k_pass2_region<false, kMode, 1>), dim3(grid), dim3(kWave), 0, st, a, nullptr);
    else if (a.agg == 2)
        hipLaunchKernelGGL((k_pass2_region<false, kMode, 2>), dim3(grid), dim3(kWave), 0, st, a, nullptr);
    else
        hipLaunchKernelGGL((k_pass2_region<false, kMode, 3>), dim3(grid), dim3(kWave), 0, st, a, nullptr);
    return true;
}

void launch_composite_pass2(const CompositeArgs &a, bool stats, uint64_t *counters, hipStream_t st) {
    const int mode = composite_mode(a.query_mode);
    if (a.agg != 0) {
        if (mode == kModeL2 && pass2_agg_region<kModeL2>(a, st)) return;
        if (mode == kModeL1 && pass2_agg_region<kModeL1>(a, st)) return;
        if (mode == kModeL2)
            pass2_agg<kModeL2>(a, counters, st);
        else if (mode == kModeL1)
            pass2_agg<kModeL1>(a, counters, st);
        return;
    }
    if (mode == kModeL2)
        pass2_ray_any<kModeL2, true>(a, stats, counters, st);
    else if (mode == kModeChannel)
        pass2_ray_any<kModeChannel, false>(a, stats, counters, st);
    else
        pass2_ray_any<kModeL1, true>(a, stats, counters, st);
}

// ---------------------------------------------------------------------------
// Aggregated queries (Section 3.5): the query objectives A(Q) from the per-ray
// A of pass 1 (zero on rays outside the mask), and the maximum over queries.
// Every sum has a fixed order (per lane in index order, then a fixed
// butterfly), so the results do not depend on scheduling.
__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// One wave per tile: lane l sums the tile's pixels l, l + 64, ... (row-major).
__global__ __launch_bounds__(kWave) void k_tile_A(CompositeArgs a, double *__restrict__ tile_A) {
    // one wave per region (up to 2 x 2 quadrants, as setup_region places
    // them): with binning tiles of 16 or 32 pixels per side a region is a
    // 16x16 pixel block on 16-pixel boundaries, the query of per-tile
    // aggregation; entry (tile << region_log) + region
    const int q = blockIdx.x;
    const int t = q >> a.region_log, rg = q & ((1 << a.region_log) - 1);
    const int v = a.tile_view[t];
    const SceneSlot &S = a.slots[0];
    const ViewDev &V = a.views[v];
    const int tl = t - V.tile_base;
    const int tx = tl % V.tiles_x, ty = tl / V.tiles_x;
    const int lane = threadIdx.x;
    const int qlx = V.tsx - 3, qly = V.tsy - 3;
    const int rlx = qlx > 1 ? qlx - 1 : 0;
    const int kxn = qlx > 0 ? 2 : 1, kyn = qly > 0 ? 2 : 1;
    const int ox = (tx << V.tsx) + kQuad * kxn * (rg & ((1 << rlx) - 1));
    const int oy = (ty << V.tsy) + kQuad * kyn * (rg >> rlx);
    const int rw = kQuad * kxn, area = rw * kQuad * kyn;
    double sum = 0.0;
    for (int k = lane; k < area; k += kWave) {
        const int px = ox + k % rw, py = oy + k / rw;
        if (px < V.W && py < V.H) sum += (double)S.ray_A[V.ray_local + (int64_t)py * V.W + px];
    }
    sum = wave_sum_f64(sum);
    if (lane == 0) tile_A[q] = sum;
}

// One wave per view: the sum of its regions' A(Q).
__global__ __launch_bounds__(kWave) void k_view_A(const ViewDev *__restrict__ views,
                                                  const double *__restrict__ tile_A, double *__restrict__ view_A,
                                                  int region_log) {
    const ViewDev &V = views[blockIdx.x];
    const int nt = (V.tiles_x * V.tiles_y) << region_log;
    const int64_t base = (int64_t)V.tile_base << region_log;
    double sum = 0.0;
    for (int t = threadIdx.x; t < nt; t += kWave) sum += tile_A[base + t];
    sum = wave_sum_f64(sum);
    if (threadIdx.x == 0) view_A[blockIdx.x] = sum;
}

// One wave: the sum over the launch's views.
__global__ __launch_bounds__(kWave) void k_total_A(const double *__restrict__ view_A, int Vc,
                                                   double *__restrict__ total) {
    double sum = 0.0;
    for (int v = threadIdx.x; v < Vc; v += kWave) sum += view_A[v];
    sum = wave_sum_f64(sum);
    if (threadIdx.x == 0) total[0] = sum;
}

void launch_query_sums(const CompositeArgs &a, int Vc, double *tile_A, double *view_A, double *total,
                       hipStream_t st) {
    if (a.total_tiles <= 0 || Vc <= 0) return;
    hipLaunchKernelGGL(k_tile_A, dim3((unsigned)(a.total_tiles << a.region_log)), dim3(kWave), 0, st, a, tile_A);
    hipLaunchKernelGGL(k_view_A, dim3(Vc), dim3(kWave), 0, st, a.views, (const double *)tile_A, view_A,
                       a.region_log);
    if (total) hipLaunchKernelGGL(k_total_A, dim3(1), dim3(kWave), 0, st, (const double *)view_A, Vc, total);
}

__device__ __forceinline__ float agg_share(uint64_t x) { return (float)((double)x * (1.0 / kAggScale)); }

__global__ __launch_bounds__(256) void k_agg_tile_max(const uint64_t *__restrict__ acc,
                                                      const uint32_t *__restrict__ lists, uint64_t n,
                                                      uint32_t *__restrict__ sens_bits) {
    const uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float s = agg_share(acc[e]);
    if (s > 0.0f) atomicMax(&sens_bits[lists[e] & kIndexMask], __float_as_uint(s));
}

__global__ __launch_bounds__(256) void k_agg_view_max(const uint64_t *__restrict__ acc, int64_t N, int Vc,
                                                      uint32_t *__restrict__ sens_bits) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= N) return;
    uint64_t m = 0;
    for (int v = 0; v < Vc; ++v) m = max(m, acc[(int64_t)v * N + g]);
    const float s = agg_share(m);
    if (s > __uint_as_float(sens_bits[g])) sens_bits[g] = __float_as_uint(s);
}

__global__ __launch_bounds__(256) void k_agg_scene_add(const uint64_t *__restrict__ acc, int64_t N,
                                                       double *__restrict__ num, double *__restrict__ den,
                                                       const double *__restrict__ launch_A) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double LA = launch_A[0];
    if (g == 0) den[0] += LA;
    if (g < N) num[g] += ((double)acc[g] * (1.0 / kAggScale)) * LA;
}

void launch_agg_finalize(int agg, const uint64_t *acc, const uint32_t *lists, uint64_t n_entries, int64_t N,
                         int Vc, uint32_t *sens_bits, double *num, double *den, const double *launch_A,
                         hipStream_t st) {
    if (agg == 1) {
        if (n_entries == 0) return;
        hipLaunchKernelGGL(k_agg_tile_max, dim3((unsigned)((n_entries + 255) / 256)), dim3(256), 0, st, acc, lists,
                           n_entries, sens_bits);
    } else if (agg == 2) {
        hipLaunchKernelGGL(k_agg_view_max, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, acc, N, Vc,
                           sens_bits);
    } else if (agg == 3) {
        hipLaunchKernelGGL(k_agg_scene_add, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, acc, N, num, den,
                           launch_A);
    }
}

__global__ __launch_bounds__(256) void k_div_f64_to_f32(const double *__restrict__ num,
                                                        const double *__restrict__ den, int64_t n,
                                                        float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double d = den[0];
    out[i] = d > 0.0 ? (float)(num[i] / d) : 0.0f;
}

void launch_div_f64_to_f32(const double *num, const double *den, int64_t n, float *out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_div_f64_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, num, den, n, out);
}

// ---------------------------------------------------------------------------
// Objectives of a weighted pruned scene (Section 3): full A, the fixed
// relaxation A^th_w = sum w_i a_i (full-scene T), and the true reduced render
// A_w with T_w = prod (1 - w_j rho_j) over retained Gaussians.  Also counts
// pairs with w rho >= 1 (Definition 2) and tracks the log-transmittance gap
// |log T - log T_w| = |sum log(1 - rho_j) - log(1 - w_j rho_j)| at every
// contributing retained pair (Assumption 1), on rays that stay valid.
// kModeL2 replaces each contribution c rho T by c (rho T)^2 (and c rho T_w by
// c (rho T_w)^2 in the reduced render).  kTrue: the reduced render and its
// diagnostics are computed (the true objective); otherwise A_w reads 0.
template <int kMode, bool kTrue>
__global__ __launch_bounds__(kWave) void k_objective(CompositeArgs a, ObjectiveArgs o,
                                                     uint64_t *__restrict__ counters) {
    static_assert(kMode != kModeChannel, "the objectives hold one query per ray");
    __shared__ float4 geo[kWave], col[kWave];
    const int nq = quad_count(a);
    int iter = 0;
    for (int qi = next_quad<false>(a, iter); qi < nq; qi = next_quad<false>(a, iter)) {
    WaveSetup w;
    if (!setup_quad(a, qi, w)) {
        if (threadIdx.x == 0) {
            const int64_t slot = (int64_t)qi * 3;
            o.tile_sums[slot] = o.tile_sums[slot + 1] = o.tile_sums[slot + 2] = 0.0;
        }
        continue;
    }
    const bool scored = w.inside && ray_selected(w.ray_mask, w.ray_global);
    const bool has_w = o.weights != nullptr;
    float T = 1.0f, A = 0.0f, Ax = 0.0f, Tw = 1.0f, At = 0.0f, gap = 0.0f, gmax = 0.0f;
    bool bad = false;
    uint32_t n_bad = 0;
    // Optional stop for the full and fixed objectives: every later term of
    // A^th_w is w_i c_i rho_i T_i <= w_max c_max T (w_max c_max T^2 for L2),
    // so once that bound is below stop_rel A the rest changes A and A^th_w by
    // less than stop_rel A.  (A_w has its own transmittance and gets no stop.)
    float stop_scale = 0.0f;
    if (o.wmax_bits) {
        const double wm = __longlong_as_double((long long)*o.wmax_bits);
        stop_scale = (float)wm * w.cmax;
    }
    bool done = !scored;
    for (uint64_t e0 = w.start; e0 < w.end; e0 += kWave) {
        if (__all(done)) break;
        const int n = has_w ? stage_slice<2>(w, e0, a.r2_log2, geo, col, nullptr, nullptr, o.weights)
                            : stage_slice<0>(w, e0, a.r2_log2, geo, col, nullptr, nullptr, nullptr);
        wave_sync();
        for (int j = 0; j < n; ++j) {
            const float4 G = geo[j], Cc = col[j];
            bool in_fp;
            const float rho = pair_rho(G, Cc, w.xl, w.yl, a.r2_log2, in_fp);
            const float cr = Cc.z * rho;
            const float rt = rho * T;
            const float aT = kMode == kModeL2 ? (Cc.z * rt) * rt : cr * T;
            A += aT;
            if (has_w) {
                const float wi = Cc.w;
                Ax = fmaf(wi, aT, Ax);
                if (kTrue && wi > 0.0f) {
                    const float wr = wi * rho;
                    if (kMode == kModeL2) {
                        const float rtw = rho * Tw;
                        At = fmaf(wi * (Cc.z * rtw), rtw, At);
                    } else {
                        At = fmaf(wi * cr, Tw, At);
                    }
                    if (rho > 0.0f && !bad) gmax = fmaxf(gmax, fabsf(gap));
                    if (wr >= 1.0f) {
                        bad = true;
                        n_bad += scored ? 1u : 0u;
                    }
                    if (!bad) gap += log1pf(-rho) - log1pf(-wr);
                    Tw = fmaf(-wr, Tw, Tw);
                } else if (kTrue && !bad) {
                    gap += log1pf(-rho);
                }
            }
            T = fmaf(-rho, T, T);
        }
        if (o.wmax_bits) done = done || ((kMode == kModeL2 ? T * T : T) * stop_scale < o.stop_rel * A);
        wave_sync();
    }
    const bool on = scored && A > 0.0f;
    if (w.inside && o.per_ray) {
        float val = o.objective == 0 ? A : (o.objective == 1 ? Ax : At);
        o.per_ray[w.ray_global] = on ? val : 0.0f;
    }
    double s0 = on ? (double)A : 0.0, s1 = on ? (double)Ax : 0.0, s2 = on ? (double)At : 0.0;
    float gm = (on && !bad) ? gmax : 0.0f;
    uint64_t nb = n_bad;
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_xor(s0, off);
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
        gm = fmaxf(gm, __shfl_xor(gm, off));
        nb += __shfl_xor(nb, off);
    }
    if (threadIdx.x == 0) {
        const int64_t slot = (((int64_t)w.gt << a.quad_log) + w.quad) * 3;
        o.tile_sums[slot + 0] = s0;
        o.tile_sums[slot + 1] = s1;
        o.tile_sums[slot + 2] = s2;
        if (nb) atomicAdd((unsigned long long *)&counters[CNT_INVALID_PAIRS], (unsigned long long)nb);
        if (gm > 0.0f) atomicMax((unsigned long long *)&counters[CNT_GAMMA_BITS], (unsigned long long)__float_as_uint(gm));
    }
    }
}

// Always the flat form (a.work is ignored).
void launch_objective(const CompositeArgs &a, const ObjectiveArgs &o, uint64_t *counters, hipStream_t st) {
    const bool l2 = composite_mode(a.query_mode) == kModeL2, tr = o.objective == 2;
    if (l2 && tr)
        hipLaunchKernelGGL((k_objective<kModeL2, true>), dim3(flat_grid(a)), dim3(kWave), 0, st, a, o, counters);
    else if (l2)
        hipLaunchKernelGGL((k_objective<kModeL2, false>), dim3(flat_grid(a)), dim3(kWave), 0, st, a, o, counters);
    else if (tr)
        hipLaunchKernelGGL((k_objective<kModeL1, true>), dim3(flat_grid(a)), dim3(kWave), 0, st, a, o, counters);
    else
        hipLaunchKernelGGL((k_objective<kModeL1, false>), dim3(flat_grid(a)), dim3(kWave), 0, st, a, o, counters);
}

// Largest value of a non-negative double array (as bits: monotone for x >= 0).
__global__ void k_max_f64(const double *__restrict__ x, int64_t n, unsigned long long *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = i < n ? (unsigned long long)__double_as_longlong(fmax(x[i], 0.0)) : 0ull;
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0 && v) atomicMax(out, v);
}

void launch_max_f64(const double *x, int64_t n, uint64_t *out_bits, hipStream_t st) {
    launch_fill_u64(out_bits, 0ull, 1, st);
    hipLaunchKernelGGL(k_max_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n,
                       (unsigned long long *)out_bits);
}

// Per-view sums of the per-wave partials: one block per view, each thread
// sums a fixed strided subset, then a fixed tree; the order never depends on
// scheduling.
__global__ __launch_bounds__(256) void k_view_sums(const double *__restrict__ tile_sums,
                                                   const ViewDev *__restrict__ views, int Vc, int quad_log,
                                                   double *__restrict__ out) {
    __shared__ double sh[3][256];
    const int v = blockIdx.x;
    const ViewDev &V = views[v];
    const int64_t lo = (int64_t)V.tile_base << quad_log, hi = lo + ((int64_t)V.tiles_x * V.tiles_y << quad_log);
    double s0 = 0, s1 = 0, s2 = 0;
    for (int64_t k = lo + threadIdx.x; k < hi; k += 256) {
        s0 += tile_sums[3 * k];
        s1 += tile_sums[3 * k + 1];
        s2 += tile_sums[3 * k + 2];
    }
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    sh[2][threadIdx.x] = s2;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[3 * v + threadIdx.x] = sh[threadIdx.x][0];
}

void launch_view_sums(const double *tile_sums, const ViewDev *views_dev, int Vc, int quad_log, double *per_view_out,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_view_sums, dim3(Vc), dim3(256), 0, st, tile_sums, views_dev, Vc, quad_log, per_view_out);
}

// Coreset-objective error of per-image objectives: out[0] = max over views
// with sum A > 0 of |sum A^th_w - sum A| / sum A, out[1] the same with the
// reduced render.  Each thread takes a fixed strided set of views, then a
// tree of maxima (order-free); one block.
__global__ __launch_bounds__(256) void k_coreset_error(const double *__restrict__ pv, int n_views,
                                                       double *__restrict__ out) {
    __shared__ double sh[2][256];
    double e0 = 0.0, e1 = 0.0;
    for (int v = threadIdx.x; v < n_views; v += 256) {
        const double A = pv[3 * v];
        if (A > 0.0) {
            e0 = fmax(e0, fabs(pv[3 * v + 1] - A) / A);
            e1 = fmax(e1, fabs(pv[3 * v + 2] - A) / A);
        }
    }
    sh[0][threadIdx.x] = e0;
    sh[1][threadIdx.x] = e1;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + off]);
            sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) out[threadIdx.x] = sh[threadIdx.x][0];
}

void launch_coreset_error(const double *per_view, int n_views, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_coreset_error, dim3(1), dim3(256), 0, st, per_view, n_views, out);
}

}  // namespace gs
