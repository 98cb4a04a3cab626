// Projection of every Gaussian into every view of a chunk (Section 3:
// camera map p -> R p + t, projected kernel k, attenuation rho = alpha k,
// front-to-back order by view depth).
//
// One thread per Gaussian loads its attributes once (coalesced SoA planes)
// and loops over the chunk's views; per view it writes a 32-byte geometry
// record, the colour factor, the packed pixel ranges and a depth key.
// Set-up runs in FP64 (the vector FP64 rate equals the non-packed FP32 rate
// on CDNA4), so the float32 record fields carry only their own rounding.
//
// Records (all float32 unless noted):
//   geo.m = mean2d as float hi + float lo (x_hi, y_hi, x_lo, y_lo)
//   geo.q = (beta, a', g', alpha) with, for Delta = pixel centre - mean,
//        u = Delta_x + beta Delta_y and P = a' u^2 + g' Delta_y^2,
//        P = -(log2 e / 2) d^2 exactly in real arithmetic, so that
//        k = exp(-d^2/2) = exp2(P).  This is the Cholesky form of the
//        conic: both terms are non-negative multiples of -1, so P has no
//        cancellation between them.
//   CB = cbar, the query colour factor: c_R + c_G + c_B (RGB sum), 1
//        (nocolor), c_R^2 + c_G^2 + c_B^2 (L2) or the largest channel (per
//        channel, where it only bounds later contributions); a float array of
//        its own, so that the compositing passes gather 4-byte values
//   XY = (x-range, y-range): the inclusive pixel ranges whose centres can
//        fall inside the r-ellipse, packed as int16 (lo | hi << 16); an
//        8-byte array of its own, gathered in depth order by k_ranges_in_order
//   R3 = (c_R, c_G, c_B, 0), written for per-channel queries only.
#include "gs_internal.hpp"

#include <hip/hip_fp16.h>

namespace gs {

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float load_attr(const void *base, int64_t idx, int f16kind) {
    // f16kind: 0 = f32, 1 = bf16, 2 = ieee f16
    if (f16kind == 0) return static_cast<const float *>(base)[idx];
    uint16_t b = static_cast<const uint16_t *>(base)[idx];
    if (f16kind == 1) return bf16_bits_to_f32(b);
    return __half2float(__ushort_as_half(b));
}

// Wave-wide maximum / minimum: an inclusive DPP scan (shifts by 1, 2, 4, 8
// inside rows of 16 lanes, then row_bcast:15 and row_bcast:31; lanes without
// a source keep their value) leaves the result in lane 63.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t identity, uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)x, kCtrl, kRowMask, 0xF, false);
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, dpp_u32<0x111, 0xF>(0u, v));
    v = max(v, dpp_u32<0x112, 0xF>(0u, v));
    v = max(v, dpp_u32<0x114, 0xF>(0u, v));
    v = max(v, dpp_u32<0x118, 0xF>(0u, v));
    v = max(v, dpp_u32<0x142, 0xA>(0u, v));
    v = max(v, dpp_u32<0x143, 0xC>(0u, v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    v = min(v, dpp_u32<0x111, 0xF>(0xFFFFFFFFu, v));
    v = min(v, dpp_u32<0x112, 0xF>(0xFFFFFFFFu, v));
    v = min(v, dpp_u32<0x114, 0xF>(0xFFFFFFFFu, v));
    v = min(v, dpp_u32<0x118, 0xF>(0xFFFFFFFFu, v));
    v = min(v, dpp_u32<0x142, 0xA>(0xFFFFFFFFu, v));
    v = min(v, dpp_u32<0x143, 0xC>(0xFFFFFFFFu, v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Real spherical harmonics (orthonormal, degree <= 3) at unit direction d.
__device__ __forceinline__ void sh_basis(double x, double y, double z, double *Y) {
    const double k00 = 0.28209479177387814;       // 1/(2 sqrt(pi))
    const double k1 = 0.48860251190291992;        // sqrt(3/(4 pi))
    const double k2a = 1.0925484305920792;        // 1/2 sqrt(15/pi)
    const double k20 = 0.31539156525252005;       // 1/4 sqrt(5/pi)
    const double k22 = 0.54627421529603959;       // 1/4 sqrt(15/pi)
    const double k33 = 0.59004358992664352;       // 1/4 sqrt(35/(2 pi))
    const double k32 = 2.8906114426405538;        // 1/2 sqrt(105/pi)
    const double k31 = 0.45704579946446572;       // 1/4 sqrt(21/(2 pi))
    const double k30 = 0.37317633259011540;       // 1/4 sqrt(7/pi)
    const double k32b = 1.4453057213202769;       // 1/4 sqrt(105/pi)
    Y[0] = k00;
    Y[1] = k1 * y;
    Y[2] = k1 * z;
    Y[3] = k1 * x;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = k2a * x * y;
    Y[5] = k2a * y * z;
    Y[6] = k20 * (3.0 * zz - 1.0);
    Y[7] = k2a * x * z;
    Y[8] = k22 * (xx - yy);
    Y[9] = k33 * y * (3.0 * xx - yy);
    Y[10] = k32 * x * y * z;
    Y[11] = k31 * y * (5.0 * zz - 1.0);
    Y[12] = k30 * z * (5.0 * zz - 3.0);
    Y[13] = k31 * x * (5.0 * zz - 1.0);
    Y[14] = k32b * z * (xx - yy);
    Y[15] = k33 * x * (xx - 3.0 * yy);
}

__device__ __forceinline__ uint32_t pack_range(int lo, int hi) {
    return (uint32_t)(uint16_t)(int16_t)lo | ((uint32_t)(uint16_t)(int16_t)hi << 16);
}

template <int kDeg, int kFmt>
__global__ __launch_bounds__(kProjThreads) void k_project(SceneDev sc, const ViewDev *__restrict__ views, int Vc,
                                                 ProjParams pp, GeoRec *__restrict__ geo, float *__restrict__ CB,
                                                 uint2 *__restrict__ XY,
                                                 float4 *__restrict__ R3, uint32_t *__restrict__ keys,
                                                 uint4 *__restrict__ part, uint64_t *__restrict__ counters,
                                                 const uint32_t *__restrict__ tile_sat) {
    const int64_t n = sc.n;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in_range = g < n;
    const int64_t gi = in_range ? g : 0;
    constexpr int kf = kFmt == 1 ? 1 : 0;   // bf16 planes
    constexpr int kh = kFmt == 1 ? 2 : 0;   // f16 planes

    double mu[3], ls[3], q[4];
    for (int c = 0; c < 3; ++c) mu[c] = load_attr(sc.mean, c * n + gi, kf);
    for (int c = 0; c < 3; ++c) ls[c] = load_attr(sc.log_scale, c * n + gi, kf);
    for (int c = 0; c < 4; ++c) q[c] = load_attr(sc.quat, c * n + gi, kh);
    const float alpha = load_attr(sc.opacity, gi, kh);
    constexpr int K = (kDeg + 1) * (kDeg + 1);
    float shc[3 * K];
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) shc[k] = load_attr(sc.sh, (int64_t)k * n + gi, kf);

    bool valid = in_range;
    double qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    bool finite = isfinite(qn2) && qn2 > 0.0 && isfinite(alpha);
    for (int c = 0; c < 3; ++c) finite = finite && isfinite(mu[c]) && isfinite(ls[c]);
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) finite = finite && isfinite(shc[k]);
    if (in_range && !finite) atomicAdd((unsigned long long *)&counters[CNT_INVALID], 1ull);
    valid = valid && finite;

    // 3D covariance Sigma = R(q) diag(exp(2 l)) R(q)^T (upper triangle).
    double S3[6] = {0, 0, 0, 0, 0, 0};
    if (valid) {
        const double inv = 1.0 / sqrt(qn2);
        const double w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
        const double Rq[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                              2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                              2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
        const double s2[3] = {exp(2.0 * ls[0]), exp(2.0 * ls[1]), exp(2.0 * ls[2])};
        int k = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b) {
                double acc = 0.0;
                for (int c = 0; c < 3; ++c) acc += Rq[3 * a + c] * s2[c] * Rq[3 * b + c];
                S3[k++] = acc;
            }
    }
    const double r = pp.footprint_sigma;
    const float cut_pad = 0.01f;

    // this block's views: group blockIdx.y of gridDim.y near-equal groups
    const int v0 = (int)((int64_t)blockIdx.y * Vc / gridDim.y);
    const int v1 = (int)((int64_t)(blockIdx.y + 1) * Vc / gridDim.y);
    for (int v = v0; v < v1; ++v) {
        const ViewDev &V = views[v];
        const double *R = V.R;
        const double px = R[0] * mu[0] + R[1] * mu[1] + R[2] * mu[2] + V.t[0];
        const double py = R[3] * mu[0] + R[4] * mu[1] + R[5] * mu[2] + V.t[1];
        const double pz = R[6] * mu[0] + R[7] * mu[1] + R[8] * mu[2] + V.t[2];
        bool vis = valid && pz > (double)pp.z_near;
        bool keep = false;   // visible and, in ray-masked runs, meeting a tile that holds a selected ray
        float4 r0 = make_float4(0, 0, 0, 0), r1 = make_float4(0, 0, 0, 0);
        uint2 xy = make_uint2(0u, 0u);
        float4 r3 = make_float4(0, 0, 0, 0);
        float cbar = 0.0f;
        if (vis) {
            const double iz = 1.0 / pz;
            // T = J R (2x3), J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]]
            const double j00 = V.fx * iz, j02 = -V.fx * px * iz * iz;
            const double j11 = V.fy * iz, j12 = -V.fy * py * iz * iz;
            double T0[3], T1[3];
            for (int c = 0; c < 3; ++c) {
                T0[c] = j00 * R[c] + j02 * R[6 + c];
                T1[c] = j11 * R[3 + c] + j12 * R[6 + c];
            }
            // Sigma_2d = T S3 T^T + delta I
            const double S[3][3] = {{S3[0], S3[1], S3[2]}, {S3[1], S3[3], S3[4]}, {S3[2], S3[4], S3[5]}};
            double u0[3], u1[3];
            for (int a = 0; a < 3; ++a) {
                u0[a] = S[a][0] * T0[0] + S[a][1] * T0[1] + S[a][2] * T0[2];
                u1[a] = S[a][0] * T1[0] + S[a][1] * T1[1] + S[a][2] * T1[2];
            }
            const double sxx = T0[0] * u0[0] + T0[1] * u0[1] + T0[2] * u0[2] + (double)pp.dilation;
            const double sxy = T0[0] * u1[0] + T0[1] * u1[1] + T0[2] * u1[2];
            const double syy = T1[0] * u1[0] + T1[1] * u1[1] + T1[2] * u1[2] + (double)pp.dilation;
            const double det = sxx * syy - sxy * sxy;
            const double mx = V.fx * px * iz + V.cx;
            const double my = V.fy * py * iz + V.cy;
            const double rx = r * sqrt(sxx), ry = r * sqrt(syy);
            double xl = ceil(mx - rx - 0.5 - cut_pad), xh = floor(mx + rx - 0.5 + cut_pad);
            double yl = ceil(my - ry - 0.5 - cut_pad), yh = floor(my + ry - 0.5 + cut_pad);
            xl = fmax(xl, 0.0); yl = fmax(yl, 0.0);
            xh = fmin(xh, (double)(V.W - 1)); yh = fmin(yh, (double)(V.H - 1));
            vis = det > 0.0 && syy > 0.0 && xl <= xh && yl <= yh;
            if (vis) {
                const double log2e = 1.4426950408889634;
                const double beta = -sxy / syy;
                const double a = syy / det;
                const double gm = 1.0 / syy;
                const float hx = (float)mx, hy = (float)my;
                r0 = make_float4(hx, hy, (float)(mx - (double)hx), (float)(my - (double)hy));
                r1 = make_float4((float)beta, (float)(-0.5 * log2e * a), (float)(-0.5 * log2e * gm), alpha);
                // colour at the direction camera centre -> mean
                double d0 = mu[0] - V.cam[0], d1 = mu[1] - V.cam[1], d2 = mu[2] - V.cam[2];
                const double dn = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                double Y[16];
                sh_basis(d0 * dn, d1 * dn, d2 * dn, Y);
                // the coefficients stay float32 in registers and are widened
                // here, per view (widened once outside the loop, their FP64
                // copies take 96 registers instead of 48 and the kernel holds
                // two waves per SIMD instead of three)
#pragma unroll
                for (int k = 0; k < 3 * K; ++k) asm volatile("" : "+v"(shc[k]));
                double c[3];
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    double acc = 0.0;
#pragma unroll
                    for (int k = 0; k < K; ++k) acc += Y[k] * (double)shc[3 * k + ch];
                    acc += 0.5;
                    c[ch] = acc > 0.0 ? acc : 0.0;
                }
                if (pp.query_mode == 1)
                    cbar = 1.0f;
                else if (pp.query_mode == 2)
                    cbar = (float)(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
                else if (pp.query_mode == 3)
                    cbar = (float)fmax(c[0], fmax(c[1], c[2]));
                else
                    cbar = (float)(c[0] + c[1] + c[2]);
                r3 = make_float4((float)c[0], (float)c[1], (float)c[2], 0.0f);
                xy = make_uint2(pack_range((int)xl, (int)xh), pack_range((int)yl, (int)yh));
                keep = true;
                if (tile_sat) {
                    // active tiles inside the tile rectangle [x0, x1) x [y0, y1)
                    const uint32_t *S = tile_sat + V.sat_base;
                    const int stride = V.tiles_x + 1;
                    const int x0 = (int)xl >> V.tsx, x1 = ((int)xh >> V.tsx) + 1;
                    const int y0 = ((int)yl >> V.tsy) * stride, y1 = (((int)yh >> V.tsy) + 1) * stride;
                    keep = S[y1 + x1] - S[y0 + x1] - S[y1 + x0] + S[y0 + x0] != 0u;
                }
            }
        }
        const int64_t o = (int64_t)v * n + gi;
        if (in_range) {
            geo[o].m = r0;
            geo[o].q = r1;
            CB[o] = cbar;
            XY[o] = xy;
            if (R3) R3[o] = r3;
            keys[o] = keep ? __float_as_uint((float)pz) : kInvisibleKey;
        }
        // per-view visible count, colour maximum and key range of this wave
        // (one wave per block), folded over the waves by k_proj_reduce (one
        // shared counter per view would take every wave's atomic in turn)
        // (colours and depths are positive: their float bits order like them;
        // the colour maximum bounds later contributions on a ray, so it
        // covers every visible Gaussian, kept or not: a ray-masked run then
        // stops its rays exactly where the unmasked run does)
        const uint64_t bal = __ballot(keep);
        const uint32_t key = __float_as_uint((float)pz);
        // Depth keys that FP32 rounding could order either way: pz within
        // 2^-40 pz of the midpoint between its float32 rounding and a float32
        // neighbour (pz > z_near > 0, so the neighbours are the next and
        // previous bit patterns).  Counted only; such keys are rare.
        if (vis) {
            const double f = (double)__uint_as_float(key);
            const double up = 0.5 * (f + (double)__uint_as_float(key + 1u));
            const double dn = 0.5 * (f + (double)__uint_as_float(key - 1u));
            const double band = ldexp(pz, -40);
            const bool amb = fabs(pz - up) <= band || fabs(pz - dn) <= band;
            const uint64_t ab = __ballot(amb);
            if (ab && (threadIdx.x & 63) == 0)
                atomicAdd((unsigned long long *)&counters[CNT_AMB_KEYS], (unsigned long long)__popcll(ab));
        }
        const uint32_t cm = wave_max_u32(vis ? __float_as_uint(cbar) : 0u);
        const uint32_t klo = wave_min_u32(keep ? key : 0xFFFFFFFFu);
        const uint32_t khi = wave_max_u32(keep ? key : 0u);
        if (threadIdx.x == 0)
            part[(int64_t)v * gridDim.x + blockIdx.x] = make_uint4((uint32_t)__popcll(bal), cm, klo, khi);
    }
}

// nvis[v] = sum, cmax[v] = maximum, kmin[v] / kmax[v] = smallest / largest
// kept depth key of the per-block values of view v (one block of 1024
// threads per view); each block's count is replaced by the kept keys of the
// blocks before it (the offsets launch_key_compact writes at).  Thread t
// takes a contiguous run of blocks so that a scan of the runs' sums (DPP
// inside each wave, then the 16 wave sums) gives those offsets.
constexpr int kReduceThreads = 1024;

__device__ __forceinline__ uint32_t wave_incl_scan_add(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
    return v;
}

__global__ __launch_bounds__(kReduceThreads) void k_proj_reduce(uint4 *__restrict__ part, int Vc, int64_t nblk,
                                                                uint32_t *__restrict__ nvis,
                                                                uint32_t *__restrict__ cmax_bits,
                                                                uint32_t *__restrict__ kmin) {
    constexpr int kW = kReduceThreads / 64;
    __shared__ uint32_t sh[4][kW];
    const int v = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t per = (nblk + kReduceThreads - 1) / kReduceThreads;
    const int64_t lo = (int64_t)threadIdx.x * per, hi = min(lo + per, nblk);
    uint4 *pv = part + (int64_t)v * nblk;
    uint32_t cnt = 0, cm = 0, klo = 0xFFFFFFFFu, khi = 0;
    for (int64_t b = lo; b < hi; ++b) {
        const uint4 q = pv[b];
        cnt += q.x;
        cm = max(cm, q.y);
        klo = min(klo, q.z);
        khi = max(khi, q.w);
    }
    const uint32_t incl = wave_incl_scan_add(cnt);
    if (lane == 63) sh[0][w] = incl;
    __syncthreads();
    uint32_t run = incl - cnt, total = 0;
    for (int k = 0; k < kW; ++k) {
        run += k < w ? sh[0][k] : 0u;
        total += sh[0][k];
    }
    for (int64_t b = lo; b < hi; ++b) {
        const uint32_t c = pv[b].x;
        pv[b].x = run;
        run += c;
    }
    for (int off = 32; off > 0; off >>= 1) {
        cm = max(cm, (uint32_t)__shfl_xor((int)cm, off));
        klo = min(klo, (uint32_t)__shfl_xor((int)klo, off));
        khi = max(khi, (uint32_t)__shfl_xor((int)khi, off));
    }
    if (lane == 0) {
        sh[1][w] = cm;
        sh[2][w] = klo;
        sh[3][w] = khi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = 0, mn = 0xFFFFFFFFu, mx = 0;
        for (int k = 0; k < kW; ++k) {
            m = max(m, sh[1][k]);
            mn = min(mn, sh[2][k]);
            mx = max(mx, sh[3][k]);
        }
        nvis[v] = total;
        cmax_bits[v] = m;
        kmin[v] = mn;
        kmin[Vc + v] = mx;
    }
}

template <int kDeg, int kFmt>
static void launch_t(const SceneDev &sc, const ViewDev *views_dev, int Vc, const ProjParams &pp, const ChunkBufs &b,
                     hipStream_t st) {
    const int64_t blocks = proj_blocks(sc.n);
    // Each wave projects its 64 Gaussians into a group of about kProjViews
    // views (the Gaussian's set-up is repeated per group): with one group a
    // 1M-Gaussian scene is 15 625 waves, five rounds and a nearly empty sixth
    // at three waves per SIMD; groups of 25 views make the last round a
    // small part of the whole.
    constexpr int kProjViews = 25;
    const int groups = std::max(1, (Vc + kProjViews - 1) / kProjViews);
    hipLaunchKernelGGL((k_project<kDeg, kFmt>), dim3((unsigned)blocks, (unsigned)groups), dim3(kProjThreads), 0, st, sc, views_dev, Vc, pp, b.R,
                       b.CB, b.XY, b.R3, b.key0, (uint4 *)b.proj_part, b.counters, b.tile_sat);
    hipLaunchKernelGGL(k_proj_reduce, dim3((unsigned)Vc), dim3(kReduceThreads), 0, st, (uint4 *)b.proj_part, Vc, blocks,
                       b.nvis, b.cmax, b.kmin);
}

// Block (g, v) moves the kept keys of Gaussians [64 g, 64 g + 64) of view v
// (one wave) to their place after the kept keys of the blocks before it (the
// offsets k_proj_reduce left), in index order.
__global__ __launch_bounds__(kProjThreads) void k_key_compact(const uint32_t *__restrict__ keys,
                                                              const uint4 *__restrict__ part, int64_t N, int64_t nblk,
                                                              uint32_t *__restrict__ kout, uint32_t *__restrict__ vout) {
    const int v = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * kProjThreads + threadIdx.x;
    const uint32_t key = i < N ? keys[(int64_t)v * N + i] : kInvisibleKey;
    const bool keep = key != kInvisibleKey;
    const uint64_t bal = __ballot(keep);
    const int lane = threadIdx.x;
    const uint32_t below = (uint32_t)__popcll(bal & (lane ? (~0ull >> (64 - lane)) : 0ull));
    const uint32_t before = part[(int64_t)v * nblk + blockIdx.x].x;
    if (keep) {
        const int64_t dst = (int64_t)v * N + before + below;
        kout[dst] = key;
        vout[dst] = (uint32_t)i;
    }
}

void launch_key_compact(const ChunkBufs &b, int Vc, int64_t N, uint32_t *kout, uint32_t *vout, hipStream_t st) {
    const int64_t blocks = proj_blocks(N);
    hipLaunchKernelGGL(k_key_compact, dim3((unsigned)blocks, (unsigned)Vc), dim3(kProjThreads), 0, st, b.key0,
                       (const uint4 *)b.proj_part, N, blocks, kout, vout);
}

void launch_project(const SceneDev &sc, const ViewDev *views_dev, int Vc, const ProjParams &pp,
                    const ChunkBufs &b, hipStream_t st) {
    using L = void (*)(const SceneDev &, const ViewDev *, int, const ProjParams &, const ChunkBufs &, hipStream_t);
    static const L table[2][4] = {{launch_t<0, 0>, launch_t<1, 0>, launch_t<2, 0>, launch_t<3, 0>},
                                  {launch_t<0, 1>, launch_t<1, 1>, launch_t<2, 1>, launch_t<3, 1>}};
    table[sc.format == 1 ? 1 : 0][sc.sh_degree](sc, views_dev, Vc, pp, b, st);
}

// Depth-ordered copy of each visible Gaussian's pixel ranges, so that the
// binning kernels read them with unit stride: xr/yr[v*N + p] for position p
// of view v's front-to-back order.
__global__ __launch_bounds__(256) void k_ranges_in_order(const uint32_t *__restrict__ sorted_g,
                                                         const uint2 *__restrict__ XY,
                                                         const uint32_t *__restrict__ nvis, int64_t N,
                                                         uint32_t *__restrict__ xr, uint32_t *__restrict__ yr, int Vc) {
    // blocks go to the XCDs in turn (block i to XCD i mod 8): block i takes
    // view 8 (i / 8 / nbx) + i mod 8, so each XCD gathers from views of its
    // own and a view's records are cached in one L2 instead of eight
    const int64_t nbx = (N + 255) / 256;
    const int64_t i = blockIdx.x, r = i >> 3;
    const int v = (int)((r / nbx) * 8 + (i & 7));
    if (v >= Vc) return;
    const int64_t p = (r % nbx) * 256 + threadIdx.x;
    if (p >= (int64_t)nvis[v]) return;
    const int64_t o = (int64_t)v * N;
    const uint2 rg = XY[o + sorted_g[o + p]];
    xr[o + p] = rg.x;
    yr[o + p] = rg.y;
}

void launch_ranges_in_order(const uint32_t *sorted_g, const ChunkBufs &b, int Vc, int64_t N, uint32_t *xr,
                            uint32_t *yr, hipStream_t st) {
    const int64_t nbx = (N + 255) / 256;
    const int64_t blocks = nbx * (((int64_t)Vc + 7) / 8) * 8;
    hipLaunchKernelGGL(k_ranges_in_order, dim3((unsigned)blocks), dim3(256), 0, st, sorted_g, b.XY, b.nvis, N, xr,
                       yr, Vc);
}

}  // namespace gs
