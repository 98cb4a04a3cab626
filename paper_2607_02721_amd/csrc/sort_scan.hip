// Segmented LSD radix sort of (u32 key, u32 value) pairs, exclusive/inclusive
// prefix sums, fills and a fixed-order float sum.
//
// Radix sort: each of n_segs segments of n_per_seg items (one segment per
// view) is sorted independently and stably by key, 8 bits per pass, 3 or 4
// passes (3 when every segment's keys, minus the segment's smallest, fit in
// 24 bits).  Blocks never straddle segments.  Once, before the passes:
//   hist_all:   every pass's digit counts per segment (one read of the keys)
//   digit_base: per segment and pass, exclusive scan of the digit counts
// Per pass:
//   scatter: each wave ranks its 1024 keys in 16 rounds of 64 with ballot
//            matching (wave-private LDS digit counters, so no block barrier
//            inside the rounds); waves then add the counts of the waves
//            before them, which keeps the sort stable; the block's start in
//            each digit's run is the digit base plus the counts of the
//            segment's earlier blocks, found by decoupled look-back.
#include "gs_internal.hpp"

namespace gs {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = kSortTile / kSortThreads;  // 16

__device__ __forceinline__ uint64_t lanemask_lt() {
    const unsigned lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lanes (among `active`) holding the same 8-bit digit as this lane.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active) {
    uint64_t m = active;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t bal = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return m;
}

// Key as the pass sees it: with kbase, visible keys relative to their
// segment's smallest one (first pass only; later passes read rebased keys).
__device__ __forceinline__ uint32_t rebase(uint32_t k, const uint32_t *kbase, int seg) {
    return (kbase && k != kInvisibleKey) ? k - kbase[seg] : k;
}

// Inclusive DPP scan of a wave (lanes without a source add 0).
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
    return v;
}

// Single-sweep form (look-back): one histogram kernel counts every pass's
// digits of the segment up front; each pass's scatter then takes its block
// number from a per-segment ticket, publishes its digit counts and sums
// those of the blocks before it (decoupled look-back), so no per-block
// histogram or offsets scan runs between the passes.
// Scratch after the status words, per segment: [4 passes][256] counts,
// [4][256] exclusive digit bases, [4] tickets (kSweepExtra words).
constexpr int kSweepExtra = 4 * 256 * 2 + 4;
constexpr uint32_t kFlagAgg = 1u << 30, kFlagPrefix = 2u << 30, kCountMask = (1u << 30) - 1u;

__global__ __launch_bounds__(kSortThreads) void k_radix_hist_all(const uint32_t *__restrict__ keys,
                                                                  int64_t n_per_seg, int passes,
                                                                  uint32_t *__restrict__ extra,
                                                                  const uint32_t *__restrict__ kbase,
                                                                  const uint32_t *__restrict__ seg_len) {
    __shared__ uint32_t cnt[4][256];
    const int seg = blockIdx.y, b = blockIdx.x;
    for (int i = threadIdx.x; i < 4 * 256; i += kSortThreads) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)seg * n_per_seg;
    const int64_t len = seg_len ? (int64_t)seg_len[seg] : n_per_seg;
    const int64_t lo = (int64_t)b * kSortTile;
    const int64_t hi = min(lo + (int64_t)kSortTile, len);
    for (int64_t i = lo + threadIdx.x; i < hi; i += kSortThreads) {
        const uint32_t k = rebase(keys[base + i], kbase, seg);
        for (int p = 0; p < passes; ++p) atomicAdd(&cnt[p][(k >> (8 * p)) & 255u], 1u);
    }
    __syncthreads();
    uint32_t *gc = extra + (int64_t)seg * kSweepExtra;
    for (int p = 0; p < passes; ++p) {
        const uint32_t c = cnt[p][threadIdx.x];
        if (c) atomicAdd(&gc[p * 256 + threadIdx.x], c);
    }
}

// One block of 256 threads per segment: exclusive scan of each pass's digit
// counts into the digit bases; the tickets are cleared here too.
__global__ __launch_bounds__(256) void k_radix_digit_base(uint32_t *__restrict__ extra, int passes) {
    __shared__ uint32_t wsum[4];
    uint32_t *e = extra + (int64_t)blockIdx.x * kSweepExtra;
    const int d = threadIdx.x, w = d >> 6, lane = d & 63;
    for (int p = 0; p < passes; ++p) {
        const uint32_t c = e[p * 256 + d];
        const uint32_t incl = wave_incl_scan_u32(c);
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        uint32_t before = incl - c;
        for (int k = 0; k < 3; ++k) before += k < w ? wsum[k] : 0u;
        e[4 * 256 + p * 256 + d] = before;
        __syncthreads();
    }
    if (d < 4) e[8 * 256 + d] = 0u;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                                 const uint32_t *__restrict__ vin,
                                                                 uint32_t *__restrict__ kout,
                                                                 uint32_t *__restrict__ vout, int64_t n_per_seg,
                                                                 int nb, int shift, int vals_are_iota,
                                                                 const uint32_t *__restrict__ kbase,
                                                                 const uint32_t *__restrict__ seg_len,
                                                                 uint32_t *__restrict__ status,
                                                                 uint32_t *__restrict__ extra, int pass,
                                                                 int n_segs) {
    // per wave and digit: the wave's count while ranking, then (thread d
    // rewrites its own column once it has read it) the block-local start of
    // the wave's run of digit d; one array instead of two keeps the block
    // under 40 KB of LDS, four blocks per CU
    __shared__ uint32_t wcnt[4][256];
    uint32_t (*wbase)[256] = wcnt;
    __shared__ uint32_t dstart[256];     // block-local start of each digit
    __shared__ uint32_t gdst[256];       // global start of the block's run of each digit
    __shared__ uint32_t wsum4[4];        // digit counts of each wave's 64 digits
    __shared__ uint32_t lkey[kSortTile], lval[kSortTile];
    __shared__ int tick;
    // blocks go to the XCDs in turn (block i to XCD i mod 8): block i works
    // on segment 8 (i / 8 / nb) + i mod 8, so each segment's scattered lines
    // are written through one L2; its place in the segment is its ticket
    const int64_t bi = blockIdx.x;
    const int seg = (int)(((bi >> 3) / nb) * 8 + (bi & 7));
    if (seg >= n_segs) return;
    int b;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t *ex = extra + (int64_t)seg * kSweepExtra;
    // block number in the order the segment's blocks started: every block
    // this one waits for below has started and publishes its counts before
    // it waits for anything
    if (threadIdx.x == 0) tick = (int)atomicAdd(&ex[8 * 256 + pass], 1u);
    __syncthreads();
    b = tick;
    // items of the segment to sort (the whole block leaves if it holds none)
    const int64_t len = seg_len ? (int64_t)seg_len[seg] : n_per_seg;
    if ((int64_t)b * kSortTile >= len) return;
    for (int i = threadIdx.x; i < 4 * 256; i += kSortThreads) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)seg * n_per_seg;
    const int64_t wlo = (int64_t)b * kSortTile + (int64_t)w * (kSortRounds * 64);
    uint32_t key[kSortRounds], val[kSortRounds], rank[kSortRounds];
#pragma unroll
    for (int k = 0; k < kSortRounds; ++k) {
        const int64_t i = wlo + k * 64 + lane;
        const bool ok = i < len;
        key[k] = ok ? rebase(kin[base + i], kbase, seg) : 0u;
        val[k] = ok ? (vals_are_iota ? (uint32_t)i : vin[base + i]) : 0u;
        const uint32_t d = (key[k] >> shift) & 255u;
        const uint64_t active = __ballot(ok);
        const uint64_t peers = match_digit(d, active);
        const uint32_t before = (uint32_t)__popcll(peers & lanemask_lt());
        const uint32_t run = ok ? wcnt[w][d] : 0u;
        rank[k] = run + before;
        // the last peer advances the wave's counter for this digit
        if (ok && (peers >> lane) == 1ull) wcnt[w][d] = run + before + 1u;
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // digit counts of the block, their exclusive scan (block-local run
    // starts) and each wave's start inside its digit's run
    {
        const int d = threadIdx.x;
        const uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
        const uint32_t tot = c0 + c1 + c2 + c3;
        {
            // publish this block's count of digit d, then add up the counts
            // of the blocks before it back to one that published its prefix
            uint32_t *st = status + (int64_t)seg * nb * 256;
            uint32_t excl = 0;
            if (b == 0) {
                __hip_atomic_store(&st[d], kFlagPrefix | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                __hip_atomic_store(&st[(int64_t)b * 256 + d], kFlagAgg | tot, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                for (int j = b - 1;; --j) {
                    uint32_t v = 0;
                    // (bounded: the block waited for has started; the bound only
                    // keeps a broken invariant from hanging the device)
                    for (int spin = 0; spin < (1 << 24); ++spin) {
                        v = __hip_atomic_load(&st[(int64_t)j * 256 + d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (v & ~kCountMask) break;
                        __builtin_amdgcn_s_sleep(1);
                    }
                    excl += v & kCountMask;
                    if ((v & kFlagPrefix) || j == 0) break;
                }
                __hip_atomic_store(&st[(int64_t)b * 256 + d], kFlagPrefix | (excl + tot), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            gdst[d] = ex[4 * 256 + pass * 256 + d] + excl;
        }
        // digits 64w .. 64w+63 are wave w's lanes: a DPP scan per wave, then
        // the sums of the waves before
        const uint32_t incl = wave_incl_scan_u32(tot);
        if (lane == 63) wsum4[w] = incl;
        __syncthreads();
        uint32_t start = incl - tot;
#pragma unroll
        for (int k = 0; k < 3; ++k) start += k < w ? wsum4[k] : 0u;
        dstart[d] = start;
        wbase[0][d] = start;
        wbase[1][d] = start + c0;
        wbase[2][d] = start + c0 + c1;
        wbase[3][d] = start + c0 + c1 + c2;
    }
    __syncthreads();
    // the block's keys in LDS in stable digit order, then written out in that
    // order: consecutive threads store consecutive positions of each digit's
    // run, so the stores of a wave cover a few runs instead of 64 scattered words
    int nvalid = 0;
#pragma unroll
    for (int k = 0; k < kSortRounds; ++k) {
        const int64_t i = wlo + k * 64 + lane;
        if (i < len) {
            const uint32_t d = (key[k] >> shift) & 255u;
            const uint32_t pos = wbase[w][d] + rank[k];
            lkey[pos] = key[k];
            lval[pos] = val[k];
        }
    }
    {
        const int64_t lo = (int64_t)b * kSortTile;
        nvalid = (int)min((int64_t)kSortTile, len - lo);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nvalid; i += kSortThreads) {
        const uint32_t kk = lkey[i];
        const uint32_t d = (kk >> shift) & 255u;
        const uint32_t dst = gdst[d] + ((uint32_t)i - dstart[d]);
        if (kout) kout[base + dst] = kk;
        vout[base + dst] = lval[i];
    }
}

hipError_t radix_sort_segments(uint32_t *key0, uint32_t *val0, uint32_t *key1, uint32_t *val1, uint32_t *hist,
                               int64_t n_per_seg, int n_segs, bool vals_are_iota, int passes,
                               const uint32_t *kbase, const uint32_t *seg_len, uint32_t **key_out,
                               uint32_t **val_out, hipStream_t st) {
    const int nb = (int)((n_per_seg + kSortTile - 1) / kSortTile);
    uint32_t *ki = key0, *vi = val0, *ko = key1, *vo = val1;
    // hist: [n_segs][256][nb] status words, then kSweepExtra words per segment
    const int64_t nstatus = (int64_t)n_segs * 256 * nb;
    uint32_t *extra = hist + nstatus;
    launch_fill_u32(extra, 0u, (int64_t)n_segs * kSweepExtra, st);
    hipLaunchKernelGGL(k_radix_hist_all, dim3(nb, n_segs), dim3(kSortThreads), 0, st, key0, n_per_seg, passes,
                       extra, kbase, seg_len);
    hipLaunchKernelGGL(k_radix_digit_base, dim3(n_segs), dim3(256), 0, st, extra, passes);
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        const uint32_t *kb = pass == 0 ? kbase : nullptr;
        launch_fill_u32(hist, 0u, nstatus, st);
        // the last pass writes the values only (nothing reads the sorted keys)
        const int64_t blocks = (int64_t)nb * ((n_segs + 7) / 8) * 8;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)blocks), dim3(kSortThreads), 0, st, ki, vi,
                           pass + 1 < passes ? ko : nullptr, vo, n_per_seg, nb, shift,
                           (pass == 0 && vals_are_iota) ? 1 : 0, kb, seg_len, hist, extra, pass, n_segs);
        uint32_t *t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    *key_out = nullptr;
    *val_out = vi;
    return hipGetLastError();
}

int64_t radix_sort_scratch_words(int64_t n_per_seg, int n_segs) {
    const int64_t nb = (n_per_seg + kSortTile - 1) / kSortTile;
    return (int64_t)n_segs * (256 * nb + kSweepExtra);
}

// ---------------------------------------------------------------------------
// Prefix sums over u64 (inputs u32 or u64), three phases with 2048-item blocks.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;

int64_t scan_tmp_elems(int64_t n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

template <typename T>
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t *sh, uint64_t *total) {
    // sh: kScanThreads entries
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        uint64_t x = t >= off ? sh[t - off] : 0ull;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    const uint64_t incl = sh[t];
    *total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const T *__restrict__ in, int64_t n,
                                                               uint64_t *__restrict__ partial) {
    __shared__ uint64_t sh[kScanThreads];
    const int64_t lo = (int64_t)blockIdx.x * kScanBlock;
    uint64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = lo + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) s += (uint64_t)in[i];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = kScanThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Exclusive scan of the block partials in place (single block); partial[nblk] = total.
__global__ __launch_bounds__(1024) void k_scan_partials(uint64_t *__restrict__ partial, int64_t nblk) {
    __shared__ uint64_t sh[1024];
    const int64_t per = (nblk + 1023) / 1024;
    const int64_t lo = threadIdx.x * per, hi = min(lo + per, nblk);
    uint64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += partial[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint64_t x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0ull;
        __syncthreads();
        sh[threadIdx.x] += x;
        __syncthreads();
    }
    uint64_t run = threadIdx.x ? sh[threadIdx.x - 1] : 0ull;
    for (int64_t i = lo; i < hi; ++i) {
        const uint64_t c = partial[i];
        partial[i] = run;
        run += c;
    }
    if (threadIdx.x == 1023) partial[nblk] = sh[1023];
}

template <typename T, bool kInclusive>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const T *__restrict__ in, int64_t n,
                                                              const uint64_t *__restrict__ partial,
                                                              uint64_t *__restrict__ out) {
    __shared__ uint64_t sh[kScanThreads];
    const int64_t lo = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = lo + k;
        v[k] = i < n ? (uint64_t)in[i] : 0ull;
        s += v[k];
    }
    uint64_t total;
    uint64_t run = block_exclusive_scan<T>(s, sh, &total) + partial[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = lo + k;
        if (kInclusive) run += v[k];
        if (i < n) out[i] = run;
        if (!kInclusive) run += v[k];
    }
}

// The inclusive apply phase over one array in place: each thread reads its
// own items before the block scan and writes the same items after it, so no
// item is read after another thread has written it (no __restrict__ here:
// input and output are the same memory).
__global__ __launch_bounds__(kScanThreads) void k_scan_apply_inplace(uint64_t *data, int64_t n,
                                                                      const uint64_t *__restrict__ partial) {
    __shared__ uint64_t sh[kScanThreads];
    const int64_t lo = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = lo + k;
        v[k] = i < n ? data[i] : 0ull;
        s += v[k];
    }
    uint64_t total;
    uint64_t run = block_exclusive_scan<uint64_t>(s, sh, &total) + partial[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = lo + k;
        run += v[k];
        if (i < n) data[i] = run;
    }
}

void scan_u64_inclusive_inplace(uint64_t *data, int64_t n, uint64_t *tmp, hipStream_t st) {
    const int64_t nblk = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_reduce<uint64_t>, dim3((unsigned)nblk), dim3(kScanThreads), 0, st, data, n, tmp);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, tmp, nblk);
    hipLaunchKernelGGL(k_scan_apply_inplace, dim3((unsigned)nblk), dim3(kScanThreads), 0, st, data, n, tmp);
}

// out[i] = sum_{j<i} in[j] for i in [0, n]; out has n+1 entries.
void scan_u32_to_u64_exclusive(const uint32_t *in, uint64_t *out, int64_t n, uint64_t *tmp, hipStream_t st) {
    const int64_t nblk = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_reduce<uint32_t>, dim3((unsigned)nblk), dim3(kScanThreads), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, tmp, nblk);
    hipLaunchKernelGGL((k_scan_apply<uint32_t, false>), dim3((unsigned)nblk), dim3(kScanThreads), 0, st, in, n,
                       tmp, out);
    // trailing total (a kernel rather than a copy, so that the sequence can be
    // captured into a graph)
    launch_copy_u64(out + n, tmp + nblk, 1, st);
}

void scan_u64_inclusive(const uint64_t *in, uint64_t *out, int64_t n, uint64_t *tmp, hipStream_t st) {
    const int64_t nblk = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_reduce<uint64_t>, dim3((unsigned)nblk), dim3(kScanThreads), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, tmp, nblk);
    hipLaunchKernelGGL((k_scan_apply<uint64_t, true>), dim3((unsigned)nblk), dim3(kScanThreads), 0, st, in, n,
                       tmp, out);
}

// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_copy_u64(uint64_t *dst, const uint64_t *src, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}
void launch_copy_u64(uint64_t *dst, const uint64_t *src, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, src, n);
}
// dst[k] = src[min(k stride, n)] for k = 0 .. ceil(n / stride).
__global__ void k_gather_u64(uint64_t *dst, const uint64_t *src, int64_t n, int64_t stride, int64_t count) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) dst[k] = src[min(k * stride, n)];
}
void launch_gather_u64(uint64_t *dst, const uint64_t *src, int64_t n, int64_t stride, hipStream_t st) {
    const int64_t count = (n + stride - 1) / stride + 1;
    hipLaunchKernelGGL(k_gather_u64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, dst, src, n, stride,
                       count);
}
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    const int64_t blocks = min((n + 255) / 256, (int64_t)65536);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
}
void launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    const int64_t blocks = min((n + 255) / 256, (int64_t)65536);
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
}

// Fixed-order sum: per-block tree sums in double, then a sequential sum of
// the block results, so the total does not depend on scheduling.
__global__ __launch_bounds__(256) void k_sum_blocks(const float *__restrict__ x, int64_t n, double *partial) {
    __shared__ double sh[256];
    const int64_t lo = (int64_t)blockIdx.x * 4096;
    double s = 0.0;
    for (int k = 0; k < 16; ++k) {
        const int64_t i = lo + (int64_t)k * 256 + threadIdx.x;
        if (i < n) s += (double)x[i];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}
__global__ void k_sum_final(const double *partial, int64_t nblk, double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int64_t i = 0; i < nblk; ++i) s += partial[i];
        *out = s;
    }
}
void launch_sum_f32_to_f64(const float *x, int64_t n, double *out, double *tmp, hipStream_t st) {
    const int64_t nblk = (n + 4095) / 4096;
    hipLaunchKernelGGL(k_sum_blocks, dim3((unsigned)nblk), dim3(256), 0, st, x, n, tmp);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, st, tmp, nblk, out);
}

}  // namespace gs
