// Per-Gaussian support and tile binning for the gfx950 rasterizer:
//   setup    - image table into the workspace, counters zeroed
//   support  - per Gaussian (FP64): support box, tile range, tile count and
//              the FP32 render record
//   scan     - exclusive prefix sum of the tile counts (per-block sums in the
//              support kernel, one workgroup over the block sums, local scans
//              in the emission kernel)
//   emit     - (tile id, Gaussian id) pairs, Gaussian-major, ascending id
//   sort     - stable LSD radix sort of the pairs by tile id (8-bit digits)
//   ranges   - [begin, end) of every tile in the sorted pairs
//
// The support box follows Algorithm 1's strict window test with the window
// replaced by R standard deviations per axis, evaluated in HR pixels:
//   { x integer : s (mu_x - R sigma_x) < x < s (mu_x + R sigma_x) }
// with the FP64 operation sequence below (no fused multiply-add), so that
// the box, the tile lists and the per-tile counts are exactly reproducible.
#include <algorithm>

#include "gs_internal.h"

namespace gs {

namespace {

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Inclusive scan of one int64 value per thread across a workgroup of
// kBlockG threads.  `tmp` holds kBlockG / 64 entries.
__device__ __forceinline__ int64_t block_inclusive_scan(int64_t v, int64_t* tmp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        int64_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) tmp[wave] = v;
    __syncthreads();
    int64_t carry = 0;
    for (int k = 0; k < wave; ++k) carry += tmp[k];
    __syncthreads();
    return v + carry;
}

__global__ void k_setup(ImgChunk chunk, int first, int count, ImgDev* dst) {
    const int t = threadIdx.x;
    if (t < count) dst[first + t] = chunk.img[t];
}

// Last image with g_begin <= i (images are validated ascending and
// disjoint); -1 if i falls in no image.
template <typename Table>
__device__ __forceinline__ int find_image(const Table& imgs, int n_img, int64_t i) {
    int lo = 0, hi = n_img - 1, ans = -1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        if (imgs[mid].g_begin <= i) { ans = mid; lo = mid + 1; } else { hi = mid - 1; }
    }
    if (ans >= 0 && i >= imgs[ans].g_begin + imgs[ans].g_count) ans = -1;
    return ans;
}

__device__ __forceinline__ bool finite_d(double v) { return __builtin_isfinite(v); }

// Support box in HR pixels, clipped to the image (see the file comment).
// Returns false when the box is empty or the parameters are invalid.
__device__ bool support_box(double s, int out_w, int out_h, double mx, double my,
                            double l11, double l21, double l22, double R, int* box) {
#pragma clang fp contract(off)
    if (!finite_d(mx) || !finite_d(my) || !finite_d(l11) || !finite_d(l21) ||
        !finite_d(l22) || !finite_d(R))
        return false;
    if (!(l11 > 0.0) || !(l22 > 0.0) || !(R > 0.0)) return false;
    const double sx = l11;
    const double sy = __dsqrt_rn(l21 * l21 + l22 * l22);
    const double lo_x = s * (mx - R * sx);
    const double hi_x = s * (mx + R * sx);
    const double lo_y = s * (my - R * sy);
    const double hi_y = s * (my + R * sy);
    double x0 = __builtin_floor(lo_x) + 1.0, x1 = __builtin_ceil(hi_x) - 1.0;
    double y0 = __builtin_floor(lo_y) + 1.0, y1 = __builtin_ceil(hi_y) - 1.0;
    if (x0 < 0.0) x0 = 0.0;
    if (y0 < 0.0) y0 = 0.0;
    if (x1 > (double)(out_w - 1)) x1 = (double)(out_w - 1);
    if (y1 > (double)(out_h - 1)) y1 = (double)(out_h - 1);
    if (x0 > x1 || y0 > y1) return false;
    box[0] = (int)x0; box[1] = (int)x1; box[2] = (int)y0; box[3] = (int)y1;
    return true;
}

// One thread per Gaussian: box, record, tile count; per-block sums of the
// pair counts, in-support areas and invalid flags.  Also clears the per-tile
// ranges and the backward accumulators (grid-stride / per Gaussian).  With a
// by-value image table (kArgTable, batches of at most kSetupChunk images) the
// first block also writes the table into the workspace for later kernels.
template <bool kArgTable>
__global__ __launch_bounds__(kBlockG) void k_support(
    ImgChunk arg_imgs, ImgDev* __restrict__ imgs, int n_img, int64_t n_gauss, int tile,
    const float* __restrict__ mean, const float* __restrict__ chol,
    const float* __restrict__ color, const float* __restrict__ opacity,
    const float* __restrict__ radius, GRec* __restrict__ recs, int32_t* __restrict__ counts,
    BlockSums* __restrict__ blocksums, int2* __restrict__ ranges, int64_t n_tiles,
    float4* __restrict__ moments, uint32_t* __restrict__ sched) {
    __shared__ int64_t tmp[3][kBlockG / 64];
    const int64_t i = (int64_t)blockIdx.x * kBlockG + threadIdx.x;

    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < kSchedWords; k += kBlockG) sched[k] = 0;

    if (kArgTable && blockIdx.x == 0 && threadIdx.x < n_img)
        imgs[threadIdx.x] = arg_imgs.img[threadIdx.x];
    for (int64_t t = i; t < n_tiles; t += (int64_t)gridDim.x * kBlockG)
        ranges[t] = make_int2(0, 0);

    int cnt = 0;
    int64_t area = 0;
    int bad = 0;
    if (i < n_gauss) {
        GRec r;
        r.x0 = 0; r.x1 = -1; r.y0 = 0; r.y1 = -1;
        r.fx = r.fy = 0.f; r.kx = r.ky = 0;
        r.a = r.e = r.g = 0.f;
        r.A[0] = r.A[1] = r.A[2] = 0.f;
        r.pad = 0;
        const int k = kArgTable ? find_image(arg_imgs.img, n_img, i) : find_image(imgs, n_img, i);
        r.img = k;
        if (k >= 0) {
            const ImgDev im = kArgTable ? arg_imgs.img[k] : imgs[k];
            const double s = im.scale;
            const double mx = mean[2 * i], my = mean[2 * i + 1];
            const double l11 = chol[3 * i], l21 = chol[3 * i + 1], l22 = chol[3 * i + 2];
            const double R = radius ? (double)radius[i] : 3.0;
            int box[4];
            const bool shape_ok = finite_d(mx) && finite_d(my) && finite_d(l11) &&
                                  finite_d(l21) && finite_d(l22) && l11 > 0.0 && l22 > 0.0;
            bad = shape_ok ? 0 : 1;
            if (support_box(s, im.out_w, im.out_h, mx, my, l11, l21, l22, R, box)) {
                // colour / opacity may be NULL when only the pairs are counted
                const double al = opacity ? (double)opacity[i] : 0.0;
                const double c0 = color ? (double)color[3 * i] : 0.0;
                const double c1 = color ? (double)color[3 * i + 1] : 0.0;
                const double c2 = color ? (double)color[3 * i + 2] : 0.0;
                const bool amp_ok = finite_d(al) && finite_d(c0) && finite_d(c1) && finite_d(c2);
                if (!amp_ok) bad = 1;
                r.x0 = box[0]; r.x1 = box[1]; r.y0 = box[2]; r.y1 = box[3];
                const double cx = s * mx, cy = s * my;
                const double lim = 1073741824.0;  // keep the integer part in int32
                const double kx = __builtin_floor(fmin(fmax(cx, -lim), lim));
                const double ky = __builtin_floor(fmin(fmax(cy, -lim), lim));
                r.kx = (int)kx; r.ky = (int)ky;
                r.fx = (float)(cx - kx);
                r.fy = (float)(cy - ky);
                r.a = (float)(kZScale / (s * l11));
                r.e = (float)(kZScale / (s * l22));
                r.g = (float)(kZScale * l21 / (s * l11 * l22));
                const double K = 1.0 / (2.0 * 3.14159265358979323846 * l11 * l22);
                if (amp_ok) {
                    r.A[0] = (float)(al * c0 * K);
                    r.A[1] = (float)(al * c1 * K);
                    r.A[2] = (float)(al * c2 * K);
                } else {
                    r.pad = 1;  // listed in tiles but contributes and receives nothing
                }
                const int tx0 = r.x0 / tile, tx1 = r.x1 / tile;
                const int ty0 = r.y0 / tile, ty1 = r.y1 / tile;
                cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
                area = (int64_t)(r.x1 - r.x0 + 1) * (r.y1 - r.y0 + 1);
            }
        }
        recs[i] = r;
        counts[i] = cnt;
        // backward accumulators start at zero (the gradient kernel re-zeroes
        // them after reading, so every backward of this forward starts clean)
        if (moments) {
            moments[2 * i] = make_float4(0.f, 0.f, 0.f, 0.f);
            moments[2 * i + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    const int64_t v0 = wave_sum_i64((int64_t)cnt);
    const int64_t v1 = wave_sum_i64(area);
    const int64_t v2 = wave_sum_i64((int64_t)bad);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { tmp[0][wave] = v0; tmp[1][wave] = v1; tmp[2][wave] = v2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        BlockSums b{0, 0, 0};
        for (int k = 0; k < kBlockG / 64; ++k) {
            b.pairs += tmp[0][k]; b.support += tmp[1][k]; b.invalid += tmp[2][k];
        }
        blocksums[blockIdx.x] = b;
    }
}

// One workgroup: exclusive scan of the per-block pair counts (in place in
// .pairs), and the header totals.
__global__ __launch_bounds__(kBlockG) void k_scan_blocks(BlockSums* __restrict__ bs, int nblk,
                                                         int64_t cap,
                                                         WsHeader* __restrict__ hdr) {
    __shared__ int64_t tmp[kBlockG / 64];
    __shared__ int64_t last;
    int64_t carry = 0, sup = 0, inv = 0;
    for (int base = 0; base < nblk; base += kBlockG) {
        const int j = base + threadIdx.x;
        int64_t v = 0;
        if (j < nblk) {
            v = bs[j].pairs;
            sup += bs[j].support;
            inv += bs[j].invalid;
        }
        const int64_t inc = block_inclusive_scan(v, tmp);
        if (j < nblk) bs[j].pairs = carry + inc - v;
        if (threadIdx.x == kBlockG - 1) last = inc;
        __syncthreads();
        carry += last;
        __syncthreads();
    }
    sup = wave_sum_i64(sup);
    inv = wave_sum_i64(inv);
    __shared__ int64_t ts[kBlockG / 64], ti[kBlockG / 64];
    if ((threadIdx.x & 63) == 0) { ts[threadIdx.x >> 6] = sup; ti[threadIdx.x >> 6] = inv; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t a = 0, b = 0;
        for (int k = 0; k < kBlockG / 64; ++k) { a += ts[k]; b += ti[k]; }
        hdr->n_pairs = carry;
        hdr->overflow = carry > cap ? 1 : 0;
        hdr->n_support = a;
        hdr->n_invalid = b;
        hdr->ordered = 0;
    }
}

// One thread per Gaussian: local exclusive scan + block offset, then the
// Gaussian's pairs in tile row-major order.  Pairs past the capacity are
// dropped (the overflow flag says so).  With kFold the block computes its
// offset from the unscanned block sums itself, and the last block writes the
// header totals (k_scan_blocks does both otherwise).
template <bool kFold>
__global__ __launch_bounds__(kBlockG) void k_emit(
    const ImgDev* __restrict__ imgs, const GRec* __restrict__ recs,
    const int32_t* __restrict__ counts, const BlockSums* __restrict__ bs, int nblk,
    int64_t n_gauss, int tile, int64_t cap, uint32_t* __restrict__ keys,
    uint32_t* __restrict__ vals, int32_t* __restrict__ offsets, WsHeader* __restrict__ hdr) {
    __shared__ int64_t tmp[kBlockG / 64];
    int64_t base;
    if (kFold) {
        const int b = blockIdx.x;
        const bool last_block = b == nblk - 1;
        int64_t lower = 0, sup = 0, inv = 0;
        for (int j = threadIdx.x; j < nblk; j += kBlockG) {
            if (j < b) lower += bs[j].pairs;
            if (last_block) { sup += bs[j].support; inv += bs[j].invalid; }
        }
        lower = wave_sum_i64(lower);
        __shared__ int64_t t3[3][kBlockG / 64];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (last_block) { sup = wave_sum_i64(sup); inv = wave_sum_i64(inv); }
        if (lane == 0) { t3[0][wave] = lower; t3[1][wave] = sup; t3[2][wave] = inv; }
        __syncthreads();
        base = 0;
        int64_t sa = 0, sb = 0;
        for (int k = 0; k < kBlockG / 64; ++k) { base += t3[0][k]; sa += t3[1][k]; sb += t3[2][k]; }
        if (last_block && threadIdx.x == 0) {
            const int64_t total = base + bs[b].pairs;
            hdr->n_pairs = total;
            hdr->overflow = total > cap ? 1 : 0;
            hdr->n_support = sa;
            hdr->n_invalid = sb;
                hdr->ordered = 0;
        hdr->ordered = 0;
        }
    } else {
        base = bs[blockIdx.x].pairs;  // scanned by k_scan_blocks
    }
    const int64_t i = (int64_t)blockIdx.x * kBlockG + threadIdx.x;
    const int cnt = i < n_gauss ? counts[i] : 0;
    const int64_t inc = block_inclusive_scan((int64_t)cnt, tmp);
    int64_t off = base + inc - cnt;
    if (i < n_gauss) offsets[i] = (int32_t)(off < cap ? off : cap);
    if (cnt == 0) return;
    const GRec r = recs[i];
    const ImgDev im = imgs[r.img];
    const int tx0 = r.x0 / tile, tx1 = r.x1 / tile;
    const int ty0 = r.y0 / tile, ty1 = r.y1 / tile;
    for (int ty = ty0; ty <= ty1; ++ty) {
        for (int tx = tx0; tx <= tx1; ++tx) {
            if (off < cap) {
                keys[off] = (uint32_t)(im.tile_base + (int64_t)ty * im.tiles_x + tx);
                vals[off] = (uint32_t)i;
            }
            ++off;
        }
    }
}

__device__ __forceinline__ int64_t pairs_in_use(const WsHeader* hdr, int64_t cap) {
    const int64_t p = hdr->n_pairs;
    return p < cap ? p : cap;
}

// Sort sources.  PairDigits: the (tile, Gaussian) pairs, keyed by the 8-bit
// digit of the tile id at `shift`.  TileDigits: the tiles themselves, keyed
// by the bucket of their list length, longest first (the longest-processing-
// time order the persistent tile kernels take their work in).
struct PairDigits {
    const uint32_t* keys;
    const uint32_t* vals;
    const WsHeader* hdr;
    int64_t cap;
    int shift;
    __device__ __forceinline__ int64_t count() const { return pairs_in_use(hdr, cap); }
    __device__ __forceinline__ int digit(int64_t i) const {
        return (int)((keys[i] >> shift) & (kRadix - 1));
    }
    __device__ __forceinline__ void load(int64_t i, int* d, uint32_t* a, uint32_t* b) const {
        *a = keys[i];
        *b = vals[i];
        *d = (int)((*a >> shift) & (kRadix - 1));
    }
};
struct PairSink {
    uint32_t* keys;
    uint32_t* vals;
    __device__ __forceinline__ void store(int64_t pos, uint32_t a, uint32_t b) const {
        keys[pos] = a;
        vals[pos] = b;
    }
};

// List length -> digit: lengths 0..127 one bucket each, then buckets 16 wide,
// everything from 2160 on in the last; digit 255 - bucket puts long lists first.
__device__ __forceinline__ int length_digit(int len) {
    const int b = len < 128 ? len : min(255, 128 + ((len - 128) >> 4));
    return (kRadix - 1) - b;
}
struct TileDigits {
    const int2* ranges;
    int64_t n_tiles;
    __device__ __forceinline__ int64_t count() const { return n_tiles; }
    __device__ __forceinline__ int digit(int64_t i) const {
        const int2 r = ranges[i];
        return length_digit(r.y - r.x);
    }
    __device__ __forceinline__ void load(int64_t i, int* d, uint32_t* a, uint32_t* b) const {
        *d = digit(i);
        *a = (uint32_t)i;
        *b = 0;
    }
};
struct OrderSink {
    uint32_t* order;
    __device__ __forceinline__ void store(int64_t pos, uint32_t a, uint32_t) const {
        order[pos] = a;
    }
};

// Per sort block: histogram of the digits.  hist is digit-major:
// hist[d * nblk + b].
template <typename Src>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(Src src, int nblk,
                                                            int32_t* __restrict__ hist) {
    __shared__ int32_t cnt[kRadix];
    const int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    const int64_t P = src.count();
    const int64_t start = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = start + (int64_t)k * kSortThreads + t;
        if (idx < P) atomicAdd(&cnt[src.digit(idx)], 1);
    }
    __syncthreads();
    hist[(int64_t)t * nblk + blockIdx.x] = cnt[t];
}

// One workgroup per digit: exclusive scan of that digit's row over blocks,
// row total into totals[d].
__global__ __launch_bounds__(kBlockG) void k_sort_rowscan(int32_t* __restrict__ hist,
                                                          int nblk,
                                                          int32_t* __restrict__ totals) {
    __shared__ int64_t tmp[kBlockG / 64];
    __shared__ int64_t last;
    int32_t* row = hist + (int64_t)blockIdx.x * nblk;
    int64_t carry = 0;
    for (int base = 0; base < nblk; base += kBlockG) {
        const int j = base + threadIdx.x;
        const int64_t v = j < nblk ? row[j] : 0;
        const int64_t inc = block_inclusive_scan(v, tmp);
        if (j < nblk) row[j] = (int32_t)(carry + inc - v);
        if (threadIdx.x == kBlockG - 1) last = inc;
        __syncthreads();
        carry += last;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = (int32_t)carry;
}

// Stable scatter of one sort block.  Items are ranked 256 at a time in index
// order: within a wave by matching the digit bit by bit with ballots, across
// the block's four waves through LDS counts.
template <typename Src, typename Dst>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    Src src, Dst dst, const int32_t* __restrict__ hist, const int32_t* __restrict__ totals,
    int nblk) {
    constexpr int kWaves = kSortThreads / 64;
    __shared__ int32_t base[kRadix];
    __shared__ int32_t wcnt[kWaves][kRadix];
    __shared__ int64_t tmp[kBlockG / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t P = src.count();
    const int64_t start = (int64_t)blockIdx.x * kSortTile;
    if (start >= P) return;  // uniform per block

    // digit base = sum of lower digits' totals + this digit's earlier blocks
    {
        const int64_t tot = totals[t];
        const int64_t inc = block_inclusive_scan(tot, tmp);
        base[t] = (int32_t)(inc - tot) + hist[(int64_t)t * nblk + blockIdx.x];
    }
    for (int k = 0; k < kWaves; ++k) wcnt[k][t] = 0;
    __syncthreads();

    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int round = 0; round < kSortItems; ++round) {
        const int64_t idx = start + (int64_t)round * kSortThreads + t;
        const bool valid = idx < P;
        uint32_t a = 0, b = 0;
        int d = 0;
        if (valid) src.load(idx, &d, &a, &b);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < kRadixBits; ++bit) {
            const bool on = (d >> bit) & 1;
            const uint64_t bal = __ballot(on);
            peers &= on ? bal : ~bal;
        }
        const int rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = base[d] + rank;
            for (int k = 0; k < wave; ++k) pos += wcnt[k][d];
            dst.store(pos, a, b);
        }
        __syncthreads();
        int add = 0;
        for (int k = 0; k < kWaves; ++k) { add += wcnt[k][t]; wcnt[k][t] = 0; }
        base[t] += add;
        __syncthreads();
    }
}

__global__ void k_mark_ordered(WsHeader* __restrict__ hdr) { hdr->ordered = 1; }

// One thread per sorted pair: the tile range boundaries.
__global__ __launch_bounds__(kBlockG) void k_ranges(const uint32_t* __restrict__ keys,
                                                    const WsHeader* __restrict__ hdr,
                                                    int64_t cap, int2* __restrict__ ranges) {
    const int64_t p = (int64_t)blockIdx.x * kBlockG + threadIdx.x;
    const int64_t P = pairs_in_use(hdr, cap);
    if (p >= P) return;
    const uint32_t k = keys[p];
    if (p == 0 || keys[p - 1] != k) ranges[k].x = (int)p;
    if (p == P - 1 || keys[p + 1] != k) ranges[k].y = (int)(p + 1);
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_support(const Layout& L, const Ws& w, const ImgDev* host_imgs,
                          const float* mean, const float* chol, const float* color,
                          const float* opacity, const float* radius, bool count_only,
                          hipStream_t st) {
    ImgChunk chunk;
    for (int k = 0; k < kSetupChunk; ++k) chunk.img[k] = ImgDev{};
    const bool by_value = L.n_img <= kSetupChunk;
    if (by_value) {
        for (int k = 0; k < L.n_img; ++k) chunk.img[k] = host_imgs[k];
    } else {
        for (int first = 0; first < L.n_img; first += kSetupChunk) {
            const int count = std::min(kSetupChunk, L.n_img - first);
            ImgChunk c;
            for (int k = 0; k < kSetupChunk; ++k) c.img[k] = k < count ? host_imgs[first + k] : ImgDev{};
            hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, st, c, first, count, w.imgs);
        }
    }
    float4* mom = reinterpret_cast<float4*>(w.moments);
    if (by_value)
        hipLaunchKernelGGL(k_support<true>, dim3(L.nblk_g), dim3(kBlockG), 0, st, chunk, w.imgs,
                           L.n_img, L.n_gauss, L.tile, mean, chol, color, opacity, radius,
                           w.recs, w.counts, w.blocksums, w.ranges, L.n_tiles, mom, w.sched);
    else
        hipLaunchKernelGGL(k_support<false>, dim3(L.nblk_g), dim3(kBlockG), 0, st, chunk, w.imgs,
                           L.n_img, L.n_gauss, L.tile, mean, chol, color, opacity, radius,
                           w.recs, w.counts, w.blocksums, w.ranges, L.n_tiles, mom, w.sched);
    if (count_only || L.nblk_g > kFoldScanBlocks)
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBlockG), 0, st, w.blocksums, L.nblk_g,
                           L.cap, w.hdr);
    return hipGetLastError();
}

hipError_t launch_emit(const Layout& L, const Ws& w, hipStream_t st) {
    if (L.nblk_g > kFoldScanBlocks)
        hipLaunchKernelGGL(k_emit<false>, dim3(L.nblk_g), dim3(kBlockG), 0, st, w.imgs, w.recs,
                           w.counts, w.blocksums, L.nblk_g, L.n_gauss, L.tile, L.cap,
                           w.keys[0], w.vals[0], w.offsets, w.hdr);
    else
        hipLaunchKernelGGL(k_emit<true>, dim3(L.nblk_g), dim3(kBlockG), 0, st, w.imgs, w.recs,
                           w.counts, w.blocksums, L.nblk_g, L.n_gauss, L.tile, L.cap,
                           w.keys[0], w.vals[0], w.offsets, w.hdr);
    return hipGetLastError();
}

hipError_t launch_sort(const Layout& L, const Ws& w, hipStream_t st) {
    int32_t* totals = w.hist + (int64_t)kRadix * L.nblk_sort;
    for (int pass = 0; pass < L.n_passes; ++pass) {
        const int src = pass & 1, dst = src ^ 1;
        const PairDigits in{w.keys[src], w.vals[src], w.hdr, L.cap, pass * kRadixBits};
        const PairSink out{w.keys[dst], w.vals[dst]};
        hipLaunchKernelGGL(k_sort_hist<PairDigits>, dim3(L.nblk_sort), dim3(kSortThreads), 0, st,
                           in, L.nblk_sort, w.hist);
        hipLaunchKernelGGL(k_sort_rowscan, dim3(kRadix), dim3(kBlockG), 0, st, w.hist,
                           L.nblk_sort, totals);
        hipLaunchKernelGGL((k_sort_scatter<PairDigits, PairSink>), dim3(L.nblk_sort),
                           dim3(kSortThreads), 0, st, in, out, w.hist, totals, L.nblk_sort);
    }
    return hipGetLastError();
}

hipError_t launch_order(const Layout& L, const Ws& w, hipStream_t st) {
    if (L.n_tiles == 0) return hipSuccess;
    int32_t* totals = w.order_hist + (int64_t)kRadix * L.nblk_order;
    const TileDigits in{w.ranges, L.n_tiles};
    hipLaunchKernelGGL(k_sort_hist<TileDigits>, dim3(L.nblk_order), dim3(kSortThreads), 0, st, in,
                       L.nblk_order, w.order_hist);
    hipLaunchKernelGGL(k_sort_rowscan, dim3(kRadix), dim3(kBlockG), 0, st, w.order_hist,
                       L.nblk_order, totals);
    hipLaunchKernelGGL((k_sort_scatter<TileDigits, OrderSink>), dim3(L.nblk_order),
                       dim3(kSortThreads), 0, st, in, OrderSink{w.order}, w.order_hist, totals,
                       L.nblk_order);
    hipLaunchKernelGGL(k_mark_ordered, dim3(1), dim3(1), 0, st, w.hdr);
    return hipGetLastError();
}

hipError_t launch_ranges(const Layout& L, const Ws& w, hipStream_t st) {
    hipLaunchKernelGGL(k_ranges, dim3(blocks_for(L.cap, kBlockG)), dim3(kBlockG), 0, st,
                       w.keys[L.n_passes & 1], w.hdr, L.cap, w.ranges);
    return hipGetLastError();
}

}  // namespace gs
