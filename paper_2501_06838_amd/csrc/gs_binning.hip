// Per-Gaussian support and tile binning for the gfx950 rasterizer:
//   setup    - image table into the workspace, counters zeroed
//   support  - per Gaussian (FP64): support box, tile range, tile count and
//              the FP32 render record
//   scan     - exclusive prefix sum of the per-Gaussian pair counts
//              (per-block sums in the support kernel, one workgroup over the
//              block sums, local scans in the emission kernel)
//   emit     - each (tile, Gaussian) pair counted into its tile with an
//              atomic, which hands the pair a place in the tile's list
//   lists    - exclusive scan of the per-tile counts (the tile ranges), every
//              Gaussian id written to its place, then each tile's list sorted
//              ascending (the atomics' order is arbitrary; the sorted lists
//              are unique)
// With GS_FLAG_RADIX_SORT the emission writes (tile id, Gaussian id) pairs
// instead, a stable LSD radix sort orders them by tile id and the ranges are
// read off the sorted keys: the same lists.
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

// Cross-lane steps on 64-bit values without LDS round trips (all 64 lanes
// active).  dpp64: the value of the lane that the DPP control names, moved as
// two 32-bit halves (0 where the control names no lane or the row is masked
// off).  swap64: the pair {value of lane l, value of lane l ^ kD} in lane
// order, kD = 16 or 32, from the gfx950 row and half-wave swaps.
template <int kCtrl, int kRowMask = 0xF>
__device__ __forceinline__ int64_t dpp64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, kCtrl,
                                                              kRowMask, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(
        0, (int)(uint32_t)((uint64_t)v >> 32), kCtrl, kRowMask, 0xF, false);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <int kD>
__device__ __forceinline__ void swap64(int64_t v, int64_t& r0, int64_t& r1) {
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)((uint64_t)v >> 32);
    const auto a = kD == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                            : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = kD == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                            : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    r0 = (int64_t)(((uint64_t)(uint32_t)b[0] << 32) | (uint32_t)a[0]);
    r1 = (int64_t)(((uint64_t)(uint32_t)b[1] << 32) | (uint32_t)a[1]);
}

// Butterfly over the wave: every lane ends with op over all 64 lanes
// (partners at lane distance 1, 2, 4, 8 by DPP: quad permutes, a quad
// reversal followed by a half-row mirror, a rotation by 8 within the row;
// 16 and 32 by the swaps).
template <typename Op>
__device__ __forceinline__ int64_t wave_butterfly(int64_t v, Op op) {
    v = op(v, dpp64<0xB1>(v));                // quad_perm [1, 0, 3, 2]
    v = op(v, dpp64<0x4E>(v));                // quad_perm [2, 3, 0, 1]
    v = op(v, dpp64<0x141>(dpp64<0x1B>(v)));  // quad_perm [3, 2, 1, 0], row_half_mirror
    v = op(v, dpp64<0x128>(v));               // row_ror:8
    int64_t r0, r1;
    swap64<16>(v, r0, r1);
    v = op(r0, r1);
    swap64<32>(v, r0, r1);
    return op(r0, r1);
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
    return wave_butterfly(v, [](int64_t a, int64_t b) { return a + b; });
}

// Inclusive scan of one value per lane across the wave: shifts by 1, 2, 4, 8
// within each row of 16, then each row adds the totals of the rows before it
// (lane 15 into rows 1 and 3, then lane 31 into rows 2 and 3).
__device__ __forceinline__ int64_t wave_inclusive_scan_i64(int64_t v) {
    v += dpp64<0x111>(v);       // row_shr:1
    v += dpp64<0x112>(v);       // row_shr:2
    v += dpp64<0x114>(v);       // row_shr:4
    v += dpp64<0x118>(v);       // row_shr:8
    v += dpp64<0x142, 0xA>(v);  // row_bcast:15
    v += dpp64<0x143, 0xC>(v);  // row_bcast:31
    return v;
}

// Inclusive scan of one int64 value per thread across a workgroup of
// kBlockG threads.  `tmp` holds kBlockG / 64 entries.
__device__ __forceinline__ int64_t block_inclusive_scan(int64_t v, int64_t* tmp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_inclusive_scan_i64(v);
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
// Returns false when the box is empty or the parameters are invalid;
// *clipped tells whether the image border cut the box.
__device__ bool support_box(double s, int out_w, int out_h, double mx, double my,
                            double l11, double l21, double l22, double R, bool centre, int* box,
                            bool* clipped) {
#pragma clang fp contract(off)
    if (!finite_d(mx) || !finite_d(my) || !finite_d(l11) || !finite_d(l21) ||
        !finite_d(l22) || !finite_d(R))
        return false;
    if (!(l11 > 0.0) || !(l22 > 0.0) || !(R > 0.0)) return false;
    const double sx = l11;
    const double sy = __dsqrt_rn(l21 * l21 + l22 * l22);
    // pixel-centre sampling: {x : s((mu - R sd) + 1/2) - 1/2 < x < ...}
    const double lo_x = centre ? s * ((mx - R * sx) + 0.5) - 0.5 : s * (mx - R * sx);
    const double hi_x = centre ? s * ((mx + R * sx) + 0.5) - 0.5 : s * (mx + R * sx);
    const double lo_y = centre ? s * ((my - R * sy) + 0.5) - 0.5 : s * (my - R * sy);
    const double hi_y = centre ? s * ((my + R * sy) + 0.5) - 0.5 : s * (my + R * sy);
    double x0 = __builtin_floor(lo_x) + 1.0, x1 = __builtin_ceil(hi_x) - 1.0;
    double y0 = __builtin_floor(lo_y) + 1.0, y1 = __builtin_ceil(hi_y) - 1.0;
    *clipped = x0 < 0.0 || y0 < 0.0 || x1 > (double)(out_w - 1) || y1 > (double)(out_h - 1);
    if (x0 < 0.0) x0 = 0.0;
    if (y0 < 0.0) y0 = 0.0;
    if (x1 > (double)(out_w - 1)) x1 = (double)(out_w - 1);
    if (y1 > (double)(out_h - 1)) y1 = (double)(out_h - 1);
    if (x0 > x1 || y0 > y1) return false;
    box[0] = (int)x0; box[1] = (int)x1; box[2] = (int)y0; box[3] = (int)y1;
    return true;
}

// Algorithm 1's own window (the rasterization ratio r): the strict test
// |x - s mu_x| < r s W, |y - s mu_y| < r s H with both sides in HR pixels
// and each axis paired with its own extent, clipped to the image; the
// Gaussian must still be valid.  Same FP64 operation sequence as the
// standard-deviation box, so boxes are reproducible bit for bit.
__device__ bool window_box(double s, int out_w, int out_h, int lr_w, int lr_h, double r,
                           double mx, double my, double l11, double l21, double l22,
                           bool centre, int* box, bool* clipped) {
#pragma clang fp contract(off)
    if (!finite_d(mx) || !finite_d(my) || !finite_d(l11) || !finite_d(l21) ||
        !finite_d(l22) || !finite_d(r))
        return false;
    if (!(l11 > 0.0) || !(l22 > 0.0) || !(r > 0.0)) return false;
    const double hx = r * (s * (double)lr_w);
    const double hy = r * (s * (double)lr_h);
    const double cx = centre ? s * (mx + 0.5) - 0.5 : s * mx;
    const double cy = centre ? s * (my + 0.5) - 0.5 : s * my;
    double x0 = __builtin_floor(cx - hx) + 1.0, x1 = __builtin_ceil(cx + hx) - 1.0;
    double y0 = __builtin_floor(cy - hy) + 1.0, y1 = __builtin_ceil(cy + hy) - 1.0;
    *clipped = x0 < 0.0 || y0 < 0.0 || x1 > (double)(out_w - 1) || y1 > (double)(out_h - 1);
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
// pair counts (and, for the radix path, the ranges), the backward
// accumulators and the device counters.  With a by-value image table
// (kArgTable, batches of at most kSetupChunk images) the first block also
// writes the table into the workspace for later kernels.
template <bool kArgTable>
__global__ __launch_bounds__(kBlockG) void k_support(
    ImgChunk arg_imgs, ImgDev* __restrict__ imgs, int n_img, int64_t n_gauss, int tile,
    const float* __restrict__ mean, const float* __restrict__ chol,
    const float* __restrict__ color, const float* __restrict__ opacity,
    const float* __restrict__ radius, double window_r, int mode, EParams* __restrict__ eparams,
    GRec* __restrict__ recs,
    int32_t* __restrict__ counts, BlockSums* __restrict__ blocksums,
    int32_t* __restrict__ tile_cnt, int2* __restrict__ ranges_clear, int64_t n_tiles,
    float4* __restrict__ moments, uint32_t* __restrict__ counters) {
    __shared__ int64_t tmp[3][kBlockG / 64];
    const int64_t i = (int64_t)blockIdx.x * kBlockG + threadIdx.x;

    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < kCounterWords; k += kBlockG) counters[k] = 0;

    if (kArgTable && blockIdx.x == 0 && threadIdx.x < n_img)
        imgs[threadIdx.x] = arg_imgs.img[threadIdx.x];
    for (int64_t t = i; t < n_tiles; t += (int64_t)gridDim.x * kBlockG) {
        tile_cnt[t] = 0;
        if (ranges_clear) ranges_clear[t] = make_int2(0, 0);  // radix-sort binning
    }

    int cnt = 0;
    int64_t area = 0;
    int bad = 0;
    if (i < n_gauss) {
        GRec r;
        r.x0 = 0; r.x1 = -1; r.y0 = 0; r.y1 = -1;
        r.fx = r.fy = 0.f; r.kx = r.ky = 0;
        r.a = r.e = r.g = 0.f;
        r.A[0] = r.A[1] = r.A[2] = 0.f;
        r.flags = 0;
        const int k = kArgTable ? find_image(arg_imgs.img, n_img, i) : find_image(imgs, n_img, i);
        r.img = k;
        if (k >= 0) {
            const ImgDev im = kArgTable ? arg_imgs.img[k] : imgs[k];
            const double s = im.scale;
            const double mx = mean[2 * i], my = mean[2 * i + 1];
            const double l11 = chol[3 * i], l21 = chol[3 * i + 1], l22 = chol[3 * i + 2];
            const double R = radius ? (double)radius[i] : 3.0;
            int box[4];
            bool clipped = false;
            const bool shape_ok = finite_d(mx) && finite_d(my) && finite_d(l11) &&
                                  finite_d(l21) && finite_d(l22) && l11 > 0.0 && l22 > 0.0;
            bad = shape_ok ? 0 : 1;
            const bool centre = (mode & GS_FLAG_PIXEL_CENTER) != 0;
            const bool has_box =
                window_r > 0.0
                    ? window_box(s, im.out_w, im.out_h, im.lr_w, im.lr_h, window_r, mx, my, l11,
                                 l21, l22, centre, box, &clipped)
                    : support_box(s, im.out_w, im.out_h, mx, my, l11, l21, l22, R, centre, box,
                                  &clipped);
            if (has_box) {
                // colour / opacity may be NULL when only the pairs are counted
                const double al = opacity ? (double)opacity[i] : 0.0;
                const double c0 = color ? (double)color[3 * i] : 0.0;
                const double c1 = color ? (double)color[3 * i + 1] : 0.0;
                const double c2 = color ? (double)color[3 * i + 2] : 0.0;
                const bool amp_ok = finite_d(al) && finite_d(c0) && finite_d(c1) && finite_d(c2);
                if (!amp_ok) bad = 1;
                r.x0 = box[0]; r.x1 = box[1]; r.y0 = box[2]; r.y1 = box[3];
                const double cx = centre ? s * (mx + 0.5) - 0.5 : s * mx;
                const double cy = centre ? s * (my + 0.5) - 0.5 : s * my;
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
                    r.flags |= kRecNoAmp;  // listed in tiles but adds and receives nothing
                }
                if (clipped) r.flags |= kRecClipped;
                if (window_r > 0.0) r.flags |= kRecCull;
                const int tx0 = r.x0 / tile, tx1 = r.x1 / tile;
                const int ty0 = r.y0 / tile, ty1 = r.y1 / tile;
                cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
                if (eparams) {
                    // elliptical support: the tile kernels rebuild its pixel
                    // masks from these; the in-support pairs are its pixels
                    r.flags |= kRecEllipse;
                    eparams[i].p0 = make_float4(mean[2 * i], mean[2 * i + 1], chol[3 * i],
                                                chol[3 * i + 1]);
                    eparams[i].p1 = make_float4(chol[3 * i + 2], (float)R, centre ? 1.f : 0.f, 0.f);
                    const double R2 = R * R;
                    for (int y = r.y0; y <= r.y1; ++y) {
                        int xa, xb;
                        ellipse_row(y, r.x0, r.x1, s, centre, mx, my, l11, l21, l22, R2, &xa,
                                    &xb);
                        if (xb >= xa) area += xb - xa + 1;
                    }
                } else {
                    area = (int64_t)(r.x1 - r.x0 + 1) * (r.y1 - r.y0 + 1);
                }
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

// First emission index of this block's Gaussians.  With kFold the block sums
// the unscanned block sums below it itself, and the last block writes the
// header totals; otherwise k_scan_blocks has done both.
template <bool kFold>
__device__ __forceinline__ int64_t emission_base(const BlockSums* __restrict__ bs, int nblk,
                                                 int64_t cap, WsHeader* __restrict__ hdr) {
    if (!kFold) return bs[blockIdx.x].pairs;
    __shared__ int64_t t3[3][kBlockG / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.x;
    const bool last_block = b == nblk - 1;
    int64_t lower = 0, sup = 0, inv = 0;
    for (int j = threadIdx.x; j < nblk; j += kBlockG) {
        if (j < b) lower += bs[j].pairs;
        if (last_block) { sup += bs[j].support; inv += bs[j].invalid; }
    }
    lower = wave_sum_i64(lower);
    if (last_block) { sup = wave_sum_i64(sup); inv = wave_sum_i64(inv); }
    if (lane == 0) { t3[0][wave] = lower; t3[1][wave] = sup; t3[2][wave] = inv; }
    __syncthreads();
    int64_t base = 0, sa = 0, sb = 0;
    for (int k = 0; k < kBlockG / 64; ++k) { base += t3[0][k]; sa += t3[1][k]; sb += t3[2][k]; }
    if (last_block && threadIdx.x == 0) {
        const int64_t total = base + bs[b].pairs;
        hdr->n_pairs = total;
        hdr->overflow = total > cap ? 1 : 0;
        hdr->n_support = sa;
        hdr->n_invalid = sb;
        hdr->ordered = 0;
    }
    return base;
}

// One thread per Gaussian: local exclusive scan + block offset (the
// Gaussian's first emission index), then the Gaussian's tiles in row-major
// order: each pair is counted into its tile (tile_cnt, cleared by the support
// kernel), and the count before the pair's increment is its place in the
// tile's list.  When the block's tiles span at most kEmitBins ids, the
// pairs are counted in LDS first and the block adds one total per tile to the
// global count (its place = the block's base + the LDS rank); otherwise each
// pair takes a global atomic.  Pairs past the capacity are neither counted
// nor placed (the overflow flag says so).
template <bool kFold, typename Table>
__global__ __launch_bounds__(kBlockG) void k_emit(
    Table imgs, const GRec* __restrict__ recs, const int32_t* __restrict__ counts,
    const BlockSums* __restrict__ bs, int nblk, int64_t n_gauss, int tile, int64_t cap,
    int32_t* __restrict__ tile_cnt, uint32_t* __restrict__ slots, int32_t* __restrict__ offsets,
    WsHeader* __restrict__ hdr) {
    __shared__ int64_t tmp[kBlockG / 64];
    __shared__ int64_t win[2][kBlockG / 64];
    __shared__ int32_t bins[kEmitBins];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // this Gaussian's count and record, read together with the block sums
    const int64_t i = (int64_t)blockIdx.x * kBlockG + threadIdx.x;
    const int cnt = i < n_gauss ? counts[i] : 0;
    GRec r;
    if (cnt > 0) r = recs[i];
    const int64_t base = emission_base<kFold>(bs, nblk, cap, hdr);
    const int64_t inc = block_inclusive_scan((int64_t)cnt, tmp);
    const int64_t off = base + inc - cnt;
    if (i < n_gauss) offsets[i] = (int32_t)(off < cap ? off : cap);

    // pairs kept, the first tile id and the box's tile geometry
    int n = 0, tx0 = 0, tx1 = -1, ty0 = 0, tiles_x = 0;
    int64_t tb = 0, lo = INT64_MAX, hi = -1;
    if (cnt > 0 && off < cap) {
        const ImgDev& im = imgs[r.img];
        tx0 = r.x0 / tile; tx1 = r.x1 / tile; ty0 = r.y0 / tile;
        const int ty1 = r.y1 / tile;
        tiles_x = im.tiles_x;
        tb = im.tile_base;
        n = (int)(cap - off < (int64_t)cnt ? cap - off : (int64_t)cnt);
        lo = tb + (int64_t)ty0 * tiles_x + tx0;
        hi = tb + (int64_t)ty1 * tiles_x + tx1;
    }
    // the block's tile window
    lo = wave_butterfly(lo, [](int64_t a, int64_t b) { return min(a, b); });
    hi = wave_butterfly(hi, [](int64_t a, int64_t b) { return max(a, b); });
    if (lane == 0) { win[0][wave] = lo; win[1][wave] = hi; }
    __syncthreads();
    int64_t wlo = win[0][0], whi = win[1][0];
    for (int k = 1; k < kBlockG / 64; ++k) { wlo = min(wlo, win[0][k]); whi = max(whi, win[1][k]); }
    if (whi < wlo) return;  // uniform: no pairs in this block

    if (whi - wlo < kEmitBins) {  // uniform
        const int nw = (int)(whi - wlo + 1);
        for (int j = threadIdx.x; j < nw; j += kBlockG) bins[j] = 0;
        __syncthreads();
        // LDS ranks; the first kKeep in registers, the rest parked in slots
        constexpr int kKeep = 8;
        uint32_t rk[kKeep];
        int tx = tx0, ty = ty0;
#pragma unroll
        for (int k = 0; k < kKeep; ++k) {
            rk[k] = 0;
            if (k < n) {
                rk[k] = (uint32_t)atomicAdd(&bins[(int)(tb + (int64_t)ty * tiles_x + tx - wlo)], 1);
                if (++tx > tx1) { tx = tx0; ++ty; }
            }
        }
        for (int k = kKeep; k < n; ++k) {
            slots[off + k] = (uint32_t)atomicAdd(&bins[(int)(tb + (int64_t)ty * tiles_x + tx - wlo)], 1);
            if (++tx > tx1) { tx = tx0; ++ty; }
        }
        __syncthreads();
        // one global atomic per tile: the block's base in the tile's list
        for (int j = threadIdx.x; j < nw; j += kBlockG) {
            const int c = bins[j];
            if (c) bins[j] = atomicAdd(&tile_cnt[wlo + j], c);
        }
        __syncthreads();
        tx = tx0; ty = ty0;
#pragma unroll
        for (int k = 0; k < kKeep; ++k) {
            if (k < n) {
                slots[off + k] = (uint32_t)bins[(int)(tb + (int64_t)ty * tiles_x + tx - wlo)] + rk[k];
                if (++tx > tx1) { tx = tx0; ++ty; }
            }
        }
        for (int k = kKeep; k < n; ++k) {
            slots[off + k] += (uint32_t)bins[(int)(tb + (int64_t)ty * tiles_x + tx - wlo)];
            if (++tx > tx1) { tx = tx0; ++ty; }
        }
        return;
    }
    // wide block: a global atomic per pair, four in flight per thread
    int tx = tx0, ty = ty0;
    for (int k0 = 0; k0 < n; k0 += 4) {
        uint32_t slot[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            slot[u] = 0;
            if (k0 + u < n) {
                slot[u] = (uint32_t)atomicAdd(&tile_cnt[tb + (int64_t)ty * tiles_x + tx], 1);
                if (++tx > tx1) { tx = tx0; ++ty; }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k0 + u < n) slots[off + k0 + u] = slot[u];
    }
}

// Radix-sort binning (GS_FLAG_RADIX_SORT).  Each Gaussian's (tile id,
// Gaussian id) pairs go in tile row-major order to its emission indices,
// Gaussian-major overall, so a stable sort by tile id leaves every tile's
// Gaussians in ascending id.  The block's threads write the block's span of
// pairs together, consecutive threads consecutive pairs (coalesced stores):
// each finds its pair's Gaussian by binary search over the block's emission
// starts in LDS and the tile from the pair's rank in the Gaussian's tile
// rectangle.
template <bool kFold, typename Table>
__global__ __launch_bounds__(kBlockG) void k_emit_pairs(
    Table imgs, const GRec* __restrict__ recs, const int32_t* __restrict__ counts,
    const BlockSums* __restrict__ bs, int nblk, int64_t n_gauss, int tile, int64_t cap,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, int32_t* __restrict__ offsets,
    WsHeader* __restrict__ hdr) {
    __shared__ int64_t tmp[kBlockG / 64];
    __shared__ int64_t s_start[kBlockG];  // block-relative emission start
    __shared__ uint32_t s_first[kBlockG];  // tile id of the rectangle's first tile
    __shared__ int32_t s_width[kBlockG];   // tiles per rectangle row
    __shared__ int32_t s_stride[kBlockG];  // tiles per image row
    __shared__ int64_t s_total;
    const int64_t base = emission_base<kFold>(bs, nblk, cap, hdr);
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kBlockG + t;
    const int cnt = i < n_gauss ? counts[i] : 0;
    const int64_t inc = block_inclusive_scan((int64_t)cnt, tmp);
    const int64_t off = base + inc - cnt;
    if (i < n_gauss) offsets[i] = (int32_t)(off < cap ? off : cap);
    s_start[t] = inc - cnt;
    s_first[t] = 0u;
    s_width[t] = 1;
    s_stride[t] = 0;
    if (cnt > 0) {
        const GRec r = recs[i];
        const ImgDev& im = imgs[r.img];
        const int tx0 = r.x0 / tile, tx1 = r.x1 / tile, ty0 = r.y0 / tile;
        s_first[t] = (uint32_t)(im.tile_base + (int64_t)ty0 * im.tiles_x + tx0);
        s_width[t] = tx1 - tx0 + 1;
        s_stride[t] = im.tiles_x;
    }
    if (t == kBlockG - 1) s_total = inc;
    __syncthreads();
    const int64_t total = s_total;
    int lo = 0;  // the pairs' Gaussians ascend with p
    for (int64_t p = t; p < total; p += kBlockG) {
        // the last Gaussian whose start is at most p (empty Gaussians share
        // their successor's start and precede it)
        int a = lo, b = kBlockG - 1;
        while (a < b) {
            const int m = (a + b + 1) >> 1;
            if (s_start[m] <= p) a = m; else b = m - 1;
        }
        lo = a;
        const int k = (int)(p - s_start[a]);  // below the Gaussian's int32 count
        const int w = s_width[a];
        const int row = k / w, col = k - row * w;
        if (base + p < cap) {
            keys[base + p] = s_first[a] + (uint32_t)row * (uint32_t)s_stride[a] + (uint32_t)col;
            vals[base + p] = (uint32_t)((int64_t)blockIdx.x * kBlockG + a);
        }
    }
}

__device__ __forceinline__ int64_t pairs_in_use(const WsHeader* hdr, int64_t cap) {
    const int64_t p = hdr->n_pairs;
    return p < cap ? p : cap;
}

// Sort source of the radix-sort binning: the (tile, Gaussian) pairs, keyed by
// the 8-bit digit of the tile id at `shift`.
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

// One thread per sorted pair: the tile range boundaries (the ranges were
// cleared to [0, 0) by the support kernel).
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

// Inclusive scan of one int64 value per thread across a workgroup of
// kScanThreads threads; `tmp` holds kScanThreads / 64 entries.
__device__ __forceinline__ int64_t scan_block_inclusive(int64_t v, int64_t* tmp) {
    constexpr int NW = kScanThreads / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_inclusive_scan_i64(v);
    if (lane == 63) tmp[wave] = v;
    __syncthreads();
    if (wave == 0) {
        const int64_t x = wave_inclusive_scan_i64(lane < NW ? tmp[lane] : 0);
        if (lane < NW) tmp[lane] = x;  // inclusive over waves
    }
    __syncthreads();
    const int64_t carry = wave > 0 ? tmp[wave - 1] : 0;
    __syncthreads();
    return v + carry;
}

// Tile-count scan, blocks of kScanTile tiles (kScanPer consecutive tiles per
// thread).  With several blocks: k_tile_sums writes each block's count,
// k_scan_sums scans them, k_tile_ranges adds the block's base.
__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const int32_t* __restrict__ tile_cnt,
                                                            int64_t n_tiles,
                                                            int64_t* __restrict__ sums) {
    __shared__ int64_t tmp[kScanThreads / 64];
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
    int64_t v = 0;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        const int64_t j = b0 + u * kScanThreads + threadIdx.x;
        if (j < n_tiles) v += tile_cnt[j];
    }
    v = wave_sum_i64(v);
    if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t b = 0;
        for (int k = 0; k < kScanThreads / 64; ++k) b += tmp[k];
        sums[blockIdx.x] = b;
    }
}

// One workgroup: exclusive scan of the block sums, in place.
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int64_t* __restrict__ sums, int nblk) {
    __shared__ int64_t tmp[kScanThreads / 64];
    __shared__ int64_t last;
    int64_t carry = 0;
    for (int base = 0; base < nblk; base += kScanThreads) {
        const int j = base + threadIdx.x;
        const int64_t v = j < nblk ? sums[j] : 0;
        const int64_t inc = scan_block_inclusive(v, tmp);
        if (j < nblk) sums[j] = carry + inc - v;
        if (threadIdx.x == kScanThreads - 1) last = inc;
        __syncthreads();
        carry += last;
        __syncthreads();
    }
}

// The tile ranges: [begin, end) from the exclusive scan of the counts
// ([0, 0) for an empty tile).  Counts are loaded and ranges stored coalesced
// through LDS (one pad word every 32, so that a thread's kScanPer consecutive
// entries are free of bank conflicts too).
__global__ __launch_bounds__(kScanThreads) void k_tile_ranges(const int32_t* __restrict__ tile_cnt,
                                                              int2* __restrict__ ranges,
                                                              int64_t n_tiles,
                                                              const int64_t* __restrict__ sums,
                                                              int multi) {
    auto lds = [](int j) { return j + (j >> 5); };
    __shared__ int64_t tmp[kScanThreads / 64];
    __shared__ int32_t sc[kScanTile + kScanTile / 32];
    __shared__ int32_t s_end;
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        const int j = u * kScanThreads + threadIdx.x;
        sc[lds(j)] = b0 + j < n_tiles ? tile_cnt[b0 + j] : 0;
    }
    __syncthreads();
    const int t0 = threadIdx.x * kScanPer;
    int c[kScanPer];
    int64_t v = 0;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        c[u] = sc[lds(t0 + u)];
        v += c[u];
    }
    const int64_t inc = scan_block_inclusive(v, tmp);  // has barriers
    int b = (int)((multi ? sums[blockIdx.x] : 0) + inc - v);
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        sc[lds(t0 + u)] = b;
        b += c[u];
    }
    if (threadIdx.x == kScanThreads - 1) s_end = b;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        const int j = u * kScanThreads + threadIdx.x;
        if (b0 + j < n_tiles) {
            const int beg = sc[lds(j)];
            const int end = j + 1 < kScanTile ? sc[lds(j + 1)] : s_end;
            ranges[b0 + j] = end > beg ? make_int2(beg, end) : make_int2(0, 0);
        }
    }
}

// One thread per Gaussian: its id written at its place in each of its tiles'
// lists (the tiles in the emission's order).  With kLocalScan (at most
// kPlaceScanTiles tiles) every block scans the tile counts into LDS itself
// and block 0 writes the tile ranges; otherwise the ranges come from the scan
// kernels.
template <bool kLocalScan, typename Table>
__global__ __launch_bounds__(kBlockG) void k_place(
    Table imgs, const GRec* __restrict__ recs, const int32_t* __restrict__ counts,
    const int32_t* __restrict__ offsets, int64_t n_gauss, int tile, int64_t cap,
    const int32_t* __restrict__ tile_cnt, int64_t n_tiles, int2* __restrict__ ranges,
    const uint32_t* __restrict__ slots, uint32_t* __restrict__ lists) {
    constexpr int kPer = kPlaceScanTiles / kBlockG;
    // LDS index of tile j: one pad word every 32, so that a thread's kPer
    // consecutive tiles and the coalesced fill are both free of bank conflicts
    auto lds = [](int j) { return j + (j >> 5); };
    __shared__ int32_t s_off[kLocalScan ? kPlaceScanTiles + kPlaceScanTiles / 32 : 1];
    __shared__ int64_t tmp[kBlockG / 64];
    // this Gaussian's inputs first: their latency overlaps the scan below
    const int64_t i = (int64_t)blockIdx.x * kBlockG + threadIdx.x;
    int cnt = 0;
    int64_t off = cap;
    GRec r;
    uint32_t sl[4] = {0u, 0u, 0u, 0u};  // the first four slots
    if (i < n_gauss) {
        cnt = counts[i];
        off = offsets[i];
        if (cnt > 0 && off < cap) {
            r = recs[i];
            const int n4 = (int)min((int64_t)min(cnt, 4), cap - off);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (u < n4) sl[u] = slots[off + u];
        }
    }
    if (kLocalScan) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int j = u * kBlockG + threadIdx.x;
            s_off[lds(j)] = j < n_tiles ? tile_cnt[j] : 0;
        }
        __syncthreads();
        const int t0 = threadIdx.x * kPer;
        int c[kPer];
        int64_t v = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            c[u] = s_off[lds(t0 + u)];
            v += c[u];
        }
        const int64_t inc = block_inclusive_scan(v, tmp);  // has barriers
        int b = (int)(inc - v);
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            s_off[lds(t0 + u)] = b;
            if (blockIdx.x == 0 && t0 + u < n_tiles)
                ranges[t0 + u] = c[u] ? make_int2(b, b + c[u]) : make_int2(0, 0);
            b += c[u];
        }
        __syncthreads();
    }
    if (cnt == 0 || off >= cap) return;
    const ImgDev& im = imgs[r.img];
    const int tx0 = r.x0 / tile, tx1 = r.x1 / tile, ty0 = r.y0 / tile;
    const int n = (int)(cap - off < (int64_t)cnt ? cap - off : (int64_t)cnt);
    const int64_t tb = im.tile_base;
    int tx = tx0, ty = ty0;
    for (int k0 = 0; k0 < n; k0 += 4) {
        int pos[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pos[u] = -1;
            if (k0 + u < n) {
                const int64_t t = tb + (int64_t)ty * im.tiles_x + tx;
                const uint32_t slot = k0 == 0 ? sl[u] : slots[off + k0 + u];
                pos[u] = (kLocalScan ? s_off[lds((int)t)] : ranges[t].x) + (int)slot;
                if (++tx > tx1) { tx = tx0; ++ty; }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (pos[u] >= 0) lists[pos[u]] = (uint32_t)i;
    }
}

// The smaller and the larger of a lane's value and the value of lane
// (lane ^ d), d in {1, 2, 4, 8, 16, 32}, without an LDS round trip: DPP lane
// moves within rows of 16 (d = 4 as a quad reversal then a half-row mirror,
// d = 8 as a rotation by 8 within the row), the row and half-wave swaps of
// gfx950 for 16 and 32 (each lane then holds both values of its pair).
template <int kD>
__device__ __forceinline__ void xor_minmax(uint32_t v, uint32_t& lo, uint32_t& hi) {
    if constexpr (kD == 16 || kD == 32) {
        const auto r = kD == 16 ? __builtin_amdgcn_permlane16_swap(v, v, false, false)
                                : __builtin_amdgcn_permlane32_swap(v, v, false, false);
        lo = min((uint32_t)r[0], (uint32_t)r[1]);
        hi = max((uint32_t)r[0], (uint32_t)r[1]);
    } else {
        const int x = (int)v;
        int p;
        if constexpr (kD == 1) {
            p = __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
        } else if constexpr (kD == 2) {
            p = __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
        } else if constexpr (kD == 4) {
            const int q = __builtin_amdgcn_update_dpp(0, x, 0x1B, 0xF, 0xF, false);  // [3,2,1,0]
            p = __builtin_amdgcn_update_dpp(0, q, 0x141, 0xF, 0xF, false);  // row_half_mirror
        } else {
            static_assert(kD == 8, "lane distance");
            p = __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);  // row_ror:8
        }
        lo = min(v, (uint32_t)p);
        hi = max(v, (uint32_t)p);
    }
}

// Ascending bitonic sort of 64 K values held K per lane across the wave:
// element i = 64 k + lane is v[k] of that lane.  Partners closer than 64 are
// exchanged across lanes, farther ones between a lane's own registers.
template <int K, int kS, int kD>
__device__ __forceinline__ void bitonic_step(uint32_t (&v)[K], int lane) {
    if constexpr (kD >= 64) {
        constexpr int kd = kD >> 6;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k & kd) continue;
            const bool up = (((k << 6) | lane) & kS) == 0;
            const uint32_t lo = min(v[k], v[k | kd]), hi = max(v[k], v[k | kd]);
            v[k] = up ? lo : hi;
            v[k | kd] = up ? hi : lo;
        }
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            uint32_t lo, hi;
            xor_minmax<kD>(v[k], lo, hi);
            const bool up = (((k << 6) | lane) & kS) == 0;
            const bool low = (lane & kD) == 0;
            v[k] = (low == up) ? lo : hi;
        }
    }
    if constexpr (kD > 1) bitonic_step<K, kS, kD / 2>(v, lane);
}

template <int K, int kS>
__device__ __forceinline__ void bitonic_stage(uint32_t (&v)[K], int lane) {
    bitonic_step<K, kS, kS / 2>(v, lane);
    if constexpr (kS < 64 * K) bitonic_stage<K, kS * 2>(v, lane);
}

template <int K>
__device__ __forceinline__ void wave_sort(uint32_t (&v)[K]) {
    bitonic_stage<K, 2>(v, threadIdx.x & 63);
}

// One wave sorts seg[0, n), n <= 64 K, in registers and writes it back.
template <int K>
__device__ __forceinline__ void wave_sort_list(uint32_t* __restrict__ seg, int n) {
    const int lane = threadIdx.x & 63;
    uint32_t v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 64 * k + lane < n ? seg[64 * k + lane] : 0xffffffffu;
    wave_sort<K>(v);
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (64 * k + lane < n) seg[64 * k + lane] = v[k];
}

// Number of entries of the ascending run a[0, n), n >= 1, below x.
__device__ __forceinline__ int count_below(const uint32_t* a, int n, uint32_t x) {
    int lo = 0;
    for (int step = 1 << (31 - __builtin_clz((unsigned)n)); step > 0; step >>= 1)
        if (lo + step <= n && a[lo + step - 1] < x) lo += step;
    return lo;
}

// Sorts seg[0, n), n <= kSegLds, ascending (distinct values) with the whole
// workgroup: each wave sorts 256-entry runs in registers into LDS, then
// every entry's rank is its place in its own run plus the entries below it
// in the other runs.  Ends with a barrier.
__device__ __forceinline__ void sort_chunk(uint32_t* __restrict__ seg, int n, uint32_t* sk) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int NW = kSegThreads / 64;
    const int runs = (n + 255) >> 8;
    for (int q = wave; q < runs; q += NW) {
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int idx = q * 256 + 64 * k + lane;
            v[k] = idx < n ? seg[idx] : 0xffffffffu;
        }
        wave_sort<4>(v);
#pragma unroll
        for (int k = 0; k < 4; ++k) sk[q * 256 + 64 * k + lane] = v[k];
    }
    __syncthreads();
    for (int i = t; i < n; i += kSegThreads) {
        const uint32_t x = sk[i];
        const int own = i >> 8;
        int pos = i & 255;
        for (int q = 0; q < runs; ++q)
            if (q != own) pos += count_below(sk + q * 256, 256, x);
        seg[pos] = x;
    }
    __syncthreads();
}

// Four tiles per workgroup: each wave sorts its tile's list in registers when
// it holds at most 256 ids; longer lists are sorted by the whole workgroup
// afterwards: up to kSegLds through LDS, beyond that in kSegLds chunks merged
// pairwise through `spare` (each entry's place: its index in its run plus the
// entries below it in the partner run).
__global__ __launch_bounds__(kSegThreads) void k_sort_lists(const int2* __restrict__ ranges,
                                                            int64_t n_tiles,
                                                            uint32_t* __restrict__ lists,
                                                            uint32_t* __restrict__ spare) {
    constexpr int NW = kSegThreads / 64;
    __shared__ uint32_t sk[kSegLds];
    __shared__ int s_long[NW];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * NW + wave;
    int2 r = make_int2(0, 0);
    if (tile < n_tiles) r = ranges[tile];
    const int n = r.y - r.x;
    if (n > 1 && n <= 64) wave_sort_list<1>(lists + r.x, n);
    else if (n > 64 && n <= 128) wave_sort_list<2>(lists + r.x, n);
    else if (n > 128 && n <= 256) wave_sort_list<4>(lists + r.x, n);
    if (lane == 0) s_long[wave] = n > 256 ? 1 : 0;
    __syncthreads();
    for (int wv = 0; wv < NW; ++wv) {
        if (!s_long[wv]) continue;  // uniform
        const int2 rl = ranges[(int64_t)blockIdx.x * NW + wv];
        const int nl = rl.y - rl.x;
        uint32_t* seg = lists + rl.x;
        if (nl <= kSegLds) {
            sort_chunk(seg, nl, sk);
            continue;
        }
        for (int c0 = 0; c0 < nl; c0 += kSegLds) sort_chunk(seg + c0, min(kSegLds, nl - c0), sk);
        uint32_t* src = seg;
        uint32_t* dst = spare + rl.x;
        for (int64_t w = kSegLds; w < nl; w *= 2) {
            for (int i = threadIdx.x; i < nl; i += kSegThreads) {
                const uint32_t x = src[i];
                const int64_t run = i / w, first = run * w;
                const int64_t p0 = (run ^ 1) * w;  // partner run
                int below = 0;
                if (p0 < nl) below = count_below(src + p0, (int)min(w, (int64_t)nl - p0), x);
                dst[min(first, p0) + (i - first) + below] = x;
            }
            __syncthreads();
            uint32_t* sw = src;
            src = dst;
            dst = sw;
        }
        if (src != seg) {
            for (int i = threadIdx.x; i < nl; i += kSegThreads) seg[i] = src[i];
            __syncthreads();
        }
    }
}

// Sort source of the tile order: the tiles themselves, keyed by the bucket
// of their list length, longest first (the longest-processing-time order the
// persistent tile kernels take their work in).
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
// row total into totals[d].  Each wave scans its own contiguous quarter of
// the row 64 entries at a time with shuffles (no barrier per chunk), the
// quarters' totals are combined once, and a second sweep adds each
// quarter's offset.
__global__ __launch_bounds__(kBlockG) void k_sort_rowscan(int32_t* __restrict__ hist,
                                                          int nblk,
                                                          int32_t* __restrict__ totals) {
    constexpr int NW = kBlockG / 64;
    __shared__ int64_t wsum[NW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t* row = hist + (int64_t)blockIdx.x * nblk;
    const int per = (nblk + NW - 1) / NW;
    const int lo = min(nblk, wave * per), hi = min(nblk, lo + per);
    int64_t carry = 0;  // within the wave's quarter
    for (int b0 = lo; b0 < hi; b0 += 64) {
        const int j = b0 + lane;
        const int64_t v = j < hi ? row[j] : 0;
        int64_t x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t u = __shfl_up(x, o, 64);
            if (lane >= o) x += u;
        }
        if (j < hi) row[j] = (int32_t)(carry + x - v);  // exclusive within the quarter
        carry += __shfl(x, 63, 64);
    }
    if (lane == 0) wsum[wave] = carry;
    __syncthreads();
    int64_t off = 0;
    for (int k = 0; k < wave; ++k) off += wsum[k];
    if (off != 0) {
        for (int j = lo + lane; j < hi; j += 64) row[j] += (int32_t)off;
    }
    if (threadIdx.x == 0) {
        int64_t tot = 0;
        for (int k = 0; k < NW; ++k) tot += wsum[k];
        totals[blockIdx.x] = (int32_t)tot;
    }
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
    const bool radix = (L.flags & GS_FLAG_RADIX_SORT) != 0;
    if (by_value)
        hipLaunchKernelGGL(k_support<true>, dim3(L.nblk_g), dim3(kBlockG), 0, st, chunk, w.imgs,
                           L.n_img, L.n_gauss, L.tile, mean, chol, color, opacity, radius,
                           L.window_r, L.flags, w.eparams, w.recs, w.counts, w.blocksums, w.tile_cnt, radix ? w.ranges : nullptr, L.n_tiles, mom,
                           w.counters);
    else
        hipLaunchKernelGGL(k_support<false>, dim3(L.nblk_g), dim3(kBlockG), 0, st, chunk, w.imgs,
                           L.n_img, L.n_gauss, L.tile, mean, chol, color, opacity, radius,
                           L.window_r, L.flags, w.eparams, w.recs, w.counts, w.blocksums, w.tile_cnt, radix ? w.ranges : nullptr, L.n_tiles, mom,
                           w.counters);
    if (count_only || L.nblk_g > kFoldScanBlocks)
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBlockG), 0, st, w.blocksums, L.nblk_g,
                           L.cap, w.hdr);
    return hipGetLastError();
}

template <typename Table>
void launch_emit_t(const Layout& L, const Ws& w, Table tab, hipStream_t st) {
    if (L.flags & GS_FLAG_RADIX_SORT) {
        uint32_t* keys = w.keys[0];
        uint32_t* vals = w.vals[0];
        if (L.nblk_g > kFoldScanBlocks)
            hipLaunchKernelGGL((k_emit_pairs<false, Table>), dim3(L.nblk_g), dim3(kBlockG), 0, st,
                               tab, w.recs, w.counts, w.blocksums, L.nblk_g, L.n_gauss, L.tile,
                               L.cap, keys, vals, w.offsets, w.hdr);
        else
            hipLaunchKernelGGL((k_emit_pairs<true, Table>), dim3(L.nblk_g), dim3(kBlockG), 0, st,
                               tab, w.recs, w.counts, w.blocksums, L.nblk_g, L.n_gauss, L.tile,
                               L.cap, keys, vals, w.offsets, w.hdr);
        return;
    }
    if (L.nblk_g > kFoldScanBlocks)
        hipLaunchKernelGGL((k_emit<false, Table>), dim3(L.nblk_g), dim3(kBlockG), 0, st, tab,
                           w.recs, w.counts, w.blocksums, L.nblk_g, L.n_gauss, L.tile, L.cap,
                           w.tile_cnt, w.slots, w.offsets, w.hdr);
    else
        hipLaunchKernelGGL((k_emit<true, Table>), dim3(L.nblk_g), dim3(kBlockG), 0, st, tab,
                           w.recs, w.counts, w.blocksums, L.nblk_g, L.n_gauss, L.tile, L.cap,
                           w.tile_cnt, w.slots, w.offsets, w.hdr);
}

hipError_t launch_emit(const Layout& L, const Ws& w, hipStream_t st) {
    if (L.n_img <= kSetupChunk && L.host_imgs) {
        ArgTable tab;
        for (int k = 0; k < kSetupChunk; ++k) tab.c.img[k] = k < L.n_img ? L.host_imgs[k] : ImgDev{};
        launch_emit_t(L, w, tab, st);
    } else {
        launch_emit_t(L, w, MemTable{w.imgs}, st);
    }
    return hipGetLastError();
}

template <typename Table>
void launch_place_t(const Layout& L, const Ws& w, Table tab, bool local_scan, hipStream_t st) {
    if (local_scan)
        hipLaunchKernelGGL((k_place<true, Table>), dim3(L.nblk_g), dim3(kBlockG), 0, st, tab,
                           w.recs, w.counts, w.offsets, L.n_gauss, L.tile, L.cap, w.tile_cnt,
                           L.n_tiles, w.ranges, w.slots, w.lists);
    else
        hipLaunchKernelGGL((k_place<false, Table>), dim3(L.nblk_g), dim3(kBlockG), 0, st, tab,
                           w.recs, w.counts, w.offsets, L.n_gauss, L.tile, L.cap, w.tile_cnt,
                           L.n_tiles, w.ranges, w.slots, w.lists);
}

// Radix-sort binning: LSD passes of 8-bit digits over the tile-id bits
// (ping-pong between the two key and value buffers; the layout puts the last
// pass's values into the lists), then the ranges from the sorted keys.
hipError_t launch_radix_lists(const Layout& L, const Ws& w, hipStream_t st) {
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
    hipLaunchKernelGGL(k_ranges, dim3(blocks_for(L.cap, kBlockG)), dim3(kBlockG), 0, st,
                       w.keys[L.n_passes & 1], w.hdr, L.cap, w.ranges);
    return hipGetLastError();
}

hipError_t launch_lists(const Layout& L, const Ws& w, hipStream_t st) {
    if (L.n_tiles == 0) return hipSuccess;
    if (L.flags & GS_FLAG_RADIX_SORT) return launch_radix_lists(L, w, st);
    // small batches: the placement blocks scan the counts themselves (each
    // reads all of them, so only while that stays a few MB)
    const bool local_scan = L.n_tiles <= kPlaceScanTiles &&
                            L.n_tiles * (int64_t)L.nblk_g <= ((int64_t)1 << 22);
    if (!local_scan) {
        const int multi = L.nblk_scan > 1 ? 1 : 0;
        if (multi) {
            hipLaunchKernelGGL(k_tile_sums, dim3(L.nblk_scan), dim3(kScanThreads), 0, st,
                               w.tile_cnt, L.n_tiles, w.scan_sums);
            hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, st, w.scan_sums,
                               L.nblk_scan);
        }
        hipLaunchKernelGGL(k_tile_ranges, dim3(L.nblk_scan), dim3(kScanThreads), 0, st,
                           w.tile_cnt, w.ranges, L.n_tiles, w.scan_sums, multi);
    }
    if (L.n_img <= kSetupChunk && L.host_imgs) {
        ArgTable tab;
        for (int k = 0; k < kSetupChunk; ++k) tab.c.img[k] = k < L.n_img ? L.host_imgs[k] : ImgDev{};
        launch_place_t(L, w, tab, local_scan, st);
    } else {
        launch_place_t(L, w, MemTable{w.imgs}, local_scan, st);
    }
    hipLaunchKernelGGL(k_sort_lists, dim3((unsigned)((L.n_tiles + kSegThreads / 64 - 1) / (kSegThreads / 64))), dim3(kSegThreads), 0,
                       st, w.ranges, L.n_tiles, w.lists, w.spare);
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

}  // namespace gs
