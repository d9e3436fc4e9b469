// Internal device structures and launchers of the gfx950 rasterizer library.
// Not part of the C ABI (include/gs_raster.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gs_raster.h"

namespace gs {

constexpr int kMlpParams = 4801;        // W1 64x8, b1 64, W2 64x64, b2 64, W3 1x64, b3 1
constexpr int kSetupChunk = 32;        // images per table chunk (kernel argument)
constexpr int kFoldScanBlocks = 2048;  // up to this many Gaussian blocks the
                                       // emission kernel scans the block sums itself
constexpr int kBlockG = 256;           // threads of per-Gaussian kernels
constexpr int kSortThreads = 256;      // tile-order radix sort workgroup
constexpr int kSortItems = 4;          // keys per thread per sort block
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRadixBits = 8;
constexpr int kScanThreads = 1024;     // tile-count scan workgroup
constexpr int kScanPer = 16;           // tiles per scan thread
constexpr int kScanTile = kScanThreads * kScanPer;
constexpr int kSegThreads = 256;       // per-tile list sort workgroup
constexpr int kSegLds = 2048;          // longest list sorted in LDS in one go
constexpr int kFinChunk = 1024;        // per-pair sums staged per gradient-kernel round
constexpr int kEmitBins = 4096;        // widest tile window counted in LDS by one emission block
constexpr int kPlaceScanTiles = 4096;  // up to this many tiles each placement block scans the
                                       // tile counts itself
// Device counters (one 64-byte line each), zeroed by every binning: the
// loss reduction's count of finished workgroups.
constexpr int kCounterStride = 16;  // words
constexpr int kLossCounterWord = 0;
constexpr int kCounterWords = kCounterStride;
constexpr int kLossSlice = 4096;  // tiles per loss-reduction workgroup (at least)
constexpr int kLossParts = 64;    // loss-reduction workgroups (at most)
// The loss reductions (the stand-alone kernel and the gradient kernel's
// appended workgroups) split the tiles the same way, so they give the same
// bits: P parts, part b summing tiles [n b / P, n (b + 1) / P).
inline int loss_parts(int64_t n_tiles) {
    const int64_t p = (n_tiles + kLossSlice - 1) / kLossSlice;
    return (int)(p < 1 ? 1 : (p > kLossParts ? kLossParts : p));
}
constexpr int kRadix = 1 << kRadixBits;

// exp(-q/2) = exp2(-(kc z)^2) with kc = sqrt(log2(e) / 2); the render
// records carry z pre-multiplied by kc so the kernels call exp2 directly.
constexpr double kZScale = 0.84932180028801904272;

// Per-image table, resident in the workspace (64 B).
struct ImgDev {
    int32_t out_w, out_h;
    int32_t tiles_x, tiles_y;
    int64_t out_offset;     // element offset of [3][out_h][out_w]
    int64_t g_begin, g_count;
    int64_t tile_base;      // first global tile id of this image
    double scale;
    int32_t lr_w, lr_h;     // LR size (the r-window's extents)
};
static_assert(sizeof(ImgDev) == 64, "ImgDev layout");

// Per-Gaussian render record written by the support kernel (64 B).
//   HR centre s*mu = (kx + fx, ky + fy), kx = floor(s*mu_x), fx in [0, 1).
//   For an HR pixel at integer (x, y): X = (x - kx) - fx, Y = (y - ky) - fy,
//   z1 = a X, z2 = e Y - g X, contribution A_c * exp2(-(z1^2 + z2^2)).
struct GRec {
    float fx, fy;
    int32_t kx, ky;
    float a, e, g;
    float A[3];
    int32_t x0, x1, y0, y1;  // support box, inclusive; x0 > x1 means none
    int32_t img;
    int32_t flags;           // kRecNoAmp | kRecClipped
};
// GRec::flags: a non-finite opacity or colour (listed in its tiles, adds and
// receives nothing); the support box was cut by the image border.
constexpr int32_t kRecNoAmp = 1;
constexpr int32_t kRecClipped = 2;
// The support is a window wider than the Gaussian (Algorithm 1's r-window):
// the tile kernels drop (block, Gaussian) records whose weights all round to
// zero.
constexpr int32_t kRecCull = 4;
// The support is the ellipse d < R inside the box: the tile kernels build the
// pixel masks from the Gaussian's exact parameters (eparams).
constexpr int32_t kRecEllipse = 8;

// Per Gaussian, for the elliptical support: {mu_x, mu_y, l11, l21},
// {l22, R, centre, 0} (the FP32 inputs, widened to FP64 where used; centre
// is 1 with GS_FLAG_PIXEL_CENTER).
struct EParams {
    float4 p0, p1;
};

// The LR coordinate HR pixel index x samples: x / s, or (x + 1/2)/s - 1/2
// with pixel-centre sampling.
__device__ __forceinline__ double sample_u(int x, double s, bool centre) {
#pragma clang fp contract(off)
    return centre ? ((double)x + 0.5) / s - 0.5 : (double)x / s;
}

// Elliptical support membership of HR pixel (x, y): d^2 < R^2 with
// z1 = (u - mu_x)/l11, z2 = ((v - mu_y) - l21 z1)/l22, d^2 = z1 z1 + z2 z2,
// evaluated in FP64 in exactly this order (IEEE division, no contraction), so
// the decision is reproducible bit for bit.
__device__ __forceinline__ bool in_ellipse(int x, int y, double s, bool centre, double mx,
                                           double my, double l11, double l21, double l22,
                                           double R2) {
#pragma clang fp contract(off)
    const double z1 = (sample_u(x, s, centre) - mx) / l11;
    const double z2 = ((sample_u(y, s, centre) - my) - l21 * z1) / l22;
    return z1 * z1 + z2 * z2 < R2;
}

// The pixels [*xa, *xb] of HR row y within [x0, x1] inside the ellipse
// (*xa > *xb when none).  Along a row d^2 is a convex quadratic, so the set
// is an interval: its ends come from the analytic roots (FP64), and the
// pixels within two of them are decided by in_ellipse itself.
__device__ __forceinline__ void ellipse_row(int y, int x0, int x1, double s, bool centre,
                                            double mx, double my, double l11, double l21,
                                            double l22, double R2, int* xa, int* xb) {
    const double c = centre ? 0.5 : 0.0;
    const double dy = sample_u(y, s, centre) - my;
    const double k = l21 / l22;
    const double A = 1.0 + k * k;
    const double B = dy * k / l22;
    const double C = (dy / l22) * (dy / l22) - R2;
    const double disc = B * B - A * C;
    const double zc = B / A;
    const double r = disc > 0.0 ? sqrt(disc) / A : 0.0;
    // HR x of z1: s (mu_x + l11 z1 + c) - c, clamped near the range
    const double lim_lo = (double)x0 - 4.0, lim_hi = (double)x1 + 4.0;
    double xl = s * (mx + l11 * (zc - r) + c) - c;
    double xh = s * (mx + l11 * (zc + r) + c) - c;
    xl = fmin(fmax(xl, lim_lo), lim_hi);
    xh = fmin(fmax(xh, lim_lo), lim_hi);
    int a = max(x0, (int)ceil(xl) - 2), b = min(x1, (int)floor(xh) + 2);
    while (a <= b && !in_ellipse(a, y, s, centre, mx, my, l11, l21, l22, R2)) ++a;
    while (b >= a && !in_ellipse(b, y, s, centre, mx, my, l11, l21, l22, R2)) --b;
    *xa = a;
    *xb = b;
}
static_assert(sizeof(GRec) == 64, "GRec layout");


// Per-block partial counts written by the support kernel.
struct BlockSums {
    int64_t pairs;    // (tile, Gaussian) pairs of the block's Gaussians
    int64_t support;  // in-support (pixel, Gaussian) pairs
    int64_t invalid;  // Gaussians flagged for invalid values
};

// Device counters at the start of the workspace (256 B reserved).
struct WsHeader {
    int64_t n_pairs;      // pairs the emission produced (may exceed capacity)
    int64_t n_invalid;    // Gaussians without support because of bad values
    int64_t n_support;    // in-support (pixel, Gaussian) pairs: sum of box areas
    int32_t overflow;     // n_pairs > capacity
    int32_t ordered;      // 1 once the tile order of this binning is complete
    uint32_t reserved[4];
};


// Host-side workspace layout for one batch shape.
struct Layout {
    int32_t n_img = 0;
    int32_t tile = 16;
    int32_t lds_batch = 256;
    int32_t flags = 0;
    int64_t n_gauss = 0;
    int64_t n_tiles = 0;
    int64_t cap = 0;          // pair capacity
    int32_t nblk_g = 0;       // blocks of per-Gaussian kernels
    int32_t nblk_scan = 0;    // blocks of the tile-count scan
    int32_t nblk_sort = 0;    // radix-sort binning: blocks of a pass at full capacity
    int32_t n_passes = 0;     // radix-sort binning: passes over the tile-id bits
    int32_t nblk_order = 0;   // blocks of the tile-order sort
    double window_r = 0.0;    // > 0: Algorithm 1's r-window support instead of the sigma box
    size_t off_order = 0, off_order_hist = 0, off_counters = 0;
    size_t off_header = 0, off_imgs = 0, off_recs = 0, off_counts = 0, off_offsets = 0,
           off_blocksums = 0, off_tile_cnt = 0, off_loss_parts = 0, off_scan_sums = 0, off_slots = 0, off_lists = 0, off_spare = 0,
           off_ranges = 0, off_moments = 0, off_tile_loss = 0, off_partials = 0,
           off_keys1 = 0, off_hist = 0, off_eparams = 0, total = 0;
    const ImgDev* host_imgs = nullptr;  // host copy of the table (valid during a call)
};

// Device pointers into one workspace.
struct Ws {
    WsHeader* hdr;
    ImgDev* imgs;
    GRec* recs;
    int32_t* counts;
    int32_t* offsets;
    BlockSums* blocksums;
    int32_t* tile_cnt;   // per tile: pairs counted by the emission
    int64_t* scan_sums;  // per scan block: tile-count sums, then their exclusive scan
    uint32_t* slots;     // per emitted pair (emission order): its place in its tile's list
    uint32_t* lists;     // per tile, its Gaussian ids ascending (tile ranges index it)
    uint32_t* spare;     // merge buffer of the longest lists' sort
    // radix-sort binning: ping-pong keys and values (keys[0] is slots; the
    // values of the last pass land in lists, the other buffer is spare)
    uint32_t* keys[2];
    uint32_t* vals[2];
    int32_t* hist;       // per sort block digit counts, then digit totals
    int2* ranges;        // per tile [begin, end) in lists ([0, 0) when empty)
    float* moments;
    double* tile_loss;
    double* loss_parts;  // per workgroup of the loss reduction: its tiles' sum
    float4* partials;    // per emitted pair (emission order): 8 backward sums (2 x float4)
    EParams* eparams;    // GS_FLAG_ELLIPSE: per Gaussian, its exact parameters (else null)
    uint32_t* order;     // tiles, longest list first (persistent kernels)
    int32_t* order_hist; // histograms of the tile-order sort
    uint32_t* counters;  // device counters (kCounterWords, zeroed by the binning)
};

inline Ws bind(const Layout& L, void* base) {
    char* b = static_cast<char*>(base);
    Ws w;
    w.hdr = reinterpret_cast<WsHeader*>(b + L.off_header);
    w.imgs = reinterpret_cast<ImgDev*>(b + L.off_imgs);
    w.recs = reinterpret_cast<GRec*>(b + L.off_recs);
    w.counts = reinterpret_cast<int32_t*>(b + L.off_counts);
    w.offsets = reinterpret_cast<int32_t*>(b + L.off_offsets);
    w.blocksums = reinterpret_cast<BlockSums*>(b + L.off_blocksums);
    w.tile_cnt = reinterpret_cast<int32_t*>(b + L.off_tile_cnt);
    w.scan_sums = reinterpret_cast<int64_t*>(b + L.off_scan_sums);
    w.slots = reinterpret_cast<uint32_t*>(b + L.off_slots);
    w.lists = reinterpret_cast<uint32_t*>(b + L.off_lists);
    w.spare = reinterpret_cast<uint32_t*>(b + L.off_spare);
    w.keys[0] = w.slots;
    w.keys[1] = L.off_keys1 ? reinterpret_cast<uint32_t*>(b + L.off_keys1) : nullptr;
    w.vals[L.n_passes & 1] = w.lists;
    w.vals[(L.n_passes & 1) ^ 1] = w.spare;
    w.hist = L.off_hist ? reinterpret_cast<int32_t*>(b + L.off_hist) : nullptr;
    w.ranges = reinterpret_cast<int2*>(b + L.off_ranges);
    w.moments = reinterpret_cast<float*>(b + L.off_moments);
    w.tile_loss = reinterpret_cast<double*>(b + L.off_tile_loss);
    w.loss_parts = reinterpret_cast<double*>(b + L.off_loss_parts);
    w.partials = reinterpret_cast<float4*>(b + L.off_partials);
    w.eparams = L.off_eparams ? reinterpret_cast<EParams*>(b + L.off_eparams) : nullptr;
    w.order = reinterpret_cast<uint32_t*>(b + L.off_order);
    w.order_hist = reinterpret_cast<int32_t*>(b + L.off_order_hist);
    w.counters = reinterpret_cast<uint32_t*>(b + L.off_counters);
    return w;
}

// Table chunk passed by value to the table-writer kernel.
struct ImgChunk {
    ImgDev img[kSetupChunk];
};

// Image table seen by the tile kernels: by value in the kernel arguments
// (batches of at most kSetupChunk images: read through the scalar cache, no
// dependent global loads) or in the workspace.
struct ArgTable {
    ImgChunk c;
    __device__ __forceinline__ const ImgDev& operator[](int i) const { return c.img[i]; }
};
struct MemTable {
    const ImgDev* p;
    __device__ __forceinline__ const ImgDev& operator[](int i) const { return p[i]; }
};

// ---- launchers (gs_binning.hip) ------------------------------------------
// Support boxes and render records (writes the image table too); with
// `count_only` the block sums are scanned right away so the header holds the
// pair total (no emission follows).
hipError_t launch_support(const Layout& L, const Ws& w, const ImgDev* host_imgs,
                          const float* mean, const float* chol, const float* color,
                          const float* opacity, const float* radius, bool count_only,
                          hipStream_t st);
// Pairs: per-Gaussian offsets, per-tile counts and each pair's place in its
// tile's list (counting atomics).
hipError_t launch_emit(const Layout& L, const Ws& w, hipStream_t st);
// Tile ranges from the counts, the Gaussian ids placed, each list sorted.
hipError_t launch_lists(const Layout& L, const Ws& w, hipStream_t st);
// Tile work order for the persistent kernels: longest list first.
hipError_t launch_order(const Layout& L, const Ws& w, hipStream_t st);

// ---- launchers (gs_render.hip) -------------------------------------------
hipError_t launch_render_fwd(const Layout& L, const Ws& w, float* out, hipStream_t st);
hipError_t launch_render_bwd(const Layout& L, const Ws& w, const float* grad_out,
                             hipStream_t st);
hipError_t launch_render_bwd_l1(const Layout& L, const Ws& w, const float* out,
                                const float* target, int64_t numel, hipStream_t st);
// Forward render, L1 gradient and backward render of each tile in one kernel.
hipError_t launch_render_fused_l1(const Layout& L, const Ws& w, float* out, const float* target,
                                  int64_t numel, hipStream_t st);
hipError_t launch_sum_loss(const Layout& L, const Ws& w, int64_t numel, double* loss,
                           hipStream_t st);
// With loss not NULL, one more workgroup writes the mean of the per-tile L1
// sums (numel output elements) to *loss.
hipError_t launch_finalize(const Layout& L, const Ws& w, const float* chol,
                           const float* color, const float* opacity, float* grad_mean,
                           float* grad_chol, float* grad_color, float* grad_opacity,
                           hipStream_t st, int64_t numel = 0, double* loss = nullptr);
// grad = sign(img - target) / numel; *loss = mean |img - target| (overwritten)
hipError_t launch_l1(const float* img, const float* target, int64_t numel, float* grad,
                     double* loss, hipStream_t st);

// ---- launchers (gs_surrogate.hip) ----------------------------------------
int64_t mlp_grad_waves(int64_t n);
hipError_t launch_mlp_features(const Layout& L, const Ws& w, const float* chol,
                               const float* color, const float* opacity,
                               const gs_mlp_norm& norm, int standardise, float* X,
                               hipStream_t st);
hipError_t launch_mlp_radius(const Layout& L, const Ws& w, const float* params,
                             const float* chol, const float* color, const float* opacity,
                             const gs_mlp_norm& norm, float* out, hipStream_t st);
hipError_t launch_mlp_forward(const float* params, const float* X, int64_t n,
                              const gs_mlp_norm& norm, int radius_mode, float* out,
                              hipStream_t st);
hipError_t launch_mlp_grad(const float* params, const float* X, const float* labels,
                           const float* dout, int64_t n, float q, float* partials,
                           float* grad, double* loss_sum, hipStream_t st);
hipError_t launch_adam(float* p, float* m, float* v, const float* grad, int t, float lr,
                       float b1, float b2, float eps, hipStream_t st);
hipError_t launch_radius_stats(const Layout& L, const Ws& w, float tau, int interior_only,
                               float* R, hipStream_t st);
hipError_t launch_closed_form_radius(const float* chol, const float* color,
                                    const float* opacity, int64_t n, double tau, double margin,
                                    float* R, hipStream_t st);
hipError_t launch_sq_error(const float* a, const float* b, int64_t n, double* sum,
                           hipStream_t st);

// ---- launchers (gs_head.hip) ---------------------------------------------
hipError_t launch_head_fwd(const gs_image* images, int32_t n_img, int32_t grid,
                           const float* raw_opacity, const float* raw_color,
                           const float* raw_sigma, const float* raw_rho, const float* offset,
                           float* mean, float* chol, float* color, float* opacity,
                           hipStream_t st);
hipError_t launch_head_bwd(int64_t n, const float* raw_opacity, const float* raw_color,
                           const float* raw_sigma, const float* raw_rho, const float* g_mean,
                           const float* g_chol, const float* g_color, const float* g_opacity,
                           float* d_opacity, float* d_color, float* d_sigma, float* d_rho,
                           float* d_offset, hipStream_t st);
hipError_t launch_psnr_y(const gs_image* images, int32_t n_img, const float* test,
                         const float* ref, int32_t crop, double* sse, double* psnr,
                         hipStream_t st);

}  // namespace gs
