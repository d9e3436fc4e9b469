// Host side of the C ABI declared in include/gs_raster.h: argument
// validation, workspace layout, kernel sequencing on the caller's stream.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "gs_internal.h"

namespace gs {
namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kMaxPairs = 2147483647LL;
// one workgroup of up to 256 threads per tile: the dispatch's work-item
// count must stay below 2^32
constexpr int64_t kMaxTiles = (int64_t)1 << 24;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

gs_status size_of(int32_t H, int32_t W, double s, int32_t* oh, int32_t* ow) {
    if (H < 1 || W < 1 || !std::isfinite(s) || !(s > 0.0)) return GS_E_INVALID;
    const double h = floor(s * (double)H + 0.5);
    const double w = floor(s * (double)W + 0.5);
    if (!(h >= 1.0) || !(w >= 1.0) || h * w >= 2147483648.0) return GS_E_INVALID;
    *oh = (int32_t)h;
    *ow = (int32_t)w;
    return GS_OK;
}

// Validates the batch description and computes the workspace layout and the
// device image table.
gs_status make_layout(const gs_config* cfg, const gs_image* images, int32_t n_img,
                      int64_t n_gauss, Layout* L, std::vector<ImgDev>* table) {
    if (n_img < 1 || images == nullptr || n_gauss < 0) return GS_E_INVALID;
    if (n_gauss > 2147483647LL) return GS_E_UNSUPPORTED;  // Gaussian ids are 32-bit
    Layout l;
    l.tile = (cfg && cfg->tile) ? cfg->tile : 16;
    if (l.tile != 8 && l.tile != 16 && l.tile != 32) return GS_E_UNSUPPORTED;
    // forward LDS batch: per tile size, the staged Gaussians per round whose
    // per-block record lists fit the LDS next to a useful occupancy
    const int dflt = l.tile == 8 ? 64 : (l.tile == 16 ? 96 : 32);
    l.lds_batch = (cfg && cfg->lds_batch) ? cfg->lds_batch : dflt;
    const bool ok_batch = (l.tile == 8 && (l.lds_batch == 32 || l.lds_batch == 64)) ||
                          (l.tile == 16 && (l.lds_batch == 64 || l.lds_batch == 96 || l.lds_batch == 112 || l.lds_batch == 128 ||
                                            l.lds_batch == 256)) ||
                          (l.tile == 32 && (l.lds_batch == 32 || l.lds_batch == 64));
    if (!ok_batch) return GS_E_UNSUPPORTED;
    l.flags = cfg ? cfg->flags : 0;
    if (l.flags & ~(GS_FLAG_PERSISTENT | GS_FLAG_ATOMIC_GRADS | GS_FLAG_RADIX_SORT |
                    GS_FLAG_PIXEL_CENTER | GS_FLAG_ELLIPSE))
        return GS_E_INVALID;
    l.window_r = cfg ? cfg->window_r : 0.0;
    if (!std::isfinite(l.window_r) || l.window_r < 0.0) return GS_E_INVALID;
    if ((l.flags & GS_FLAG_ELLIPSE) && l.window_r > 0.0) return GS_E_INVALID;
    // the elliptical tile kernels exist at each tile size's default batch only
    if ((l.flags & GS_FLAG_ELLIPSE) && l.lds_batch != dflt) return GS_E_UNSUPPORTED;
    l.n_img = n_img;
    l.n_gauss = n_gauss;

    table->assign(n_img, ImgDev{});
    int64_t tiles = 0, prev_end = 0;
    std::vector<std::pair<int64_t, int64_t>> blocks;
    for (int k = 0; k < n_img; ++k) {
        const gs_image& im = images[k];
        int32_t oh, ow;
        if (size_of(im.lr_h, im.lr_w, im.scale, &oh, &ow) != GS_OK) return GS_E_INVALID;
        if (im.g_begin < 0 || im.g_count < 0 || im.g_begin < prev_end ||
            im.g_begin + im.g_count > n_gauss)
            return GS_E_INVALID;  // Gaussian ranges ascending and disjoint
        prev_end = im.g_begin + im.g_count;
        if (im.out_offset < 0) return GS_E_INVALID;
        blocks.emplace_back(im.out_offset, im.out_offset + 3LL * oh * ow);
        ImgDev& d = (*table)[k];
        d.out_w = ow;
        d.out_h = oh;
        d.tiles_x = (ow + l.tile - 1) / l.tile;
        d.tiles_y = (oh + l.tile - 1) / l.tile;
        d.out_offset = im.out_offset;
        d.g_begin = im.g_begin;
        d.g_count = im.g_count;
        d.tile_base = tiles;
        d.scale = im.scale;
        d.lr_w = im.lr_w;
        d.lr_h = im.lr_h;
        tiles += (int64_t)d.tiles_x * d.tiles_y;
    }
    std::sort(blocks.begin(), blocks.end());
    for (size_t k = 1; k < blocks.size(); ++k)
        if (blocks[k].first < blocks[k - 1].second) return GS_E_INVALID;  // outputs overlap
    if (tiles >= kMaxTiles) return GS_E_UNSUPPORTED;
    l.n_tiles = tiles;

    int64_t cap = (cfg && cfg->pair_capacity) ? cfg->pair_capacity : n_gauss * 16;
    if (cap < 1) cap = 1;
    if (cap > kMaxPairs) return GS_E_UNSUPPORTED;
    l.cap = cap;
    l.nblk_g = (int32_t)std::max<int64_t>(1, (n_gauss + kBlockG - 1) / kBlockG);
    l.nblk_scan = (int32_t)std::max<int64_t>(1, (tiles + kScanTile - 1) / kScanTile);
    if (l.flags & GS_FLAG_RADIX_SORT) {
        int bits = 0;
        while (bits < 32 && ((int64_t)1 << bits) < tiles) ++bits;
        l.n_passes = (bits + kRadixBits - 1) / kRadixBits;
        l.nblk_sort = (int32_t)std::max<int64_t>(1, (cap + kSortTile - 1) / kSortTile);
    }
    l.nblk_order = (int32_t)std::max<int64_t>(1, (tiles + kSortTile - 1) / kSortTile);

    // Capacity-independent sections first, so a small workspace can run the
    // counting kernels of a larger layout.
    size_t off = 0;
    l.off_header = off; off = align_up(off + sizeof(WsHeader));
    l.off_imgs = off; off = align_up(off + sizeof(ImgDev) * (size_t)n_img);
    l.off_recs = off; off = align_up(off + sizeof(GRec) * (size_t)n_gauss);
    l.off_counts = off; off = align_up(off + sizeof(int32_t) * (size_t)n_gauss);
    l.off_offsets = off; off = align_up(off + sizeof(int32_t) * (size_t)n_gauss);
    l.off_blocksums = off; off = align_up(off + sizeof(BlockSums) * (size_t)l.nblk_g);
    l.off_ranges = off; off = align_up(off + sizeof(int2) * (size_t)tiles);
    l.off_tile_cnt = off; off = align_up(off + sizeof(int32_t) * (size_t)tiles);
    l.off_moments = off; off = align_up(off + sizeof(float) * 8 * (size_t)n_gauss);
    if (l.flags & GS_FLAG_ELLIPSE) {
        l.off_eparams = off;
        off = align_up(off + sizeof(EParams) * (size_t)n_gauss);
    }
    l.off_tile_loss = off; off = align_up(off + sizeof(double) * (size_t)tiles);
    l.off_loss_parts = off;
    off = align_up(off + sizeof(double) * (size_t)std::max<int64_t>(
                             kLossParts, (tiles + kLossSlice - 1) / kLossSlice + 1));
    l.off_order = off; off = align_up(off + sizeof(uint32_t) * (size_t)tiles);
    l.off_order_hist = off;
    off = align_up(off + sizeof(int32_t) * ((size_t)kRadix * l.nblk_order + kRadix));
    l.off_counters = off; off = align_up(off + sizeof(uint32_t) * kCounterWords);
    l.off_scan_sums = off; off = align_up(off + sizeof(int64_t) * (size_t)l.nblk_scan);
    l.off_slots = off; off = align_up(off + sizeof(uint32_t) * (size_t)cap);
    l.off_lists = off; off = align_up(off + sizeof(uint32_t) * (size_t)cap);
    l.off_spare = off; off = align_up(off + sizeof(uint32_t) * (size_t)cap);
    if (l.flags & GS_FLAG_RADIX_SORT) {
        l.off_keys1 = off; off = align_up(off + sizeof(uint32_t) * (size_t)cap);
        l.off_hist = off;
        off = align_up(off + sizeof(int32_t) * ((size_t)kRadix * l.nblk_sort + kRadix));
    }
    l.off_partials = off; off = align_up(off + sizeof(float) * 8 * (size_t)cap);
    l.total = off;
    l.host_imgs = table->data();
    *L = l;
    return GS_OK;
}

// Number of output elements (3 per HR pixel) over the whole batch.
int64_t batch_numel(const std::vector<ImgDev>& table) {
    int64_t n = 0;
    for (const ImgDev& d : table) n += 3LL * d.out_w * d.out_h;
    return n;
}

// Bytes of the capacity-independent prefix of a layout.
size_t counting_bytes(const Layout& L) { return L.off_slots; }

gs_status check_gauss_ptrs(int64_t n, const float* a, const float* b, const float* c,
                           const float* d) {
    if (n > 0 && (!a || !b || !c || !d)) return GS_E_INVALID;
    return GS_OK;
}

gs_status dev(hipError_t e) { return e == hipSuccess ? GS_OK : GS_E_DEVICE; }

#define GS_TRY(x)                                 \
    do {                                          \
        const gs_status _s = (x);                 \
        if (_s != GS_OK) return _s;               \
    } while (0)

gs_status run_binning(const Layout& L, const Ws& w, const std::vector<ImgDev>& table,
                      const float* mean, const float* chol, const float* color,
                      const float* opacity, const float* radius, hipStream_t st) {
    if (radius && L.window_r > 0.0) return GS_E_INVALID;  // one support rule at a time
    GS_TRY(dev(launch_support(L, w, table.data(), mean, chol, color, opacity, radius, false,
                              st)));
    GS_TRY(dev(launch_emit(L, w, st)));
    GS_TRY(dev(launch_lists(L, w, st)));
    if (L.flags & GS_FLAG_PERSISTENT) GS_TRY(dev(launch_order(L, w, st)));
    return GS_OK;
}

// Device scratch of gs_raster_step_l1_noalloc: the workspace of one step
// lives here instead of in caller memory.  Each device holds its own copy
// from module load until the process ends.  In host code the array's name is
// only a stand-in; its device address comes from hipGetSymbolAddress, once
// per device, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[GS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on first use).
gs_status scratch_ptr(void** out) {
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess) return GS_E_DEVICE;
    if (d < 0 || d >= kMaxDevices) return GS_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[d]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return GS_E_DEVICE;
        g_scratch_ptr[d] = p;
    }
    *out = g_scratch_ptr[d];
    return GS_OK;
}

__global__ void k_overflow_flag(const WsHeader* h, int32_t* dst) {
    if (threadIdx.x == 0) *dst = h->overflow ? 1 : 0;
}

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" {

int32_t gs_abi_version(void) { return GS_ABI_VERSION; }

const char* gs_status_string(gs_status st) {
    switch (st) {
        case GS_OK: return "ok";
        case GS_E_INVALID: return "invalid argument";
        case GS_E_CAPACITY: return "pair capacity exceeded";
        case GS_E_DEVICE: return "HIP runtime error";
        case GS_E_UNSUPPORTED: return "unsupported configuration";
        case GS_E_WORKSPACE: return "workspace missing or too small";
        default: return "unknown status";
    }
}

gs_status gs_output_size(int32_t H, int32_t W, double s, int32_t* out_h, int32_t* out_w) {
    if (!out_h || !out_w) return GS_E_INVALID;
    return size_of(H, W, s, out_h, out_w);
}

gs_status gs_workspace_size(const gs_config* cfg, const gs_image* images, int32_t n_img,
                            int64_t n_gauss, size_t* bytes) {
    if (!bytes) return GS_E_INVALID;
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    *bytes = L.total;
    return GS_OK;
}

gs_status gs_raster_bin(const gs_config* cfg, const gs_image* images, int32_t n_img,
                        const float* mean, const float* chol, const float* color,
                        const float* opacity, const float* radius, int64_t n_gauss,
                        void* workspace, size_t ws_bytes, void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    GS_TRY(check_gauss_ptrs(n_gauss, mean, chol, color, opacity));
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;
    return run_binning(L, bind(L, workspace), table, mean, chol, color, opacity, radius,
                       static_cast<hipStream_t>(stream));
}

gs_status gs_raster_render(const gs_config* cfg, const gs_image* images, int32_t n_img,
                           int64_t n_gauss, void* workspace, size_t ws_bytes, float* out,
                           void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    if (!out) return GS_E_INVALID;
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;
    return dev(launch_render_fwd(L, bind(L, workspace), out, static_cast<hipStream_t>(stream)));
}

gs_status gs_raster_forward(const gs_config* cfg, const gs_image* images, int32_t n_img,
                            const float* mean, const float* chol, const float* color,
                            const float* opacity, const float* radius, int64_t n_gauss,
                            void* workspace, size_t ws_bytes, float* out, void* stream) {
    if (!out) return GS_E_INVALID;
    GS_TRY(gs_raster_bin(cfg, images, n_img, mean, chol, color, opacity, radius, n_gauss,
                         workspace, ws_bytes, stream));
    return gs_raster_render(cfg, images, n_img, n_gauss, workspace, ws_bytes, out, stream);
}

gs_status gs_raster_render_backward(const gs_config* cfg, const gs_image* images,
                                    int32_t n_img, int64_t n_gauss, void* workspace,
                                    size_t ws_bytes, const float* grad_out, void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    if (!grad_out) return GS_E_INVALID;
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;
    return dev(launch_render_bwd(L, bind(L, workspace), grad_out,
                                 static_cast<hipStream_t>(stream)));
}

gs_status gs_raster_render_backward_l1(const gs_config* cfg, const gs_image* images,
                                       int32_t n_img, int64_t n_gauss, void* workspace,
                                       size_t ws_bytes, const float* out, const float* target,
                                       void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    if (!out || !target) return GS_E_INVALID;
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;
    return dev(launch_render_bwd_l1(L, bind(L, workspace), out, target, batch_numel(table),
                                    static_cast<hipStream_t>(stream)));
}

gs_status gs_raster_render_fused_l1(const gs_config* cfg, const gs_image* images,
                                    int32_t n_img, int64_t n_gauss, void* workspace,
                                    size_t ws_bytes, float* out, const float* target,
                                    void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    if (!out || !target) return GS_E_INVALID;
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;
    return dev(launch_render_fused_l1(L, bind(L, workspace), out, target, batch_numel(table),
                                      static_cast<hipStream_t>(stream)));
}

gs_status gs_raster_step_l1(const gs_config* cfg, const gs_image* images, int32_t n_img,
                            const float* mean, const float* chol, const float* color,
                            const float* opacity, const float* radius, int64_t n_gauss,
                            void* workspace, size_t ws_bytes, float* out, const float* target,
                            float* grad_mean, float* grad_chol, float* grad_color,
                            float* grad_opacity, double* loss, void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    GS_TRY(check_gauss_ptrs(n_gauss, mean, chol, color, opacity));
    if (!out || !target) return GS_E_INVALID;
    if (n_gauss > 0 && (!grad_mean || !grad_chol || !grad_color || !grad_opacity))
        return GS_E_INVALID;
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Ws w = bind(L, workspace);
    GS_TRY(run_binning(L, w, table, mean, chol, color, opacity, radius, st));
    GS_TRY(dev(launch_render_fused_l1(L, w, out, target, batch_numel(table), st)));
    return dev(launch_finalize(L, w, chol, color, opacity, grad_mean, grad_chol, grad_color,
                               grad_opacity, st, batch_numel(table), loss));
}

gs_status gs_raster_step_l1_noalloc(const gs_config* cfg, const gs_image* images,
                                    int32_t n_img, const float* mean, const float* chol,
                                    const float* color, const float* opacity,
                                    const float* radius, int64_t n_gauss, float* out,
                                    const float* target, float* grad_mean, float* grad_chol,
                                    float* grad_color, float* grad_opacity, double* loss,
                                    int32_t* overflow, void* stream) {
    gs_config c = cfg ? *cfg : gs_config{};
    Layout L;
    std::vector<ImgDev> table;
    if (c.pair_capacity == 0) {
        // the largest pair capacity whose layout fits the scratch array
        c.pair_capacity = 1;
        GS_TRY(make_layout(&c, images, n_img, n_gauss, &L, &table));
        const size_t base = L.total;
        c.pair_capacity = 1 << 20;
        GS_TRY(make_layout(&c, images, n_img, n_gauss, &L, &table));
        const size_t per_pair = (L.total - base + ((1 << 20) - 2)) / ((1 << 20) - 1);
        const size_t slack = 16 * 256;  // alignment of the per-pair sections
        if (base + slack + per_pair > GS_NOALLOC_SCRATCH_BYTES) return GS_E_WORKSPACE;
        c.pair_capacity =
            (int64_t)std::min<size_t>((GS_NOALLOC_SCRATCH_BYTES - base - slack) / per_pair,
                                      (size_t)2147483647);
    }
    GS_TRY(make_layout(&c, images, n_img, n_gauss, &L, &table));
    if (L.total > GS_NOALLOC_SCRATCH_BYTES) return GS_E_WORKSPACE;
    void* ws = nullptr;
    GS_TRY(scratch_ptr(&ws));
    GS_TRY(gs_raster_step_l1(&c, images, n_img, mean, chol, color, opacity, radius, n_gauss, ws,
                             GS_NOALLOC_SCRATCH_BYTES, out, target, grad_mean, grad_chol,
                             grad_color, grad_opacity, loss, stream));
    if (overflow) {
        hipLaunchKernelGGL(k_overflow_flag, dim3(1), dim3(64), 0,
                           static_cast<hipStream_t>(stream), bind(L, ws).hdr, overflow);
        return dev(hipGetLastError());
    }
    return GS_OK;
}

gs_status gs_l1_loss_value(const gs_config* cfg, const gs_image* images, int32_t n_img,
                           int64_t n_gauss, const void* workspace, size_t ws_bytes,
                           double* loss, void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    if (!loss) return GS_E_INVALID;
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;
    return dev(launch_sum_loss(L, bind(L, const_cast<void*>(workspace)), batch_numel(table),
                               loss, static_cast<hipStream_t>(stream)));
}

gs_status gs_raster_gradients(const gs_config* cfg, const gs_image* images, int32_t n_img,
                              const float* chol, const float* color, const float* opacity,
                              int64_t n_gauss, void* workspace, size_t ws_bytes,
                              float* grad_mean, float* grad_chol, float* grad_color,
                              float* grad_opacity, void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    if (n_gauss > 0 && (!chol || !color || !opacity || !grad_mean || !grad_chol ||
                        !grad_color || !grad_opacity))
        return GS_E_INVALID;
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;
    return dev(launch_finalize(L, bind(L, workspace), chol, color, opacity, grad_mean,
                               grad_chol, grad_color, grad_opacity,
                               static_cast<hipStream_t>(stream)));
}

gs_status gs_raster_backward(const gs_config* cfg, const gs_image* images, int32_t n_img,
                             const float* mean, const float* chol, const float* color,
                             const float* opacity, const float* radius, int64_t n_gauss,
                             void* workspace, size_t ws_bytes, const float* grad_out,
                             float* grad_mean, float* grad_chol, float* grad_color,
                             float* grad_opacity, void* stream) {
    (void)radius;
    GS_TRY(check_gauss_ptrs(n_gauss, mean, chol, color, opacity));
    GS_TRY(gs_raster_render_backward(cfg, images, n_img, n_gauss, workspace, ws_bytes,
                                     grad_out, stream));
    return gs_raster_gradients(cfg, images, n_img, chol, color, opacity, n_gauss, workspace,
                               ws_bytes, grad_mean, grad_chol, grad_color, grad_opacity,
                               stream);
}

gs_status gs_raster_backward_l1(const gs_config* cfg, const gs_image* images, int32_t n_img,
                                const float* chol, const float* color, const float* opacity,
                                int64_t n_gauss, void* workspace, size_t ws_bytes,
                                const float* out, const float* target, float* grad_mean,
                                float* grad_chol, float* grad_color, float* grad_opacity,
                                double* loss, void* stream) {
    GS_TRY(gs_raster_render_backward_l1(cfg, images, n_img, n_gauss, workspace, ws_bytes, out,
                                        target, stream));
    GS_TRY(gs_raster_gradients(cfg, images, n_img, chol, color, opacity, n_gauss, workspace,
                               ws_bytes, grad_mean, grad_chol, grad_color, grad_opacity,
                               stream));
    if (loss)
        GS_TRY(gs_l1_loss_value(cfg, images, n_img, n_gauss, workspace, ws_bytes, loss, stream));
    return GS_OK;
}

gs_status gs_l1_loss_grad(const float* img, const float* target, int64_t numel,
                          float* grad, double* loss, void* stream) {
    if (numel < 0 || !loss) return GS_E_INVALID;
    if (numel > 0 && (!img || !target || !grad)) return GS_E_INVALID;
    return dev(launch_l1(img, target, numel, grad, loss, static_cast<hipStream_t>(stream)));
}

gs_status gs_diagnostics(const gs_config* cfg, const gs_image* images, int32_t n_img,
                         int64_t n_gauss, const void* workspace, size_t ws_bytes,
                         int64_t* n_pairs, int32_t* overflow, int64_t* n_invalid,
                         int64_t* n_support, void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    if (!workspace || ws_bytes < counting_bytes(L)) return GS_E_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    WsHeader h;
    GS_TRY(dev(hipMemcpyAsync(&h, static_cast<const char*>(workspace) + L.off_header,
                              sizeof h, hipMemcpyDeviceToHost, st)));
    GS_TRY(dev(hipStreamSynchronize(st)));
    if (n_pairs) *n_pairs = h.n_pairs;
    if (overflow) *overflow = h.overflow;
    if (n_invalid) *n_invalid = h.n_invalid;
    if (n_support) *n_support = h.n_support;
    return h.overflow ? GS_E_CAPACITY : GS_OK;
}

gs_status gs_count_pairs(const gs_config* cfg, const gs_image* images, int32_t n_img,
                         const float* mean, const float* chol, const float* radius,
                         int64_t n_gauss, void* workspace, size_t ws_bytes,
                         int64_t* n_pairs, void* stream) {
    if (!n_pairs) return GS_E_INVALID;
    Layout L;
    std::vector<ImgDev> table;
    gs_config c = cfg ? *cfg : gs_config{};
    c.pair_capacity = 1;
    GS_TRY(make_layout(&c, images, n_img, n_gauss, &L, &table));
    if (n_gauss > 0 && (!mean || !chol)) return GS_E_INVALID;
    if (radius && L.window_r > 0.0) return GS_E_INVALID;
    if (!workspace || ws_bytes < counting_bytes(L)) return GS_E_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Ws w = bind(L, workspace);
    // colour and opacity do not change the box: passed as NULL, the support
    // kernel leaves the record's amplitudes at zero.  Only the counting
    // kernels run, so nothing past the capacity-independent prefix is touched.
    GS_TRY(dev(launch_support(L, w, table.data(), mean, chol, nullptr, nullptr, radius, true,
                              st)));
    WsHeader h;
    GS_TRY(dev(hipMemcpyAsync(&h, static_cast<char*>(workspace) + L.off_header, sizeof h,
                              hipMemcpyDeviceToHost, st)));
    GS_TRY(dev(hipStreamSynchronize(st)));
    *n_pairs = h.n_pairs;
    return GS_OK;
}

gs_status gs_mlp_features(const gs_image* images, int32_t n_img, const float* chol,
                          const float* color, const float* opacity, int64_t n_gauss,
                          const gs_mlp_norm* norm, float* feats, void* stream) {
    if (n_gauss > 0 && (!chol || !color || !opacity || !feats)) return GS_E_INVALID;
    gs_mlp_norm nm{};
    if (norm) {
        nm = *norm;
        for (int k = 0; k < 8; ++k)
            if (!(nm.sd[k] > 0.f) || !std::isfinite(nm.mu[k])) return GS_E_INVALID;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    // one launch per chunk of images (the chunk's table travels by value)
    for (int first = 0; first < n_img; first += kSetupChunk) {
        const int count = std::min(kSetupChunk, n_img - first);
        std::vector<gs_image> sub(images + first, images + first + count);
        const int64_t g0 = sub.front().g_begin;
        const int64_t g1 = sub.back().g_begin + sub.back().g_count;
        for (auto& im : sub) { im.g_begin -= g0; im.out_offset = 0; }
        // out_offset is irrelevant here; make the blocks disjoint for validation
        int64_t off = 0;
        for (auto& im : sub) {
            int32_t oh, ow;
            GS_TRY(size_of(im.lr_h, im.lr_w, im.scale, &oh, &ow));
            im.out_offset = off;
            off += 3LL * oh * ow;
        }
        Layout L;
        std::vector<ImgDev> table;
        GS_TRY(make_layout(nullptr, sub.data(), count, g1 - g0, &L, &table));
        Ws w{};
        GS_TRY(dev(launch_mlp_features(L, w, chol + 3 * g0, color + 3 * g0, opacity + g0, nm,
                                       norm ? 1 : 0, feats + 8 * g0, st)));
    }
    return GS_OK;
}

gs_status gs_mlp_radius(const gs_image* images, int32_t n_img, const float* params,
                        const float* chol, const float* color, const float* opacity,
                        int64_t n_gauss, const gs_mlp_norm* norm, float* radius, void* stream) {
    if (!norm) return GS_E_INVALID;
    if (n_gauss > 0 && (!params || !chol || !color || !opacity || !radius)) return GS_E_INVALID;
    const gs_mlp_norm nm = *norm;
    for (int k = 0; k < 8; ++k)
        if (!(nm.sd[k] > 0.f) || !std::isfinite(nm.mu[k])) return GS_E_INVALID;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // one launch per chunk of images (the chunk's table travels by value)
    for (int first = 0; first < n_img; first += kSetupChunk) {
        const int count = std::min(kSetupChunk, n_img - first);
        std::vector<gs_image> sub(images + first, images + first + count);
        const int64_t g0 = sub.front().g_begin;
        const int64_t g1 = sub.back().g_begin + sub.back().g_count;
        int64_t off = 0;
        for (auto& im : sub) {
            im.g_begin -= g0;
            int32_t oh, ow;
            GS_TRY(size_of(im.lr_h, im.lr_w, im.scale, &oh, &ow));
            im.out_offset = off;  // irrelevant here; disjoint blocks for validation
            off += 3LL * oh * ow;
        }
        Layout L;
        std::vector<ImgDev> table;
        GS_TRY(make_layout(nullptr, sub.data(), count, g1 - g0, &L, &table));
        Ws w{};
        GS_TRY(dev(launch_mlp_radius(L, w, params, chol + 3 * g0, color + 3 * g0, opacity + g0,
                                     nm, radius + g0, st)));
    }
    return GS_OK;
}

gs_status gs_mlp_forward(const float* params, const float* feats, int64_t n,
                         const gs_mlp_norm* norm, float* out, void* stream) {
    if (n < 0) return GS_E_INVALID;
    if (n > 0 && (!params || !feats || !out)) return GS_E_INVALID;
    gs_mlp_norm nm{};
    if (norm) nm = *norm;
    return dev(launch_mlp_forward(params, feats, n, nm, norm ? 1 : 0, out,
                                  static_cast<hipStream_t>(stream)));
}

gs_status gs_mlp_workspace_size(int64_t n, size_t* bytes) {
    if (!bytes || n < 0) return GS_E_INVALID;
    *bytes = sizeof(float) * (size_t)kMlpParams * (size_t)mlp_grad_waves(n);
    return GS_OK;
}

gs_status gs_mlp_grad(const float* params, const float* feats, const float* labels,
                      const float* dout, int64_t n, float quantile, void* workspace,
                      size_t ws_bytes, float* grad, double* loss_sum, void* stream) {
    if (n < 1 || !params || !feats || !grad || (!labels && !dout)) return GS_E_INVALID;
    if (labels && !(quantile > 0.f && quantile < 1.f)) return GS_E_INVALID;
    size_t need = 0;
    GS_TRY(gs_mlp_workspace_size(n, &need));
    if (!workspace || ws_bytes < need) return GS_E_WORKSPACE;
    return dev(launch_mlp_grad(params, feats, labels, dout, n, quantile,
                               static_cast<float*>(workspace), grad, labels ? loss_sum : nullptr,
                               static_cast<hipStream_t>(stream)));
}

gs_status gs_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                      float lr, void* stream) {
    if (!params || !m || !v || !grad || step < 1 || !(lr > 0.f)) return GS_E_INVALID;
    return dev(launch_adam(params, m, v, grad, step, lr, 0.9f, 0.999f, 1e-8f,
                           static_cast<hipStream_t>(stream)));
}

gs_status gs_radius_stats(const gs_config* cfg, const gs_image* images, int32_t n_img,
                          int64_t n_gauss, const void* workspace, size_t ws_bytes, float tau,
                          int32_t interior_only, float* radius, void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    if (n_gauss > 0 && !radius) return GS_E_INVALID;
    if (!(tau > 0.f)) return GS_E_INVALID;
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;
    return dev(launch_radius_stats(L, bind(L, const_cast<void*>(workspace)), tau,
                                   interior_only ? 1 : 0, radius,
                                   static_cast<hipStream_t>(stream)));
}

gs_status gs_closed_form_radius(const float* chol, const float* color, const float* opacity,
                                int64_t n_gauss, double tau, double margin, float* radius,
                                void* stream) {
    if (n_gauss < 0 || !(tau > 0.0) || !std::isfinite(tau) || !std::isfinite(margin))
        return GS_E_INVALID;
    if (n_gauss > 0 && (!chol || !color || !opacity || !radius)) return GS_E_INVALID;
    return dev(launch_closed_form_radius(chol, color, opacity, n_gauss, tau, margin, radius,
                                         static_cast<hipStream_t>(stream)));
}

gs_status gs_sq_error(const float* a, const float* b, int64_t n, double* sum, void* stream) {
    if (n < 0 || (n > 0 && (!a || !b || !sum))) return GS_E_INVALID;
    return dev(launch_sq_error(a, b, n, sum, static_cast<hipStream_t>(stream)));
}

gs_status gs_gaussian_head_forward(const gs_image* images, int32_t n_img, int32_t grid,
                                   const float* raw_opacity, const float* raw_color,
                                   const float* raw_sigma, const float* raw_rho,
                                   const float* offset, int64_t n_gauss, float* mean,
                                   float* chol, float* color, float* opacity, void* stream) {
    if (n_img < 1 || !images || grid < 1 || n_gauss < 0) return GS_E_INVALID;
    int64_t prev_end = 0;
    for (int k = 0; k < n_img; ++k) {
        const gs_image& im = images[k];
        if (im.lr_h < 1 || im.lr_w < 1) return GS_E_INVALID;
        // grid coordinates stay exact in FP32
        if ((int64_t)grid * std::max(im.lr_h, im.lr_w) >= (1 << 23)) return GS_E_UNSUPPORTED;
        if (im.g_count != (int64_t)grid * grid * im.lr_h * im.lr_w) return GS_E_INVALID;
        if (im.g_begin < prev_end || im.g_begin + im.g_count > n_gauss) return GS_E_INVALID;
        prev_end = im.g_begin + im.g_count;
    }
    if (n_gauss > 0 && (!raw_opacity || !raw_color || !raw_sigma || !raw_rho || !offset ||
                        !mean || !chol || !color || !opacity))
        return GS_E_INVALID;
    return dev(launch_head_fwd(images, n_img, grid, raw_opacity, raw_color, raw_sigma, raw_rho,
                               offset, mean, chol, color, opacity,
                               static_cast<hipStream_t>(stream)));
}

gs_status gs_gaussian_head_backward(int64_t n_gauss, const float* raw_opacity,
                                    const float* raw_color, const float* raw_sigma,
                                    const float* raw_rho, const float* grad_mean,
                                    const float* grad_chol, const float* grad_color,
                                    const float* grad_opacity, float* d_opacity,
                                    float* d_color, float* d_sigma, float* d_rho,
                                    float* d_offset, void* stream) {
    if (n_gauss < 0) return GS_E_INVALID;
    if (n_gauss > 0 && (!raw_opacity || !raw_color || !raw_sigma || !raw_rho || !grad_mean ||
                        !grad_chol || !grad_color || !grad_opacity || !d_opacity ||
                        !d_color || !d_sigma || !d_rho || !d_offset))
        return GS_E_INVALID;
    return dev(launch_head_bwd(n_gauss, raw_opacity, raw_color, raw_sigma, raw_rho, grad_mean,
                               grad_chol, grad_color, grad_opacity, d_opacity, d_color, d_sigma,
                               d_rho, d_offset, static_cast<hipStream_t>(stream)));
}

gs_status gs_psnr_y(const gs_image* images, int32_t n_img, const float* test, const float* ref,
                    int32_t crop, double* sse, double* psnr, void* stream) {
    if (n_img < 1 || !images || crop < 0 || !test || !ref || !sse || !psnr)
        return GS_E_INVALID;
    std::vector<std::pair<int64_t, int64_t>> blocks;
    for (int k = 0; k < n_img; ++k) {
        int32_t oh, ow;
        GS_TRY(size_of(images[k].lr_h, images[k].lr_w, images[k].scale, &oh, &ow));
        if (images[k].out_offset < 0) return GS_E_INVALID;
        blocks.emplace_back(images[k].out_offset, images[k].out_offset + 3LL * oh * ow);
    }
    std::sort(blocks.begin(), blocks.end());
    for (size_t k = 1; k < blocks.size(); ++k)
        if (blocks[k].first < blocks[k - 1].second) return GS_E_INVALID;
    return dev(launch_psnr_y(images, n_img, test, ref, crop, sse, psnr,
                             static_cast<hipStream_t>(stream)));
}

struct gs_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

gs_status gs_graph_create(const gs_config* cfg, const gs_image* images, int32_t n_img,
                          const float* mean, const float* chol, const float* color,
                          const float* opacity, const float* radius, int64_t n_gauss,
                          void* workspace, size_t ws_bytes, float* out, const float* target,
                          float* grad_mean, float* grad_chol, float* grad_color,
                          float* grad_opacity, double* loss, gs_graph* graph_out) {
    if (!graph_out) return GS_E_INVALID;
    *graph_out = nullptr;
    // validate everything before capturing (a failed call inside a capture
    // would leave the capture half-built)
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    GS_TRY(check_gauss_ptrs(n_gauss, mean, chol, color, opacity));
    if (!out || (radius && L.window_r > 0.0)) return GS_E_INVALID;
    if (target && n_gauss > 0 && (!grad_mean || !grad_chol || !grad_color || !grad_opacity))
        return GS_E_INVALID;
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;

    hipStream_t cs;
    GS_TRY(dev(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)));
    gs_status st = GS_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return GS_E_DEVICE;
    }
    if (target)
        st = gs_raster_step_l1(cfg, images, n_img, mean, chol, color, opacity, radius, n_gauss,
                               workspace, ws_bytes, out, target, grad_mean, grad_chol,
                               grad_color, grad_opacity, loss, cs);
    else
        st = gs_raster_forward(cfg, images, n_img, mean, chol, color, opacity, radius,
                               n_gauss, workspace, ws_bytes, out, cs);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (st != GS_OK || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return st != GS_OK ? st : GS_E_DEVICE;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return GS_E_DEVICE;
    }
    gs_graph h = new (std::nothrow) gs_graph_s;
    if (!h) {
        (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(g);
        return GS_E_DEVICE;
    }
    h->graph = g;
    h->exec = ex;
    *graph_out = h;
    return GS_OK;
}

gs_status gs_graph_launch(gs_graph graph, void* stream) {
    if (!graph || !graph->exec) return GS_E_INVALID;
    return dev(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
}

gs_status gs_graph_destroy(gs_graph graph) {
    if (!graph) return GS_OK;
    hipError_t e1 = hipSuccess, e2 = hipSuccess;
    if (graph->exec) e1 = hipGraphExecDestroy(graph->exec);
    if (graph->graph) e2 = hipGraphDestroy(graph->graph);
    delete graph;
    return (e1 == hipSuccess && e2 == hipSuccess) ? GS_OK : GS_E_DEVICE;
}

gs_status gs_tile_lists(const gs_config* cfg, const gs_image* images, int32_t n_img,
                        int64_t n_gauss, const void* workspace, size_t ws_bytes,
                        int32_t* ranges_host, int32_t* gids_host, int64_t max_pairs,
                        int64_t* n_tiles_out, int64_t* n_pairs_out, void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char* b = static_cast<const char*>(workspace);
    WsHeader h;
    GS_TRY(dev(hipMemcpyAsync(&h, b + L.off_header, sizeof h, hipMemcpyDeviceToHost, st)));
    GS_TRY(dev(hipStreamSynchronize(st)));
    if (n_tiles_out) *n_tiles_out = L.n_tiles;
    if (n_pairs_out) *n_pairs_out = h.n_pairs;
    if (h.overflow) return GS_E_CAPACITY;
    if (ranges_host)
        GS_TRY(dev(hipMemcpyAsync(ranges_host, b + L.off_ranges, sizeof(int2) * L.n_tiles,
                                  hipMemcpyDeviceToHost, st)));
    if (gids_host) {
        if (max_pairs < h.n_pairs) return GS_E_INVALID;
        GS_TRY(dev(hipMemcpyAsync(gids_host, b + L.off_lists, sizeof(uint32_t) * h.n_pairs,
                                  hipMemcpyDeviceToHost, st)));
    }
    return dev(hipStreamSynchronize(st));
}

gs_status gs_tile_order(const gs_config* cfg, const gs_image* images, int32_t n_img,
                        int64_t n_gauss, const void* workspace, size_t ws_bytes,
                        uint32_t* order_host, int64_t max_tiles, int32_t* ordered,
                        void* stream) {
    Layout L;
    std::vector<ImgDev> table;
    GS_TRY(make_layout(cfg, images, n_img, n_gauss, &L, &table));
    if (!workspace || ws_bytes < L.total) return GS_E_WORKSPACE;
    if (order_host && max_tiles < L.n_tiles) return GS_E_INVALID;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char* b = static_cast<const char*>(workspace);
    WsHeader h;
    GS_TRY(dev(hipMemcpyAsync(&h, b + L.off_header, sizeof h, hipMemcpyDeviceToHost, st)));
    if (order_host)
        GS_TRY(dev(hipMemcpyAsync(order_host, b + L.off_order, sizeof(uint32_t) * L.n_tiles,
                                  hipMemcpyDeviceToHost, st)));
    GS_TRY(dev(hipStreamSynchronize(st)));
    if (ordered) *ordered = h.ordered;
    return GS_OK;
}

}  // extern "C"
