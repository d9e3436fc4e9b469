/*
 * gs_raster.h -- C ABI of the MI355X (gfx950) scale-aware, differentiable 2D
 * Gaussian rasterizer of GSASR (arXiv 2501.06838, Sec. 3.1, Eq. 1-4,
 * Algorithm 1).
 *
 * The library renders, for each image of a batch, the super-resolved image
 *     I_SR(x, y; s) = sum_i alpha_i c_i f_i(x/s, y/s)            (Eq. 1, 2, 4)
 * on the HR grid x in [0, out_w-1], y in [0, out_h-1], where f_i is the
 * bivariate normal density of Eq. 2 and each Gaussian only touches the HR
 * pixels inside its support box (Algorithm 1's strict window test, with the
 * half-window equal to R standard deviations per axis; R = 3 on the exact
 * path):
 *     { x : s (mu_x - R sigma_x) < x < s (mu_x + R sigma_x) } x (same for y).
 * It also returns the gradients of a loss w.r.t. every Gaussian property
 * (the paper's renderer is differentiable, Sec. 3.1 "Fast Rasterization").
 *
 * Conventions shared by every entry point
 *   - Units: mu and the covariance are in LR pixels, LR pixel centres at
 *     integer coordinates (Eq. 3 samples integer x in [0, W-1]).  HR pixel
 *     (x, y) samples the Gaussians at (x/s, y/s) (Eq. 4).
 *   - HR size: out_h = floor(s H + 0.5), out_w = floor(s W + 0.5) in FP64
 *     (Algorithm 1 allocates an sH x sW image; a non-integer product is
 *     rounded half up).
 *   - Covariance: Cholesky factor L = [[l11, 0], [l21, l22]] of Sigma, i.e.
 *     sigma_x = l11, sigma_y = sqrt(l21^2 + l22^2), rho = l21 / sigma_y
 *     (Sec. 3.1's sigma_x, sigma_y, rho).  l11 > 0 and l22 > 0; a Gaussian
 *     violating that, or holding a non-finite value, has no support: it adds
 *     nothing, gets zero gradients, and is counted (gs_diagnostics).
 *   - Memory: every array argument named "device" is device memory owned by
 *     the caller, FP32, C-contiguous.  gs_image arrays are host memory.  The
 *     library allocates nothing on the device and keeps no global state:
 *     calls on different streams with different workspaces may run
 *     concurrently.  (The one exception is gs_raster_step_l1_noalloc, whose
 *     workspace is a library-owned device array shared by its calls.)
 *   - Streams: stream is a hipStream_t passed as void* (NULL = default
 *     stream).  Every device entry point only enqueues work on it and returns
 *     without synchronising, unless marked "synchronising".
 *   - Errors: arguments that can be checked on the host make the call return
 *     an error with nothing enqueued.  Data-dependent problems never fault:
 *     pair-list overflow is flagged in the workspace (see gs_diagnostics).
 */
#ifndef GS_RASTER_H
#define GS_RASTER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_ABI_VERSION 3

typedef int32_t gs_status;
enum {
    GS_OK = 0,
    GS_E_INVALID = -1,     /* bad argument (host-checked), nothing enqueued  */
    GS_E_CAPACITY = -2,    /* (tile, Gaussian) pairs exceeded pair_capacity  */
    GS_E_DEVICE = -3,      /* a HIP runtime call failed                       */
    GS_E_UNSUPPORTED = -4, /* valid but unsupported configuration             */
    GS_E_WORKSPACE = -5    /* workspace missing or smaller than required      */
};

/* One image of a batch (host memory).  Its Gaussians are entries
 * [g_begin, g_begin + g_count) of the packed Gaussian arrays; its output is
 * the planar block [3][out_h][out_w] starting at element out_offset of the
 * output (and of the upstream gradient).  Images may not overlap in either. */
typedef struct {
    int32_t lr_h, lr_w;   /* H, W >= 1                                       */
    double scale;         /* s: finite, > 0                                  */
    int64_t g_begin;      /* first Gaussian of this image                    */
    int64_t g_count;      /* number of Gaussians (may be 0)                  */
    int64_t out_offset;   /* element offset of the [3][out_h][out_w] block   */
} gs_image;

/* Launch configuration.  Zero fields take defaults. */
typedef struct {
    int32_t tile;          /* square HR tile side: 8, 16 (default) or 32     */
    int32_t lds_batch;     /* Gaussians the tile kernels stage in LDS per
                              round: tile 8: 32 or 64 (default 64); tile 16:
                              64, 96 (default), 112, 128 or 256; tile 32: 32
                              (default) or 64.  Neither the image nor the
                              gradients depend on it.                        */
    int32_t flags;         /* GS_FLAG_* (other bits: GS_E_INVALID)           */
    int32_t reserved;
    int64_t pair_capacity; /* max (tile, Gaussian) pairs the workspace holds;
                              0 = n_gauss * 16 (use gs_count_pairs to size)  */
    double window_r;       /* 0: each Gaussian's support is the box of R
                              standard deviations (R = 3, or the radius
                              array of the pruned path).  > 0: Algorithm 1's
                              own window with rasterization ratio r
                              (Sec. 3.1 "Fast Rasterization"): the strict
                              test |x - s mu_x| < r s W, |y - s mu_y| < r s H
                              in HR pixels, each axis with its own extent,
                              the same for every Gaussian of an image; the
                              radius array must then be NULL.  Negative or
                              non-finite: GS_E_INVALID.                      */
} gs_config;

/* flags */
#define GS_FLAG_PERSISTENT 0x1   /* tile kernels run persistent: a grid of as
                                    many workgroups as fit on the device walks
                                    the tiles longest list first (the binning
                                    builds that order) in a fixed snake
                                    schedule.  Results are bitwise those of
                                    the default one-workgroup-per-tile launch.*/
#define GS_FLAG_ATOMIC_GRADS 0x2 /* backward: one FP32 global atomic per (tile,
                                    Gaussian, sum) instead of per-pair partial
                                    sums reduced in a fixed order (default)    */
#define GS_FLAG_RADIX_SORT 0x4   /* binning: emit every (tile id, Gaussian id)
                                    pair and sort them with the device LSD
                                    radix sort (8-bit digits over the tile-id
                                    bits) instead of counting each pair into
                                    its tile and sorting every tile's list
                                    (default).  Same lists, bitwise.           */
#define GS_FLAG_PIXEL_CENTER 0x8 /* alternative reading of Eq. 4: HR pixel x
                                    samples the LR coordinate (x + 1/2)/s - 1/2
                                    (pixel centres of both grids aligned)
                                    instead of x/s; boxes and windows move with
                                    it (HR centre s (mu + 1/2) - 1/2).          */
#define GS_FLAG_ELLIPSE 0x10     /* alternative reading of the truncation: a
                                    pixel of the box is in the support only if
                                    its Mahalanobis distance d (d^2 = z1^2 +
                                    z2^2, z1 = (u - mu_x)/l11, z2 = ((v - mu_y)
                                    - l21 z1)/l22, evaluated in FP64 in that
                                    order) is below R; tile lists still follow
                                    the box.  Not with window_r > 0
                                    (GS_E_INVALID); lds_batch must be 0 or
                                    the tile size's default
                                    (GS_E_UNSUPPORTED).                        */

/* ABI version of the loaded library (GS_ABI_VERSION). */
int32_t gs_abi_version(void);

/* Short English text for a status code (static storage). */
const char* gs_status_string(gs_status st);

/* HR size of one image: out_h = floor(s H + 0.5), out_w = floor(s W + 0.5)
 * (Algorithm 1's sH x sW image).  GS_E_INVALID if H, W < 1, s not finite or
 * <= 0, or out_h * out_w >= 2^31. */
gs_status gs_output_size(int32_t H, int32_t W, double s, int32_t* out_h, int32_t* out_w);

/* Bytes of device workspace needed by gs_raster_forward / backward for this
 * batch layout (cfg may be NULL for defaults).  The workspace holds the
 * per-Gaussian render records, the per-tile lists of Gaussian ids and their
 * ranges, and the backward's per-pair sums; it is written by the forward and
 * read by the matching backward, so it must persist between the two.
 * GS_E_UNSUPPORTED if the batch has 2^24 tiles or more. */
gs_status gs_workspace_size(const gs_config* cfg, const gs_image* images, int32_t n_img,
                            int64_t n_gauss, size_t* bytes);

/* Forward render (Eq. 4 with Algorithm 1's truncated support) of a batch.
 *   mean    device [n_gauss][2]  (mu_x, mu_y)
 *   chol    device [n_gauss][3]  (l11, l21, l22)
 *   color   device [n_gauss][3]  peak RGB c (not clamped)
 *   opacity device [n_gauss]     alpha (not clamped)
 *   radius  device [n_gauss] support half-widths R_i in standard deviations
 *           (the pruned path), or NULL for R = 3 everywhere (exact path)
 *   out     device, each image's [3][out_h][out_w] block at its out_offset;
 *           every pixel of every block is written (background 0).
 * Kernels: per-Gaussian support box and tile count, prefix sum, pair
 * emission (each pair counted into its tile), per-tile ranges (prefix sum of
 * the tile counts), the Gaussian ids placed into the tiles' lists and each
 * list sorted ascending, and the per-tile render.  Within a tile, Gaussians
 * are summed in ascending index, so the result is bitwise deterministic for a given configuration. */
gs_status gs_raster_forward(const gs_config* cfg, const gs_image* images, int32_t n_img,
                            const float* mean, const float* chol, const float* color,
                            const float* opacity, const float* radius, int64_t n_gauss,
                            void* workspace, size_t ws_bytes, float* out, void* stream);

/* First stage of gs_raster_forward: support boxes, tile counts, prefix sum,
 * pair emission, per-tile ranges and the sorted per-tile lists, all into the
 * workspace.
 * Arguments as for gs_raster_forward. */
gs_status gs_raster_bin(const gs_config* cfg, const gs_image* images, int32_t n_img,
                        const float* mean, const float* chol, const float* color,
                        const float* opacity, const float* radius, int64_t n_gauss,
                        void* workspace, size_t ws_bytes, void* stream);

/* Second stage of gs_raster_forward: the per-tile render (one kernel) from
 * the workspace left by gs_raster_bin into out (layout as for
 * gs_raster_forward). */
gs_status gs_raster_render(const gs_config* cfg, const gs_image* images, int32_t n_img,
                           int64_t n_gauss, void* workspace, size_t ws_bytes, float* out,
                           void* stream);

/* Backward of gs_raster_forward for upstream gradient grad_out = dL/dI
 * (device, same layout as out).  Uses the workspace left by the forward of
 * the same inputs.  Writes (overwrites) dL/d(mean) [n][2], dL/d(chol) [n][3],
 * dL/d(color) [n][3] and dL/d(opacity) [n] (all device).  The support box is
 * held fixed (its derivative is zero almost everywhere).  Each tile reduces
 * its (tile, Gaussian) sums in registers and LDS and stores them per pair;
 * the gradient stage adds a Gaussian's pairs in a fixed order, so the result
 * is bitwise deterministic (with GS_FLAG_ATOMIC_GRADS the tiles add into
 * per-Gaussian FP32 accumulators with global atomics instead: not bitwise
 * deterministic). */
gs_status gs_raster_backward(const gs_config* cfg, const gs_image* images, int32_t n_img,
                             const float* mean, const float* chol, const float* color,
                             const float* opacity, const float* radius, int64_t n_gauss,
                             void* workspace, size_t ws_bytes, const float* grad_out,
                             float* grad_mean, float* grad_chol, float* grad_color,
                             float* grad_opacity, void* stream);

/* First stage of gs_raster_backward: the per-tile backward render (one
 * kernel).  Stores, per (tile, Gaussian) pair, the eight sums the gradients
 * are made of in the workspace (with GS_FLAG_ATOMIC_GRADS: adds them into
 * per-Gaussian accumulators, which start at zero after a forward and after
 * every gs_raster_gradients).  grad_out: device, layout of out. */
gs_status gs_raster_render_backward(const gs_config* cfg, const gs_image* images,
                                    int32_t n_img, int64_t n_gauss, void* workspace,
                                    size_t ws_bytes, const float* grad_out, void* stream);

/* Second stage of gs_raster_backward: per Gaussian, turns the accumulated
 * sums into dL/d(mean, chol, color, opacity) (overwritten) and clears them. */
gs_status gs_raster_gradients(const gs_config* cfg, const gs_image* images, int32_t n_img,
                              const float* chol, const float* color, const float* opacity,
                              int64_t n_gauss, void* workspace, size_t ws_bytes,
                              float* grad_mean, float* grad_chol, float* grad_color,
                              float* grad_opacity, void* stream);

/* Backward render fused with the L1 training loss (Sec. 3.2, "Rendering"):
 * the upstream gradient sign(out - target) / numel (numel = all output
 * elements of the batch, sign(0) = 0) is formed per tile from the rendered
 * image `out` of the matching forward and `target` (device, layout of out)
 * and never stored; each tile's sum |out - target| is kept in the workspace
 * for gs_l1_loss_value.  Otherwise as gs_raster_render_backward. */
gs_status gs_raster_render_backward_l1(const gs_config* cfg, const gs_image* images,
                                       int32_t n_img, int64_t n_gauss, void* workspace,
                                       size_t ws_bytes, const float* out, const float* target,
                                       void* stream);

/* gs_raster_render followed by gs_raster_render_backward_l1, in one kernel:
 * per tile, the image is summed, stored to out, turned into the L1 gradient
 * sign(out - target) / numel against target (with the tile's share of the
 * loss) and fed to the backward render over the same staged Gaussians.  The
 * workspace must hold a gs_raster_bin of the same batch.  Results are those
 * of the two separate calls (the image bitwise). */
gs_status gs_raster_render_fused_l1(const gs_config* cfg, const gs_image* images,
                                    int32_t n_img, int64_t n_gauss, void* workspace,
                                    size_t ws_bytes, float* out, const float* target,
                                    void* stream);

/* One whole training step of the L1 loss (Sec. 3.2, "Rendering"):
 * gs_raster_bin, gs_raster_render_fused_l1, gs_raster_gradients and, when
 * loss is not NULL, gs_l1_loss_value.  Arguments as for those calls. */
gs_status gs_raster_step_l1(const gs_config* cfg, const gs_image* images, int32_t n_img,
                            const float* mean, const float* chol, const float* color,
                            const float* opacity, const float* radius, int64_t n_gauss,
                            void* workspace, size_t ws_bytes, float* out, const float* target,
                            float* grad_mean, float* grad_chol, float* grad_color,
                            float* grad_opacity, double* loss, void* stream);

/* Bytes of the device scratch array behind gs_raster_step_l1_noalloc. */
#define GS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* gs_raster_step_l1 without a caller workspace and without any device
 * allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * workspace is a library-owned device array of GS_NOALLOC_SCRATCH_BYTES
 * (64 MiB), one per device, held from library load until the process ends;
 * the call runs on the current device, which must be the stream's.
 *   - cfg->pair_capacity = 0 (or cfg NULL) takes the largest capacity whose
 *     layout fits the array; a layout larger than the array (an explicit
 *     capacity, or many Gaussians or tiles) returns GS_E_WORKSPACE with
 *     nothing enqueued.
 *   - overflow (device int32, may be NULL) is set, in stream order, to 1 if
 *     the step's pairs exceeded that capacity (its outputs are then
 *     undefined), else 0.
 *   - The first call on a device looks the array's address up
 *     (hipGetSymbolAddress); make it outside graph capture.
 *   - Every call on one device shares the array, and each call overwrites
 *     what the previous one left there: calls that overlap on one device
 *     (two streams, two threads) race.  Serialise them.
 * Otherwise as gs_raster_step_l1 (same kernels, same results). */
gs_status gs_raster_step_l1_noalloc(const gs_config* cfg, const gs_image* images,
                                    int32_t n_img, const float* mean, const float* chol,
                                    const float* color, const float* opacity,
                                    const float* radius, int64_t n_gauss, float* out,
                                    const float* target, float* grad_mean, float* grad_chol,
                                    float* grad_color, float* grad_opacity, double* loss,
                                    int32_t* overflow, void* stream);

/* Mean L1 loss of the last gs_raster_render_backward_l1 in this workspace,
 * written to *loss (device double). */
gs_status gs_l1_loss_value(const gs_config* cfg, const gs_image* images, int32_t n_img,
                           int64_t n_gauss, const void* workspace, size_t ws_bytes,
                           double* loss, void* stream);

/* gs_raster_render_backward_l1 + gs_raster_gradients (+ gs_l1_loss_value
 * when loss is not NULL): the training step's backward for the L1 loss. */
gs_status gs_raster_backward_l1(const gs_config* cfg, const gs_image* images, int32_t n_img,
                                const float* chol, const float* color, const float* opacity,
                                int64_t n_gauss, void* workspace, size_t ws_bytes,
                                const float* out, const float* target, float* grad_mean,
                                float* grad_chol, float* grad_color, float* grad_opacity,
                                double* loss, void* stream);

/* L1 training loss (Sec. 3.2, "Rendering": rendered SR image against the HR target)
 * and its gradient: grad = sign(img - target) / numel with sign(0) = 0.
 * img, target, grad: device [numel]; loss: device double, overwritten with
 * the mean of |img - target| (0 when numel is 0). */
gs_status gs_l1_loss_grad(const float* img, const float* target, int64_t numel,
                          float* grad, double* loss, void* stream);

/* Synchronising.  Counts of the last forward in this workspace: total
 * (tile, Gaussian) pairs, overflow flag (pairs > capacity: the output of
 * that forward is undefined), Gaussians flagged for invalid values, and the
 * number of in-support (HR pixel, Gaussian) pairs (the sum of the support
 * box areas: the work the method itself must do).  Any output pointer may be
 * NULL.  Returns GS_E_CAPACITY when the overflow flag is set. */
gs_status gs_diagnostics(const gs_config* cfg, const gs_image* images, int32_t n_img,
                         int64_t n_gauss, const void* workspace, size_t ws_bytes,
                         int64_t* n_pairs, int32_t* overflow, int64_t* n_invalid,
                         int64_t* n_support, void* stream);

/* Synchronising.  Exact number of (tile, Gaussian) pairs the forward of
 * these Gaussians would emit: runs the support/count kernels in the given
 * workspace (which only needs gs_workspace_size with pair_capacity = 1) and
 * reads the total back.  Use it to size pair_capacity. */
gs_status gs_count_pairs(const gs_config* cfg, const gs_image* images, int32_t n_img,
                         const float* mean, const float* chol, const float* radius,
                         int64_t n_gauss, void* workspace, size_t ws_bytes,
                         int64_t* n_pairs, void* stream);

/* Synchronising.  Copies the tile lists of the last forward to the host:
 * ranges_host [n_tiles][2] = [begin, end) into gids_host (empty tiles
 * [0, 0)); gids_host [max_pairs] the Gaussian indices, tile after tile, in
 * ascending index within a tile.  Tiles are numbered row-major within an
 * image and image after image.  n_tiles_out and n_pairs_out receive the
 * sizes; pass NULL arrays to query them.  GS_E_CAPACITY if the lists
 * overflowed, GS_E_INVALID if max_pairs is too small. */
gs_status gs_tile_lists(const gs_config* cfg, const gs_image* images, int32_t n_img,
                        int64_t n_gauss, const void* workspace, size_t ws_bytes,
                        int32_t* ranges_host, int32_t* gids_host, int64_t max_pairs,
                        int64_t* n_tiles_out, int64_t* n_pairs_out, void* stream);

/* Synchronising.  The work order of the persistent tile kernels written by
 * the last gs_raster_bin / gs_raster_forward in this workspace with
 * GS_FLAG_PERSISTENT: order_host [n_tiles] receives every tile id once,
 * longest list first (longest-processing-time order of a batch of uneven
 * images; lists of equal length bucket keep ascending tile id), and *ordered
 * is 1 when that order is complete (0 after a binning without the flag, in
 * which case the persistent kernels take tiles in id order).  order_host may
 * be NULL; max_tiles is its length (GS_E_INVALID if below n_tiles). */
gs_status gs_tile_order(const gs_config* cfg, const gs_image* images, int32_t n_img,
                        int64_t n_gauss, const void* workspace, size_t ws_bytes,
                        uint32_t* order_host, int64_t max_tiles, int32_t* ordered,
                        void* stream);

/* ---- learned support radius (pruned rasterization) ----------------------
 *
 * A small MLP predicts, per Gaussian and scale, the support half-width R (in
 * standard deviations) beyond which the Gaussian's own contribution
 * alpha max(c) f (Eq. 1, 2) stays below a threshold tau; the pruned render
 * passes R as `radius` to gs_raster_forward, so fewer (tile, Gaussian) pairs
 * are binned and evaluated.  The exact 3-sigma box remains the fallback.
 * Network: features [log s, log sigma_x, log sigma_y, rho, alpha, c_r, c_g,
 * c_b] (Sec. 3.1's properties minus the position, plus the scale),
 * standardised; 8 -> 64 -> 64 -> 1 with ReLU; BF16 matrix-core products with
 * FP32 accumulation.  Parameters: FP32 master copy, GS_MLP_PARAMS floats in
 * the order W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [1][64], b3 [1]. */
#define GS_MLP_PARAMS 4801

typedef struct {
    float mu[8], sd[8];      /* training mean / standard deviation per feature */
    float fmin[8], fmax[8];  /* training range of the standardised features   */
    float margin;            /* added to the prediction (calibrated)          */
    float reserved[3];
} gs_mlp_norm;

/* Features of every Gaussian of the batch (device feats [n_gauss][8]),
 * standardised with norm (host) or raw when norm is NULL. */
gs_status gs_mlp_features(const gs_image* images, int32_t n_img, const float* chol,
                          const float* color, const float* opacity, int64_t n_gauss,
                          const gs_mlp_norm* norm, float* feats, void* stream);

/* MLP forward on n standardised feature rows (device).  norm NULL: out[n] is
 * the raw prediction; otherwise out[n] is the support half-width for the
 * pruned path: min(max(prediction + margin, 0), 3), or 3 (the exact box) when
 * a feature lies outside [fmin, fmax] or the prediction is not finite. */
gs_status gs_mlp_forward(const float* params, const float* feats, int64_t n,
                         const gs_mlp_norm* norm, float* out, void* stream);

/* gs_mlp_features (standardised with norm) followed by gs_mlp_forward with
 * norm, in one kernel that forms the features inside the network's first
 * layer: radius (device [n_gauss]) receives the support half-width of every
 * Gaussian of the batch, bitwise as the two calls.  norm must not be NULL. */
gs_status gs_mlp_radius(const gs_image* images, int32_t n_img, const float* params,
                        const float* chol, const float* color, const float* opacity,
                        int64_t n_gauss, const gs_mlp_norm* norm, float* radius, void* stream);

/* Device workspace bytes of gs_mlp_grad for n rows. */
gs_status gs_mlp_workspace_size(int64_t n, size_t* bytes);

/* Gradient of the mean pinball (quantile) loss against labels (device [n]),
 * or, when labels is NULL, of sum_i dout_i * prediction_i for a given
 * upstream gradient dout (device [n]).  grad: device [GS_MLP_PARAMS],
 * overwritten (sums over the batch in a fixed order).  loss_sum (device
 * double, may be NULL) is incremented by the mean pinball loss. */
gs_status gs_mlp_grad(const float* params, const float* feats, const float* labels,
                      const float* dout, int64_t n, float quantile, void* workspace,
                      size_t ws_bytes, float* grad, double* loss_sum, void* stream);

/* One Adam step (Kingma & Ba: beta1 0.9, beta2 0.999, eps 1e-8) on the FP32
 * master parameters; m, v: device [GS_MLP_PARAMS]; step counts from 1. */
gs_status gs_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                      float lr, void* stream);

/* Training labels from the exact rasterizer: per Gaussian, the largest
 * Mahalanobis distance over the HR pixels of its 3-sigma box whose own
 * contribution alpha max(c) f is at least tau (0 if none).  Uses the
 * workspace of a gs_raster_bin / gs_raster_forward with radius NULL;
 * radius: device [n_gauss].  With interior_only != 0, a Gaussian whose
 * support box the image border cuts gets -1 instead (its label would be cut
 * by the border too: training takes the Gaussians with labels >= 0). */
gs_status gs_radius_stats(const gs_config* cfg, const gs_image* images, int32_t n_img,
                          int64_t n_gauss, const void* workspace, size_t ws_bytes, float tau,
                          int32_t interior_only, float* radius, void* stream);

/* The support radius of the method without the learned part (the control
 * the learned radius is compared with): the Mahalanobis distance at which a
 * Gaussian's own peak contribution alpha max(c) f (Eq. 1, 2) falls to tau,
 *     R = min(max(sqrt(2 ln(max(alpha max(c) K / tau, 1))) + margin, 0), 3),
 * K = 1 / (2 pi sigma_x sigma_y sqrt(1 - rho^2)) = 1 / (2 pi l11 l22), in FP64;
 * 3 (the exact box) for l11 <= 0, l22 <= 0 or non-finite values.
 * chol [n][3], color [n][3], opacity [n], radius [n]: device.  tau > 0. */
gs_status gs_closed_form_radius(const float* chol, const float* color, const float* opacity,
                                int64_t n_gauss, double tau, double margin, float* radius,
                                void* stream);

/* sum (a_i - b_i)^2 over n elements, ADDED to *sum (device double): the
 * squared error behind the PSNR of a pruned render against the exact one. */
gs_status gs_sq_error(const float* a, const float* b, int64_t n, double* sum, void* stream);

/* ---- graph capture (HIP graphs) ---------------------------------------- */

/* Opaque executable graph of one whole pass over a fixed batch layout and
 * fixed device pointers. */
typedef struct gs_graph_s* gs_graph;

/* ---- Gaussian primary head (Sec. 3.2, "Gaussian Primary Head" and
 * "Gaussian Embedding") ------------------------------------------------------
 * Turns the raw outputs of the five property heads into the rasterizer's
 * inputs, per Gaussian:
 *     alpha = sigmoid(a), c = sigmoid(r) per channel, sigma = sigmoid(u) per
 *     axis, rho = tanh(v), mu = p + o (no activation on the offset o),
 *     chol = (sigma_x, rho sigma_y, sigma_y sqrt(1 - rho^2)).
 * p is the Gaussian's reference position: image k holds grid^2 H W Gaussians
 * (the paper's m = grid^2 per LR pixel), entry j of its range (row-major)
 * sits at the centre of cell (j mod grid W, j div grid W) of a
 * (grid H) x (grid W) grid of equal cells over the image area
 * [-1/2, W - 1/2] x [-1/2, H - 1/2]: p = ((2 col + 1 - grid) / (2 grid), same
 * for the row).  Device arrays, FP32, C-contiguous:
 *   raw_opacity [N], raw_color [N][3], raw_sigma [N][2], raw_rho [N],
 *   offset [N][2]; outputs mean [N][2], chol [N][3], color [N][3],
 *   opacity [N] (the layouts of gs_raster_forward).
 * images: host array; only lr_h, lr_w, g_begin and g_count are read; each
 * g_count must be grid^2 lr_h lr_w, ranges ascending and disjoint within
 * [0, n_gauss) (GS_E_INVALID otherwise; GS_E_UNSUPPORTED if grid * max(H, W)
 * >= 2^23).  Gaussians between the images' ranges are left untouched.  A raw
 * rho so large that tanh rounds to +-1 gives l22 = 0 (no support). */
gs_status gs_gaussian_head_forward(const gs_image* images, int32_t n_img, int32_t grid,
                                   const float* raw_opacity, const float* raw_color,
                                   const float* raw_sigma, const float* raw_rho,
                                   const float* offset, int64_t n_gauss, float* mean,
                                   float* chol, float* color, float* opacity, void* stream);

/* Backward of gs_gaussian_head_forward: from the gradients w.r.t. mean,
 * chol, color and opacity (e.g. gs_raster_backward's), the gradients w.r.t.
 * the raw outputs (overwritten; the layouts of the raw inputs):
 *   d_opacity = g_opacity sigmoid'(a), d_color = g_color sigmoid'(r),
 *   d_sigma = (g_l11, g_l21 rho + g_l22 sqrt(1 - rho^2)) sigmoid'(u),
 *   d_rho = (g_l21 sigma_y - g_l22 sigma_y rho / sqrt(1 - rho^2)) (1 - rho^2),
 *   d_offset = g_mean. */
gs_status gs_gaussian_head_backward(int64_t n_gauss, const float* raw_opacity,
                                    const float* raw_color, const float* raw_sigma,
                                    const float* raw_rho, const float* grad_mean,
                                    const float* grad_chol, const float* grad_color,
                                    const float* grad_opacity, float* d_opacity,
                                    float* d_color, float* d_sigma, float* d_rho,
                                    float* d_offset, void* stream);

/* ---- Y-channel PSNR (Sec. 4.1, evaluation protocols) ------------------------
 * Per image k of the batch layout (images as for gs_raster_forward: the
 * planar [3][out_h][out_w] block at out_offset of test and ref, device FP32,
 * RGB on [0, 1]): the BT.601 luma Y = (16 + 65.481 R + 128.553 G +
 * 24.966 B) / 255 of both, the sum of squared Y differences over the pixels
 * at least `crop` pixels inside every border (FP64; written to sse[k]) and
 * psnr[k] = 10 log10(count / sse[k]) (+inf for equal images, NaN when the
 * crop leaves no pixel).  sse and psnr: device double [n_img], overwritten.
 * No clamping or quantisation.  Partial sums are added with FP64 atomics, so
 * the last bits of sse may differ between calls. */
gs_status gs_psnr_y(const gs_image* images, int32_t n_img, const float* test, const float* ref,
                    int32_t crop, double* sse, double* psnr, void* stream);

/* Captures, on a private stream, gs_raster_step_l1 (when target is not
 * NULL) or gs_raster_forward (when it is) with the same arguments, and
 * instantiates the result: replaying it runs the whole training step (or
 * forward pass) with one launch.  Kernel arguments, including the image
 * table, are baked in; the pointed-to device data is read at replay time, so
 * the caller may update the Gaussians in place between replays.  The pair
 * capacity must hold for every replay (check gs_diagnostics).  Arguments as
 * for gs_raster_forward / gs_raster_backward_l1.  No memset nodes are used.
 * The graph owns host resources only; destroy it with gs_graph_destroy. */
gs_status gs_graph_create(const gs_config* cfg, const gs_image* images, int32_t n_img,
                          const float* mean, const float* chol, const float* color,
                          const float* opacity, const float* radius, int64_t n_gauss,
                          void* workspace, size_t ws_bytes, float* out, const float* target,
                          float* grad_mean, float* grad_chol, float* grad_color,
                          float* grad_opacity, double* loss, gs_graph* graph);

/* Enqueues one replay on stream. */
gs_status gs_graph_launch(gs_graph graph, void* stream);

/* Releases the graph (NULL is a no-op). */
gs_status gs_graph_destroy(gs_graph graph);

/* Vector-ALU throughput probe (roofline calibration, not part of the
 * method): `blocks` workgroups of 256 threads, each thread running 8
 * independent FP32 chains of `iters` steps.  kind 0: one FMA per chain and
 * step (2 FLOP); kind 1: one exp2 per chain and step; kind 2: five FMA-class
 * operations and one exp2 per chain and step (the shape of the render's
 * per-pixel work); kinds 3-5: one FMA per chain and step followed by a lane
 * mask, a select on an SGPR-pair mask (3), a select on a mask read with
 * readfirstlane (4), a one-bit field extract ANDed into the value (5), so
 * that a mask's cost is the step time minus kind 0's.  The caller times the
 * launch on `stream` and owns `out` (device, blocks x 256 floats,
 * overwritten).  Compiled like every kernel of the library (packed FP32
 * instructions disabled).  GS_E_INVALID for kind outside 0..5, blocks or
 * iters below 1, or a NULL out. */
gs_status gs_valu_probe(int32_t kind, int32_t blocks, int32_t iters, float* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_RASTER_H */
