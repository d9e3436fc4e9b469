// Gaussian primary head (Sec. 3.2, "Gaussian Primary Head", "Gaussian
// Embedding") and the Y-channel PSNR of the evaluation protocol (Sec. 4.1).
//
// Head: per Gaussian, the five heads' raw outputs become the properties of
// Sec. 3.1 and the rasterizer's inputs in one pass:
//   alpha = sigmoid(a), c = sigmoid(r), sigma = sigmoid(u), rho = tanh(v),
//   mu = p + o (p: the reference position, the centre of cell (col, row) of a
//   (g H) x (g W) grid over the LR image area, LR pixel centres at integers),
//   L = [[sigma_x, 0], [rho sigma_y, sigma_y sqrt(1 - rho^2)]].
// The backward carries the gradients of (mu, L, c, alpha) back to the raw
// outputs.  Everything is elementwise and HBM-bound: 36 B read and 36 B
// written per Gaussian forward; 28 B of raw outputs and 36 B of gradients
// read, 36 B written backward.  Numerically stable forms: with e = exp(-|x|),
// sigmoid(x) sigmoid(-x) = e / (1 + e)^2; with t = exp(-|v|),
// sqrt(1 - tanh^2 v) = sech v = 2 t / (1 + t^2), and tanh v from expm1, so no
// 1 - x cancellation occurs anywhere.
//
// Y-PSNR: per image, the sum of squared differences of the BT.601 luma
// (65.481 R + 128.553 G + 24.966 B) / 255 between two planar RGB images
// (the +16 offset cancels), without a border of `crop` pixels, in FP64, and
// 10 log10(count / sum).  Workgroups never straddle images; each adds its
// partial sum with one FP64 atomic (the last bits of the sum depend on their
// order).
#include <math.h>

#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kHeadThreads = 256;
constexpr int kPsnrThreads = 256;
constexpr int kPsnrPer = 16;  // pixels per thread

struct HeadImg {
    int64_t g_begin, g_count;
    int32_t gw;      // grid points per row: g W
    int32_t two_g;   // 2 g
    int32_t g;
    int32_t pad;
};
struct HeadTable {
    HeadImg img[kSetupChunk];
    int32_t n;
};

__device__ __forceinline__ int head_image(const HeadTable& t, int64_t i) {
    int lo = 0, hi = t.n - 1, ans = 0;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        if (t.img[mid].g_begin <= i) { ans = mid; lo = mid + 1; } else { hi = mid - 1; }
    }
    return ans;
}

// sigmoid(x) and sigmoid(x) sigmoid(-x)
__device__ __forceinline__ void sigmoid2(float x, float& s, float& ds) {
    const float e = expf(-fabsf(x));
    const float inv = 1.f / (1.f + e);
    s = x >= 0.f ? inv : e * inv;
    ds = e * inv * inv;
}

// tanh(v) and sech(v) = sqrt(1 - tanh^2 v)
__device__ __forceinline__ void tanh_sech(float v, float& th, float& sh) {
    const float av = fabsf(v);
    const float m = expm1f(-2.f * av);  // exp(-2|v|) - 1, in (-1, 0]
    const float t = -m / (2.f + m);
    th = v < 0.f ? -t : t;
    const float e = expf(-av);
    sh = 2.f * e / (1.f + e * e);
}

// Reference position of local Gaussian k of an image: (2 col + 1 - g) / (2 g)
// per axis, an exact integer over an exact integer, rounded once.
__device__ __forceinline__ float2 ref_pos(const HeadImg& im, int64_t k) {
    const int64_t row = k / im.gw, col = k - row * im.gw;
    return make_float2((float)(2 * col + 1 - im.g) / (float)im.two_g,
                       (float)(2 * row + 1 - im.g) / (float)im.two_g);
}

__global__ __launch_bounds__(kHeadThreads) void k_head_fwd(
    HeadTable tab, int64_t g0, int64_t n, const float* __restrict__ raw_opacity,
    const float* __restrict__ raw_color, const float* __restrict__ raw_sigma,
    const float* __restrict__ raw_rho, const float* __restrict__ offset,
    float* __restrict__ mean, float* __restrict__ chol, float* __restrict__ color,
    float* __restrict__ opacity) {
    const int64_t j = (int64_t)blockIdx.x * kHeadThreads + threadIdx.x;
    if (j >= n) return;
    const int64_t i = g0 + j;
    const HeadImg& im = tab.img[head_image(tab, j)];
    if (j - im.g_begin >= im.g_count) return;  // between two images' ranges
    const float2 p = ref_pos(im, j - im.g_begin);
    float s, ds;
    sigmoid2(raw_opacity[i], s, ds);
    opacity[i] = s;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        sigmoid2(raw_color[3 * i + c], s, ds);
        color[3 * i + c] = s;
    }
    float sx, sy;
    sigmoid2(raw_sigma[2 * i], sx, ds);
    sigmoid2(raw_sigma[2 * i + 1], sy, ds);
    float th, sh;
    tanh_sech(raw_rho[i], th, sh);
    chol[3 * i] = sx;
    chol[3 * i + 1] = th * sy;
    chol[3 * i + 2] = sh * sy;
    mean[2 * i] = p.x + offset[2 * i];
    mean[2 * i + 1] = p.y + offset[2 * i + 1];
}

__global__ __launch_bounds__(kHeadThreads) void k_head_bwd(
    int64_t n, const float* __restrict__ raw_opacity, const float* __restrict__ raw_color,
    const float* __restrict__ raw_sigma, const float* __restrict__ raw_rho,
    const float* __restrict__ g_mean, const float* __restrict__ g_chol,
    const float* __restrict__ g_color, const float* __restrict__ g_opacity,
    float* __restrict__ d_opacity, float* __restrict__ d_color, float* __restrict__ d_sigma,
    float* __restrict__ d_rho, float* __restrict__ d_offset) {
    const int64_t i = (int64_t)blockIdx.x * kHeadThreads + threadIdx.x;
    if (i >= n) return;
    float s, ds;
    sigmoid2(raw_opacity[i], s, ds);
    d_opacity[i] = g_opacity[i] * ds;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        sigmoid2(raw_color[3 * i + c], s, ds);
        d_color[3 * i + c] = g_color[3 * i + c] * ds;
    }
    float sx, dsx, sy, dsy, th, sh;
    sigmoid2(raw_sigma[2 * i], sx, dsx);
    sigmoid2(raw_sigma[2 * i + 1], sy, dsy);
    tanh_sech(raw_rho[i], th, sh);
    const float g11 = g_chol[3 * i], g21 = g_chol[3 * i + 1], g22 = g_chol[3 * i + 2];
    d_sigma[2 * i] = g11 * dsx;
    d_sigma[2 * i + 1] = (g21 * th + g22 * sh) * dsy;
    // d rho / d v = sech^2: (g21 sy - g22 sy th / sech) sech^2
    d_rho[i] = (g21 * sh - g22 * th) * sy * sh;
    d_offset[2 * i] = g_mean[2 * i];
    d_offset[2 * i + 1] = g_mean[2 * i + 1];
}

struct PsnrImg {
    int64_t out_offset;
    int64_t block_begin;  // first workgroup of this image
    int32_t h, w;
};
struct PsnrTable {
    PsnrImg img[kSetupChunk];
    int32_t n;
    int32_t first;        // index of img[0] in the batch
};

__global__ void k_zero_f64(double* __restrict__ p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ __launch_bounds__(kPsnrThreads) void k_psnr_sse(PsnrTable tab,
                                                         const float* __restrict__ a,
                                                         const float* __restrict__ b,
                                                         int32_t crop,
                                                         double* __restrict__ sse) {
    __shared__ double part[kPsnrThreads / 64];
    int k = 0;
    {
        int lo = 0, hi = tab.n - 1;
        while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            if (tab.img[mid].block_begin <= (int64_t)blockIdx.x) { k = mid; lo = mid + 1; }
            else { hi = mid - 1; }
        }
    }
    const PsnrImg& im = tab.img[k];
    const int64_t plane = (int64_t)im.h * im.w;
    const int64_t base = ((int64_t)blockIdx.x - im.block_begin) * (kPsnrThreads * kPsnrPer);
    const float* pa = a + im.out_offset;
    const float* pb = b + im.out_offset;
    double s = 0.0;
#pragma unroll 4
    for (int q = 0; q < kPsnrPer; ++q) {
        const int64_t p = base + (int64_t)q * kPsnrThreads + threadIdx.x;
        if (p < plane) {
            bool in = true;
            if (crop > 0) {  // uniform; plane < 2^31 (validated), so 32-bit division
                const int y = (int)p / im.w, x = (int)p - y * im.w;
                in = y >= crop && y < im.h - crop && x >= crop && x < im.w - crop;
            }
            if (in) {
                const double d = (65.481 * ((double)pa[p] - (double)pb[p]) +
                                  128.553 * ((double)pa[plane + p] - (double)pb[plane + p]) +
                                  24.966 * ((double)pa[2 * plane + p] - (double)pb[2 * plane + p])) /
                                 255.0;
                s += d * d;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kPsnrThreads / 64; ++w) t += part[w];
        atomicAdd(sse + tab.first + k, t);
    }
}

// 10 log10(count / sse) per image of the chunk: +inf for identical images,
// NaN when the crop leaves no pixel.
__global__ void k_psnr_final(PsnrTable tab, int32_t crop, const double* __restrict__ sse,
                             double* __restrict__ psnr) {
    const int k = threadIdx.x;
    if (k >= tab.n) return;
    const PsnrImg& im = tab.img[k];
    const int64_t ch = im.h - 2 * (int64_t)crop, cw = im.w - 2 * (int64_t)crop;
    const double cnt = (ch > 0 && cw > 0) ? (double)(ch * cw) : 0.0;
    const double e = sse[tab.first + k];
    double r;
    if (cnt == 0.0) r = __builtin_nan("");
    else if (e == 0.0) r = __builtin_inf();
    else r = 10.0 * log10(cnt / e);
    psnr[tab.first + k] = r;
}

}  // namespace

hipError_t launch_head_fwd(const gs_image* images, int32_t n_img, int32_t grid,
                           const float* raw_opacity, const float* raw_color,
                           const float* raw_sigma, const float* raw_rho, const float* offset,
                           float* mean, float* chol, float* color, float* opacity,
                           hipStream_t st) {
    for (int first = 0; first < n_img; first += kSetupChunk) {
        const int cnt = n_img < first + kSetupChunk ? n_img - first : kSetupChunk;
        HeadTable tab{};
        tab.n = cnt;
        const int64_t g0 = images[first].g_begin;
        int64_t n = 0;
        for (int k = 0; k < cnt; ++k) {
            const gs_image& im = images[first + k];
            tab.img[k].g_begin = im.g_begin - g0;
            tab.img[k].g_count = im.g_count;
            tab.img[k].gw = grid * im.lr_w;
            tab.img[k].two_g = 2 * grid;
            tab.img[k].g = grid;
            n = im.g_begin + im.g_count - g0;
        }
        if (n == 0) continue;
        hipLaunchKernelGGL(k_head_fwd, dim3((unsigned)((n + kHeadThreads - 1) / kHeadThreads)),
                           dim3(kHeadThreads), 0, st, tab, g0, n, raw_opacity, raw_color,
                           raw_sigma, raw_rho, offset, mean, chol, color, opacity);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_head_bwd(int64_t n, const float* raw_opacity, const float* raw_color,
                           const float* raw_sigma, const float* raw_rho, const float* g_mean,
                           const float* g_chol, const float* g_color, const float* g_opacity,
                           float* d_opacity, float* d_color, float* d_sigma, float* d_rho,
                           float* d_offset, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_head_bwd, dim3((unsigned)((n + kHeadThreads - 1) / kHeadThreads)),
                       dim3(kHeadThreads), 0, st, n, raw_opacity, raw_color, raw_sigma, raw_rho,
                       g_mean, g_chol, g_color, g_opacity, d_opacity, d_color, d_sigma, d_rho,
                       d_offset);
    return hipGetLastError();
}

hipError_t launch_psnr_y(const gs_image* images, int32_t n_img, const float* test,
                         const float* ref, int32_t crop, double* sse, double* psnr,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_zero_f64, dim3((n_img + 255) / 256), dim3(256), 0, st, sse, n_img);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr int64_t kPix = kPsnrThreads * kPsnrPer;
    for (int first = 0; first < n_img; first += kSetupChunk) {
        const int cnt = n_img < first + kSetupChunk ? n_img - first : kSetupChunk;
        PsnrTable tab{};
        tab.n = cnt;
        tab.first = first;
        int64_t blocks = 0;
        for (int k = 0; k < cnt; ++k) {
            const gs_image& im = images[first + k];
            int32_t oh = 0, ow = 0;
            gs_output_size(im.lr_h, im.lr_w, im.scale, &oh, &ow);
            tab.img[k].out_offset = im.out_offset;
            tab.img[k].block_begin = blocks;
            tab.img[k].h = oh;
            tab.img[k].w = ow;
            blocks += ((int64_t)oh * ow + kPix - 1) / kPix;
        }
        hipLaunchKernelGGL(k_psnr_sse, dim3((unsigned)blocks), dim3(kPsnrThreads), 0, st, tab,
                           test, ref, crop, sse);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_psnr_final, dim3(1), dim3(64), 0, st, tab, crop, sse, psnr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace gs
