/*
 * FP64 CPU oracle for the scale-aware 2D Gaussian rasterizer of GSASR
 * (arXiv 2501.06838).  TEST INFRASTRUCTURE ONLY: it is called by the test
 * suite, by the smoke check and by the benchmark's CPU-baseline leg, and by
 * nothing on the product path.  It shares no code, header or constant with
 * the HIP library.
 *
 * Everything is plain double-precision C, written for readability: one loop
 * per definition, in the order the paper states it.  FP32 inputs are widened
 * to double by the caller (exactly).
 *
 * Paper passages followed (section / equation / algorithm of the paper):
 *   Sec. 3.1, 2D GS representation: Gaussian properties alpha, mu, sigma, rho, c.
 *   Eq. 1  G(x,y) = alpha * c * f(x,y).
 *   Eq. 2  f(x,y) = (2 pi sx sy sqrt(1-rho^2))^-1 *
 *                   exp(-(dx^2/sx^2 - 2 rho dx dy/(sx sy) + dy^2/sy^2) / (2 (1-rho^2))).
 *   Eq. 4  I_SR(x,y;s) = sum_i G_i(x/s, y/s).
 *   Algorithm 1 (scale-aware rasterization): zero image of size (sH, sW, 3);
 *     for each Gaussian, for each HR pixel inside a strict box window around
 *     the centre, add G_i(x/s, y/s).
 *   Sec. 3.1 "Fast Rasterization": differentiable renderer (gradients w.r.t.
 *     all Gaussian properties).
 *
 * Readings taken where the paper is silent or garbled (all listed in the
 * design notes of this repository):
 *   - mu, sigma are in LR pixels; LR pixel centres sit at integer coordinates
 *     (Eq. 3 samples integer x in [0, W-1]).
 *   - The HR image has floor(s*H + 0.5) x floor(s*W + 0.5) pixels.
 *   - The window of Algorithm 1 is replaced by the axis-aligned box of
 *     +-R standard deviations per axis (R = 3 on the exact path), keeping the
 *     algorithm's strict "<" test, expressed in HR pixels:
 *         { x integer : s*(mu_x - R*sx) < x < s*(mu_x + R*sx) }.
 *   - The covariance is passed as its Cholesky factor L = [[l11,0],[l21,l22]]:
 *         sx = l11, sy = sqrt(l21^2 + l22^2), rho = l21 / sy.
 *   - Gradients treat the box as fixed (its derivative is zero almost
 *     everywhere).
 *   - A Gaussian with a non-finite value, l11 <= 0 or l22 <= 0 has no support.
 *
 * Build (done by the repository's build step):
 *   gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared gs_oracle.c -o libgsoracle.so -lm
 * -ffp-contract=off matters: the support box is defined by an exact FP64
 * operation sequence with no fused multiply-add.  OpenMP is used only by the
 * *_mt variants, which time the oracle on several cores.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* HR image size: Algorithm 1 allocates an (sH, sW, 3) image; for a
 * non-integer product the size is rounded half up. */
int or_output_size(int32_t H, int32_t W, double s, int32_t* out_h, int32_t* out_w)
{
    if (H < 1 || W < 1 || !isfinite(s) || !(s > 0.0)) return -1;
    double h = floor(s * (double)H + 0.5);
    double w = floor(s * (double)W + 0.5);
    if (h < 1.0 || w < 1.0 || h * w >= 2147483648.0) return -1;
    *out_h = (int32_t)h;
    *out_w = (int32_t)w;
    return 0;
}

/* Support of one Gaussian in HR pixels (Algorithm 1's strict box test, with
 * the half-window R standard deviations on each axis), clipped to the image.
 * rect = {x0, x1, y0, y1}, inclusive.  Returns 1 if non-empty, else 0. */
int or_support_rect(double s, int32_t out_w, int32_t out_h,
                    double mx, double my, double l11, double l21, double l22,
                    double R, int32_t rect[4])
{
    rect[0] = 0; rect[1] = -1; rect[2] = 0; rect[3] = -1;
    if (!isfinite(mx) || !isfinite(my) || !isfinite(l11) || !isfinite(l21) ||
        !isfinite(l22) || !isfinite(R))
        return 0;
    if (!(l11 > 0.0) || !(l22 > 0.0) || !(R > 0.0)) return 0;

    double sx = l11;
    double sy = sqrt(l21 * l21 + l22 * l22);

    double lo_x = s * (mx - R * sx);
    double hi_x = s * (mx + R * sx);
    double lo_y = s * (my - R * sy);
    double hi_y = s * (my + R * sy);

    /* smallest integer strictly above lo, largest strictly below hi */
    double x0 = floor(lo_x) + 1.0, x1 = ceil(hi_x) - 1.0;
    double y0 = floor(lo_y) + 1.0, y1 = ceil(hi_y) - 1.0;
    if (x0 < 0.0) x0 = 0.0;
    if (y0 < 0.0) y0 = 0.0;
    if (x1 > (double)(out_w - 1)) x1 = (double)(out_w - 1);
    if (y1 > (double)(out_h - 1)) y1 = (double)(out_h - 1);
    if (x0 > x1 || y0 > y1) return 0;

    rect[0] = (int32_t)x0; rect[1] = (int32_t)x1;
    rect[2] = (int32_t)y0; rect[3] = (int32_t)y1;
    return 1;
}

/* Support modes (bits of `mode`), alternative readings of Eq. 4 and of the
 * truncation:
 *   OR_PIXEL_CENTER: HR pixel x samples the LR coordinate u = (x + 1/2)/s - 1/2
 *     (pixel centres of both grids aligned) instead of the literal u = x/s;
 *     every box, window and weight moves with it (the HR centre becomes
 *     s (mu + 1/2) - 1/2).
 *   OR_ELLIPSE: within the box, only pixels with Mahalanobis distance d < R
 *     (d^2 = z1^2 + z2^2 of Eq. 2) are in the support (box test first). */
#define OR_PIXEL_CENTER 1
#define OR_ELLIPSE 2

/* The LR coordinate HR pixel index x samples. */
static double sample_u(int32_t x, double s, int32_t mode)
{
    if (mode & OR_PIXEL_CENTER) return ((double)x + 0.5) / s - 0.5;
    return (double)x / s;
}

/* Squared Mahalanobis distance (Eq. 2's quadratic form in the Cholesky
 * coordinates) of HR pixel (x, y), in this exact operation sequence:
 *   z1 = (u - mx) / l11,  z2 = ((v - my) - l21 z1) / l22,  d2 = z1 z1 + z2 z2. */
double or_pixel_d2(int32_t x, int32_t y, double s, int32_t mode, double mx, double my,
                   double l11, double l21, double l22)
{
    double z1 = (sample_u(x, s, mode) - mx) / l11;
    double z2 = ((sample_u(y, s, mode) - my) - l21 * z1) / l22;
    return z1 * z1 + z2 * z2;
}

/* Box of one Gaussian (Algorithm 1's strict window test with the
 * half-window R standard deviations per axis), for either sampling
 * convention: {x : s((mx - R sx) + c) - c < x < s((mx + R sx) + c) - c},
 * c = 1/2 with OR_PIXEL_CENTER, else the literal box (c = 0). */
int or_support_rect_m(double s, int32_t out_w, int32_t out_h, double mx, double my, double l11,
                      double l21, double l22, double R, int32_t mode, int32_t rect[4])
{
    if (!(mode & OR_PIXEL_CENTER))
        return or_support_rect(s, out_w, out_h, mx, my, l11, l21, l22, R, rect);
    rect[0] = 0; rect[1] = -1; rect[2] = 0; rect[3] = -1;
    if (!isfinite(mx) || !isfinite(my) || !isfinite(l11) || !isfinite(l21) ||
        !isfinite(l22) || !isfinite(R))
        return 0;
    if (!(l11 > 0.0) || !(l22 > 0.0) || !(R > 0.0)) return 0;
    double sx = l11;
    double sy = sqrt(l21 * l21 + l22 * l22);
    double lo_x = s * ((mx - R * sx) + 0.5) - 0.5;
    double hi_x = s * ((mx + R * sx) + 0.5) - 0.5;
    double lo_y = s * ((my - R * sy) + 0.5) - 0.5;
    double hi_y = s * ((my + R * sy) + 0.5) - 0.5;
    double x0 = floor(lo_x) + 1.0, x1 = ceil(hi_x) - 1.0;
    double y0 = floor(lo_y) + 1.0, y1 = ceil(hi_y) - 1.0;
    if (x0 < 0.0) x0 = 0.0;
    if (y0 < 0.0) y0 = 0.0;
    if (x1 > (double)(out_w - 1)) x1 = (double)(out_w - 1);
    if (y1 > (double)(out_h - 1)) y1 = (double)(out_h - 1);
    if (x0 > x1 || y0 > y1) return 0;
    rect[0] = (int32_t)x0; rect[1] = (int32_t)x1;
    rect[2] = (int32_t)y0; rect[3] = (int32_t)y1;
    return 1;
}

/* Support of one Gaussian under Algorithm 1's own window, the rasterization
 * ratio r of Sec. 3.1 "Fast Rasterization": the strict test |x - mu_x| < r s H,
 * |y - mu_y| < r s W, read with both sides in HR pixels (the HR centre is
 * s mu) and each axis paired with its own image extent (x with W, y with H):
 *     { x integer : s mx - r (s W) < x < s mx + r (s W) }, same for y with H,
 * clipped to the image.  The Gaussian must still be valid (finite, l11 > 0,
 * l22 > 0).  With OR_PIXEL_CENTER the window is centred on s (mu + 1/2) - 1/2.
 * rect = {x0, x1, y0, y1}; returns 1 if non-empty, else 0. */
int or_window_rect(double s, int32_t out_w, int32_t out_h, int32_t H, int32_t W, double r,
                   double mx, double my, double l11, double l21, double l22, int32_t mode,
                   int32_t rect[4])
{
    rect[0] = 0; rect[1] = -1; rect[2] = 0; rect[3] = -1;
    if (!isfinite(mx) || !isfinite(my) || !isfinite(l11) || !isfinite(l21) ||
        !isfinite(l22) || !isfinite(r))
        return 0;
    if (!(l11 > 0.0) || !(l22 > 0.0) || !(r > 0.0)) return 0;
    double hx = r * (s * (double)W);
    double hy = r * (s * (double)H);
    double cx = s * mx, cy = s * my;
    if (mode & OR_PIXEL_CENTER) {  /* HR centre of the pixel-centre convention */
        cx = s * (mx + 0.5) - 0.5;
        cy = s * (my + 0.5) - 0.5;
    }
    double x0 = floor(cx - hx) + 1.0, x1 = ceil(cx + hx) - 1.0;
    double y0 = floor(cy - hy) + 1.0, y1 = ceil(cy + hy) - 1.0;
    if (x0 < 0.0) x0 = 0.0;
    if (y0 < 0.0) y0 = 0.0;
    if (x1 > (double)(out_w - 1)) x1 = (double)(out_w - 1);
    if (y1 > (double)(out_h - 1)) y1 = (double)(out_h - 1);
    if (x0 > x1 || y0 > y1) return 0;
    rect[0] = (int32_t)x0; rect[1] = (int32_t)x1;
    rect[2] = (int32_t)y0; rect[3] = (int32_t)y1;
    return 1;
}

/* 1 if the image border cuts the support box of a valid Gaussian (some
 * integer x or y passing the strict window test lies outside the image),
 * 0 if the box lies inside the image, -1 if the Gaussian is invalid.  Used to
 * select the Gaussians whose support-radius labels the border does not cut. */
int or_box_cut(double s, int32_t out_w, int32_t out_h,
               double mx, double my, double l11, double l21, double l22, double R)
{
    if (!isfinite(mx) || !isfinite(my) || !isfinite(l11) || !isfinite(l21) ||
        !isfinite(l22) || !isfinite(R))
        return -1;
    if (!(l11 > 0.0) || !(l22 > 0.0) || !(R > 0.0)) return -1;
    double sx = l11;
    double sy = sqrt(l21 * l21 + l22 * l22);
    double x0 = floor(s * (mx - R * sx)) + 1.0, x1 = ceil(s * (mx + R * sx)) - 1.0;
    double y0 = floor(s * (my - R * sy)) + 1.0, y1 = ceil(s * (my + R * sy)) - 1.0;
    return (x0 < 0.0 || y0 < 0.0 || x1 > (double)(out_w - 1) || y1 > (double)(out_h - 1)) ? 1 : 0;
}

/* Eq. 2 in its printed (sigma_x, sigma_y, rho) form, at offset (dx, dy). */
static double eq2_density(double dx, double dy, double sx, double sy, double rho)
{
    double d = 1.0 - rho * rho;
    double q = (dx * dx / (sx * sx) - 2.0 * rho * dx * dy / (sx * sy) + dy * dy / (sy * sy)) / d;
    return exp(-0.5 * q) / (2.0 * OR_PI * sx * sy * sqrt(d));
}

static void chol_to_eq2(double l11, double l21, double l22, double* sx, double* sy, double* rho)
{
    *sx = l11;
    *sy = sqrt(l21 * l21 + l22 * l22);
    *rho = l21 / *sy;
}

static double radius_of(const double* radius, int64_t i)
{
    return radius ? radius[i] : 3.0;
}

/* The support rect of Gaussian i: Algorithm 1's r-window when window_r > 0,
 * else the box of radius[i] (NULL: 3) standard deviations per axis. */
static int rect_of(int64_t i, int32_t H, int32_t W, double s, int32_t oh, int32_t ow,
                   const double* mean, const double* chol, const double* radius,
                   double window_r, int32_t mode, int32_t r[4])
{
    if (window_r > 0.0)
        return or_window_rect(s, ow, oh, H, W, window_r, mean[2 * i], mean[2 * i + 1],
                              chol[3 * i], chol[3 * i + 1], chol[3 * i + 2], mode, r);
    return or_support_rect_m(s, ow, oh, mean[2 * i], mean[2 * i + 1], chol[3 * i],
                             chol[3 * i + 1], chol[3 * i + 2], radius_of(radius, i), mode, r);
}

/* Whether HR pixel (x, y) of Gaussian i's box is in its support: always for
 * the box readings; with OR_ELLIPSE (not with the r-window), d^2 < R^2. */
static int in_support(int64_t i, int32_t x, int32_t y, double s, int32_t mode,
                      const double* mean, const double* chol, const double* radius,
                      double window_r)
{
    if (!(mode & OR_ELLIPSE) || window_r > 0.0) return 1;
    double R = radius_of(radius, i);
    return or_pixel_d2(x, y, s, mode, mean[2 * i], mean[2 * i + 1], chol[3 * i],
                       chol[3 * i + 1], chol[3 * i + 2]) < R * R;
}

/* Adds every Gaussian's contribution to the HR rows [y_lo, y_hi) of one image
 * (Algorithm 1's loops with Eq. 1, 2, 4, restricted to those rows): for each
 * Gaussian in ascending order, for each pixel of its support box in the rows,
 * out += alpha c f(x/s, y/s).  out is the whole [3][out_h][out_w] image. */
static void forward_rows(int32_t H, int32_t W, int32_t oh, int32_t ow, double s, int64_t n,
                         const double* mean, const double* chol, const double* color,
                         const double* opacity, const double* radius, double window_r,
                         int32_t mode, int32_t y_lo, int32_t y_hi, double* out)
{
    int64_t plane = (int64_t)oh * ow;
    for (int64_t i = 0; i < n; ++i) {
        const double mx = mean[2 * i], my = mean[2 * i + 1];
        const double l11 = chol[3 * i], l21 = chol[3 * i + 1], l22 = chol[3 * i + 2];
        int32_t r[4];
        if (!rect_of(i, H, W, s, oh, ow, mean, chol, radius, window_r, mode, r)) continue;
        if (!isfinite(opacity[i]) || !isfinite(color[3 * i]) || !isfinite(color[3 * i + 1]) ||
            !isfinite(color[3 * i + 2]))
            continue;
        const int32_t ya = r[2] > y_lo ? r[2] : y_lo;
        const int32_t yb = r[3] < y_hi - 1 ? r[3] : y_hi - 1;
        double sx, sy, rho;
        chol_to_eq2(l11, l21, l22, &sx, &sy, &rho);
        for (int32_t y = ya; y <= yb; ++y) {
            for (int32_t x = r[0]; x <= r[1]; ++x) {
                if (!in_support(i, x, y, s, mode, mean, chol, radius, window_r)) continue;
                double f = eq2_density(sample_u(x, s, mode) - mx, sample_u(y, s, mode) - my, sx,
                                       sy, rho);
                for (int c = 0; c < 3; ++c)
                    out[c * plane + (int64_t)y * ow + x] += opacity[i] * color[3 * i + c] * f; /* Eq. 1 */
            }
        }
    }
}

/* Forward render of one image (Algorithm 1 with Eq. 1, 2, 4).
 * mean [n][2] (mu_x, mu_y); chol [n][3] (l11, l21, l22); color [n][3];
 * opacity [n]; radius [n] or NULL (NULL = 3 standard deviations);
 * window_r > 0 takes Algorithm 1's r-window instead (radius ignored); mode
 * holds the OR_* support bits.  out [3][out_h][out_w] is overwritten. */
void or_forward(int32_t H, int32_t W, double s, int64_t n,
                const double* mean, const double* chol, const double* color,
                const double* opacity, const double* radius, double window_r, int32_t mode,
                double* out)
{
    int32_t oh, ow;
    if (or_output_size(H, W, s, &oh, &ow) != 0) return;
    memset(out, 0, sizeof(double) * 3 * (size_t)oh * (size_t)ow);
    forward_rows(H, W, oh, ow, s, n, mean, chol, color, opacity, radius, window_r, mode, 0, oh,
                 out);
}

/* or_forward on up to nthreads host threads (OpenMP), for timing the oracle
 * on all cores: bands of HR rows are rendered independently, each pixel
 * still summing its Gaussians in ascending order, so the result is bitwise
 * that of or_forward. */
void or_forward_mt(int32_t H, int32_t W, double s, int64_t n,
                   const double* mean, const double* chol, const double* color,
                   const double* opacity, const double* radius, double window_r, int32_t mode,
                   double* out, int32_t nthreads)
{
    int32_t oh, ow;
    if (or_output_size(H, W, s, &oh, &ow) != 0) return;
    memset(out, 0, sizeof(double) * 3 * (size_t)oh * (size_t)ow);
    const int32_t band = 32;
    const int32_t nb = (oh + band - 1) / band;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t y1 = (b + 1) * band < oh ? (b + 1) * band : oh;
        forward_rows(H, W, oh, ow, s, n, mean, chol, color, opacity, radius, window_r, mode,
                     b * band, y1, out);
    }
}

/* Gradients of a loss L w.r.t. every Gaussian property, given the upstream
 * image gradient grad_out = dL/dI_SR [3][out_h][out_w] of one image.
 *
 * Derived directly from Eq. 1 and Eq. 2 in the (sx, sy, rho) form, then
 * carried to the Cholesky parameters by the chain rule:
 *   with a = dx/sx, b = dy/sy, D = 1 - rho^2, Q = (a^2 - 2 rho a b + b^2)/D,
 *   log f = -Q/2 - log(2 pi) - log sx - log sy - log(D)/2, and
 *   d log f / d mu_x  = (a - rho b) / (D sx)
 *   d log f / d mu_y  = (b - rho a) / (D sy)
 *   d log f / d sx    = (a^2 - rho a b) / (D sx) - 1/sx
 *   d log f / d sy    = (b^2 - rho a b) / (D sy) - 1/sy
 *   d log f / d rho   = (a b D - rho (a^2 - 2 rho a b + b^2)) / D^2 + rho / D
 *   sx = l11, sy = sqrt(l21^2 + l22^2), rho = l21 / sy:
 *   d sy/d l21 = l21/sy, d sy/d l22 = l22/sy,
 *   d rho/d l21 = l22^2/sy^3, d rho/d l22 = -l21 l22/sy^3.
 * Outputs are overwritten: grad_mean [n][2], grad_chol [n][3],
 * grad_color [n][3], grad_opacity [n]. */
/* The gradients of Gaussian i (see or_backward). */
static void backward_one(int64_t i, int32_t H, int32_t W, int32_t oh, int32_t ow, double s,
                         const double* mean, const double* chol, const double* color,
                         const double* opacity, const double* radius, double window_r,
                         int32_t mode, const double* grad_out,
                         double* grad_mean, double* grad_chol, double* grad_color,
                         double* grad_opacity)
{
    int64_t plane = (int64_t)oh * ow;
    const double mx = mean[2 * i], my = mean[2 * i + 1];
    const double l11 = chol[3 * i], l21 = chol[3 * i + 1], l22 = chol[3 * i + 2];
    const double al = opacity[i];
    const double* c = color + 3 * i;
    int32_t r[4];
    if (!rect_of(i, H, W, s, oh, ow, mean, chol, radius, window_r, mode, r)) return;
    if (!isfinite(al) || !isfinite(c[0]) || !isfinite(c[1]) || !isfinite(c[2])) return;
    double sx, sy, rho;
    chol_to_eq2(l11, l21, l22, &sx, &sy, &rho);
    const double D = 1.0 - rho * rho;

    double g_mx = 0, g_my = 0, g_sx = 0, g_sy = 0, g_rho = 0, g_al = 0;
    double g_c[3] = {0, 0, 0};
    for (int32_t y = r[2]; y <= r[3]; ++y) {
        for (int32_t x = r[0]; x <= r[1]; ++x) {
            if (!in_support(i, x, y, s, mode, mean, chol, radius, window_r)) continue;
            const double dx = sample_u(x, s, mode) - mx, dy = sample_u(y, s, mode) - my;
            const double f = eq2_density(dx, dy, sx, sy, rho);
            const int64_t p = (int64_t)y * ow + x;
            double gc_dot = 0.0; /* sum_c dL/dI_c * c_c */
            for (int k = 0; k < 3; ++k) {
                const double g = grad_out[k * plane + p];
                g_c[k] += g * al * f;          /* dI_c/dc_c = alpha f      */
                gc_dot += g * c[k];
            }
            g_al += gc_dot * f;                /* dI_c/dalpha = c_c f      */
            const double wf = gc_dot * al * f; /* dL/dlog f                 */
            const double a = dx / sx, b = dy / sy;
            g_mx += wf * (a - rho * b) / (D * sx);
            g_my += wf * (b - rho * a) / (D * sy);
            g_sx += wf * ((a * a - rho * a * b) / (D * sx) - 1.0 / sx);
            g_sy += wf * ((b * b - rho * a * b) / (D * sy) - 1.0 / sy);
            g_rho += wf * ((a * b * D - rho * (a * a - 2.0 * rho * a * b + b * b)) / (D * D) + rho / D);
        }
    }
    const double sy3 = sy * sy * sy;
    grad_mean[2 * i] = g_mx;
    grad_mean[2 * i + 1] = g_my;
    grad_chol[3 * i] = g_sx;
    grad_chol[3 * i + 1] = g_sy * (l21 / sy) + g_rho * (l22 * l22 / sy3);
    grad_chol[3 * i + 2] = g_sy * (l22 / sy) + g_rho * (-l21 * l22 / sy3);
    for (int k = 0; k < 3; ++k) grad_color[3 * i + k] = g_c[k];
    grad_opacity[i] = g_al;
}

void or_backward(int32_t H, int32_t W, double s, int64_t n,
                 const double* mean, const double* chol, const double* color,
                 const double* opacity, const double* radius, double window_r, int32_t mode,
                 const double* grad_out,
                 double* grad_mean, double* grad_chol, double* grad_color, double* grad_opacity)
{
    int32_t oh, ow;
    memset(grad_mean, 0, sizeof(double) * 2 * (size_t)n);
    memset(grad_chol, 0, sizeof(double) * 3 * (size_t)n);
    memset(grad_color, 0, sizeof(double) * 3 * (size_t)n);
    memset(grad_opacity, 0, sizeof(double) * (size_t)n);
    if (or_output_size(H, W, s, &oh, &ow) != 0) return;
    for (int64_t i = 0; i < n; ++i)
        backward_one(i, H, W, oh, ow, s, mean, chol, color, opacity, radius, window_r, mode,
                     grad_out, grad_mean, grad_chol, grad_color, grad_opacity);
}

/* or_backward on up to nthreads host threads (OpenMP), for timing the
 * oracle on all cores: Gaussians are independent, so the result is bitwise
 * that of or_backward. */
void or_backward_mt(int32_t H, int32_t W, double s, int64_t n,
                    const double* mean, const double* chol, const double* color,
                    const double* opacity, const double* radius, double window_r,
                    int32_t mode, const double* grad_out,
                    double* grad_mean, double* grad_chol, double* grad_color,
                    double* grad_opacity, int32_t nthreads)
{
    int32_t oh, ow;
    memset(grad_mean, 0, sizeof(double) * 2 * (size_t)n);
    memset(grad_chol, 0, sizeof(double) * 3 * (size_t)n);
    memset(grad_color, 0, sizeof(double) * 3 * (size_t)n);
    memset(grad_opacity, 0, sizeof(double) * (size_t)n);
    if (or_output_size(H, W, s, &oh, &ow) != 0) return;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 256) num_threads(nthreads)
    for (int64_t i = 0; i < n; ++i)
        backward_one(i, H, W, oh, ow, s, mean, chol, color, opacity, radius, window_r, mode,
                     grad_out, grad_mean, grad_chol, grad_color, grad_opacity);
}

/* Tile lists of one image: tiles are tw x th HR pixels, numbered row-major
 * (ty * tiles_x + tx).  A Gaussian is listed in every tile its support box
 * touches, i.e. tiles floor(x0/tw)..floor(x1/tw) by floor(y0/th)..floor(y1/th);
 * each list is in ascending Gaussian index.  counts[tiles] is overwritten;
 * lists (may be NULL) receives the concatenation of the lists in tile order
 * when cap is at least the total number of pairs, which is returned.
 * Two plain passes: count per tile; then visit the Gaussians in ascending
 * order again and append each to its tiles' lists. */
int64_t or_tile_lists(int32_t H, int32_t W, double s, int64_t n,
                      const double* mean, const double* chol, const double* radius,
                      double window_r, int32_t mode, int32_t tw, int32_t th, int32_t* counts,
                      int32_t* lists, int64_t cap)
{
    int32_t oh, ow;
    if (tw < 1 || th < 1 || or_output_size(H, W, s, &oh, &ow) != 0) return -1;
    const int32_t tiles_x = (ow + tw - 1) / tw, tiles_y = (oh + th - 1) / th;
    const int64_t n_tiles = (int64_t)tiles_x * tiles_y;
    memset(counts, 0, sizeof(int32_t) * (size_t)n_tiles);

    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t r[4];
        if (!rect_of(i, H, W, s, oh, ow, mean, chol, radius, window_r, mode, r)) continue;
        for (int32_t ty = r[2] / th; ty <= r[3] / th; ++ty)
            for (int32_t tx = r[0] / tw; tx <= r[1] / tw; ++tx) {
                counts[(int64_t)ty * tiles_x + tx] += 1;
                ++total;
            }
    }
    if (!lists || cap < total) return total;

    /* fill[t] = where the next entry of tile t goes */
    int64_t start = 0;
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_tiles > 0 ? n_tiles : 1));
    if (!fill) return -1;
    for (int64_t t = 0; t < n_tiles; ++t) { fill[t] = start; start += counts[t]; }
    for (int64_t i = 0; i < n; ++i) {
        int32_t r[4];
        if (!rect_of(i, H, W, s, oh, ow, mean, chol, radius, window_r, mode, r)) continue;
        for (int32_t ty = r[2] / th; ty <= r[3] / th; ++ty)
            for (int32_t tx = r[0] / tw; tx <= r[1] / tw; ++tx)
                lists[fill[(int64_t)ty * tiles_x + tx]++] = (int32_t)i;
    }
    free(fill);
    return total;
}

/* Number of in-support (pixel, Gaussian) pairs of one image, and the support
 * boxes themselves (rects [n][4] may be NULL). */
int64_t or_support_pairs(int32_t H, int32_t W, double s, int64_t n,
                         const double* mean, const double* chol, const double* radius,
                         double window_r, int32_t mode, int32_t* rects)
{
    int32_t oh, ow;
    if (or_output_size(H, W, s, &oh, &ow) != 0) return -1;
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t r[4];
        int ok = rect_of(i, H, W, s, oh, ow, mean, chol, radius, window_r, mode, r);
        if (rects) memcpy(rects + 4 * i, r, sizeof r);
        if (!ok) continue;
        if (!(mode & OR_ELLIPSE) || window_r > 0.0) {
            total += (int64_t)(r[1] - r[0] + 1) * (r[3] - r[2] + 1);
            continue;
        }
        for (int32_t y = r[2]; y <= r[3]; ++y)
            for (int32_t x = r[0]; x <= r[1]; ++x)
                total += in_support(i, x, y, s, mode, mean, chol, radius, window_r);
    }
    return total;
}

/* Values of the HR image of one image at selected pixels (xs[k], ys[k]):
 * Eq. 4 summed over every Gaussian whose support box holds the pixel, in
 * ascending Gaussian order.  out [3][npix].  Used to check renders too large
 * to evaluate whole. */
void or_pixel_values(int32_t H, int32_t W, double s, int64_t n,
                     const double* mean, const double* chol, const double* color,
                     const double* opacity, const double* radius, double window_r,
                     int32_t mode, int64_t npix, const int32_t* xs, const int32_t* ys, double* out)
{
    int32_t oh, ow;
    memset(out, 0, sizeof(double) * 3 * (size_t)npix);
    if (or_output_size(H, W, s, &oh, &ow) != 0) return;
    for (int64_t i = 0; i < n; ++i) {
        const double mx = mean[2 * i], my = mean[2 * i + 1];
        const double l11 = chol[3 * i], l21 = chol[3 * i + 1], l22 = chol[3 * i + 2];
        int32_t r[4];
        if (!rect_of(i, H, W, s, oh, ow, mean, chol, radius, window_r, mode, r)) continue;
        if (!isfinite(opacity[i]) || !isfinite(color[3 * i]) || !isfinite(color[3 * i + 1]) ||
            !isfinite(color[3 * i + 2]))
            continue;
        double sx, sy, rho;
        chol_to_eq2(l11, l21, l22, &sx, &sy, &rho);
        for (int64_t k = 0; k < npix; ++k) {
            const int32_t x = xs[k], y = ys[k];
            if (x < r[0] || x > r[1] || y < r[2] || y > r[3]) continue;
            if (!in_support(i, x, y, s, mode, mean, chol, radius, window_r)) continue;
            double f = eq2_density(sample_u(x, s, mode) - mx, sample_u(y, s, mode) - my, sx, sy,
                                   rho);
            for (int c = 0; c < 3; ++c) out[c * npix + k] += opacity[i] * color[3 * i + c] * f;
        }
    }
}

/* Support-radius labels of one image for the learned pruning: for each
 * Gaussian, the largest Mahalanobis distance d (LR units, d^2 = the Eq. 2
 * quadratic form) over the HR pixels of its exact support box whose own
 * contribution alpha * max_c(c_c) * f (Eq. 1, 2) is at least tau; 0 if no
 * pixel qualifies or the Gaussian has no support.  R [n] is overwritten. */
void or_radius_labels(int32_t H, int32_t W, double s, int64_t n,
                      const double* mean, const double* chol, const double* color,
                      const double* opacity, double tau, double* R)
{
    int32_t oh, ow;
    for (int64_t i = 0; i < n; ++i) R[i] = 0.0;
    if (or_output_size(H, W, s, &oh, &ow) != 0) return;
    for (int64_t i = 0; i < n; ++i) {
        const double mx = mean[2 * i], my = mean[2 * i + 1];
        const double l11 = chol[3 * i], l21 = chol[3 * i + 1], l22 = chol[3 * i + 2];
        int32_t r[4];
        if (!or_support_rect(s, ow, oh, mx, my, l11, l21, l22, 3.0, r)) continue;
        double cmax = color[3 * i];
        if (color[3 * i + 1] > cmax) cmax = color[3 * i + 1];
        if (color[3 * i + 2] > cmax) cmax = color[3 * i + 2];
        double sx, sy, rho;
        chol_to_eq2(l11, l21, l22, &sx, &sy, &rho);
        const double D = 1.0 - rho * rho;
        double best = 0.0;
        for (int32_t y = r[2]; y <= r[3]; ++y) {
            for (int32_t x = r[0]; x <= r[1]; ++x) {
                const double dx = (double)x / s - mx, dy = (double)y / s - my;
                const double q = (dx * dx / (sx * sx) - 2.0 * rho * dx * dy / (sx * sy) +
                                  dy * dy / (sy * sy)) / D;
                const double f = exp(-0.5 * q) / (2.0 * OR_PI * sx * sy * sqrt(D));
                if (opacity[i] * cmax * f >= tau && q > best * best) best = sqrt(q);
            }
        }
        R[i] = best;
    }
}
