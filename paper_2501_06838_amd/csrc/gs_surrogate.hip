// Learned support radius for pruned rasterization (gfx950).
//
//   k_mlp_features  per Gaussian: [log s, log sigma_x, log sigma_y, rho, alpha, c]
//                   standardised with the training statistics
//   k_mlp_forward   3-layer MLP 8 -> 64 -> 64 -> 1 on BF16 matrix cores
//                   (v_mfma_f32_16x16x16_bf16, FP32 accumulation); optional
//                   epilogue: support half-width min(pred + margin, 3), or 3
//                   when a feature lies outside the training range
//   k_mlp_grad      forward + backward of a batch (pinball loss or a given
//                   upstream gradient); per-wave partial gradients, matrix
//                   products of the backward also on BF16 matrix cores
//   k_grad_reduce   fixed-order sum of the per-wave partials
//   k_adam          Adam on the FP32 master weights
//   k_radius_stats  labels: per Gaussian, the largest Mahalanobis distance
//                   over in-box HR pixels whose own contribution is >= tau,
//                   from the exact rasterizer's tile pairs
//   k_sq_error      sum of squared differences (PSNR of pruned vs exact)
//
// Matrix-core layout (16x16x16, lane l, g = l / 16, c = l % 16, e = 0..3):
//   A (M x K): A[c][4g + e];  B (K x N): B[4g + e][c];  C (M x N): C[4g + e][c].
// Activations are kept transposed (features x Gaussians), so a layer's C
// tile is, element for element, the B operand of the next layer.
#include "gs_internal.h"

namespace gs {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 8, kHid = 64;
// flat parameter layout: W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [1][64], b3 [1]
constexpr int kOffW1 = 0, kOffB1 = 512, kOffW2 = 576, kOffB2 = 4672, kOffW3 = 4736,
              kOffB3 = 4800;
constexpr int kMlpThreads = 256;

// FP32 -> BF16 bits, round to nearest even (inputs are finite).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16, round to nearest even (the hardware conversion)
__device__ __forceinline__ short bf16_bits(float x) {
    const f32x2 v = {x, 0.f};
    const bf16x2_t b = __builtin_convertvector(v, bf16x2_t);
    return (short)(__builtin_bit_cast(uint32_t, b) & 0xFFFFu);
}
// max(acc + b, 0) of a C tile as the BF16 B operand of the next layer
__device__ __forceinline__ bf16x4 relu_bf16(f32x4 acc, const float* b) {
    const f32x2 lo = {fmaxf(acc[0] + b[0], 0.f), fmaxf(acc[1] + b[1], 0.f)};
    const f32x2 hi = {fmaxf(acc[2] + b[2], 0.f), fmaxf(acc[3] + b[3], 0.f)};
    const uint32_t l = __builtin_bit_cast(uint32_t, __builtin_convertvector(lo, bf16x2_t));
    const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(hi, bf16x2_t));
    bf16x4 r;
    r[0] = (short)(l & 0xFFFFu);
    r[1] = (short)(l >> 16);
    r[2] = (short)(h & 0xFFFFu);
    r[3] = (short)(h >> 16);
    return r;
}
__device__ __forceinline__ float bf16_value(short b) {
    return __uint_as_float(((uint32_t)(uint16_t)b) << 16);
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Weights of one workgroup in LDS as BF16: W1 (64 x 16, inputs 8..15 zero),
// W2 (64 x 64), W3 padded to 16 x 64 (rows 1..15 zero).
struct MlpLds {
    short w1[kHid][16];
    short w2[kHid][kHid];
    short w3[kHid];
};

__device__ void stage_weights(const float* __restrict__ params, MlpLds& L) {
    for (int i = threadIdx.x; i < kHid * 16; i += blockDim.x) {
        const int o = i / 16, k = i % 16;
        L.w1[o][k] = k < kIn ? bf16_bits(params[kOffW1 + o * kIn + k]) : (short)0;
    }
    for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x)
        L.w2[i / kHid][i % kHid] = bf16_bits(params[kOffW2 + i]);
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) L.w3[i] = bf16_bits(params[kOffW3 + i]);
}

// A tile of W (rows m0.., cols k0..) in the A layout.
__device__ __forceinline__ bf16x4 a_tile_w1(const MlpLds& L, int p, int g, int c) {
    bf16x4 a;
    for (int e = 0; e < 4; ++e) a[e] = L.w1[16 * p + c][4 * g + e];
    return a;
}
__device__ __forceinline__ bf16x4 a_tile_w2(const MlpLds& L, int q, int p, int g, int c) {
    bf16x4 a;
    for (int e = 0; e < 4; ++e) a[e] = L.w2[16 * q + c][16 * p + 4 * g + e];
    return a;
}
__device__ __forceinline__ bf16x4 a_tile_w2t(const MlpLds& L, int p, int q, int g, int c) {
    // rows of W2^T = input units 16p + c, columns = output units 16q + 4g + e
    bf16x4 a;
    for (int e = 0; e < 4; ++e) a[e] = L.w2[16 * q + 4 * g + e][16 * p + c];
    return a;
}
__device__ __forceinline__ bf16x4 a_tile_w3(const MlpLds& L, int q, int g, int c) {
    bf16x4 a;
    for (int e = 0; e < 4; ++e) a[e] = c == 0 ? L.w3[16 * q + 4 * g + e] : (short)0;
    return a;
}

// Forward of one tile of 16 Gaussians (columns).  X: standardised features
// [n][8].  Returns the prediction of column c in every lane of column c, and
// keeps the pre-activations (Z1, Z2) and the BF16 activations for a backward.
struct FwdTile {
    f32x4 z1[4], z2[4];   // pre-activations, C layout
    bf16x4 h1[4], h2[4];  // BF16 activations = B operands of the next layer
    bf16x4 x;             // BF16 input, B operand
    float pred;
};

__device__ __forceinline__ void mlp_tile_forward(const float* __restrict__ X, int64_t n,
                                                 int64_t n0, const bf16x4* w1, const bf16x4* w2,
                                                 const bf16x4* w3,
                                                 const float* __restrict__ params,
                                                 FwdTile& f) {
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    const int64_t col = n0 + c;
    for (int e = 0; e < 4; ++e) {
        const int k = 4 * g + e;
        const float v = (k < kIn && col < n) ? X[col * kIn + k] : 0.f;
        f.x[e] = bf16_bits(v);
    }
    for (int p = 0; p < 4; ++p) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(w1[p], f.x, acc);
        for (int e = 0; e < 4; ++e) {
            const float z = acc[e] + params[kOffB1 + 16 * p + 4 * g + e];
            f.z1[p][e] = z;
            f.h1[p][e] = bf16_bits(fmaxf(z, 0.f));
        }
    }
    for (int q = 0; q < 4; ++q) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int p = 0; p < 4; ++p) acc = mfma(w2[4 * q + p], f.h1[p], acc);
        for (int e = 0; e < 4; ++e) {
            const float z = acc[e] + params[kOffB2 + 16 * q + 4 * g + e];
            f.z2[q][e] = z;
            f.h2[q][e] = bf16_bits(fmaxf(z, 0.f));
        }
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int q = 0; q < 4; ++q) acc = mfma(w3[q], f.h2[q], acc);
    // row 0 of the output tile sits in lanes g == 0, element 0
    const float out = acc[0] + params[kOffB3];
    f.pred = __shfl(out, c, 64);
}

__global__ __launch_bounds__(kMlpThreads) void k_mlp_forward(
    const float* __restrict__ params, const float* __restrict__ X, int64_t n,
    gs_mlp_norm norm, int radius_mode, float* __restrict__ out) {
    __shared__ MlpLds L;
    stage_weights(params, L);
    __syncthreads();
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    bf16x4 w1[4], w2[16], w3[4];
    for (int p = 0; p < 4; ++p) w1[p] = a_tile_w1(L, p, g, c);
    for (int q = 0; q < 4; ++q)
        for (int p = 0; p < 4; ++p) w2[4 * q + p] = a_tile_w2(L, q, p, g, c);
    for (int q = 0; q < 4; ++q) w3[q] = a_tile_w3(L, q, g, c);
    const int64_t wave = ((int64_t)blockIdx.x * kMlpThreads + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * kMlpThreads) >> 6;
    for (int64_t n0 = wave * 16; n0 < n; n0 += nwaves * 16) {
        FwdTile f;
        mlp_tile_forward(X, n, n0, w1, w2, w3, params, f);
        const int64_t col = n0 + c;
        if (g == 0 && col < n) {
            float r = f.pred;
            if (radius_mode) {
                bool inside = isfinite(r);
                for (int k = 0; k < kIn; ++k) {
                    const float v = X[col * kIn + k];
                    inside = inside && v >= norm.fmin[k] && v <= norm.fmax[k];
                }
                r = inside ? fminf(fmaxf(r + norm.margin, 0.f), 3.f) : 3.f;
            }
            out[col] = r;
        }
    }
}

// Transposes a C-layout 16x16 tile (rows 4g+e, column c) into an A-layout
// tile (row c, columns 4g+e) through a per-wave LDS scratch.
__device__ __forceinline__ bf16x4 c_to_a(short (*buf)[16], const bf16x4 v) {
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    for (int e = 0; e < 4; ++e) buf[4 * g + e][c] = v[e];
    __threadfence_block();  // the wave's LDS writes complete before the reads
    bf16x4 a;
    for (int e = 0; e < 4; ++e) a[e] = buf[c][4 * g + e];
    __threadfence_block();  // reads complete before the scratch is reused
    return a;
}

// One batch gradient.  mode 0: pinball loss on labels (quantile q, mean over
// n_total); mode 1: upstream gradient dout given.  Each wave accumulates its
// Gaussian tiles and writes its partial gradient (flat layout) to
// partials[wave][kMlpParams]; k_grad_reduce sums the waves in a fixed order.
__global__ __launch_bounds__(kMlpThreads) void k_mlp_grad(
    const float* __restrict__ params, const float* __restrict__ X,
    const float* __restrict__ labels, const float* __restrict__ dout, int64_t n, float q,
    int mode, float* __restrict__ partials, double* __restrict__ loss_sum) {
    __shared__ MlpLds L;
    __shared__ short tbuf[kMlpThreads / 64][16][16];
    stage_weights(params, L);
    __syncthreads();
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15, wv = threadIdx.x >> 6;
    bf16x4 w1[4], w2[16], w3[4];
    for (int p = 0; p < 4; ++p) w1[p] = a_tile_w1(L, p, g, c);
    for (int qq = 0; qq < 4; ++qq)
        for (int p = 0; p < 4; ++p) w2[4 * qq + p] = a_tile_w2(L, qq, p, g, c);
    for (int qq = 0; qq < 4; ++qq) w3[qq] = a_tile_w3(L, qq, g, c);
    short (*buf)[16] = tbuf[wv];

    f32x4 dW2[16], dW1[4];
    for (int i = 0; i < 16; ++i) dW2[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < 4; ++i) dW1[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dW3[4][4], db2[4][4], db1[4][4], db3 = 0.f;
    for (int i = 0; i < 4; ++i)
        for (int e = 0; e < 4; ++e) dW3[i][e] = db2[i][e] = db1[i][e] = 0.f;
    double lsum = 0.0;

    const int64_t wave = ((int64_t)blockIdx.x * kMlpThreads + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * kMlpThreads) >> 6;
    const float inv_n = 1.0f / (float)n;
    for (int64_t n0 = wave * 16; n0 < n; n0 += nwaves * 16) {
        FwdTile f;
        mlp_tile_forward(X, n, n0, w1, w2, w3, params, f);
        const int64_t col = n0 + c;
        const bool live = col < n;
        float d = 0.f;
        if (live) {
            if (mode == 0) {
                const float u = labels[col] - f.pred;
                d = (u > 0.f ? -q : 1.f - q) * inv_n;
                if (g == 0) lsum += (double)(u > 0.f ? q * u : (q - 1.f) * u);
            } else {
                d = dout[col];
            }
        }
        const float d3b = bf16_value(bf16_bits(d));
        if (g == 0) db3 += d;
        // layer 3: dW3[k] += d3b * h2[k];  dZ2 = d3b * W3[k] * (z2 > 0)
        bf16x4 dz2b[4];
        for (int qq = 0; qq < 4; ++qq) {
            for (int e = 0; e < 4; ++e) {
                const int k = 16 * qq + 4 * g + e;
                dW3[qq][e] += d3b * bf16_value(f.h2[qq][e]);
                const float dz = f.z2[qq][e] > 0.f ? d3b * bf16_value(L.w3[k]) : 0.f;
                db2[qq][e] += dz;
                dz2b[qq][e] = bf16_bits(dz);
            }
        }
        // dH1 = W2^T dZ2 (matrix cores), dZ1 = dH1 * (z1 > 0)
        bf16x4 dz1b[4];
        for (int p = 0; p < 4; ++p) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int qq = 0; qq < 4; ++qq) acc = mfma(a_tile_w2t(L, p, qq, g, c), dz2b[qq], acc);
            for (int e = 0; e < 4; ++e) {
                const float dz = f.z1[p][e] > 0.f ? acc[e] : 0.f;
                db1[p][e] += dz;
                dz1b[p][e] = bf16_bits(dz);
            }
        }
        // weight gradients: the batch is the reduction dimension
        bf16x4 h1t[4];  // B operand: H1^T tile p (rows = Gaussians, cols = units)
        for (int p = 0; p < 4; ++p) h1t[p] = c_to_a(buf, f.h1[p]);
        for (int qq = 0; qq < 4; ++qq) {
            const bf16x4 a = c_to_a(buf, dz2b[qq]);  // dZ2 tile as A (units x Gaussians)
            for (int p = 0; p < 4; ++p) dW2[4 * qq + p] = mfma(a, h1t[p], dW2[4 * qq + p]);
        }
        // X^T as B: rows = Gaussians 4g+e, column c = feature
        bf16x4 xb;
        for (int e = 0; e < 4; ++e) {
            const int64_t cc = n0 + 4 * g + e;
            xb[e] = (c < kIn && cc < n) ? bf16_bits(X[cc * kIn + c]) : (short)0;
        }
        for (int p = 0; p < 4; ++p) {
            const bf16x4 a = c_to_a(buf, dz1b[p]);
            dW1[p] = mfma(a, xb, dW1[p]);
        }
    }

    // reduce the per-lane vector sums over the 16 columns of each lane group
    for (int o = 1; o < 16; o <<= 1) {
        for (int i = 0; i < 4; ++i)
            for (int e = 0; e < 4; ++e) {
                dW3[i][e] += __shfl_xor(dW3[i][e], o, 64);
                db2[i][e] += __shfl_xor(db2[i][e], o, 64);
                db1[i][e] += __shfl_xor(db1[i][e], o, 64);
            }
    }
    for (int o = 1; o < 64; o <<= 1) {
        db3 += __shfl_xor(db3, o, 64);
        lsum += __shfl_xor(lsum, o, 64);
    }
    float* P = partials + wave * kMlpParams;
    // dW2, dW1 in C layout: tile (q, p) element e -> row 16q + 4g + e, col 16p + c
    for (int qq = 0; qq < 4; ++qq)
        for (int p = 0; p < 4; ++p)
            for (int e = 0; e < 4; ++e)
                P[kOffW2 + (16 * qq + 4 * g + e) * kHid + 16 * p + c] = dW2[4 * qq + p][e];
    for (int p = 0; p < 4; ++p)
        for (int e = 0; e < 4; ++e)
            if (c < kIn) P[kOffW1 + (16 * p + 4 * g + e) * kIn + c] = dW1[p][e];
    if (c == 0) {
        for (int i = 0; i < 4; ++i)
            for (int e = 0; e < 4; ++e) {
                const int k = 16 * i + 4 * g + e;
                P[kOffW3 + k] = dW3[i][e];
                P[kOffB2 + k] = db2[i][e];
                P[kOffB1 + k] = db1[i][e];
            }
    }
    if (l == 0) {
        P[kOffB3] = db3;
        if (loss_sum) atomicAdd(loss_sum, lsum / (double)n);
    }
}

__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ partials,
                                                     int64_t nwaves, float* __restrict__ grad) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kMlpParams) return;
    float s = 0.f;
    for (int64_t w = 0; w < nwaves; ++w) s += partials[w * kMlpParams + i];
    grad[i] = s;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ m,
                                              float* __restrict__ v,
                                              const float* __restrict__ grad, int t, float lr,
                                              float b1, float b2, float eps) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kMlpParams) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.f - powf(b1, (float)t));
    const float vh = vi / (1.f - powf(b2, (float)t));
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// The image a Gaussian belongs to (images hold ascending Gaussian ranges).
template <typename Table>
__device__ __forceinline__ int image_of(const Table& imgs, int n_img, int64_t i) {
    int lo = 0, hi = n_img - 1, k = 0;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        if (imgs[mid].g_begin <= i) { k = mid; lo = mid + 1; } else { hi = mid - 1; }
    }
    return k;
}

// Raw features of a Gaussian at scale s: [log s, log sigma_x, log sigma_y,
// rho, alpha, c_r, c_g, c_b] with sigma_x = l11, sigma_y = sqrt(l21^2 + l22^2),
// rho = l21 / sigma_y (fixed operation order: the same bits wherever used).
// Features 0..3 from (s, l11, l21, l22), features 4..7 from (alpha, c).
__device__ __forceinline__ void shape_features(double s, float l11, float l21, float l22,
                                               float* f) {
    const float sy = sqrtf(__builtin_fmaf(l21, l21, l22 * l22));
    f[0] = logf((float)s);
    f[1] = logf(l11);
    f[2] = logf(sy);
    f[3] = l21 / sy;
}

__device__ __forceinline__ float standardised(float f, int k, const gs_mlp_norm& norm) {
    return (f - norm.mu[k]) / norm.sd[k];
}

// Features of every Gaussian, standardised: (f - mu) / sd.
template <typename Table>
__global__ __launch_bounds__(256) void k_mlp_features(Table imgs, int n_img, int64_t n_gauss,
                                                      const float* __restrict__ chol,
                                                      const float* __restrict__ color,
                                                      const float* __restrict__ opacity,
                                                      gs_mlp_norm norm, int standardise,
                                                      float* __restrict__ X) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_gauss) return;
    const double s = imgs[image_of(imgs, n_img, i)].scale;
    float f[kIn];
    shape_features(s, chol[3 * i], chol[3 * i + 1], chol[3 * i + 2], f);
    f[4] = opacity[i];
    f[5] = color[3 * i];
    f[6] = color[3 * i + 1];
    f[7] = color[3 * i + 2];
    for (int j = 0; j < kIn; ++j) X[i * kIn + j] = standardise ? standardised(f[j], j, norm) : f[j];
}

// Features, MLP forward and pruned radius in one kernel: per tile of 16
// Gaussians, lane (g, c) forms features 4g..4g+3 of Gaussian c (the MFMA B
// operand) straight from the Gaussian parameters; the range check combines
// lanes g = 0 and 1.  Same bits as k_mlp_features + k_mlp_forward.
constexpr int kRadiusThreads = 1024;  // one workgroup per CU shares the staged weights

template <typename Table>
__global__ __launch_bounds__(kRadiusThreads) void k_mlp_radius(
    Table imgs, int n_img, int64_t n, const float* __restrict__ chol,
    const float* __restrict__ color, const float* __restrict__ opacity,
    const float* __restrict__ params, gs_mlp_norm norm, float* __restrict__ out) {
    __shared__ MlpLds L;
    stage_weights(params, L);
    __syncthreads();
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    bf16x4 w1[4], w2[16], w3[4];
    for (int p = 0; p < 4; ++p) w1[p] = a_tile_w1(L, p, g, c);
    for (int q = 0; q < 4; ++q)
        for (int p = 0; p < 4; ++p) w2[4 * q + p] = a_tile_w2(L, q, p, g, c);
    for (int q = 0; q < 4; ++q) w3[q] = a_tile_w3(L, q, g, c);
    float b1[4][4], b2[4][4];
    for (int p = 0; p < 4; ++p)
        for (int e = 0; e < 4; ++e) {
            b1[p][e] = params[kOffB1 + 16 * p + 4 * g + e];
            b2[p][e] = params[kOffB2 + 16 * p + 4 * g + e];
        }
    const float b3 = params[kOffB3];
    // this lane's four features' standardisation and range, in registers (an
    // index into the by-value struct would read it from memory every tile)
    float nmu[4], nsd[4], nlo[4], nhi[4];
    for (int e = 0; e < 4; ++e) {
        const int k = g < 2 ? 4 * g + e : 0;
        nmu[e] = norm.mu[k];
        nsd[e] = norm.sd[k];
        nlo[e] = norm.fmin[k];
        nhi[e] = norm.fmax[k];
    }
    const float margin = norm.margin;
    const int64_t wave = ((int64_t)blockIdx.x * kRadiusThreads + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * kRadiusThreads) >> 6;
    // lanes g = 0 read (l11, l21, l22, scale), lanes g = 1 (alpha, c): the raw
    // values of the next tile are loaded while the current one is computed
    auto fetch = [&](int64_t n0, float* v, double* s) {
        const int64_t col = n0 + c;
        v[0] = v[1] = v[2] = v[3] = 0.f;
        *s = 1.0;
        if (col >= n) return;
        if (g == 0) {
            v[0] = chol[3 * col]; v[1] = chol[3 * col + 1]; v[2] = chol[3 * col + 2];
            *s = imgs[image_of(imgs, n_img, col)].scale;
        } else if (g == 1) {
            v[0] = opacity[col]; v[1] = color[3 * col]; v[2] = color[3 * col + 1];
            v[3] = color[3 * col + 2];
        }
    };
    float nv[4];
    double ns;
    fetch(wave * 16, nv, &ns);
    for (int64_t n0 = wave * 16; n0 < n; n0 += nwaves * 16) {
        const int64_t col = n0 + c;
        float rv[4] = {nv[0], nv[1], nv[2], nv[3]};
        const double rs = ns;
        fetch(n0 + nwaves * 16, nv, &ns);
        bf16x4 x;
        bool inside = true;
        if (g < 2 && col < n) {
            float f[4];
            if (g == 0) shape_features(rs, rv[0], rv[1], rv[2], f);
            else { f[0] = rv[0]; f[1] = rv[1]; f[2] = rv[2]; f[3] = rv[3]; }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float v = (f[e] - nmu[e]) / nsd[e];
                inside = inside && v >= nlo[e] && v <= nhi[e];
                x[e] = bf16_bits(v);
            }
        } else {
            for (int e = 0; e < 4; ++e) x[e] = 0;
        }
        bf16x4 h1[4], h2[4];
        for (int p = 0; p < 4; ++p) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma(w1[p], x, acc);
            h1[p] = relu_bf16(acc, b1[p]);
        }
        for (int q = 0; q < 4; ++q) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int p = 0; p < 4; ++p) acc = mfma(w2[4 * q + p], h1[p], acc);
            h2[q] = relu_bf16(acc, b2[q]);
        }
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int q = 0; q < 4; ++q) acc = mfma(w3[q], h2[q], acc);
        const float pred = acc[0] + b3;  // row 0 of the output tile: lanes g == 0
        const bool in_hi = __shfl_xor((int)inside, 16, 64) != 0;  // features 4..7
        if (g == 0 && col < n) {
            float r = pred;
            r = (inside && in_hi && isfinite(r)) ? fminf(fmaxf(r + margin, 0.f), 3.f) : 3.f;
            out[col] = r;
        }
    }
}

// Labels from the exact rasterizer's render records (workspace of a forward
// with the exact 3-sigma boxes): per Gaussian, walk its box and keep the
// largest z1^2 + z2^2 among pixels with max_c(A_c) * w >= tau (A_c =
// alpha c_c K, w = exp(-(z1^2 + z2^2) / 2)); FP32 bits in best.  With
// interior_only, a Gaussian whose box the image border cut gets -1 (its
// label would be cut too).
__global__ __launch_bounds__(256) void k_radius_stats(const GRec* __restrict__ recs,
                                                      int64_t n, float tau, int interior_only,
                                                      uint32_t* __restrict__ best) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const GRec r = recs[i];
    float m = 0.f;
    if (r.x0 <= r.x1 && r.y0 <= r.y1 && !(r.flags & kRecNoAmp)) {
        const float amax = fmaxf(r.A[0], fmaxf(r.A[1], r.A[2]));
        const float inv_kc2 = (float)(1.0 / (kZScale * kZScale));
        for (int y = r.y0; y <= r.y1; ++y) {
            const float Y = (float)(y - r.ky) - r.fy;
            for (int x = r.x0; x <= r.x1; ++x) {
                const float X = (float)(x - r.kx) - r.fx;
                const float z1 = r.a * X, z2 = r.e * Y - r.g * X;
                const float q = z1 * z1 + z2 * z2;
                if (amax * __builtin_amdgcn_exp2f(-q) >= tau) m = fmaxf(m, q * inv_kc2);
            }
        }
    }
    if (interior_only && (r.flags & kRecClipped)) m = -1.f;
    best[i] = __float_as_uint(m);
}

__global__ __launch_bounds__(256) void k_sqrt_labels(const uint32_t* __restrict__ best,
                                                     int64_t n, float* __restrict__ R) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float v = __uint_as_float(best[i]);
    R[i] = v < 0.f ? -1.f : sqrtf(v);
}

// The closed-form support radius of the method without the learned part:
// the Mahalanobis distance d at which a Gaussian's own peak contribution
// alpha max(c) K exp(-d^2 / 2) (Eq. 1, 2; K = 1 / (2 pi sigma_x sigma_y
// sqrt(1 - rho^2)) = 1 / (2 pi l11 l22)) falls to tau, plus a margin, capped
// at 3: R = min(sqrt(2 ln(max(alpha max(c) K / tau, 1))) + margin, 3).
// Invalid values give 3 (the exact box decides).
__global__ __launch_bounds__(256) void k_closed_form_radius(
    const float* __restrict__ chol, const float* __restrict__ color,
    const float* __restrict__ opacity, int64_t n, double tau, double margin,
    float* __restrict__ R) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double l11 = chol[3 * i], l22 = chol[3 * i + 2];
    const double al = opacity[i];
    const double cm = fmax((double)color[3 * i], fmax((double)color[3 * i + 1],
                                                      (double)color[3 * i + 2]));
    const double K = 1.0 / (2.0 * 3.14159265358979323846 * l11 * l22);
    const double ratio = al * cm * K / tau;
    double r = 3.0;
    if (l11 > 0.0 && l22 > 0.0 && __builtin_isfinite(ratio)) {
        r = sqrt(2.0 * log(fmax(ratio, 1.0))) + margin;
        r = fmin(fmax(r, 0.0), 3.0);
    }
    R[i] = (float)r;
}

__global__ __launch_bounds__(256) void k_sq_error(const float* __restrict__ a,
                                                  const float* __restrict__ b, int64_t n,
                                                  double* __restrict__ sum) {
    __shared__ double part[4];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const double d = (double)a[i] - (double)b[i];
        s += d * d;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(sum, part[0] + part[1] + part[2] + part[3]);
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

int64_t mlp_grad_waves(int64_t n) {
    // enough waves to fill the chip, each with several 16-Gaussian tiles
    int64_t tiles = (n + 15) / 16;
    int64_t waves = tiles < 1024 ? tiles : 1024;
    return waves < 4 ? 4 : (waves + 3) / 4 * 4;
}

hipError_t launch_mlp_features(const Layout& L, const Ws& w, const float* chol,
                               const float* color, const float* opacity,
                               const gs_mlp_norm& norm, int standardise, float* X,
                               hipStream_t st) {
    if (L.n_gauss == 0) return hipSuccess;
    const dim3 grid(blocks_for(L.n_gauss, 256));
    if (L.n_img <= kSetupChunk && L.host_imgs) {
        ArgTable tab;
        for (int k = 0; k < kSetupChunk; ++k) tab.c.img[k] = k < L.n_img ? L.host_imgs[k] : ImgDev{};
        hipLaunchKernelGGL(k_mlp_features<ArgTable>, grid, dim3(256), 0, st, tab, L.n_img,
                           L.n_gauss, chol, color, opacity, norm, standardise, X);
    } else {
        hipLaunchKernelGGL(k_mlp_features<MemTable>, grid, dim3(256), 0, st, MemTable{w.imgs},
                           L.n_img, L.n_gauss, chol, color, opacity, norm, standardise, X);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_radius(const Layout& L, const Ws& w, const float* params,
                             const float* chol, const float* color, const float* opacity,
                             const gs_mlp_norm& norm, float* out, hipStream_t st) {
    if (L.n_gauss == 0) return hipSuccess;
    const int64_t tiles = (L.n_gauss + 15) / 16;
    int nb = (int)((tiles + 63) / 64);  // 16 waves, about four tiles each
    if (nb > 256) nb = 256;
    if (nb < 1) nb = 1;
    if (L.n_img <= kSetupChunk && L.host_imgs) {
        ArgTable tab;
        for (int k = 0; k < kSetupChunk; ++k) tab.c.img[k] = k < L.n_img ? L.host_imgs[k] : ImgDev{};
        hipLaunchKernelGGL(k_mlp_radius<ArgTable>, dim3(nb), dim3(kRadiusThreads), 0, st, tab,
                           L.n_img, L.n_gauss, chol, color, opacity, params, norm, out);
    } else {
        hipLaunchKernelGGL(k_mlp_radius<MemTable>, dim3(nb), dim3(kRadiusThreads), 0, st,
                           MemTable{w.imgs}, L.n_img, L.n_gauss, chol, color, opacity, params,
                           norm, out);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* params, const float* X, int64_t n,
                              const gs_mlp_norm& norm, int radius_mode, float* out,
                              hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int64_t tiles = (n + 15) / 16;
    int nb = (int)((tiles + 3) / 4);
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(k_mlp_forward, dim3(nb), dim3(kMlpThreads), 0, st, params, X, n, norm,
                       radius_mode, out);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* params, const float* X, const float* labels,
                           const float* dout, int64_t n, float q, float* partials,
                           float* grad, double* loss_sum, hipStream_t st) {
    const int64_t waves = mlp_grad_waves(n);
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)(waves / 4)), dim3(kMlpThreads), 0, st,
                       params, X, labels, dout, n, q, labels ? 0 : 1, partials, loss_sum);
    hipLaunchKernelGGL(k_grad_reduce, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, st,
                       partials, waves, grad);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* grad, int t, float lr,
                       float b1, float b2, float eps, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, st, p, m, v,
                       grad, t, lr, b1, b2, eps);
    return hipGetLastError();
}

hipError_t launch_radius_stats(const Layout& L, const Ws& w, float tau, int interior_only,
                               float* R, hipStream_t st) {
    uint32_t* best = reinterpret_cast<uint32_t*>(R);  // FP32 bits, then sqrt in place
    if (L.n_gauss == 0) return hipSuccess;
    hipLaunchKernelGGL(k_radius_stats, dim3(blocks_for(L.n_gauss, 256)), dim3(256), 0, st,
                       w.recs, L.n_gauss, tau, interior_only, best);
    hipLaunchKernelGGL(k_sqrt_labels, dim3(blocks_for(L.n_gauss, 256)), dim3(256), 0, st,
                       best, L.n_gauss, R);
    return hipGetLastError();
}

hipError_t launch_closed_form_radius(const float* chol, const float* color,
                                    const float* opacity, int64_t n, double tau, double margin,
                                    float* R, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_closed_form_radius, dim3(blocks_for(n, 256)), dim3(256), 0, st, chol,
                       color, opacity, n, tau, margin, R);
    return hipGetLastError();
}

hipError_t launch_sq_error(const float* a, const float* b, int64_t n, double* sum,
                           hipStream_t st) {
    if (n == 0) return hipSuccess;
    int nb = blocks_for(n, 256 * 8);
    if (nb > 256) nb = 256;
    hipLaunchKernelGGL(k_sq_error, dim3(nb), dim3(256), 0, st, a, b, n, sum);
    return hipGetLastError();
}

}  // namespace gs
