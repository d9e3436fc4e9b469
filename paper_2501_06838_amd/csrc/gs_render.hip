// Per-tile forward and backward evaluation for the gfx950 rasterizer.
//
// Forward (Eq. 1, 2, 4): one workgroup per T x T HR tile.  Each round stages
// up to one Gaussian per thread of the tile's sorted list in LDS, builds for
// every 8 x 8 pixel block of the tile the compacted list of staged Gaussians
// touching it together with the 64-bit lane mask of the block's pixels inside
// the support box, and then every wave sums, for each of its pixels, the
// listed Gaussians in ascending index: lane = pixel, wave-uniform Gaussian,
// out-of-box lanes masked by the SGPR lane mask (no per-pixel compare).
// Planar stores of the finished tile are coalesced along rows.
//
// Backward: one workgroup per tile.  The tile's upstream gradient is staged
// in LDS; the (Gaussian, pixel) pairs of each round are flattened (box area
// prefix sums in LDS) and split into equal contiguous chunks, one per lane,
// so every lane does the same number of pair evaluations whatever the box
// sizes.  A lane accumulates the eight per-Gaussian moments in registers,
// flushes them into the round's LDS accumulators when it leaves a Gaussian,
// and the workgroup issues one FP32 global atomic per (tile, Gaussian,
// moment).  The finalize kernel turns moments into parameter gradients.
#include "gs_internal.h"

namespace gs {

namespace {

__device__ __forceinline__ int tile_image(const ImgDev* imgs, int n_img, int64_t tile) {
    int lo = 0, hi = n_img - 1, ans = 0;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        if (imgs[mid].tile_base <= tile) { ans = mid; lo = mid + 1; } else { hi = mid - 1; }
    }
    return ans;
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ uint64_t rows_mask(int r0, int r1) {
    // bits [8 r0, 8 (r1 + 1)) of a 64-bit word, 0 <= r0 <= r1 <= 7
    const uint64_t hi = (r1 >= 7) ? ~0ull : ((1ull << (8 * (r1 + 1))) - 1ull);
    const uint64_t lo = (1ull << (8 * r0)) - 1ull;
    return hi & ~lo;
}

template <int T>
struct TileShape {
    static constexpr int kThreads = (T * T >= 256) ? 256 : T * T;
    static constexpr int kWaves = kThreads / 64;
    static constexpr int kBlocksX = T / 8;
    static constexpr int kBlocks = kBlocksX * kBlocksX;
    static constexpr int kBlocksPerWave = kBlocks / kWaves;
    static constexpr int kBatch = kThreads;
};

template <int T>
__global__ __launch_bounds__(TileShape<T>::kThreads) void k_render_fwd(
    const ImgDev* __restrict__ imgs, int n_img, const GRec* __restrict__ recs,
    const uint32_t* __restrict__ gids, const int2* __restrict__ ranges,
    float* __restrict__ out) {
    using S = TileShape<T>;
    constexpr int NB = S::kBlocks, B = S::kBatch;
    __shared__ float4 sp0[B];          // {x-origin minus kx, y-origin minus ky, fx, fy}
    __shared__ float4 sp1[B];          // {a, e, g, A0}
    __shared__ float2 sp2[B];          // {A1, A2}
    __shared__ uint64_t smask[NB][B];  // compacted lane masks per 8x8 block
    __shared__ uint16_t slist[NB][B];  // compacted staged indices per block
    __shared__ int scount[NB];
    __shared__ int wcount[S::kWaves][NB];

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t tile = blockIdx.x;
    const int k_img = tile_image(imgs, n_img, tile);
    const ImgDev im = imgs[k_img];
    const int64_t lt = tile - im.tile_base;
    const int px0 = (int)(lt % im.tiles_x) * T, py0 = (int)(lt / im.tiles_x) * T;
    const int2 rg = ranges[tile];

    float acc[S::kBlocksPerWave][3];
    float dxf[S::kBlocksPerWave], dyf[S::kBlocksPerWave];
#pragma unroll
    for (int m = 0; m < S::kBlocksPerWave; ++m) {
        const int j = wave + S::kWaves * m;
        dxf[m] = (float)((j % S::kBlocksX) * 8 + (lane & 7));
        dyf[m] = (float)((j / S::kBlocksX) * 8 + (lane >> 3));
        acc[m][0] = acc[m][1] = acc[m][2] = 0.f;
    }

    for (int base = rg.x; base < rg.y; base += B) {
        const int nb = min(B, rg.y - base);
        uint64_t my_mask[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) my_mask[j] = 0;
        if (t < nb) {
            const GRec r = recs[gids[base + t]];
            const int lx0 = max(r.x0 - px0, 0), lx1 = min(r.x1 - px0, T - 1);
            const int ly0 = max(r.y0 - py0, 0), ly1 = min(r.y1 - py0, T - 1);
            sp0[t] = make_float4((float)(px0 - r.kx), (float)(py0 - r.ky), r.fx, r.fy);
            sp1[t] = make_float4(r.a, r.e, r.g, r.A[0]);
            sp2[t] = make_float2(r.A[1], r.A[2]);
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int bx = (j % S::kBlocksX) * 8, by = (j / S::kBlocksX) * 8;
                const int c0 = max(lx0, bx) - bx, c1 = min(lx1, bx + 7) - bx;
                const int r0 = max(ly0, by) - by, r1 = min(ly1, by + 7) - by;
                if (c0 <= c1 && r0 <= r1) {
                    const uint64_t cols = ((1ull << (c1 - c0 + 1)) - 1ull) << c0;
                    my_mask[j] = (cols * 0x0101010101010101ull) & rows_mask(r0, r1);
                }
            }
        }
        // compaction, preserving the staged (ascending Gaussian) order
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const uint64_t bal = __ballot(my_mask[j] != 0);
            if (lane == 0) wcount[wave][j] = __popcll(bal);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const uint64_t bal = __ballot(my_mask[j] != 0);
            if (my_mask[j] != 0) {
                int pos = __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
                for (int w = 0; w < wave; ++w) pos += wcount[w][j];
                slist[j][pos] = (uint16_t)t;
                smask[j][pos] = my_mask[j];
            }
        }
        if (t < NB) {
            int c = 0;
            for (int w = 0; w < S::kWaves; ++w) c += wcount[w][t];
            scount[t] = c;
        }
        __syncthreads();

#pragma unroll
        for (int m = 0; m < S::kBlocksPerWave; ++m) {
            const int j = wave + S::kWaves * m;
            const int cnt = scount[j];
            for (int q = 0; q < cnt; ++q) {
                const int k = __builtin_amdgcn_readfirstlane(slist[j][q]);
                const uint64_t mk = smask[j][q];
                const uint32_t mlo = __builtin_amdgcn_readfirstlane((uint32_t)mk);
                const uint32_t mhi = __builtin_amdgcn_readfirstlane((uint32_t)(mk >> 32));
                const uint64_t mask = ((uint64_t)mhi << 32) | mlo;
                const float4 p0 = sp0[k];
                const float4 p1 = sp1[k];
                const float2 p2 = sp2[k];
                const float X = (p0.x + dxf[m]) - p0.z;
                const float Y = (p0.y + dyf[m]) - p0.w;
                const float z1 = p1.x * X;
                const float z2 = p1.y * Y - p1.z * X;
                float w = fast_exp2(-(z1 * z1 + z2 * z2));
                w = __builtin_amdgcn_inverse_ballot_w64(mask) ? w : 0.f;
                acc[m][0] += p1.w * w;
                acc[m][1] += p2.x * w;
                acc[m][2] += p2.y * w;
            }
        }
        __syncthreads();
    }

    const int64_t plane = (int64_t)im.out_w * im.out_h;
    float* o = out + im.out_offset;
#pragma unroll
    for (int m = 0; m < S::kBlocksPerWave; ++m) {
        const int x = px0 + (int)dxf[m], y = py0 + (int)dyf[m];
        if (x < im.out_w && y < im.out_h) {
            const int64_t p = (int64_t)y * im.out_w + x;
            o[p] = acc[m][0];
            o[plane + p] = acc[m][1];
            o[2 * plane + p] = acc[m][2];
        }
    }
}

// kL1: the upstream gradient is the L1 loss's, sign(out - target) / numel,
// formed here from the rendered image and the target (it is never stored),
// and the tile's share of sum |out - target| goes to tile_loss[tile].
template <int T, bool kL1>
__global__ __launch_bounds__(TileShape<T>::kThreads) void k_render_bwd(
    const ImgDev* __restrict__ imgs, int n_img, const GRec* __restrict__ recs,
    const uint32_t* __restrict__ gids, const int2* __restrict__ ranges,
    const float* __restrict__ grad_out, const float* __restrict__ target, float inv_numel,
    double* __restrict__ tile_loss, float* __restrict__ moments) {
    using S = TileShape<T>;
    constexpr int NT = S::kThreads, B = S::kBatch;
    __shared__ float4 gt[T * T];     // upstream gradient of the tile, {g0, g1, g2, 0}
    __shared__ float4 sq0[B];        // {X at box start, Y at box start, a, e}
    __shared__ float4 sq1[B];        // {g, A0, A1, A2}
    __shared__ int4 sq2[B];          // {first pixel index, box width, area, -}
    __shared__ int pfx[B + 1];
    __shared__ float acc[8][B];      // moment-major: lanes flushing different Gaussians hit different banks
    __shared__ int64_t tmp[NT / 64];

    const int t = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int k_img = tile_image(imgs, n_img, tile);
    const ImgDev im = imgs[k_img];
    const int64_t lt = tile - im.tile_base;
    const int px0 = (int)(lt % im.tiles_x) * T, py0 = (int)(lt / im.tiles_x) * T;
    const int2 rg = ranges[tile];
    if (!kL1 && rg.y <= rg.x) return;  // uniform: nothing listed in this tile

    const int64_t plane = (int64_t)im.out_w * im.out_h;
    const float* g = grad_out + im.out_offset;
    double lsum = 0.0;
    for (int p = t; p < T * T; p += NT) {
        const int x = px0 + (p % T), y = py0 + (p / T);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (x < im.out_w && y < im.out_h) {
            const int64_t q = (int64_t)y * im.out_w + x;
            if (kL1) {
                const float* tg = target + im.out_offset;
                float gv[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float d = g[c * plane + q] - tg[c * plane + q];
                    gv[c] = d > 0.f ? inv_numel : (d < 0.f ? -inv_numel : 0.f);
                    lsum += fabs((double)g[c * plane + q] - (double)tg[c * plane + q]);
                }
                v = make_float4(gv[0], gv[1], gv[2], 0.f);
            } else {
                v = make_float4(g[q], g[plane + q], g[2 * plane + q], 0.f);
            }
        }
        gt[p] = v;
    }
    if (kL1) {
        for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
        __shared__ double lpart[NT / 64];
        if ((t & 63) == 0) lpart[t >> 6] = lsum;
        __syncthreads();
        if (t == 0) {
            double sum = 0.0;
            for (int k = 0; k < NT / 64; ++k) sum += lpart[k];
            tile_loss[tile] = sum;
        }
        if (rg.y <= rg.x) return;  // uniform
    }

    for (int base = rg.x; base < rg.y; base += B) {
        const int nb = min(B, rg.y - base);
        uint32_t my_gid = 0;
        int area = 0;
        if (t < nb) {
            my_gid = gids[base + t];
            const GRec r = recs[my_gid];
            const int lx0 = max(r.x0 - px0, 0), lx1 = min(r.x1 - px0, T - 1);
            const int ly0 = max(r.y0 - py0, 0), ly1 = min(r.y1 - py0, T - 1);
            const int w = lx1 - lx0 + 1, h = ly1 - ly0 + 1;
            area = (r.pad == 0) ? w * h : 0;  // dead Gaussians get nothing
            const float X0 = (float)(px0 + lx0 - r.kx) - r.fx;
            const float Y0 = (float)(py0 + ly0 - r.ky) - r.fy;
            sq0[t] = make_float4(X0, Y0, r.a, r.e);
            sq1[t] = make_float4(r.g, r.A[0], r.A[1], r.A[2]);
            sq2[t] = make_int4(ly0 * T + lx0, w, area, 0);
        }
        // exclusive prefix of box areas (block-wide)
        {
            const int lane = t & 63, wave = t >> 6;
            int v = area;
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(v, o, 64);
                if (lane >= o) v += u;
            }
            if (lane == 63) tmp[wave] = v;
            __syncthreads();
            int carry = 0;
            for (int k = 0; k < wave; ++k) carry += (int)tmp[k];
            pfx[t] = carry + v - area;
            if (t == NT - 1) pfx[NT] = carry + v;
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) acc[m][t] = 0.f;
        __syncthreads();

        const int total = pfx[NT];
        const int L = (total + NT - 1) / NT;
        const int j0 = min(t * L, total), j1 = min(j0 + L, total);
        // Every lane ends with the partial sums of the last Gaussian of its
        // chunk in m0..m7 (key k); Gaussians finished strictly inside the
        // chunk are flushed to LDS on the way (at most one lane of a wave
        // finishes a given Gaussian, so those adds never collide in a wave).
        int key = 0x7fffffff;  // lanes without pairs: never merged with a Gaussian
        float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f, m5 = 0.f, m6 = 0.f, m7 = 0.f;
        if (j0 < j1) {
            // staged entry holding flat pair j0: last k with pfx[k] <= j0
            int lo = 0, hi = nb - 1, k = 0;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                if (pfx[mid] <= j0) { k = mid; lo = mid + 1; } else { hi = mid - 1; }
            }
            // skip empty entries (area 0) sharing the prefix (bounded by nb)
            while (k < nb - 1 && sq2[k].z == 0) ++k;
            float4 q0 = sq0[k], q1 = sq1[k];
            int4 q2 = sq2[k];
            int r = j0 - pfx[k];
            int ry = r / q2.y, rx = r - ry * q2.y;
            int pix = q2.x + ry * T + rx;
            float X = q0.x + (float)rx, Y = q0.y + (float)ry;
            int left = q2.z - r;  // pairs of this Gaussian still to visit
            for (int j = j0; j < j1; ++j) {
                const float4 G = gt[pix];
                const float z1 = q0.z * X;
                const float z2 = q0.w * Y - q1.x * X;
                const float w = fast_exp2(-(z1 * z1 + z2 * z2));
                m0 += G.x * w;
                m1 += G.y * w;
                m2 += G.z * w;
                const float hw = (q1.y * G.x + q1.z * G.y + q1.w * G.z) * w;
                const float t1 = hw * z1, t2 = hw * z2;
                m3 += t1;
                m4 += t2;
                m5 += t1 * z1;
                m6 += t1 * z2;
                m7 += t2 * z2;
                // advance within the box (row-major)
                ++rx;
                ++pix;
                X += 1.0f;
                if (rx == q2.y) {
                    rx = 0;
                    ++ry;
                    pix += T - q2.y;
                    X = q0.x;
                    Y += 1.0f;
                }
                if (--left == 0 && j + 1 < j1) {
                    atomicAdd(&acc[0][k], m0); atomicAdd(&acc[1][k], m1);
                    atomicAdd(&acc[2][k], m2); atomicAdd(&acc[3][k], m3);
                    atomicAdd(&acc[4][k], m4); atomicAdd(&acc[5][k], m5);
                    atomicAdd(&acc[6][k], m6); atomicAdd(&acc[7][k], m7);
                    m0 = m1 = m2 = m3 = m4 = m5 = m6 = m7 = 0.f;
                    do { ++k; } while (k < nb - 1 && sq2[k].z == 0);
                    q0 = sq0[k]; q1 = sq1[k]; q2 = sq2[k];
                    rx = 0; ry = 0; pix = q2.x;
                    X = q0.x; Y = q0.y;
                    left = q2.z;
                }
            }
            key = k;
        }
        // Chunk ends: lanes sharing a last Gaussian are contiguous in the wave
        // (keys ascend with the lane), so a segmented suffix sum leaves each
        // segment's total in its first lane, which alone adds it to LDS.
        {
            const int lane = t & 63;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int kk = __shfl_down(key, o, 64);
                const float v0 = __shfl_down(m0, o, 64), v1 = __shfl_down(m1, o, 64);
                const float v2 = __shfl_down(m2, o, 64), v3 = __shfl_down(m3, o, 64);
                const float v4 = __shfl_down(m4, o, 64), v5 = __shfl_down(m5, o, 64);
                const float v6 = __shfl_down(m6, o, 64), v7 = __shfl_down(m7, o, 64);
                if (lane + o < 64 && kk == key) {
                    m0 += v0; m1 += v1; m2 += v2; m3 += v3;
                    m4 += v4; m5 += v5; m6 += v6; m7 += v7;
                }
            }
            const int kprev = __shfl_up(key, 1, 64);
            if (j0 < j1 && (lane == 0 || kprev != key)) {
                atomicAdd(&acc[0][key], m0); atomicAdd(&acc[1][key], m1);
                atomicAdd(&acc[2][key], m2); atomicAdd(&acc[3][key], m3);
                atomicAdd(&acc[4][key], m4); atomicAdd(&acc[5][key], m5);
                atomicAdd(&acc[6][key], m6); atomicAdd(&acc[7][key], m7);
            }
        }
        __syncthreads();
        if (t < nb && area > 0) {
            float* dst = moments + (int64_t)my_gid * 8;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const float v = acc[m][t];
                if (v != 0.f) atomicAdd(dst + m, v);
            }
        }
        __syncthreads();
    }
}

// Moments -> gradients, per Gaussian, in FP64.  With K = 1/(2 pi l11 l22),
// w = exp(-(z1^2 + z2^2)/2), z1 = (x/s - mu_x)/l11,
// z2 = ((y/s - mu_y) - l21 z1)/l22, H = sum_c A_c dL/dI_c:
//   dL/dA_c = sum G_c w;   S_m = sum H w m for m in {z1, z2, z1^2, z1 z2, z2^2};
//   S_1 = sum_c A_c dL/dA_c;
//   d mu_x = (S_z1 - S_z2 l21/l22)/l11,   d mu_y = S_z2/l22,
//   d l11 = (S_z1z1 - S_1 - S_z1z2 l21/l22)/l11,   d l21 = S_z1z2/l22,
//   d l22 = (S_z2z2 - S_1)/l22,   d c_c = alpha K dL/dA_c,
//   d alpha = K sum_c c_c dL/dA_c.
// The render accumulates z scaled by kc, hence the kc and kc^2 divisions.
__global__ __launch_bounds__(kBlockG) void k_finalize(
    const GRec* __restrict__ recs, int64_t n_gauss, const float* __restrict__ chol,
    const float* __restrict__ color, const float* __restrict__ opacity,
    float* __restrict__ moments, float* __restrict__ grad_mean,
    float* __restrict__ grad_chol, float* __restrict__ grad_color,
    float* __restrict__ grad_opacity) {
    const int64_t i = (int64_t)blockIdx.x * kBlockG + threadIdx.x;
    if (i >= n_gauss) return;
    const GRec r = recs[i];
    double gm0 = 0, gm1 = 0, gl0 = 0, gl1 = 0, gl2 = 0, gc0 = 0, gc1 = 0, gc2 = 0, ga = 0;
    float m[8];
    {
        float4* mp = reinterpret_cast<float4*>(moments + i * 8);
        const float4 u = mp[0], v = mp[1];
        m[0] = u.x; m[1] = u.y; m[2] = u.z; m[3] = u.w;
        m[4] = v.x; m[5] = v.y; m[6] = v.z; m[7] = v.w;
        mp[0] = make_float4(0.f, 0.f, 0.f, 0.f);  // ready for the next backward
        mp[1] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (r.x0 <= r.x1 && r.pad == 0) {
        const double l11 = chol[3 * i], l21 = chol[3 * i + 1], l22 = chol[3 * i + 2];
        const double al = opacity[i];
        const double c0 = color[3 * i], c1 = color[3 * i + 1], c2 = color[3 * i + 2];
        const double K = 1.0 / (2.0 * 3.14159265358979323846 * l11 * l22);
        const double G0 = m[0], G1 = m[1], G2 = m[2];
        const double kc = kZScale;
        const double Sz1 = m[3] / kc, Sz2 = m[4] / kc;
        const double Sz11 = m[5] / (kc * kc), Sz12 = m[6] / (kc * kc), Sz22 = m[7] / (kc * kc);
        const double S1 = al * K * (c0 * G0 + c1 * G1 + c2 * G2);
        const double b = l21 / l22;
        gm0 = (Sz1 - Sz2 * b) / l11;
        gm1 = Sz2 / l22;
        gl0 = (Sz11 - S1 - Sz12 * b) / l11;
        gl1 = Sz12 / l22;
        gl2 = (Sz22 - S1) / l22;
        gc0 = al * K * G0;
        gc1 = al * K * G1;
        gc2 = al * K * G2;
        ga = K * (c0 * G0 + c1 * G1 + c2 * G2);
    }
    grad_mean[2 * i] = (float)gm0;
    grad_mean[2 * i + 1] = (float)gm1;
    grad_chol[3 * i] = (float)gl0;
    grad_chol[3 * i + 1] = (float)gl1;
    grad_chol[3 * i + 2] = (float)gl2;
    grad_color[3 * i] = (float)gc0;
    grad_color[3 * i + 1] = (float)gc1;
    grad_color[3 * i + 2] = (float)gc2;
    grad_opacity[i] = (float)ga;
}

__global__ __launch_bounds__(kBlockG) void k_l1(const float* __restrict__ img,
                                                const float* __restrict__ tgt, int64_t numel,
                                                float* __restrict__ grad,
                                                double* __restrict__ loss_sum) {
    __shared__ double tmp[kBlockG / 64];
    const float inv = (float)(1.0 / (double)numel);
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlockG + threadIdx.x; i < numel;
         i += (int64_t)gridDim.x * kBlockG) {
        const float d = img[i] - tgt[i];
        grad[i] = d > 0.f ? inv : (d < 0.f ? -inv : 0.f);
        s += fabs((double)img[i] - (double)tgt[i]);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int k = 0; k < kBlockG / 64; ++k) b += tmp[k];
        atomicAdd(loss_sum, b);
    }
}

// One workgroup: mean of the per-tile L1 partial sums.
__global__ __launch_bounds__(1024) void k_sum_loss(const double* __restrict__ tile_loss,
                                                   int64_t n_tiles, double inv_numel,
                                                   double* __restrict__ loss) {
    __shared__ double part[1024 / 64];
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < n_tiles; t += 1024) s += tile_loss[t];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int k = 0; k < 1024 / 64; ++k) sum += part[k];
        *loss = sum * inv_numel;
    }
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_sum_loss(const Layout& L, const Ws& w, int64_t numel, double* loss,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(1024), 0, st, w.tile_loss, L.n_tiles,
                       1.0 / (double)numel, loss);
    return hipGetLastError();
}

hipError_t launch_render_fwd(const Layout& L, const Ws& w, float* out, hipStream_t st) {
    const uint32_t* gids = (L.n_passes & 1) ? w.vals[1] : w.vals[0];
    const dim3 grid((unsigned)L.n_tiles);
    switch (L.tile) {
        case 8:
            hipLaunchKernelGGL(k_render_fwd<8>, grid, dim3(TileShape<8>::kThreads), 0, st,
                               w.imgs, L.n_img, w.recs, gids, w.ranges, out);
            break;
        case 16:
            hipLaunchKernelGGL(k_render_fwd<16>, grid, dim3(TileShape<16>::kThreads), 0, st,
                               w.imgs, L.n_img, w.recs, gids, w.ranges, out);
            break;
        case 32:
            hipLaunchKernelGGL(k_render_fwd<32>, grid, dim3(TileShape<32>::kThreads), 0, st,
                               w.imgs, L.n_img, w.recs, gids, w.ranges, out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool kL1>
static hipError_t launch_bwd_t(const Layout& L, const Ws& w, const float* grad_out,
                               const float* target, float inv_numel, hipStream_t st) {
    const uint32_t* gids = (L.n_passes & 1) ? w.vals[1] : w.vals[0];
    const dim3 grid((unsigned)L.n_tiles);
    switch (L.tile) {
        case 8:
            hipLaunchKernelGGL((k_render_bwd<8, kL1>), grid, dim3(TileShape<8>::kThreads), 0, st,
                               w.imgs, L.n_img, w.recs, gids, w.ranges, grad_out, target,
                               inv_numel, w.tile_loss, w.moments);
            break;
        case 16:
            hipLaunchKernelGGL((k_render_bwd<16, kL1>), grid, dim3(TileShape<16>::kThreads), 0, st,
                               w.imgs, L.n_img, w.recs, gids, w.ranges, grad_out, target,
                               inv_numel, w.tile_loss, w.moments);
            break;
        case 32:
            hipLaunchKernelGGL((k_render_bwd<32, kL1>), grid, dim3(TileShape<32>::kThreads), 0, st,
                               w.imgs, L.n_img, w.recs, gids, w.ranges, grad_out, target,
                               inv_numel, w.tile_loss, w.moments);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_render_bwd(const Layout& L, const Ws& w, const float* grad_out,
                             hipStream_t st) {
    return launch_bwd_t<false>(L, w, grad_out, nullptr, 0.f, st);
}

hipError_t launch_render_bwd_l1(const Layout& L, const Ws& w, const float* out,
                                const float* target, int64_t numel, hipStream_t st) {
    return launch_bwd_t<true>(L, w, out, target, (float)(1.0 / (double)numel), st);
}

hipError_t launch_finalize(const Layout& L, const Ws& w, const float* chol,
                           const float* color, const float* opacity, float* grad_mean,
                           float* grad_chol, float* grad_color, float* grad_opacity,
                           hipStream_t st) {
    if (L.n_gauss == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(blocks_for(L.n_gauss, kBlockG)), dim3(kBlockG), 0, st,
                       w.recs, L.n_gauss, chol, color, opacity, w.moments, grad_mean,
                       grad_chol, grad_color, grad_opacity);
    return hipGetLastError();
}

hipError_t launch_l1(const float* img, const float* target, int64_t numel, float* grad,
                     double* loss_sum, hipStream_t st) {
    if (numel == 0) return hipSuccess;
    // at most 256 workgroups: each adds one double to *loss_sum, and atomics
    // on a single address serialise
    int nb = blocks_for(numel, kBlockG * 4);
    if (nb > 256) nb = 256;
    hipLaunchKernelGGL(k_l1, dim3(nb), dim3(kBlockG), 0, st, img, target, numel, grad,
                       loss_sum);
    return hipGetLastError();
}

}  // namespace gs
