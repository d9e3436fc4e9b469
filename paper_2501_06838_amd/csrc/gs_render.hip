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
// in LDS and the listed Gaussians are compacted per 8x8 block as in the
// forward; a wave puts one Gaussian of a block's list on each lane and walks
// the block's pixels with all lanes together, so every lane accumulates the
// eight per-Gaussian sums of its own Gaussian in registers.  The tile's sums
// per (tile, Gaussian) are stored once, in sorted pair order (or added into
// per-Gaussian accumulators with global atomics); the finalize kernel turns
// them into parameter gradients.
#include <algorithm>

#include "gs_internal.h"

namespace gs {

namespace {

template <typename Table>
__device__ __forceinline__ int tile_image(const Table& imgs, int n_img, int64_t tile) {
    int lo = 0, hi = n_img - 1, ans = 0;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        if (imgs[mid].tile_base <= tile) { ans = mid; lo = mid + 1; } else { hi = mid - 1; }
    }
    return ans;
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// v + the value of the lane that the DPP control kCtrl names (all lanes
// active, so every lane reads a valid partner), for an FP64 value moved as
// its two 32-bit halves.
template <int kCtrl>
__device__ __forceinline__ double dpp_add(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, 0xF, 0xF, false);
    return v + __hiloint2double(hi, lo);
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

// Waves per SIMD the tile kernels are compiled for (their register
// budget).  The backward and fused kernels are latency bound, so at 16 x 16
// the budget follows the workgroups the LDS fits per CU: eight with 64 or 96
// Gaussians per round (64 VGPRs), seven with 112 (72), six with 128 (80); a
// few values spill, outside the pixel loops.  The forward kernel at 16 x 16
// holds eight workgroups per CU up to 112 Gaussians per round and seven with
// 128 (its LDS).  Elsewhere
// (and for the elliptical supports, whose FP64 mask building needs more) the
// compiler's own register count decides.
template <int T, int B, bool kEll>
struct BwdOccupancy {
    static constexpr int kMinWaves = (T != 16 || kEll) ? 1
                                   : (B == 64 || B == 96) ? 8
                                   : B == 112             ? 7
                                   : B == 128             ? 6
                                                          : 1;
    static constexpr int kFwdMinWaves = (T != 16 || kEll || B > 128) ? 1 : B == 128 ? 7 : 8;
};

// Persistent tile kernels: a grid of the resident workgroups walks the items
// (the longest-first tile order) in a fixed snake schedule: round r gives
// item r G + b to workgroup b on even rounds and r G + G - 1 - b on odd ones,
// so every workgroup's share alternates long and short lists (the static
// longest-processing-time heuristic).  No counters: work queues taken with
// same-address atomics serialise across the XCDs (about one atomic per 100 ns
// per address here), which cost more than the tiles' imbalance.
template <typename Body>
__device__ __forceinline__ void run_persistent(int64_t n_items, Body body) {
    const int64_t G = gridDim.x, b = blockIdx.x;
    for (int64_t r = 0;; ++r) {
        const int64_t item = r * G + ((r & 1) ? G - 1 - b : b);
        if (item >= n_items) break;  // uniform
        body(item);
        __syncthreads();  // the LDS is reused by the next item
    }
}

// Gaussians staged per round (lds_batch).  Per 8x8 block of the tile the
// staged Gaussians touching it are compacted, in staged (ascending Gaussian)
// order, into a list of 40-byte records:
//   l0 = {z1, z2 at the block's first pixel, a, e}
//   l1 = {g, A0, A1, A2}
//   mk = pixel mask, its low 32 bits (lanes 0-31) in mk[0], its high
//        32 bits (lanes 32-63) in mk[1].
// For the block's pixel (dx, dy): z1 = z1_0 + a dx, z2 = z2_0 + e dy - g dx, and the
// Gaussian's contribution is A_c exp2(-(z1^2 + z2^2)) where the mask is set.
template <int T, int B>
struct StageLds {
    static constexpr int NB = TileShape<T>::kBlocks;
    static_assert(B % 4 == 0, "the forward reads four mask halves per LDS load");
    float4 l0[NB][B];
    float4 l1[NB][B];
    alignas(16) uint32_t mk[2][NB][B];  // mask halves: [0] lanes 0-31, [1] lanes 32-63
    int scount[NB];
    int wcount[TileShape<T>::kWaves][NB];
    uint8_t slot[NB][B];  // staged Gaussian t's position in block j's list
};

template <int T, int B>
struct FwdLds {
    StageLds<T, B> st;
};

// Backward and fused kernels: the records and the tile's upstream gradient.
// The eight sums of a (block, staged Gaussian) record overwrite its l0 and
// l1 entries once the backward has read them (only the lane that owns a
// record reads it), so the sums need no LDS of their own.
template <int T, int B>
struct BwdLds {
    StageLds<T, B> st;
    float4 gt[T * T];       // upstream gradient of the tile, {g0, g1, g2, 0}
    double lpart[4 * TileShape<T>::kWaves];  // per row of 16 lanes
};

// What a staging thread keeps about its Gaussian for the backward's sums.
struct StagedMine {
    uint32_t gid;
    uint32_t touch;  // bit j: the Gaussian's box meets block j
    int64_t e;       // emission index of this (tile, Gaussian) pair
};

// Tile geometry and list.
struct TileInfo {
    ImgDev im;
    int tx, ty;      // tile coordinates within the image
    int px0, py0;    // HR origin
    int2 rg;
};

// A record whose box has q = z1^2 + z2^2 (log2-scaled) above kQCull
// everywhere adds exactly zero: its FP32 weights exp2(-q) < 2^-159 round to
// zero.  Such records are dropped at staging when the support is a window
// much wider than the Gaussian (Algorithm 1's r-window), which leaves every
// sum bit for bit as it was.
constexpr float kQCull = 160.f;

// A lower bound of q = (a X + z10)^2 + (e Y - g X + z20)^2 over the real box
// [x0, x1] x [y0, y1] (a, e > 0): z1 and z2 are linear, so each one's
// smallest square over the box follows from its range (z1 over x0..x1, z2
// over the four corners), and q is at least their sum.
__device__ __forceinline__ float box_qlow(float a, float e, float g, float z10, float z20,
                                          float x0, float x1, float y0, float y1) {
    const float u0 = __builtin_fmaf(a, x0, z10), u1 = __builtin_fmaf(a, x1, z10);
    const float d1 = u0 > 0.f ? u0 : (u1 < 0.f ? -u1 : 0.f);
    const float gx0 = __builtin_fmaf(-g, x0, z20), gx1 = __builtin_fmaf(-g, x1, z20);
    const float v0 = __builtin_fmaf(e, y0, fminf(gx0, gx1));
    const float v1 = __builtin_fmaf(e, y1, fmaxf(gx0, gx1));
    const float d2 = v0 > 0.f ? v0 : (v1 < 0.f ? -v1 : 0.f);
    return __builtin_fmaf(d1, d1, d2 * d2);
}

// Stages entries [base, base + nb) of the tile's sorted list (Gaussian ids)
// from the Gaussians' render records and builds the per-block record lists.
// Ends with a barrier.
// Pixel masks of an elliptical record: row by row, the pixels of the box
// within the tile whose Mahalanobis distance is below R (ellipse_row: the
// same FP64 predicate as the definition), split over the tile's blocks.
template <int T>
__device__ void ellipse_masks(const EParams& ep, double s, const TileInfo& ti, int lx0, int lx1,
                              int ly0, int ly1, uint64_t (&mask)[TileShape<T>::kBlocks]) {
    using S = TileShape<T>;
    const double mx = ep.p0.x, my = ep.p0.y, l11 = ep.p0.z, l21 = ep.p0.w, l22 = ep.p1.x;
    const double R = ep.p1.y;
    const bool centre = ep.p1.z != 0.f;
    for (int ly = ly0; ly <= ly1; ++ly) {
        int xa, xb;
        ellipse_row(ti.py0 + ly, ti.px0 + lx0, ti.px0 + lx1, s, centre, mx, my, l11, l21, l22,
                    R * R, &xa, &xb);
        if (xa > xb) continue;
        xa -= ti.px0;
        xb -= ti.px0;
        const int byi = ly >> 3, ry = ly & 7;
#pragma unroll
        for (int j = 0; j < S::kBlocks; ++j) {
            if (j / S::kBlocksX != byi) continue;
            const int bx = (j % S::kBlocksX) * 8;
            const int c0 = max(xa, bx) - bx, c1 = min(xb, bx + 7) - bx;
            if (c0 <= c1)
                mask[j] |= (uint64_t)(((1u << (c1 - c0 + 1)) - 1u) << c0) << (8 * ry);
        }
    }
}

template <int T, int B, bool kEll>
__device__ __forceinline__ StagedMine stage_round(StageLds<T, B>& st,
                                                  const uint32_t* __restrict__ svals,
                                                  const GRec* __restrict__ recs,
                                                  const int32_t* __restrict__ offsets,
                                                  const EParams* __restrict__ eparams,
                                                  const TileInfo& ti, int base, int nb) {
    using S = TileShape<T>;
    constexpr int NB = S::kBlocks;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    StagedMine mine{0u, 0u, 0};
    GRec r;
    float kxr = 0.f, kyr = 0.f;
    uint64_t my_mask[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) my_mask[j] = 0;
    if (t < nb) {
        mine.gid = svals[base + t];
        r = recs[mine.gid];
        // this pair's emission index: the Gaussian's offset plus the tile's
        // row-major rank in the Gaussian's tile range
        const int tx0 = r.x0 / T, tx1 = r.x1 / T, ty0 = r.y0 / T;
        mine.e = (int64_t)offsets[mine.gid] + (int64_t)(ti.ty - ty0) * (tx1 - tx0 + 1) +
                 (ti.tx - tx0);
        // tile origin minus the integer part of the HR centre (exact)
        kxr = (float)(ti.px0 - r.kx);
        kyr = (float)(ti.py0 - r.ky);
        const int lx0 = max(r.x0 - ti.px0, 0), lx1 = min(r.x1 - ti.px0, T - 1);
        const int ly0 = max(r.y0 - ti.py0, 0), ly1 = min(r.y1 - ti.py0, T - 1);
        const bool cull = (r.flags & kRecCull) != 0;
        if constexpr (kEll) {
            // every listed record is elliptical
            if (lx0 <= lx1 && ly0 <= ly1)
                ellipse_masks<T>(eparams[mine.gid], ti.im.scale, ti, lx0, lx1, ly0, ly1, my_mask);
        } else if (lx0 <= lx1 && ly0 <= ly1) {
            // the box's tile columns and tile rows as bit sets; per block
            // column its 8 column bits repeated in every byte, per block row
            // its rows 0-3 and 4-7 as bytes of ones; a block's mask is their AND
            const uint32_t tc = (~0u << lx0) & (~0u >> (31 - lx1));
            const uint32_t tr = (~0u << ly0) & (~0u >> (31 - ly1));
            uint32_t rep[S::kBlocksX], rlo[S::kBlocksX], rhi[S::kBlocksX];
#pragma unroll
            for (int b = 0; b < S::kBlocksX; ++b) {
                const uint32_t c8 = (tc >> (8 * b)) & 255u;
                const uint32_t c16 = c8 | (c8 << 8);
                rep[b] = c16 | (c16 << 16);
                const uint32_t r8 = (tr >> (8 * b)) & 255u;
                // bit k of a nibble to byte k (k = 0..3), then each byte 1 -> 255
                const uint32_t l1 = ((r8 & 15u) * 0x00204081u) & 0x01010101u;
                const uint32_t h1 = ((r8 >> 4) * 0x00204081u) & 0x01010101u;
                rlo[b] = (l1 << 8) - l1;
                rhi[b] = (h1 << 8) - h1;
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int jx = j % S::kBlocksX, jy = j / S::kBlocksX;
                const uint32_t lo = rep[jx] & rlo[jy], hi = rep[jx] & rhi[jy];
                if ((lo | hi) == 0u) continue;
                if (cull) {
                    const int bx = jx * 8, by = jy * 8;
                    const int c0 = max(lx0, bx) - bx, c1 = min(lx1, bx + 7) - bx;
                    const int r0 = max(ly0, by) - by, r1 = min(ly1, by + 7) - by;
                    const float Xb = (kxr + (float)bx) - r.fx;
                    const float Yb = (kyr + (float)by) - r.fy;
                    if (box_qlow(r.a, r.e, r.g, r.a * Xb, r.e * Yb - r.g * Xb, (float)c0,
                                 (float)c1, (float)r0, (float)r1) > kQCull)
                        continue;
                }
                my_mask[j] = ((uint64_t)hi << 32) | lo;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const uint64_t bal = __ballot(my_mask[j] != 0);
        if (lane == 0) st.wcount[wave][j] = __popcll(bal);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const uint64_t bal = __ballot(my_mask[j] != 0);
        if (my_mask[j] != 0) {
            int pos = __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
            for (int w = 0; w < wave; ++w) pos += st.wcount[w][j];
            const int bx = (j % S::kBlocksX) * 8, by = (j / S::kBlocksX) * 8;
            // block origin relative to the HR centre: exact integer part, one
            // rounding for the fraction
            const float Xb = (kxr + (float)bx) - r.fx;
            const float Yb = (kyr + (float)by) - r.fy;
            st.l0[j][pos] = make_float4(r.a * Xb, r.e * Yb - r.g * Xb, r.a, r.e);
            st.l1[j][pos] = make_float4(r.g, r.A[0], r.A[1], r.A[2]);
            st.mk[0][j][pos] = (uint32_t)my_mask[j];
            st.mk[1][j][pos] = (uint32_t)(my_mask[j] >> 32);
            st.slot[j][t] = (uint8_t)pos;
            mine.touch |= 1u << j;
        }
    }
    if (t < NB) {
        int c = 0;
        for (int w = 0; w < S::kWaves; ++w) c += st.wcount[w][t];
        st.scount[t] = c;
        if (c & 1) {  // an odd list gets an empty record (zero mask, zero amplitude)
            st.l0[t][c] = make_float4(0.f, 0.f, 0.f, 0.f);
            st.l1[t][c] = make_float4(0.f, 0.f, 0.f, 0.f);
            st.mk[0][t][c] = 0u;
            st.mk[1][t][c] = 0u;
        }
    }
    __syncthreads();
    return mine;
}

// Forward sums of one round: lane = pixel of the wave's blocks, the block's
// records in list order (wave-uniform coefficients).  Each lane reads its own
// half of the records' pixel masks (four records per LDS read) and clears its
// weight where its bit is 0: a sign-extended one-bit field ANDed into the
// weight's bits, which gives the same +0 as a select.
template <int T, int B>
__device__ __forceinline__ void fwd_round(const StageLds<T, B>& st,
                                          float (&acc)[TileShape<T>::kBlocksPerWave][3]) {
    using S = TileShape<T>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float lxf = (float)(lane & 7), lyf = (float)(lane >> 3);
    const int bit = lane & 31;
#pragma unroll
    for (int m = 0; m < S::kBlocksPerWave; ++m) {
        const int j = wave + S::kWaves * m;
        const uint32_t* mk = st.mk[lane >> 5][j];
        auto rec = [&](int q, uint32_t mh) {
            const float4 a0 = st.l0[j][q], a1 = st.l1[j][q];
            const float z1 = __builtin_fmaf(a0.z, lxf, a0.x);
            const float z2 = __builtin_fmaf(a0.w, lyf, __builtin_fmaf(-a1.x, lxf, a0.y));
            const float w = fast_exp2(-(z1 * z1 + z2 * z2));
            const uint32_t keep = (uint32_t)__builtin_amdgcn_sbfe((int32_t)mh, bit, 1);
            const float wm = __uint_as_float(__float_as_uint(w) & keep);
            acc[m][0] += a1.y * wm;
            acc[m][1] += a1.z * wm;
            acc[m][2] += a1.w * wm;
        };
        // records four at a time (an odd list ends with the staging's empty
        // record, so a list is walked in pairs)
        const int cnt = __builtin_amdgcn_readfirstlane(st.scount[j]);  // uniform
        const int cntp = (cnt + 1) & ~1;
        int q = 0;
        for (; q + 4 <= cntp; q += 4) {
            const uint4 mh = *reinterpret_cast<const uint4*>(mk + q);
            rec(q, mh.x);
            rec(q + 1, mh.y);
            rec(q + 2, mh.z);
            rec(q + 3, mh.w);
        }
        if (q < cntp) {  // uniform
            const uint2 mh = *reinterpret_cast<const uint2*>(mk + q);
            rec(q, mh.x);
            rec(q + 1, mh.y);
        }
    }
}

// Backward sums of one round.  The (block, Gaussian) records of all blocks,
// block after block, go 64 to a wave, one per lane; a pass walks the
// block-local pixels of the union of its lanes' boxes with all lanes
// together, each lane reading the upstream gradient of its own block, so the
// loop is uniform and each lane accumulates the eight sums of its own
// Gaussian in registers (no cross-lane reduction, no atomics).  A lane's
// values depend only on its own record, never on which records share its
// pass.  Each (block, staged Gaussian) writes its sums once, over the l0 and
// l1 entries of the record it came from.  Idle lanes of the last pass read
// entry (0, 0), which may already hold sums; their masks are zero and they
// write nothing.  Ends with a barrier.
// One lane's eight backward sums over the block-local pixels [cx0, cx1] x
// [ry0, ry1] (the pass's union of boxes; kFull: the whole block, no bounds
// checks).  The lane's own box is a rectangle: a column outside it gets a far
// z1 and a row outside it a far z2 (1e19: the squares stay finite, the
// weight underflows to 0, and 0 times the finite z is 0), so no pixel needs a
// select.  Column by column: z1 is constant down a column, so the z1 moments
// follow from the column's sums of H w, H w z2 and H w z2^2
// (H = sum_c A_c G_c).  rec0 = {z1, z2 at the block's first pixel, a, e},
// rec1 = {g, A0, A1, A2}.  kMask (elliptical supports): the record's pixel
// mask decides every pixel instead.
template <int T, bool kFull, bool kMask>
__device__ __forceinline__ void bwd_columns(const float4* __restrict__ gcol, uint32_t colset,
                                            uint32_t rows, uint32_t mlo, uint32_t mhi, int cx0,
                                            int cx1, int ry0, int ry1, float4 rec0, float4 rec1,
                                            float (&m)[8]) {
    constexpr float kFar = 1e19f;
    const float a = rec0.z, e = rec0.w, gg = rec1.x;
    float zr[8];  // e ry inside the lane's rows, far outside
#pragma unroll
    for (int ry = 0; ry < 8; ++ry)
        zr[ry] = (kMask || ((rows >> ry) & 1u)) ? e * (float)ry : kFar;
#pragma unroll
    for (int cx = 0; cx < 8; ++cx) {
        if (!kFull && (cx < cx0 || cx > cx1)) continue;  // uniform
        const float z1 = (kMask || ((colset >> cx) & 1u)) ? __builtin_fmaf(a, (float)cx, rec0.x)
                                                          : kFar;
        const float z1sq = z1 * z1;
        const float zb = __builtin_fmaf(-gg, (float)cx, rec0.y);
        float sa = 0.f, sb = 0.f, sc = 0.f;
#pragma unroll
        for (int ry = 0; ry < 8; ++ry) {
            if (!kFull && (ry < ry0 || ry > ry1)) continue;  // uniform
            const float4 G = gcol[ry * T + cx];
            const float z2 = zr[ry] + zb;
            float w = fast_exp2(-__builtin_fmaf(z2, z2, z1sq));
            if (kMask) w = (((ry < 4 ? mlo : mhi) >> (8 * (ry & 3) + cx)) & 1u) ? w : 0.f;
            m[0] = __builtin_fmaf(G.x, w, m[0]);
            m[1] = __builtin_fmaf(G.y, w, m[1]);
            m[2] = __builtin_fmaf(G.z, w, m[2]);
            const float hw =
                __builtin_fmaf(rec1.y, G.x, __builtin_fmaf(rec1.z, G.y, rec1.w * G.z)) * w;
            const float hz = hw * z2;
            sa += hw;
            sb += hz;
            sc = __builtin_fmaf(hz, z2, sc);
        }
        m[3] = __builtin_fmaf(z1, sa, m[3]);
        m[4] += sb;
        m[5] = __builtin_fmaf(z1sq, sa, m[5]);
        m[6] = __builtin_fmaf(z1, sb, m[6]);
        m[7] += sc;
    }
}

template <int T, int B, bool kEll>
__device__ __forceinline__ void bwd_round(BwdLds<T, B>& sm) {
    using S = TileShape<T>;
    constexpr int NB = S::kBlocks, NW = S::kWaves;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int total = 0;
#pragma unroll
    for (int j = 0; j < NB; ++j) total += sm.st.scount[j];
    total = __builtin_amdgcn_readfirstlane(total);  // uniform
    for (int f0 = wave * 64; f0 < total; f0 += NW * 64) {
        const int f = f0 + lane;
        const bool active = f < total;
        int j = 0, pos = f;
#pragma unroll
        for (int k = 0; k + 1 < NB; ++k) {
            if (j == k && pos >= sm.st.scount[k]) { pos -= sm.st.scount[k]; j = k + 1; }
        }
        if (!active) { j = 0; pos = 0; }
        const float4 c0 = sm.st.l0[j][pos], c1 = sm.st.l1[j][pos];
        const uint32_t mlo = active ? sm.st.mk[0][j][pos] : 0u;
        const uint32_t mhi = active ? sm.st.mk[1][j][pos] : 0u;
        const int bx = (j % S::kBlocksX) * 8, by = (j / S::kBlocksX) * 8;
        // the lane's block-local columns (bits of cm) and rows (bits of rows):
        // its pixels are row-convex, so its rows run from the first to the
        // last nonzero byte of the mask
        uint32_t cm = mlo | mhi;
        cm |= cm >> 16;
        cm |= cm >> 8;
        cm &= 255u;
        const uint64_t mm = ((uint64_t)mhi << 32) | mlo;
        uint32_t rows = 0u;
        if (mm != 0ull) {
            const int r0 = __builtin_ctzll(mm) >> 3, r1 = (63 - __builtin_clzll(mm)) >> 3;
            rows = (255u << r0) & (255u >> (7 - r1));
        }
        const float4* gcol = &sm.gt[by * T + bx];
        float m[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        // the pass walks the bounding box of its lanes' boxes: the whole block
        // when some lane has column 0, some column 7, some row 0 and some row 7
        const bool full = __ballot(cm & 1u) != 0ull && __ballot(cm & 128u) != 0ull &&
                          __ballot(rows & 1u) != 0ull && __ballot(rows & 128u) != 0ull;
        if (!kEll && full) {  // uniform
            bwd_columns<T, true, false>(gcol, cm, rows, mlo, mhi, 0, 7, 0, 7, c0, c1, m);
        } else {
            uint32_t any = cm | (rows << 8);
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) any |= (uint32_t)__shfl_xor((int)any, o, 64);
            any = __builtin_amdgcn_readfirstlane(any);
            const int cx0 = __builtin_ctz(any & 255u), cx1 = 31 - __builtin_clz(any & 255u);
            const int ry0 = __builtin_ctz(any >> 8), ry1 = 31 - __builtin_clz(any >> 8);
            if constexpr (kEll)  // elliptical supports: the pixel mask decides
                bwd_columns<T, false, true>(gcol, cm, rows, mlo, mhi, cx0, cx1, ry0, ry1, c0, c1,
                                            m);
            else
                bwd_columns<T, false, false>(gcol, cm, rows, mlo, mhi, cx0, cx1, ry0, ry1, c0,
                                             c1, m);
        }
        const float m0 = m[0], m1 = m[1], m2 = m[2], m3 = m[3], m4 = m[4], m5 = m[5],
                    m6 = m[6], m7 = m[7];
        if (active) {
            // in place of the record this lane read (no other lane reads it)
            sm.st.l0[j][pos] = make_float4(m0, m1, m2, m3);
            sm.st.l1[j][pos] = make_float4(m4, m5, m6, m7);
        }
    }
    __syncthreads();
}

// The round's sums per (tile, Gaussian): blocks added in ascending order,
// stored per sorted pair (or added with global atomics).  Ends with a barrier
// unless it is the tile's last round (the LDS is not read again).
template <int T, int B>
__device__ __forceinline__ void bwd_round_store(BwdLds<T, B>& sm, StagedMine mine, bool last,
                                                int nb, float* __restrict__ moments,
                                                float4* __restrict__ partials,
                                                int atomic_grads) {
    constexpr int NB = TileShape<T>::kBlocks;
    const int t = threadIdx.x;
    if (t < nb) {
        float4 u = make_float4(0.f, 0.f, 0.f, 0.f), v = u;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (mine.touch & (1u << j)) {
                const int p = sm.st.slot[j][t];
                const float4 a0 = sm.st.l0[j][p], a1 = sm.st.l1[j][p];
                u.x += a0.x; u.y += a0.y; u.z += a0.z; u.w += a0.w;
                v.x += a1.x; v.y += a1.y; v.z += a1.z; v.w += a1.w;
            }
        }
        if (atomic_grads) {
            // one FP32 global atomic per (tile, Gaussian, sum)
            float* dst = moments + (int64_t)mine.gid * 8;
            const float vals[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (vals[m] != 0.f) atomicAdd(dst + m, vals[m]);
        } else {
            // the (tile, Gaussian) sums at the pair's emission index, so each
            // Gaussian's pairs lie together; the gradient kernel adds them in
            // that (fixed) order
            float4* dst = partials + 2 * mine.e;
            dst[0] = u;
            dst[1] = v;
        }
    }
    if (!last) __syncthreads();  // uniform
}

template <int T, typename Table>
__device__ __forceinline__ TileInfo tile_info(const Table& imgs, int n_img,
                                              const int2* __restrict__ ranges, int64_t tile) {
    TileInfo ti;
    const int k_img = tile_image(imgs, n_img, tile);
    ti.im = imgs[k_img];
    const int64_t lt = tile - ti.im.tile_base;
    ti.tx = (int)(lt % ti.im.tiles_x);
    ti.ty = (int)(lt / ti.im.tiles_x);
    ti.px0 = ti.tx * T;
    ti.py0 = ti.ty * T;
    ti.rg = ranges[tile];
    return ti;
}

template <int T, int B, bool kEll, typename Table>
__device__ __forceinline__ void fwd_tile(FwdLds<T, B>& sm, const Table& imgs, int n_img,
                                         const uint32_t* __restrict__ svals, const GRec* __restrict__ recs,
    const int32_t* __restrict__ offsets, const EParams* __restrict__ eparams,
                                         const int2* __restrict__ ranges,
                                         float* __restrict__ out, int64_t tile) {
    using S = TileShape<T>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const TileInfo ti = tile_info<T>(imgs, n_img, ranges, tile);
    float acc[S::kBlocksPerWave][3];
#pragma unroll
    for (int m = 0; m < S::kBlocksPerWave; ++m) acc[m][0] = acc[m][1] = acc[m][2] = 0.f;
    for (int base = ti.rg.x; base < ti.rg.y; base += B) {
        stage_round<T, B, kEll>(sm.st, svals, recs, offsets, eparams, ti, base, min(B, ti.rg.y - base));
        fwd_round<T, B>(sm.st, acc);
        __syncthreads();
    }
    const int64_t plane = (int64_t)ti.im.out_w * ti.im.out_h;
    float* o = out + ti.im.out_offset;
#pragma unroll
    for (int m = 0; m < S::kBlocksPerWave; ++m) {
        const int j = wave + S::kWaves * m;
        const int x = ti.px0 + (j % S::kBlocksX) * 8 + (lane & 7);
        const int y = ti.py0 + (j / S::kBlocksX) * 8 + (lane >> 3);
        if (x < ti.im.out_w && y < ti.im.out_h) {
            const int64_t p = (int64_t)y * ti.im.out_w + x;
            o[p] = acc[m][0];
            o[plane + p] = acc[m][1];
            o[2 * plane + p] = acc[m][2];
        }
    }
}

// Reduces the tile's L1 partial sum (one per thread) into tile_loss[tile].
template <int T, int B>
__device__ __forceinline__ void tile_loss_sum(BwdLds<T, B>& sm, double lsum,
                                              double* __restrict__ tile_loss, int64_t tile) {
    constexpr int NW = TileShape<T>::kWaves;
    // butterflies within each row of 16 lanes (lane pairs i^1, i^2, then the
    // mirrored halves of 8 and of 16): every lane of a row ends with the same
    // row sum, with no LDS round trip
    lsum = dpp_add<0xB1>(lsum);   // quad_perm [1, 0, 3, 2]
    lsum = dpp_add<0x4E>(lsum);   // quad_perm [2, 3, 0, 1]
    lsum = dpp_add<0x141>(lsum);  // row_half_mirror
    lsum = dpp_add<0x140>(lsum);  // row_mirror
    if ((threadIdx.x & 15) == 0) sm.lpart[threadIdx.x >> 4] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int k = 0; k < 4 * NW; ++k) sum += sm.lpart[k];
        tile_loss[tile] = sum;
    }
}

// kL1: the upstream gradient is the L1 loss's, sign(out - target) / numel,
// formed here from the rendered image and the target (it is never stored),
// and the tile's share of sum |out - target| goes to tile_loss[tile].
template <int T, int B, bool kL1, bool kEll, typename Table>
__device__ __forceinline__ void bwd_tile(
    BwdLds<T, B>& sm, const Table& imgs, int n_img, const uint32_t* __restrict__ svals, const GRec* __restrict__ recs,
    const int32_t* __restrict__ offsets, const EParams* __restrict__ eparams,
    const int2* __restrict__ ranges, const float* __restrict__ grad_out,
    const float* __restrict__ target, float inv_numel, double* __restrict__ tile_loss,
    float* __restrict__ moments, float4* __restrict__ partials, int atomic_grads,
    int64_t tile) {
    using S = TileShape<T>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const TileInfo ti = tile_info<T>(imgs, n_img, ranges, tile);
    if (!kL1 && ti.rg.y <= ti.rg.x) return;  // uniform: nothing listed in this tile

    // the fused kernel's pixel-to-thread mapping, so that the tile's L1 sum
    // is added in the same order (bitwise the same loss)
    const int64_t plane = (int64_t)ti.im.out_w * ti.im.out_h;
    const float* g = grad_out + ti.im.out_offset;
    double lsum = 0.0;
#pragma unroll
    for (int m = 0; m < S::kBlocksPerWave; ++m) {
        const int j = wave + S::kWaves * m;
        const int lx = (j % S::kBlocksX) * 8 + (lane & 7);
        const int ly = (j / S::kBlocksX) * 8 + (lane >> 3);
        const int p = ly * T + lx;
        const int x = ti.px0 + lx, y = ti.py0 + ly;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (x < ti.im.out_w && y < ti.im.out_h) {
            const int64_t q = (int64_t)y * ti.im.out_w + x;
            if (kL1) {
                const float* tg = target + ti.im.out_offset;
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
        sm.gt[p] = v;
    }
    if (kL1) tile_loss_sum<T, B>(sm, lsum, tile_loss, tile);  // has a barrier

    for (int base = ti.rg.x; base < ti.rg.y; base += B) {
        const int nb = min(B, ti.rg.y - base);
        const StagedMine mine = stage_round<T, B, kEll>(sm.st, svals, recs, offsets, eparams, ti, base, nb);
        bwd_round<T, B, kEll>(sm);
        bwd_round_store<T, B>(sm, mine, base + B >= ti.rg.y, nb, moments, partials,
                              atomic_grads);
    }
}

// Forward, L1 gradient and backward of one tile in one pass: the image is
// summed in registers and stored; each lane forms the L1 gradient of its own
// pixels from them and the target into LDS (with the tile's L1 sum); the
// backward then runs over the same records, which stay staged when the
// tile's list fits one round.
template <int T, int B, bool kEll, typename Table>
__device__ __forceinline__ void fused_tile(
    BwdLds<T, B>& sm, const Table& imgs, int n_img, const uint32_t* __restrict__ svals, const GRec* __restrict__ recs,
    const int32_t* __restrict__ offsets, const EParams* __restrict__ eparams,
    const int2* __restrict__ ranges, float* __restrict__ out, const float* __restrict__ target,
    float inv_numel, double* __restrict__ tile_loss, float* __restrict__ moments,
    float4* __restrict__ partials, int atomic_grads, int64_t tile) {
    using S = TileShape<T>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const TileInfo ti = tile_info<T>(imgs, n_img, ranges, tile);
    float acc[S::kBlocksPerWave][3];
#pragma unroll
    for (int m = 0; m < S::kBlocksPerWave; ++m) acc[m][0] = acc[m][1] = acc[m][2] = 0.f;
    const bool one_round = ti.rg.y - ti.rg.x <= B;
    StagedMine mine{0u, 0u, 0};
    for (int base = ti.rg.x; base < ti.rg.y; base += B) {
        mine = stage_round<T, B, kEll>(sm.st, svals, recs, offsets, eparams, ti, base, min(B, ti.rg.y - base));
        fwd_round<T, B>(sm.st, acc);
        if (!one_round) __syncthreads();
    }
    const int64_t plane = (int64_t)ti.im.out_w * ti.im.out_h;
    float* o = out + ti.im.out_offset;
    const float* tg = target + ti.im.out_offset;
    double lsum = 0.0;
#pragma unroll
    for (int m = 0; m < S::kBlocksPerWave; ++m) {
        const int j = wave + S::kWaves * m;
        const int lx = (j % S::kBlocksX) * 8 + (lane & 7);
        const int ly = (j / S::kBlocksX) * 8 + (lane >> 3);
        const int x = ti.px0 + lx, y = ti.py0 + ly;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (x < ti.im.out_w && y < ti.im.out_h) {
            const int64_t p = (int64_t)y * ti.im.out_w + x;
            o[p] = acc[m][0];
            o[plane + p] = acc[m][1];
            o[2 * plane + p] = acc[m][2];
            float gv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float tv = tg[c * plane + p];
                const float d = acc[m][c] - tv;
                gv[c] = d > 0.f ? inv_numel : (d < 0.f ? -inv_numel : 0.f);
                lsum += fabs((double)acc[m][c] - (double)tv);
            }
            v = make_float4(gv[0], gv[1], gv[2], 0.f);
        }
        sm.gt[ly * T + lx] = v;
    }
    tile_loss_sum<T, B>(sm, lsum, tile_loss, tile);  // has a barrier
    if (ti.rg.y <= ti.rg.x) return;  // uniform
    if (one_round) {
        bwd_round<T, B, kEll>(sm);
        bwd_round_store<T, B>(sm, mine, true, ti.rg.y - ti.rg.x, moments, partials,
                              atomic_grads);
        return;
    }
    for (int base = ti.rg.x; base < ti.rg.y; base += B) {
        const int nb = min(B, ti.rg.y - base);
        mine = stage_round<T, B, kEll>(sm.st, svals, recs, offsets, eparams, ti, base, nb);
        bwd_round<T, B, kEll>(sm);
        bwd_round_store<T, B>(sm, mine, base + B >= ti.rg.y, nb, moments, partials,
                              atomic_grads);
    }
}

// One workgroup per tile: workgroups are dealt round-robin to the 8 XCDs
// (workgroup b runs on XCD b % 8).  Runs of kXcdRun consecutive tiles go to
// one XCD, so neighbouring tiles of a row, which gather many of the same
// render records, share an L2, while the runs still rotate over the XCDs
// (heavy regions of uneven batches stay spread).  The ragged end keeps its
// order.
constexpr int64_t kXcds = 8;
constexpr int64_t kXcdRun = 16;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n) {
    const int64_t full = n / (kXcds * kXcdRun) * (kXcds * kXcdRun);
    if (b >= full) return b;
    const int64_t x = b % kXcds, k = b / kXcds;
    return (k / kXcdRun) * (kXcds * kXcdRun) + x * kXcdRun + (k % kXcdRun);
}

// One tile per workgroup (grid of n_tiles, XCD-aware order), or, with
// `persistent`, a grid sized to the resident workgroups that walks the longest-first tile order
// (without a tile order from the matching binning, items are tiles).
template <int T, int B, bool kEll, typename Table>
__global__ __launch_bounds__(TileShape<T>::kThreads)
__attribute__((amdgpu_waves_per_eu(BwdOccupancy<T, B, kEll>::kFwdMinWaves, 8))) void k_render_fwd(
    Table imgs, int n_img, const uint32_t* __restrict__ svals, const GRec* __restrict__ recs,
    const int32_t* __restrict__ offsets, const EParams* __restrict__ eparams,
    const int2* __restrict__ ranges, float* __restrict__ out,
    const uint32_t* __restrict__ order, const WsHeader* __restrict__ hdr, int64_t n_tiles,
    int persistent) {
    __shared__ FwdLds<T, B> sm;
    if (!persistent) {
        fwd_tile<T, B, kEll>(sm, imgs, n_img, svals, recs, offsets, eparams, ranges, out, xcd_tile(blockIdx.x, n_tiles));
        return;
    }
    const bool ordered = hdr->ordered != 0;
    run_persistent(n_tiles, [&](int64_t item) {
        const int64_t tile = ordered ? (int64_t)order[item] : item;
        if (tile < n_tiles) fwd_tile<T, B, kEll>(sm, imgs, n_img, svals, recs, offsets, eparams, ranges, out, tile);
    });
}

template <int T, int B, bool kL1, bool kEll, typename Table>
__global__ __launch_bounds__(TileShape<T>::kThreads)
__attribute__((amdgpu_waves_per_eu(BwdOccupancy<T, B, kEll>::kMinWaves, 8))) void k_render_bwd(
    Table imgs, int n_img, const uint32_t* __restrict__ svals, const GRec* __restrict__ recs,
    const int32_t* __restrict__ offsets, const EParams* __restrict__ eparams,
    const int2* __restrict__ ranges, const float* __restrict__ grad_out,
    const float* __restrict__ target, float inv_numel, double* __restrict__ tile_loss,
    float* __restrict__ moments, float4* __restrict__ partials, int atomic_grads,
    const uint32_t* __restrict__ order, const WsHeader* __restrict__ hdr, int64_t n_tiles,
    int persistent) {
    __shared__ BwdLds<T, B> sm;
    if (!persistent) {
        bwd_tile<T, B, kL1, kEll>(sm, imgs, n_img, svals, recs, offsets, eparams, ranges, grad_out, target, inv_numel,
                            tile_loss, moments, partials, atomic_grads, xcd_tile(blockIdx.x, n_tiles));
        return;
    }
    const bool ordered = hdr->ordered != 0;
    run_persistent(n_tiles, [&](int64_t item) {
        const int64_t tile = ordered ? (int64_t)order[item] : item;
        if (tile < n_tiles)
            bwd_tile<T, B, kL1, kEll>(sm, imgs, n_img, svals, recs, offsets, eparams, ranges, grad_out, target, inv_numel,
                                tile_loss, moments, partials, atomic_grads, tile);
    });
}

template <int T, int B, bool kEll, typename Table>
__global__ __launch_bounds__(TileShape<T>::kThreads)
__attribute__((amdgpu_waves_per_eu(BwdOccupancy<T, B, kEll>::kMinWaves, 8))) void k_render_fused(
    Table imgs, int n_img, const uint32_t* __restrict__ svals, const GRec* __restrict__ recs,
    const int32_t* __restrict__ offsets, const EParams* __restrict__ eparams,
    const int2* __restrict__ ranges, float* __restrict__ out,
    const float* __restrict__ target, float inv_numel, double* __restrict__ tile_loss,
    float* __restrict__ moments, float4* __restrict__ partials, int atomic_grads,
    const uint32_t* __restrict__ order, const WsHeader* __restrict__ hdr, int64_t n_tiles,
    int persistent) {
    __shared__ BwdLds<T, B> sm;
    if (!persistent) {
        fused_tile<T, B, kEll>(sm, imgs, n_img, svals, recs, offsets, eparams, ranges, out, target, inv_numel, tile_loss,
                         moments, partials, atomic_grads, xcd_tile(blockIdx.x, n_tiles));
        return;
    }
    const bool ordered = hdr->ordered != 0;
    run_persistent(n_tiles, [&](int64_t item) {
        const int64_t tile = ordered ? (int64_t)order[item] : item;
        if (tile < n_tiles)
            fused_tile<T, B, kEll>(sm, imgs, n_img, svals, recs, offsets, eparams, ranges, out, target, inv_numel, tile_loss,
                             moments, partials, atomic_grads, tile);
    });
}

// Distributed L1 loss value: workgroup `part` of `nparts` sums the per-tile
// L1 sums of tiles [lo, hi) into parts[part]; the last workgroup to finish
// adds the nparts sums in part order and writes the mean to *loss, then
// resets the counter.  Every order is fixed, so the value is reproducible
// whichever workgroup finishes last.  All threads of the workgroup call it.
__device__ __forceinline__ void loss_reduce(const double* __restrict__ tile_loss, int64_t lo,
                                            int64_t hi, double* __restrict__ parts,
                                            int nparts, int part, uint32_t* __restrict__ counter,
                                            double inv_numel, double* __restrict__ loss) {
    __shared__ double red[kBlockG / 64];
    __shared__ int s_last;
    auto block_sum = [&](double v) {
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        double sum = 0.0;
        for (int k = 0; k < kBlockG / 64; ++k) sum += red[k];
        __syncthreads();
        return sum;
    };
    // eight independent loads in flight per thread, combined in a fixed order
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t t = lo + threadIdx.x;
    for (; t + 7 * kBlockG < hi; t += 8 * kBlockG) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += tile_loss[t + u * kBlockG];
    }
    for (; t < hi; t += kBlockG) a[0] += tile_loss[t];
    const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    const double bs = block_sum(s);
    if (threadIdx.x == 0) {
        parts[part] = bs;
        __threadfence();  // the part is visible before it is counted
        s_last = atomicAdd(counter, 1u) == (uint32_t)nparts - 1 ? 1 : 0;
    }
    __syncthreads();
    if (!s_last) return;  // uniform
    __threadfence();
    const volatile double* vp = parts;
    double t2 = 0.0;
    for (int k = threadIdx.x; k < nparts; k += kBlockG) t2 += vp[k];
    const double total = block_sum(t2);
    if (threadIdx.x == 0) {
        *loss = total * inv_numel;
        atomicExch(counter, 0u);
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
    float* __restrict__ moments, const int32_t* __restrict__ counts,
    const int32_t* __restrict__ offsets, const float4* __restrict__ partials, int64_t cap,
    int atomic_grads, float* __restrict__ grad_mean, float* __restrict__ grad_chol,
    float* __restrict__ grad_color, float* __restrict__ grad_opacity,
    const double* __restrict__ tile_loss, int64_t n_tiles, double inv_numel,
    double* __restrict__ loss, double* __restrict__ loss_parts, uint32_t* __restrict__ counter) {
    // with the loss, loss_parts(n_tiles) workgroups past the Gaussians' sum
    // the per-tile L1 sums
    const int64_t nbg = (n_gauss + kBlockG - 1) / kBlockG;
    if (loss && (int64_t)blockIdx.x >= nbg) {  // uniform
        const int64_t P = (int64_t)gridDim.x - nbg, b = (int64_t)blockIdx.x - nbg;
        loss_reduce(tile_loss, n_tiles * b / P, n_tiles * (b + 1) / P, loss_parts, (int)P, (int)b,
                    counter, inv_numel, loss);
        return;
    }
    const int64_t i = (int64_t)blockIdx.x * kBlockG + threadIdx.x;
    float m[8];
    for (int k = 0; k < 8; ++k) m[k] = 0.f;
    if (!atomic_grads && (int64_t)blockIdx.x * kBlockG < n_gauss) {  // uniform
        // this Gaussian's pairs, stored at their emission indices (tile
        // row-major within the Gaussian), added in that order; the pairs at
        // or past the capacity were never emitted.  The block's Gaussians
        // own one contiguous span of pairs, staged through LDS in coalesced
        // chunks.
        __shared__ float4 sp[kFinChunk][2];
        const int64_t g0 = (int64_t)blockIdx.x * kBlockG;
        const int64_t gl = min(g0 + kBlockG, n_gauss) - 1;
        const int64_t s0 = offsets[g0];
        const int64_t s1 = min((int64_t)offsets[gl] + counts[gl], cap);
        int64_t e0 = 0, e1 = 0;
        if (i < n_gauss) {
            e0 = offsets[i];
            e1 = min(e0 + counts[i], cap);
        }
        for (int64_t c0 = s0; c0 < s1; c0 += kFinChunk) {  // uniform
            const int len = (int)min((int64_t)kFinChunk, s1 - c0);
            for (int k = threadIdx.x; k < len; k += kBlockG) {
                sp[k][0] = partials[2 * (c0 + k)];
                sp[k][1] = partials[2 * (c0 + k) + 1];
            }
            __syncthreads();
            const int64_t a = max(e0, c0), b = min(e1, c0 + len);
            for (int64_t e = a; e < b; ++e) {
                const float4 u = sp[e - c0][0], v = sp[e - c0][1];
                m[0] += u.x; m[1] += u.y; m[2] += u.z; m[3] += u.w;
                m[4] += v.x; m[5] += v.y; m[6] += v.z; m[7] += v.w;
            }
            __syncthreads();
        }
    }
    if (i >= n_gauss) return;
    const GRec r = recs[i];
    double gm0 = 0, gm1 = 0, gl0 = 0, gl1 = 0, gl2 = 0, gc0 = 0, gc1 = 0, gc2 = 0, ga = 0;
    if (atomic_grads) {
        float4* mp = reinterpret_cast<float4*>(moments + i * 8);
        const float4 u = mp[0], v = mp[1];
        m[0] = u.x; m[1] = u.y; m[2] = u.z; m[3] = u.w;
        m[4] = v.x; m[5] = v.y; m[6] = v.z; m[7] = v.w;
        mp[0] = make_float4(0.f, 0.f, 0.f, 0.f);  // ready for the next backward
        mp[1] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (r.x0 <= r.x1 && !(r.flags & kRecNoAmp)) {
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

__global__ void k_zero_double(double* __restrict__ p) { *p = 0.0; }

// L1 gradient sign(img - tgt) / numel per element; each workgroup adds its
// share of the mean |img - tgt| to *loss (zeroed by k_zero_double first).
__global__ __launch_bounds__(kBlockG) void k_l1(const float* __restrict__ img,
                                                const float* __restrict__ tgt, int64_t numel,
                                                float* __restrict__ grad,
                                                double* __restrict__ loss) {
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
        atomicAdd(loss, b / (double)numel);
    }
}

// The L1 loss value alone: loss_parts(n_tiles) workgroups, split as the
// gradient kernel's loss workgroups split the tiles.
__global__ __launch_bounds__(kBlockG) void k_sum_loss(const double* __restrict__ tile_loss,
                                                      int64_t n_tiles, double inv_numel,
                                                      double* __restrict__ loss,
                                                      double* __restrict__ parts,
                                                      uint32_t* __restrict__ counter) {
    const int64_t P = gridDim.x, b = blockIdx.x;
    loss_reduce(tile_loss, n_tiles * b / P, n_tiles * (b + 1) / P, parts, (int)P, (int)b,
                counter, inv_numel, loss);
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_sum_loss(const Layout& L, const Ws& w, int64_t numel, double* loss,
                           hipStream_t st) {
    const int nb = loss_parts(L.n_tiles);
    hipLaunchKernelGGL(k_sum_loss, dim3(nb), dim3(kBlockG), 0, st, w.tile_loss, L.n_tiles,
                       1.0 / (double)numel, loss, w.loss_parts, w.counters + kLossCounterWord);
    return hipGetLastError();
}

// Grid of a tile kernel: one workgroup per tile, or, persistent, as many as
// fit on the device at once (never more than the tiles).
static hipError_t tile_grid(const Layout& L, const void* kernel, int threads, unsigned* grid) {
    *grid = (unsigned)L.n_tiles;
    if (!(L.flags & GS_FLAG_PERSISTENT)) return hipSuccess;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0);
    if (e != hipSuccess) return e;
    // exactly the resident workgroups: a workgroup's first item is fixed by
    // its index, so one that could only start once another has left would
    // hold its item back until the end
    const int64_t resident = (int64_t)std::max(cus, 1) * std::max(per_cu, 1);
    *grid = (unsigned)std::min<int64_t>(L.n_tiles, resident);
    return hipSuccess;
}

template <int T, int B, bool kEll, typename Table>
static hipError_t launch_fwd_tb(const Layout& L, const Ws& w, const Table& tab, float* out,
                                hipStream_t st) {
    const auto kernel = k_render_fwd<T, B, kEll, Table>;
    unsigned grid = 0;
    const hipError_t e = tile_grid(L, reinterpret_cast<const void*>(kernel),
                                   TileShape<T>::kThreads, &grid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(TileShape<T>::kThreads), 0, st, tab, L.n_img,
                       w.lists, w.recs, w.offsets, w.eparams, w.ranges, out, w.order, w.hdr, L.n_tiles,
                       (L.flags & GS_FLAG_PERSISTENT) ? 1 : 0);
    return hipGetLastError();
}

template <typename Table>
static hipError_t launch_fwd_t(const Layout& L, const Ws& w, const Table& tab, float* out,
                               hipStream_t st) {
    if (L.flags & GS_FLAG_ELLIPSE) {  // one batch per tile size (the default)
        if (L.tile == 8) return launch_fwd_tb<8, 64, true>(L, w, tab, out, st);
        if (L.tile == 16) return launch_fwd_tb<16, 96, true>(L, w, tab, out, st);
        if (L.tile == 32) return launch_fwd_tb<32, 32, true>(L, w, tab, out, st);
        return hipErrorInvalidValue;
    }
    const int b = L.lds_batch;
    switch (L.tile) {
        case 8:
            if (b == 32) return launch_fwd_tb<8, 32, false>(L, w, tab, out, st);
            if (b == 64) return launch_fwd_tb<8, 64, false>(L, w, tab, out, st);
            break;
        case 16:
            if (b == 64) return launch_fwd_tb<16, 64, false>(L, w, tab, out, st);
            if (b == 96) return launch_fwd_tb<16, 96, false>(L, w, tab, out, st);
            if (b == 112) return launch_fwd_tb<16, 112, false>(L, w, tab, out, st);
            if (b == 128) return launch_fwd_tb<16, 128, false>(L, w, tab, out, st);
            if (b == 256) return launch_fwd_tb<16, 256, false>(L, w, tab, out, st);
            break;
        case 32:
            if (b == 32) return launch_fwd_tb<32, 32, false>(L, w, tab, out, st);
            if (b == 64) return launch_fwd_tb<32, 64, false>(L, w, tab, out, st);
            break;
        default:
            break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_render_fwd(const Layout& L, const Ws& w, float* out, hipStream_t st) {
    if (L.n_tiles == 0) return hipSuccess;
    if (L.n_img <= kSetupChunk && L.host_imgs) {
        ArgTable tab;
        for (int k = 0; k < kSetupChunk; ++k) tab.c.img[k] = k < L.n_img ? L.host_imgs[k] : ImgDev{};
        return launch_fwd_t(L, w, tab, out, st);
    }
    return launch_fwd_t(L, w, MemTable{w.imgs}, out, st);
}

template <int T, int B, bool kL1, bool kEll, typename Table>
static hipError_t launch_bwd_tt(const Layout& L, const Ws& w, const Table& tab,
                                const float* grad_out, const float* target, float inv_numel,
                                hipStream_t st) {
    const auto kernel = k_render_bwd<T, B, kL1, kEll, Table>;
    unsigned grid = 0;
    const hipError_t e = tile_grid(L, reinterpret_cast<const void*>(kernel),
                                   TileShape<T>::kThreads, &grid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(TileShape<T>::kThreads), 0, st, tab, L.n_img,
                       w.lists, w.recs, w.offsets, w.eparams, w.ranges, grad_out, target, inv_numel, w.tile_loss, w.moments,
                       w.partials, (L.flags & GS_FLAG_ATOMIC_GRADS) ? 1 : 0, w.order, w.hdr,
                       L.n_tiles, (L.flags & GS_FLAG_PERSISTENT) ? 1 : 0);
    return hipGetLastError();
}

template <bool kL1, typename Table>
static hipError_t launch_bwd_t(const Layout& L, const Ws& w, const Table& tab,
                               const float* grad_out, const float* target, float inv_numel,
                               hipStream_t st) {
    if (L.flags & GS_FLAG_ELLIPSE) {  // one batch per tile size (the default)
        if (L.tile == 8)
            return launch_bwd_tt<8, 64, kL1, true>(L, w, tab, grad_out, target, inv_numel, st);
        if (L.tile == 16)
            return launch_bwd_tt<16, 96, kL1, true>(L, w, tab, grad_out, target, inv_numel, st);
        if (L.tile == 32)
            return launch_bwd_tt<32, 32, kL1, true>(L, w, tab, grad_out, target, inv_numel, st);
        return hipErrorInvalidValue;
    }
    const int b = L.lds_batch;
    switch (L.tile) {
        case 8:
            if (b == 32) return launch_bwd_tt<8, 32, kL1, false>(L, w, tab, grad_out, target, inv_numel, st);
            if (b == 64) return launch_bwd_tt<8, 64, kL1, false>(L, w, tab, grad_out, target, inv_numel, st);
            break;
        case 16:
            if (b == 64) return launch_bwd_tt<16, 64, kL1, false>(L, w, tab, grad_out, target, inv_numel, st);
            if (b == 96) return launch_bwd_tt<16, 96, kL1, false>(L, w, tab, grad_out, target, inv_numel, st);
            if (b == 112) return launch_bwd_tt<16, 112, kL1, false>(L, w, tab, grad_out, target, inv_numel, st);
            if (b == 128)
                return launch_bwd_tt<16, 128, kL1, false>(L, w, tab, grad_out, target, inv_numel, st);
            if (b == 256)
                return launch_bwd_tt<16, 256, kL1, false>(L, w, tab, grad_out, target, inv_numel, st);
            break;
        case 32:
            if (b == 32) return launch_bwd_tt<32, 32, kL1, false>(L, w, tab, grad_out, target, inv_numel, st);
            if (b == 64) return launch_bwd_tt<32, 64, kL1, false>(L, w, tab, grad_out, target, inv_numel, st);
            break;
        default:
            break;
    }
    return hipErrorInvalidValue;
}

template <bool kL1>
static hipError_t launch_bwd_any(const Layout& L, const Ws& w, const float* grad_out,
                                 const float* target, float inv_numel, hipStream_t st) {
    if (L.n_tiles == 0) return hipSuccess;
    if (L.n_img <= kSetupChunk && L.host_imgs) {
        ArgTable tab;
        for (int k = 0; k < kSetupChunk; ++k) tab.c.img[k] = k < L.n_img ? L.host_imgs[k] : ImgDev{};
        return launch_bwd_t<kL1>(L, w, tab, grad_out, target, inv_numel, st);
    }
    return launch_bwd_t<kL1>(L, w, MemTable{w.imgs}, grad_out, target, inv_numel, st);
}

hipError_t launch_render_bwd(const Layout& L, const Ws& w, const float* grad_out,
                             hipStream_t st) {
    return launch_bwd_any<false>(L, w, grad_out, nullptr, 0.f, st);
}

hipError_t launch_render_bwd_l1(const Layout& L, const Ws& w, const float* out,
                                const float* target, int64_t numel, hipStream_t st) {
    return launch_bwd_any<true>(L, w, out, target, (float)(1.0 / (double)numel), st);
}

template <int T, int B, bool kEll, typename Table>
static hipError_t launch_fused_tt(const Layout& L, const Ws& w, const Table& tab, float* out,
                                  const float* target, float inv_numel, hipStream_t st) {
    const auto kernel = k_render_fused<T, B, kEll, Table>;
    unsigned grid = 0;
    const hipError_t e = tile_grid(L, reinterpret_cast<const void*>(kernel),
                                   TileShape<T>::kThreads, &grid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(TileShape<T>::kThreads), 0, st, tab, L.n_img,
                       w.lists, w.recs, w.offsets, w.eparams, w.ranges, out, target, inv_numel, w.tile_loss, w.moments,
                       w.partials, (L.flags & GS_FLAG_ATOMIC_GRADS) ? 1 : 0, w.order, w.hdr,
                       L.n_tiles, (L.flags & GS_FLAG_PERSISTENT) ? 1 : 0);
    return hipGetLastError();
}

template <typename Table>
static hipError_t launch_fused_t(const Layout& L, const Ws& w, const Table& tab, float* out,
                                 const float* target, float inv_numel, hipStream_t st) {
    if (L.flags & GS_FLAG_ELLIPSE) {  // one batch per tile size (the default)
        if (L.tile == 8) return launch_fused_tt<8, 64, true>(L, w, tab, out, target, inv_numel, st);
        if (L.tile == 16)
            return launch_fused_tt<16, 96, true>(L, w, tab, out, target, inv_numel, st);
        if (L.tile == 32)
            return launch_fused_tt<32, 32, true>(L, w, tab, out, target, inv_numel, st);
        return hipErrorInvalidValue;
    }
    const int b = L.lds_batch;
    switch (L.tile) {
        case 8:
            if (b == 32) return launch_fused_tt<8, 32, false>(L, w, tab, out, target, inv_numel, st);
            if (b == 64) return launch_fused_tt<8, 64, false>(L, w, tab, out, target, inv_numel, st);
            break;
        case 16:
            if (b == 64) return launch_fused_tt<16, 64, false>(L, w, tab, out, target, inv_numel, st);
            if (b == 96) return launch_fused_tt<16, 96, false>(L, w, tab, out, target, inv_numel, st);
            if (b == 112) return launch_fused_tt<16, 112, false>(L, w, tab, out, target, inv_numel, st);
            if (b == 128) return launch_fused_tt<16, 128, false>(L, w, tab, out, target, inv_numel, st);
            if (b == 256) return launch_fused_tt<16, 256, false>(L, w, tab, out, target, inv_numel, st);
            break;
        case 32:
            if (b == 32) return launch_fused_tt<32, 32, false>(L, w, tab, out, target, inv_numel, st);
            if (b == 64) return launch_fused_tt<32, 64, false>(L, w, tab, out, target, inv_numel, st);
            break;
        default:
            break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_render_fused_l1(const Layout& L, const Ws& w, float* out, const float* target,
                                  int64_t numel, hipStream_t st) {
    if (L.n_tiles == 0) return hipSuccess;
    const float inv = (float)(1.0 / (double)numel);
    if (L.n_img <= kSetupChunk && L.host_imgs) {
        ArgTable tab;
        for (int k = 0; k < kSetupChunk; ++k) tab.c.img[k] = k < L.n_img ? L.host_imgs[k] : ImgDev{};
        return launch_fused_t(L, w, tab, out, target, inv, st);
    }
    return launch_fused_t(L, w, MemTable{w.imgs}, out, target, inv, st);
}

hipError_t launch_finalize(const Layout& L, const Ws& w, const float* chol,
                           const float* color, const float* opacity, float* grad_mean,
                           float* grad_chol, float* grad_color, float* grad_opacity,
                           hipStream_t st, int64_t numel, double* loss) {
    const int nb_loss = loss_parts(L.n_tiles);
    const int nb = (int)blocks_for(L.n_gauss, kBlockG) + (loss ? nb_loss : 0);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(nb), dim3(kBlockG), 0, st, w.recs, L.n_gauss, chol,
                       color, opacity, w.moments, w.counts, w.offsets, w.partials, L.cap,
                       (L.flags & GS_FLAG_ATOMIC_GRADS) ? 1 : 0, grad_mean, grad_chol,
                       grad_color, grad_opacity, w.tile_loss, L.n_tiles,
                       loss ? 1.0 / (double)numel : 0.0, loss, w.loss_parts,
                       w.counters + kLossCounterWord);
    return hipGetLastError();
}

hipError_t launch_l1(const float* img, const float* target, int64_t numel, float* grad,
                     double* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_double, dim3(1), dim3(1), 0, st, loss);
    if (numel == 0) return hipGetLastError();
    // at most 256 workgroups: each adds one double to *loss, and atomics
    // on a single address serialise
    int nb = blocks_for(numel, kBlockG * 4);
    if (nb > 256) nb = 256;
    hipLaunchKernelGGL(k_l1, dim3(nb), dim3(kBlockG), 0, st, img, target, numel, grad, loss);
    return hipGetLastError();
}

}  // namespace gs
