// Vector-ALU throughput probe for the roofline of the tile kernels: long
// chains of independent FP32 operations whose launch the caller times, so
// that the FP32 issue rate the library is compiled for (packed FP32
// instructions disabled), the cost of the hardware exp2 and the issue cost
// of the lane-mask forms the tile kernels choose between are measured on
// the device at hand rather than taken from a datasheet.  Not part of the
// rasterizer.
#include "gs_raster.h"

#include <hip/hip_runtime.h>

namespace gs {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kChains = 8;  // independent chains per thread

// kind 0: 8 chains of FMAs (2 FLOP each).  kind 1: 8 chains of exp2(-x).
// kind 2: per step z = fma(z, b, c), w = exp2(-z^2), acc = fma(w, b, acc),
// z = fma(w, c, z) * 0.5 (five FMA-class operations and one exp).
// Kinds 3-5: one FMA per chain and step followed by a per-lane mask, so the
// mask's issue cost is the step time minus kind 0's: kind 3 a select on a
// loop-invariant SGPR-pair lane mask; kind 4 a lane mask read from a VGPR
// word with readfirstlane (the other half formed on the scalar unit), then a
// select; kind 5 a sign-extended one-bit field of a VGPR word (bit = lane
// mod 32) ANDed into the value's bits.  The kind 4 and 5 words advance by an
// integer add each step.
__global__ __launch_bounds__(kProbeThreads) void k_valu_probe(int kind, int iters, float b,
                                                              float c, uint32_t mlo, uint32_t mhi,
                                                              float* __restrict__ out) {
    float a[kChains], acc[kChains];
    uint32_t u[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        a[i] = 0.1f + (float)threadIdx.x * 1e-4f + (float)i * 0.01f;
        acc[i] = 0.f;
        u[i] = 0x3c3c3c3cu ^ (threadIdx.x * 0x9E3779B9u) ^ (uint32_t)i;
    }
    const uint64_t m = ((uint64_t)mhi << 32) | mlo;
    const int bit = threadIdx.x & 31;
    if (kind == 0) {
#pragma unroll 4
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < kChains; ++i) a[i] = __builtin_fmaf(a[i], b, c);
        }
    } else if (kind == 1) {
#pragma unroll 4
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < kChains; ++i) a[i] = __builtin_amdgcn_exp2f(-a[i]);
        }
    } else if (kind == 2) {
#pragma unroll 4
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < kChains; ++i) {
                const float z1 = __builtin_fmaf(a[i], b, c);
                const float w = __builtin_amdgcn_exp2f(-(z1 * z1));
                acc[i] = __builtin_fmaf(w, b, acc[i]);
                a[i] = __builtin_fmaf(w, c, z1) * 0.5f;
            }
        }
    } else if (kind == 3) {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < kChains; ++i) {
                const float v = __builtin_fmaf(a[i], b, c);
                a[i] = __builtin_amdgcn_inverse_ballot_w64(m) ? v : c;
            }
        }
    } else if (kind == 4) {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < kChains; ++i) {
                const float v = __builtin_fmaf(a[i], b, c);
                const uint32_t lo = __builtin_amdgcn_readfirstlane(u[i]);
                const uint32_t hi = __builtin_amdgcn_readfirstlane(u[i] ^ 0x5555u);
                a[i] = __builtin_amdgcn_inverse_ballot_w64(((uint64_t)hi << 32) | lo) ? v : c;
                u[i] += 0x01010101u;
            }
        }
    } else {
#pragma unroll 4
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < kChains; ++i) {
                const float v = __builtin_fmaf(a[i], b, c);
                const uint32_t keep = (uint32_t)__builtin_amdgcn_sbfe((int32_t)u[i], bit, 1);
                a[i] = __uint_as_float(__float_as_uint(v) & keep);
                u[i] += 0x01010101u;
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i] + acc[i] + (float)(u[i] & 1u);
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;  // keeps the chains live
}

}  // namespace
}  // namespace gs

extern "C" gs_status gs_valu_probe(int32_t kind, int32_t blocks, int32_t iters, float* out,
                                   void* stream) {
    if (kind < 0 || kind > 5 || blocks < 1 || iters < 1 || out == nullptr) return GS_E_INVALID;
    hipLaunchKernelGGL(gs::k_valu_probe, dim3(blocks), dim3(gs::kProbeThreads), 0,
                       static_cast<hipStream_t>(stream), (int)kind, (int)iters, 0.999f, 1e-3f,
                       0x0f0f0f0fu, 0x33333333u, out);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_E_DEVICE;
}
