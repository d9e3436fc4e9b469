// Vector-ALU throughput probe for the roofline of the tile kernels: long
// chains of independent FP32 operations whose launch the caller times, so
// that the FP32 issue rate the library is compiled for (packed FP32
// instructions disabled) and the cost of the hardware exp2 are measured on
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
__global__ __launch_bounds__(kProbeThreads) void k_valu_probe(int kind, int iters, float b,
                                                              float c, float* __restrict__ out) {
    float a[kChains], acc[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        a[i] = 0.1f + (float)threadIdx.x * 1e-4f + (float)i * 0.01f;
        acc[i] = 0.f;
    }
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
    } else {
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
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i] + acc[i];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;  // keeps the chains live
}

}  // namespace
}  // namespace gs

extern "C" gs_status gs_valu_probe(int32_t kind, int32_t blocks, int32_t iters, float* out,
                                   void* stream) {
    if (kind < 0 || kind > 2 || blocks < 1 || iters < 1 || out == nullptr) return GS_E_INVALID;
    hipLaunchKernelGGL(gs::k_valu_probe, dim3(blocks), dim3(gs::kProbeThreads), 0,
                       static_cast<hipStream_t>(stream), (int)kind, (int)iters, 0.999f, 1e-3f,
                       out);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_E_DEVICE;
}
