// Matrix-core throughput probes: the measured ceilings beside which the
// matchers' rates are read. Every wavefront runs `iters` rounds of four
// independent accumulator chains of one MFMA shape (operands held in
// registers, so nothing but the matrix cores is exercised) and folds its
// accumulators into one value per wavefront, written to `out` so that no
// work can be removed.
#include "internal.h"

namespace lpsift {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef int intx4 __attribute__((ext_vector_type(4)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef int intx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kProbeBlocks = 2048;   // 8 per compute unit, 4 wavefronts each

template <int kKind>
__global__ __launch_bounds__(256) void mfma_probe_kernel(int64_t iters, float* out)
{
    const int lane = threadIdx.x & 63;
    const float x = 1.0f + (float)lane * 1e-3f;
    float r = 0.0f;
    if (kKind == LPSIFT_PROBE_MFMA_F32) {
        floatx16 c[4] = {};
        for (int64_t i = 0; i < iters; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) c[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, x, c[k], 0, 0, 0);
        for (int k = 0; k < 4; ++k)
            for (int e = 0; e < 16; ++e) r += c[k][e];
    } else if (kKind == LPSIFT_PROBE_MFMA_BF16) {
        bf16x8 a;
        for (int e = 0; e < 8; ++e) a[e] = (__bf16)x;
        floatx16 c[4] = {};
        for (int64_t i = 0; i < iters; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) c[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, c[k], 0, 0, 0);
        for (int k = 0; k < 4; ++k)
            for (int e = 0; e < 16; ++e) r += c[k][e];
    } else if (kKind == LPSIFT_PROBE_MFMA_FP8) {
        intx8 a;
        for (int e = 0; e < 8; ++e) a[e] = 0x38383838 + lane;   // E4M3 values near 1
        floatx16 c[4] = {};
        for (int64_t i = 0; i < iters; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                c[k] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, a, c[k], 0, 0, 0, 0, 0, 0);
        for (int k = 0; k < 4; ++k)
            for (int e = 0; e < 16; ++e) r += c[k][e];
    } else {
        intx4 a = {1 + lane, 2, 3, 4};
        intx16 c[4] = {};
        for (int64_t i = 0; i < iters; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) c[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, a, c[k], 0, 0, 0);
        for (int k = 0; k < 4; ++k)
            for (int e = 0; e < 16; ++e) r += (float)c[k][e];
    }
    if (lane == 0) out[blockIdx.x * 4 + (threadIdx.x >> 6)] = r;
}

}  // namespace

int64_t probe_out_floats()
{
    return (int64_t)kProbeBlocks * 4;
}

double probe_ops(int kind, int64_t iters)
{
    // multiply-adds x 2 per MFMA: 32x32x2, 32x32x16, 32x32x64, 32x32x32
    const double k = kind == LPSIFT_PROBE_MFMA_F32 ? 2 : kind == LPSIFT_PROBE_MFMA_BF16 ? 16
                   : kind == LPSIFT_PROBE_MFMA_FP8 ? 64 : 32;
    return 2.0 * 32 * 32 * k * 4.0 * (double)iters * probe_out_floats();
}

int launch_probe(int kind, int64_t iters, float* out, hipStream_t s)
{
    const dim3 g(kProbeBlocks), b(256);
    switch (kind) {
    case LPSIFT_PROBE_MFMA_F32:
        hipLaunchKernelGGL(mfma_probe_kernel<LPSIFT_PROBE_MFMA_F32>, g, b, 0, s, iters, out);
        break;
    case LPSIFT_PROBE_MFMA_BF16:
        hipLaunchKernelGGL(mfma_probe_kernel<LPSIFT_PROBE_MFMA_BF16>, g, b, 0, s, iters, out);
        break;
    case LPSIFT_PROBE_MFMA_FP8:
        hipLaunchKernelGGL(mfma_probe_kernel<LPSIFT_PROBE_MFMA_FP8>, g, b, 0, s, iters, out);
        break;
    default:
        hipLaunchKernelGGL(mfma_probe_kernel<LPSIFT_PROBE_MFMA_I8>, g, b, 0, s, iters, out);
        break;
    }
    return hipGetLastError() == hipSuccess ? LPSIFT_OK : LPSIFT_EHIP;
}

}  // namespace lpsift
