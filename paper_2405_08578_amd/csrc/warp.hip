// Warping registered images into one canvas and blending them (the stitched
// output of Sec. 4, Fig. 2(f) and Fig. 9).
//
// warp_blend_kernel: a 256-thread workgroup owns a 128 x 8 pixel canvas
// tile, each thread four consecutive pixels of one row. Images whose canvas
// bounding box (from the host, one pixel of margin) misses the tile are
// skipped by the whole workgroup. For the others, each pixel's reference
// point goes through the image's inverse transform in double; a covered
// pixel takes the bilinear sample and the feather weight
// min(x + 1, w - x, y + 1, h - y), summed in double in image order; the
// canvas gets sum(weight x sample) / sum(weight) rounded to float once and
// the number of covering images. Each canvas pixel is written once.
#include "internal.h"

namespace lpsift {
namespace {

constexpr int kTileW = 128, kTileH = 8;

__global__ __launch_bounds__(256) void warp_blend_kernel(WarpArgs a)
{
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int tu0 = blockIdx.x * kTileW, tv0 = blockIdx.y * kTileH;
    const int u0 = tu0 + tx * 4;
    const int v = tv0 + ty;
    double acc[4] = {0.0, 0.0, 0.0, 0.0}, sw[4] = {0.0, 0.0, 0.0, 0.0};
    int cnt[4] = {0, 0, 0, 0};
    const double py = (double)v + a.y0;
    for (int k = 0; k < a.n; ++k) {
        const WarpImg& I = a.img[k];
        if (I.bx1 <= tu0 || I.bx0 >= tu0 + kTileW || I.by1 <= tv0 || I.by0 >= tv0 + kTileH)
            continue;
        const double* m = I.hi;
        const double rx = m[1] * py + m[2], ry = m[4] * py + m[5], rz = m[7] * py + m[8];
        const double wm1 = (double)(I.w - 1), hm1 = (double)(I.h - 1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int u = u0 + j;
            if (u >= a.W || v >= a.H) continue;
            const double px = (double)u + a.x0;
            const double iz = 1.0 / (m[6] * px + rz);
            const double qx = (m[0] * px + rx) * iz, qy = (m[3] * px + ry) * iz;
            if (!(qx >= 0.0 && qx <= wm1 && qy >= 0.0 && qy <= hm1)) continue;
            const int ix = (int)qx, iy = (int)qy;          // qx, qy >= 0: truncation = floor
            const double fx = qx - (double)ix, fy = qy - (double)iy;
            const int ix1 = ix + 1 < I.w ? ix + 1 : I.w - 1;
            const int iy1 = iy + 1 < I.h ? iy + 1 : I.h - 1;
            const uint8_t* r0 = I.data + (int64_t)iy * I.pitch;
            const uint8_t* r1 = I.data + (int64_t)iy1 * I.pitch;
            const double top = (1.0 - fx) * (double)r0[ix] + fx * (double)r0[ix1];
            const double bot = (1.0 - fx) * (double)r1[ix] + fx * (double)r1[ix1];
            const double val = (1.0 - fy) * top + fy * bot;
            const double wgt = fmin(fmin(qx + 1.0, (double)I.w - qx), fmin(qy + 1.0, (double)I.h - qy));
            acc[j] += wgt * val;
            sw[j] += wgt;
            ++cnt[j];
        }
    }
    if (v >= a.H) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int u = u0 + j;
        if (u >= a.W) continue;
        const int64_t o = (int64_t)v * a.W + u;
        a.canvas[o] = sw[j] > 0.0 ? (float)(acc[j] / sw[j]) : 0.0f;
        if (a.count) a.count[o] = (uint8_t)cnt[j];
    }
}

}  // namespace

int launch_warp_blend(const WarpArgs& a, hipStream_t stream)
{
    if (a.W == 0 || a.H == 0) return LPSIFT_OK;
    TimedScope ts(LPSIFT_KERNEL_WARP, stream);
    hipLaunchKernelGGL(warp_blend_kernel, dim3((a.W + kTileW - 1) / kTileW, (a.H + kTileH - 1) / kTileH),
                       dim3(256), 0, stream, a);
    return hipGetLastError() == hipSuccess ? LPSIFT_OK : LPSIFT_EHIP;
}

}  // namespace lpsift
