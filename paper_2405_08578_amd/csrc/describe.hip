// Orientation assignment and SIFT description at the detected window extrema
// (Sec. 2.3, Eq. 3-5).
//
// Three kernels, all enqueued by launch_describe:
//  1. disc_tables_kernel: for every scale, the integer offsets of the
//     orientation disc (radius round(1.5 w_s)) and of the descriptor disc
//     (radius w_s sqrt(2) (d+1)/2, which circumscribes the rotated d+1 cell
//     square where trilinear weights can be non-zero), row-major.
//  2. polar_field_kernel: the Eq. 5 gradient of every pixel once, as
//     (magnitude, angle in turns in [0, 1)); border pixels get magnitude 0.
//     Each image pixel is visited by ~10 keypoint supports, so the atan2 and
//     the square root are paid once per pixel instead of once per visit.
//  3. orient_describe_kernel: one wavefront per keypoint. Lane l walks the
//     l-th contiguous 1/64 of the disc table, so the 64 lanes of one step are
//     spread over the whole support and their votes land in different cells;
//     votes go to a per-wave histogram in LDS with ds_add_f32. The histogram
//     is private to the wave, so its accumulation order is fixed by the
//     instruction stream. Orientation (36 bins, smoothing, argmax, parabola),
//     then the 128-bin descriptor, normalisation, clipping at 0.2 and
//     renormalisation happen in the same wave; the descriptor row is stored
//     with two coalesced 256-byte writes.
#include "internal.h"

namespace lpsift {
namespace {

constexpr float kTwoPiInv = 0.15915494309189535f;  // 1 / (2 pi)

// Images per launch (keeps the by-value kernel arguments small).
constexpr int kDescBatch = 8;

// ---------------------------------------------------------------- tables --

struct TableArgs {
    int32_t n_tables;
    int32_t r2[2 * LPSIFT_MAX_SCALES];
    int32_t off[2 * LPSIFT_MAX_SCALES];
};

__device__ inline int32_t pack_offset(int dx, int dy)
{
    return (int32_t)((uint32_t)(dx & 0xFFFF) | ((uint32_t)dy << 16));
}

// One workgroup per table; thread t writes rows dy = -R + t, -R + t + 256, ...
__global__ __launch_bounds__(256) void disc_tables_kernel(TableArgs a, int32_t* tables)
{
    const int t = blockIdx.x;
    const int r2 = a.r2[t];
    const int R = isqrt_floor(r2);
    int32_t* out = tables + a.off[t];
    for (int dy = -R + (int)threadIdx.x; dy <= R; dy += blockDim.x) {
        int start = 0;
        for (int y = -R; y < dy; ++y) start += 2 * isqrt_floor(r2 - y * y) + 1;
        const int hw = isqrt_floor(r2 - dy * dy);
        for (int dx = -hw; dx <= hw; ++dx) out[start + dx + hw] = pack_offset(dx, dy);
    }
}

// ---------------------------------------------------------- gradient field --

struct FieldImg {
    const uint8_t* data;
    int64_t pitch;
    int32_t h, w;
    float2* field;
};

struct FieldArgs {
    int32_t n_images;
    FieldImg img[kDescBatch];
};

// grid: (ceil(w/64), h, image); block 64 lanes along a row.
__global__ __launch_bounds__(64) void polar_field_kernel(FieldArgs a)
{
    const FieldImg& I = a.img[blockIdx.z];
    const int r = blockIdx.y;
    const int c = blockIdx.x * 64 + threadIdx.x;
    if (r >= I.h || c >= I.w) return;
    float2 out = make_float2(0.0f, 0.0f);
    if (r >= 1 && r <= I.h - 2 && c >= 1 && c <= I.w - 2) {
        const uint8_t* p = I.data + (int64_t)r * I.pitch + c;
        const int av = (int)p[I.pitch] - (int)p[-I.pitch];   // along rows
        const int bv = (int)p[1] - (int)p[-1];               // along columns
        const float f = sqrtf((float)(av * av + bv * bv));
        if (f > 0.0f) {
            float t = atan2f((float)av, (float)bv) * kTwoPiInv;
            if (t < 0.0f) t += 1.0f;
            if (t >= 1.0f) t -= 1.0f;
            out = make_float2(f, t);
        }
    }
    I.field[(int64_t)r * I.w + c] = out;
}

// ------------------------------------------------------ orient + describe --

struct DescImg {
    const float2* field;
    int32_t h, w;
    const int32_t* x;
    const int32_t* y;
    float* theta;
    float* desc;
};

struct DescArgs {   // passed by value: keep well under 4 KB
    int32_t n_images;
    int32_t n_scales;
    ScaleGeom geom[LPSIFT_MAX_SCALES];
    // Work is ordered by scale, largest first, so the longest waves start first.
    // Scale s (in that order) covers work items [scale_begin[s], scale_begin[s+1]).
    int64_t scale_begin[LPSIFT_MAX_SCALES + 1];
    int32_t scale_of[LPSIFT_MAX_SCALES];
    // Within a scale, image i covers [img_begin[s][i], img_begin[s][i+1]) and its
    // slots of that scale start at slot_base[s][i].
    int64_t img_begin[LPSIFT_MAX_SCALES][kDescBatch + 1];
    int64_t slot_base[LPSIFT_MAX_SCALES][kDescBatch];
    DescImg img[kDescBatch];
};

__device__ inline float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__global__ __launch_bounds__(64) void orient_describe_kernel(DescArgs a, const int32_t* tables)
{
    __shared__ float hist[128 + 36];
    const int lane = threadIdx.x;
    const int64_t item = blockIdx.x;

    // locate (scale, image, slot) of this work item
    int so = 0;
    while (so + 1 < a.n_scales && item >= a.scale_begin[so + 1]) ++so;
    int im = 0;
    while (im + 1 < a.n_images && item >= a.img_begin[so][im + 1]) ++im;
    const int64_t slot = a.slot_base[so][im] + (item - a.img_begin[so][im]);
    const DescImg& I = a.img[im];
    const ScaleGeom& G = a.geom[a.scale_of[so]];
    const int kx = I.x[slot], ky = I.y[slot];
    const float2* field = I.field;
    const int W = I.w, H = I.h;

    // ---- orientation histogram ----
    float* ho = hist + 128;
    if (lane < 36) ho[lane] = 0.0f;
    __syncthreads();
    {
        const int n = G.n_orient;
        const int per = (n + 63) / 64;
        const int32_t* tab = tables + G.off_orient;
        for (int it = 0; it < per; ++it) {
            const int j = lane * per + it;
            if (j >= n) break;
            const int32_t e = tab[j];
            const int dx = (int)(int16_t)(e & 0xFFFF), dy = e >> 16;
            const int px = kx + dx, py = ky + dy;
            if (px < 0 || px >= W || py < 0 || py >= H) continue;
            const float2 ft = field[(int64_t)py * W + px];
            if (ft.x == 0.0f) continue;
            const float wt = ft.x * exp2f((float)(dx * dx + dy * dy) * G.k_orient);
            const float t = ft.y * 36.0f;
            const float k0f = floorf(t);
            const float fr = t - k0f;
            int k0 = (int)k0f;
            if (k0 >= 36) k0 -= 36;
            const int k1 = (k0 == 35) ? 0 : k0 + 1;
            atomicAdd(&ho[k0], (1.0f - fr) * wt);
            atomicAdd(&ho[k1], fr * wt);
        }
    }
    __syncthreads();

    // smoothing, argmax (lowest bin on ties), parabolic refinement
    float sm = -1.0f;
    if (lane < 36) {
        sm = (ho[(lane + 34) % 36] + 4.0f * ho[(lane + 35) % 36] + 6.0f * ho[lane]
              + 4.0f * ho[(lane + 1) % 36] + ho[(lane + 2) % 36]) / 16.0f;
    }
    float bv = sm;
    int bk = lane;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(bv, off);
        const int ok = __shfl_xor(bk, off);
        if (ov > bv || (ov == bv && ok < bk)) {
            bv = ov;
            bk = ok;
        }
    }
    const float hm = __shfl(sm, (bk + 35) % 36);
    const float hp = __shfl(sm, (bk + 1) % 36);
    const float den = hm - 2.0f * bv + hp;
    const float offp = (den != 0.0f) ? 0.5f * (hm - hp) / den : 0.0f;
    const float th_turns = ((float)bk + offp) / 36.0f;
    if (lane == 0) I.theta[slot] = th_turns * 6.283185307179586f;

    // ---- descriptor histogram ----
    hist[lane] = 0.0f;
    hist[lane + 64] = 0.0f;
    __syncthreads();
    {
        float sn, cs;
        sincospif(2.0f * th_turns, &sn, &cs);
        const float iw = G.inv_ws;
        const int n = G.n_desc;
        const int per = (n + 63) / 64;
        const int32_t* tab = tables + G.off_desc;
        for (int it = 0; it < per; ++it) {
            const int j = lane * per + it;
            if (j >= n) break;
            const int32_t e = tab[j];
            const int dx = (int)(int16_t)(e & 0xFFFF), dy = e >> 16;
            const int px = kx + dx, py = ky + dy;
            if (px < 0 || px >= W || py < 0 || py >= H) continue;
            const float2 ft = field[(int64_t)py * W + px];
            if (ft.x == 0.0f) continue;
            // offset rotated by -theta0, in subregion units
            const float u = (cs * (float)dx + sn * (float)dy) * iw;
            const float v = (cs * (float)dy - sn * (float)dx) * iw;
            if (fabsf(u) >= 2.5f || fabsf(v) >= 2.5f) continue;   // no cell reachable
            const float m = ft.x * exp2f((float)(dx * dx + dy * dy) * G.k_desc);
            float rel = ft.y - th_turns;
            rel -= floorf(rel);
            const float t = rel * 8.0f;
            const float o0f = floorf(t);
            const float fo = t - o0f;
            int o0 = (int)o0f;
            if (o0 >= 8) o0 -= 8;
            const int o1 = (o0 + 1) & 7;
            const float cu = u + 1.5f, cv = v + 1.5f;
            const float ix0f = floorf(cu), iy0f = floorf(cv);
            const float fx = cu - ix0f, fy = cv - iy0f;
            const int ix0 = (int)ix0f, iy0 = (int)iy0f;
#pragma unroll
            for (int jy = 0; jy < 2; ++jy) {
                const int iy = iy0 + jy;
                if (iy < 0 || iy > 3) continue;
                const float wy = jy ? fy : 1.0f - fy;
#pragma unroll
                for (int jx = 0; jx < 2; ++jx) {
                    const int ix = ix0 + jx;
                    if (ix < 0 || ix > 3) continue;
                    const float wxy = m * (jx ? fx : 1.0f - fx) * wy;
                    float* cell = hist + (iy * 4 + ix) * 8;
                    atomicAdd(cell + o0, wxy * (1.0f - fo));
                    atomicAdd(cell + o1, wxy * fo);
                }
            }
        }
    }
    __syncthreads();

    // normalise, clip at 0.2, normalise again
    float d0 = hist[lane], d1 = hist[lane + 64];
    float nrm = fmaxf(sqrtf(wave_sum(d0 * d0 + d1 * d1)), 1e-12f);
    d0 = fminf(d0 / nrm, 0.2f);
    d1 = fminf(d1 / nrm, 0.2f);
    nrm = fmaxf(sqrtf(wave_sum(d0 * d0 + d1 * d1)), 1e-12f);
    float* out = I.desc + slot * 128;
    out[lane] = d0 / nrm;
    out[lane + 64] = d1 / nrm;
}

size_t field_offset(const Geometry& g)
{
    return align_up((size_t)g.table_entries * 4, 256);
}

}  // namespace

size_t describe_workspace_bytes(const lpsift_image* imgs, int n, const Geometry& g)
{
    size_t b = field_offset(g);
    for (int i = 0; i < n; ++i)
        b += align_up((size_t)imgs[i].height * (size_t)imgs[i].width * sizeof(float2), 256);
    return b;
}

int launch_describe(const lpsift_image* imgs, int n, const lpsift_keypoints* kps,
                    const Geometry& g, void* ws, float* const* theta, float* const* desc,
                    hipStream_t stream)
{
    char* base = static_cast<char*>(ws);
    int32_t* tables = reinterpret_cast<int32_t*>(base);

    TableArgs ta{};
    ta.n_tables = 2 * g.n_scales;
    for (int s = 0; s < g.n_scales; ++s) {
        ta.r2[2 * s] = g.s[s].r2_orient;
        ta.off[2 * s] = g.s[s].off_orient;
        ta.r2[2 * s + 1] = g.s[s].r2_desc;
        ta.off[2 * s + 1] = g.s[s].off_desc;
    }
    hipLaunchKernelGGL(disc_tables_kernel, dim3(ta.n_tables), dim3(256), 0, stream, ta, tables);
    if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;

    size_t foff = field_offset(g);
    for (int b0 = 0; b0 < n; b0 += kDescBatch) {
        const int nb = (n - b0 < kDescBatch) ? n - b0 : kDescBatch;
        FieldArgs fa{};
        DescArgs da{};
        fa.n_images = nb;
        da.n_images = nb;
        da.n_scales = g.n_scales;
        int maxw = 0, maxh = 0;
        for (int i = 0; i < nb; ++i) {
            const lpsift_image& im = imgs[b0 + i];
            float2* field = reinterpret_cast<float2*>(base + foff);
            foff += align_up((size_t)im.height * (size_t)im.width * sizeof(float2), 256);
            fa.img[i] = FieldImg{im.data, im.pitch, im.height, im.width, field};
            maxw = im.width > maxw ? im.width : maxw;
            maxh = im.height > maxh ? im.height : maxh;
            const lpsift_keypoints& kp = kps[b0 + i];
            da.img[i] = DescImg{field, im.height, im.width, kp.x, kp.y, theta[b0 + i], desc[b0 + i]};
        }
        hipLaunchKernelGGL(polar_field_kernel, dim3((maxw + 63) / 64, maxh, nb), dim3(64), 0,
                           stream, fa);
        if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;

        // work items: scales from the largest, images in order within a scale
        int64_t item = 0;
        for (int so = 0; so < g.n_scales; ++so) {
            const int s = g.n_scales - 1 - so;
            da.geom[s] = g.s[s];
            da.scale_of[so] = s;
            da.scale_begin[so] = item;
            for (int i = 0; i < nb; ++i) {
                const lpsift_image& im = imgs[b0 + i];
                int64_t slot = 0;
                for (int t = 0; t < s; ++t)
                    slot += 2 * n_windows(im.height, g.L[t]) * n_windows(im.width, g.L[t]);
                const int64_t cnt = 2 * n_windows(im.height, g.L[s]) * n_windows(im.width, g.L[s]);
                da.img_begin[so][i] = item;
                da.slot_base[so][i] = slot;
                item += cnt;
            }
            da.img_begin[so][nb] = item;
        }
        da.scale_begin[g.n_scales] = item;
        if (item > 0) {
            hipLaunchKernelGGL(orient_describe_kernel, dim3((unsigned)item), dim3(64), 0, stream,
                               da, tables);
            if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;
        }
    }
    return LPSIFT_OK;
}

}  // namespace lpsift
