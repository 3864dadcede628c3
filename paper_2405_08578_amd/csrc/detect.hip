// Multiscale window extrema (Sec. 2.2, Eq. 2) with the Eq. 1 ramp folded into
// an exact integer key.
//
// Nested window sets with windows of at most 128 px (the fast path):
// One workgroup owns a T x T tile of one image, T a multiple of the largest
// window side (about 128 px; the largest window is at most 128). The tile is
// staged once in LDS with coalesced 4-byte loads; every pixel becomes the key
//     value << 16 | row_in_tile << 8 | col_in_tile
// whose unsigned order is (intensity, raster index) inside the tile, i.e. the
// order Eq. 1 induces for any 0 < alpha < 1/(rows*cols). Level 0 windows are
// reduced by groups of lanes (cross-lane shuffles); every larger window, which
// the nesting condition makes a union of whole child windows, is the max / min
// of its children's keys. Each window's extrema and integer pixel sum are
// written to their fixed keypoint slots; nothing is compacted, so the output
// is deterministic and no atomics are needed.
#include "internal.h"

namespace lpsift {
namespace {

struct DetectImg {
    const uint8_t* data;
    int64_t pitch;
    int32_t h, w;
    int32_t tiles_x;
    int32_t tile_begin;        // first global tile index of this image
    int32_t* x;
    int32_t* y;
    uint8_t* scale;
    int8_t* type;
    uint8_t* value;
    float* contrast;
    int64_t base[LPSIFT_MAX_SCALES];   // first slot of each scale
};

struct DetectArgs {
    int32_t n_images;
    int32_t n_scales;
    int32_t T;                  // tile side
    int32_t Tp;                 // LDS row stride of the tile (multiple of 4)
    int32_t L[LPSIFT_MAX_SCALES];
    int32_t lvl_off[LPSIFT_MAX_SCALES];  // LDS word offset of each level's records
    int32_t tile_words;         // LDS word offset of the pixel tile
    DetectImg img[kMaxBatch];
};

constexpr int kThreads = 256;

typedef unsigned short ushort2v __attribute__((ext_vector_type(2)));

// Lane-wise max / min of two pairs of 16-bit keys (v_pk_max_u16 / v_pk_min_u16).
__device__ inline uint32_t pk_max(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(ushort2v, a),
                                                                  __builtin_bit_cast(ushort2v, b)));
}

__device__ inline uint32_t pk_min(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(ushort2v, a),
                                                                  __builtin_bit_cast(ushort2v, b)));
}

__device__ inline void write_kp(const DetectImg& I, int s, int64_t slot, int ox, int oy,
                                uint32_t key, uint32_t sum, uint32_t n, int8_t type)
{
    const uint32_t v = key >> 16;
    I.x[slot] = ox + (int32_t)(key & 255u);
    I.y[slot] = oy + (int32_t)((key >> 8) & 255u);
    I.scale[slot] = (uint8_t)s;
    I.type[slot] = type;
    I.value[slot] = (uint8_t)v;
    // |v n - sum| and 255 n are integers below 2^24: one correctly rounded division
    const int64_t num = (int64_t)v * n - (int64_t)sum;
    I.contrast[slot] = (float)(num < 0 ? -num : num) / (float)(255u * n);
}

__global__ __launch_bounds__(kThreads) void detect_kernel(DetectArgs args)
{
    extern __shared__ uint32_t smem[];
    const int tile = blockIdx.x;
    int im = 0;
    for (int i = 1; i < args.n_images; ++i)
        if (tile >= args.img[i].tile_begin) im = i;
    const DetectImg& I = args.img[im];
    const int T = args.T, Tp = args.Tp;
    const int local = tile - I.tile_begin;
    const int ty = local / I.tiles_x, tx = local - ty * I.tiles_x;
    const int ox = tx * T, oy = ty * T;
    const int tw = min(T, I.w - ox), th = min(T, I.h - oy);
    uint8_t* pix = reinterpret_cast<uint8_t*>(smem + args.tile_words);
    const int tid = threadIdx.x;

    // ---- stage the tile in LDS ----
    {
        const uint8_t* tile0 = I.data + (int64_t)oy * I.pitch + ox;
        const uintptr_t al = reinterpret_cast<uintptr_t>(tile0) | (uintptr_t)I.pitch;
        const bool al4 = (al & 3u) == 0;
        // 16- or 8-byte row pieces where the tile's address, the pitch and
        // the tile's width allow them (the LDS tile starts 16-byte aligned)
        if ((al & 15u) == 0 && (Tp & 15) == 0 && (tw & 15) == 0) {
            const int gpr = tw / 16;
            for (int idx = tid; idx < th * gpr; idx += kThreads) {
                const int r = idx / gpr, c = (idx - r * gpr) * 16;
                *reinterpret_cast<uint4*>(pix + r * Tp + c) =
                    *reinterpret_cast<const uint4*>(tile0 + (int64_t)r * I.pitch + c);
            }
        } else if ((al & 7u) == 0 && (Tp & 7) == 0 && (tw & 7) == 0) {
            const int gpr = tw / 8;
            for (int idx = tid; idx < th * gpr; idx += kThreads) {
                const int r = idx / gpr, c = (idx - r * gpr) * 8;
                *reinterpret_cast<uint2*>(pix + r * Tp + c) =
                    *reinterpret_cast<const uint2*>(tile0 + (int64_t)r * I.pitch + c);
            }
        } else {
        const int gpr = Tp / 4;
        for (int idx = tid; idx < th * gpr; idx += kThreads) {
            const int r = idx / gpr, c = (idx - r * gpr) * 4;
            if (c >= tw) continue;
            const uint8_t* src = tile0 + (int64_t)r * I.pitch + c;
            uint8_t* dst = pix + r * Tp + c;
            if (al4 && c + 4 <= tw) {
                *reinterpret_cast<uint32_t*>(dst) = *reinterpret_cast<const uint32_t*>(src);
            } else {
                for (int k = 0; k < 4 && c + k < tw; ++k) dst[k] = src[k];
            }
        }
        }
    }
    __syncthreads();

    // ---- level 0: groups of G lanes per window ----
    // Packed form (first window side a multiple of 4): a lane reads its rows
    // 4 pixels at a time and keeps 16-bit keys value << 8 | (row count << lc
    // | column in window), which order its pixels as (value, raster index)
    // do; two v_perm_b32 build four keys, v_pk_max_u16 / v_pk_min_u16 keep the
    // extremes and v_sad_u8 adds the four pixels. The lane's extremes are then
    // expanded to tile keys.
    {
        const int L0 = args.L[0];
        const int n0 = T / L0, nw = n0 * n0;
        int G = 1;
        while (G < 64 && 2 * G <= L0 && 2 * G * nw <= kThreads) G *= 2;
        const int groups = kThreads / G;
        const int g = tid % G, grp = tid / G;
        const int rows_pl = (L0 + G - 1) / G;   // rows per lane
        int lc = 0, rb = 0;
        while ((1 << lc) < L0) ++lc;
        while ((1 << rb) < rows_pl) ++rb;
        const bool packed = (L0 % 4) == 0 && lc + rb <= 8;
        uint32_t* rec = smem + args.lvl_off[0];
        const int nbx = (int)n_windows(I.w, L0);
        for (int wb = 0; wb < nw; wb += groups) {   // uniform trip count for the shuffles
            const int wi = wb + grp;
            uint32_t kmax = 0u, kmin = 0xFFFFFFFFu, sum = 0u;
            int r0 = 0, c0 = 0;
            bool valid = false;
            if (wi < nw) {
                const int wy = wi / n0, wx = wi - wy * n0;
                r0 = wy * L0;
                c0 = wx * L0;
                valid = r0 < th && c0 < tw;
                const int r1 = min(r0 + L0, th), c1 = min(c0 + L0, tw);
                if (packed) {
                    uint32_t pmax = 0u, pmin = 0xFFFFFFFFu;
                    int ri = 0;
                    for (int r = r0 + g; r < r1; r += G, ++ri) {
                        const uint8_t* row = pix + r * Tp;
                        uint32_t cbytes = (uint32_t)(ri << lc) * 0x01010101u + 0x03020100u;
                        int c = c0;
                        for (; c + 4 <= c1; c += 4, cbytes += 0x04040404u) {
                            const uint32_t w4 = *reinterpret_cast<const uint32_t*>(row + c);
                            // keys of columns c, c + 1 and c + 2, c + 3
                            const uint32_t lo = __builtin_amdgcn_perm(w4, cbytes, 0x05010400u);
                            const uint32_t hi = __builtin_amdgcn_perm(w4, cbytes, 0x07030602u);
                            pmax = pk_max(pmax, pk_max(lo, hi));
                            pmin = pk_min(pmin, pk_min(lo, hi));
                            sum = __builtin_amdgcn_sad_u8(w4, 0u, sum);
                        }
                        for (; c < c1; ++c) {   // the image's ragged right edge
                            const uint32_t v = row[c];
                            const uint32_t k = (v << 8) | (uint32_t)((ri << lc) | (c - c0));
                            pmax = pk_max(pmax, k | (k << 16));
                            pmin = pk_min(pmin, k | (k << 16));
                            sum += v;
                        }
                    }
                    if (ri > 0) {   // the lane saw pixels: expand its two keys
                        const uint32_t km = max(pmax & 0xFFFFu, pmax >> 16);
                        const uint32_t kn = min(pmin & 0xFFFFu, pmin >> 16);
                        const uint32_t msk = (1u << lc) - 1u;
                        kmax = ((km >> 8) << 16) |
                               ((uint32_t)(r0 + g + (int)((km & 255u) >> lc) * G) << 8) |
                               (uint32_t)(c0 + (int)(km & msk));
                        kmin = ((kn >> 8) << 16) |
                               ((uint32_t)(r0 + g + (int)((kn & 255u) >> lc) * G) << 8) |
                               (uint32_t)(c0 + (int)(kn & msk));
                    }
                } else {
                    for (int r = r0 + g; r < r1; r += G) {
                        const uint8_t* row = pix + r * Tp;
                        for (int c = c0; c < c1; ++c) {
                            const uint32_t v = row[c];
                            const uint32_t key = (v << 16) | ((uint32_t)r << 8) | (uint32_t)c;
                            kmax = max(kmax, key);
                            kmin = min(kmin, key);
                            sum += v;
                        }
                    }
                }
            }
            for (int off = G / 2; off > 0; off >>= 1) {
                kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off));
                kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, off));
                sum += (uint32_t)__shfl_xor((int)sum, off);
            }
            if (valid && g == 0) {
                rec[3 * wi + 0] = kmax;
                rec[3 * wi + 1] = kmin;
                rec[3 * wi + 2] = sum;
                const int wy = wi / n0, wx = wi - wy * n0;
                const int64_t by = (int64_t)ty * n0 + wy, bx = (int64_t)tx * n0 + wx;
                const int64_t slot = I.base[0] + 2 * (by * nbx + bx);
                const uint32_t n = (uint32_t)((min(r0 + L0, th) - r0) * (min(c0 + L0, tw) - c0));
                write_kp(I, 0, slot, ox, oy, kmax, sum, n, +1);
                write_kp(I, 0, slot + 1, ox, oy, kmin, sum, n, -1);
            }
        }
    }

    // ---- larger windows: merge whole children ----
    for (int s = 1; s < args.n_scales; ++s) {
        __syncthreads();
        const int Ls = args.L[s], Lc = args.L[s - 1];
        const int ns = T / Ls, nc = T / Lc, m = Ls / Lc;
        const uint32_t* crec = smem + args.lvl_off[s - 1];
        uint32_t* rec = smem + args.lvl_off[s];
        const int nbx = (int)n_windows(I.w, Ls);
        for (int wi = tid; wi < ns * ns; wi += kThreads) {
            const int wy = wi / ns, wx = wi - wy * ns;
            const int r0 = wy * Ls, c0 = wx * Ls;
            if (r0 >= th || c0 >= tw) continue;
            uint32_t kmax = 0u, kmin = 0xFFFFFFFFu, sum = 0u;
            for (int cy = 0; cy < m; ++cy) {
                const int cwy = wy * m + cy;
                if (cwy * Lc >= th) break;
                for (int cx = 0; cx < m; ++cx) {
                    const int cwx = wx * m + cx;
                    if (cwx * Lc >= tw) break;
                    const uint32_t* c = crec + 3 * (cwy * nc + cwx);
                    kmax = max(kmax, c[0]);
                    kmin = min(kmin, c[1]);
                    sum += c[2];
                }
            }
            rec[3 * wi + 0] = kmax;
            rec[3 * wi + 1] = kmin;
            rec[3 * wi + 2] = sum;
            const int64_t by = (int64_t)ty * ns + wy, bx = (int64_t)tx * ns + wx;
            const int64_t slot = I.base[s] + 2 * (by * nbx + bx);
            const uint32_t n = (uint32_t)((min(r0 + Ls, th) - r0) * (min(c0 + Ls, tw) - c0));
            write_kp(I, s, slot, ox, oy, kmax, sum, n, +1);
            write_kp(I, s, slot + 1, ox, oy, kmin, sum, n, -1);
        }
    }
}

// ---- any window set: one workgroup per window ----
//
// For L sets that are not nested, or with windows above 128 px, each window
// is reduced on its own: key (value << 32 | y W + x) orders pixels exactly as
// Eq. 1 does over the whole image (max: largest value, then largest raster
// index; min: smallest value, then smallest index), and the window's integer
// pixel sum gives the contrast, divided in double and rounded once to FP32.

struct WinArgs {
    int32_t n_images;
    int32_t n_scales;
    int32_t L[LPSIFT_MAX_SCALES];
    int64_t first[kMaxBatch][LPSIFT_MAX_SCALES];   // first workgroup of (image, scale)
    DetectImg img[kMaxBatch];
};

__device__ inline uint64_t max_u64(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ inline uint64_t min_u64(uint64_t a, uint64_t b) { return a < b ? a : b; }

__global__ __launch_bounds__(kThreads) void detect_window_kernel(WinArgs a)
{
    __shared__ uint64_t smax[kThreads / 64], smin[kThreads / 64];
    __shared__ uint32_t ssum[kThreads / 64];
    // (image, scale, window) of this workgroup
    const int64_t wg = blockIdx.x;
    int im = 0, s = 0;
    for (int i = 0; i < a.n_images; ++i)
        for (int t = 0; t < a.n_scales; ++t)
            if (wg >= a.first[i][t]) {
                im = i;
                s = t;
            }
    const DetectImg& I = a.img[im];
    const int L = a.L[s];
    const int64_t nbx = (I.w + L - 1) / L;
    const int64_t win = wg - a.first[im][s];
    const int by = (int)(win / nbx), bx = (int)(win - (int64_t)by * nbx);
    const int x0 = bx * L, y0 = by * L;
    const int ww = min(L, I.w - x0), wh = min(L, I.h - y0);
    const int64_t npx = (int64_t)ww * wh;

    uint64_t kmax = 0ull, kmin = ~0ull;
    uint32_t sum = 0u;
    for (int64_t p = threadIdx.x; p < npx; p += kThreads) {
        const int r = (int)(p / ww), c = (int)(p - (int64_t)r * ww);
        const int y = y0 + r, x = x0 + c;
        const uint32_t v = I.data[(int64_t)y * I.pitch + x];
        const uint64_t key = ((uint64_t)v << 32) | (uint32_t)(y * I.w + x);
        kmax = max_u64(kmax, key);
        kmin = min_u64(kmin, key);
        sum += v;
    }
    for (int off = 32; off > 0; off >>= 1) {
        kmax = max_u64(kmax, (uint64_t)__shfl_xor((long long)kmax, off));
        kmin = min_u64(kmin, (uint64_t)__shfl_xor((long long)kmin, off));
        sum += (uint32_t)__shfl_xor((int)sum, off);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        smax[wave] = kmax;
        smin[wave] = kmin;
        ssum[wave] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kThreads / 64; ++k) {
            kmax = max_u64(kmax, smax[k]);
            kmin = min_u64(kmin, smin[k]);
            sum += ssum[k];
        }
        const int64_t slot = I.base[s] + 2 * win;
        const uint64_t keys[2] = {kmax, kmin};
        for (int t = 0; t < 2; ++t) {
            const uint32_t v = (uint32_t)(keys[t] >> 32);
            const uint32_t idx = (uint32_t)keys[t];
            I.x[slot + t] = (int32_t)(idx % (uint32_t)I.w);
            I.y[slot + t] = (int32_t)(idx / (uint32_t)I.w);
            I.scale[slot + t] = (uint8_t)s;
            I.type[slot + t] = t == 0 ? (int8_t)1 : (int8_t)-1;
            I.value[slot + t] = (uint8_t)v;
            const int64_t num = (int64_t)v * npx - (int64_t)sum;
            I.contrast[slot + t] =
                (float)((double)(num < 0 ? -num : num) / (255.0 * (double)npx));
        }
    }
}

bool nested_small(const Geometry& g)
{
    for (int s = 1; s < g.n_scales; ++s)
        if (g.L[s] % g.L[s - 1] != 0) return false;
    return g.L[g.n_scales - 1] <= 128;
}

int launch_window_detect(const lpsift_image* imgs, int n, const Geometry& g,
                         const lpsift_keypoints* out, hipStream_t stream)
{
    for (int b0 = 0; b0 < n; b0 += kMaxBatch) {
        const int nb = (n - b0 < kMaxBatch) ? n - b0 : kMaxBatch;
        WinArgs a{};
        a.n_images = nb;
        a.n_scales = g.n_scales;
        for (int s = 0; s < g.n_scales; ++s) a.L[s] = g.L[s];
        int64_t wgs = 0;
        for (int i = 0; i < nb; ++i) {
            const lpsift_image& im = imgs[b0 + i];
            const lpsift_keypoints& kp = out[b0 + i];
            DetectImg& d = a.img[i];
            d.data = im.data;
            d.pitch = im.pitch;
            d.h = im.height;
            d.w = im.width;
            d.x = kp.x;
            d.y = kp.y;
            d.scale = kp.scale;
            d.type = kp.type;
            d.value = kp.value;
            d.contrast = kp.contrast;
            int64_t base = 0;
            for (int s = 0; s < g.n_scales; ++s) {
                const int64_t nw = n_windows(im.height, g.L[s]) * n_windows(im.width, g.L[s]);
                d.base[s] = base;
                base += 2 * nw;
                a.first[i][s] = wgs;
                wgs += nw;
            }
        }
        if (wgs > 0x7FFFFFFF) return LPSIFT_EINVAL;
        {
            TimedScope ts(LPSIFT_KERNEL_DETECT, stream);
            hipLaunchKernelGGL(detect_window_kernel, dim3((unsigned)wgs), dim3(kThreads), 0, stream,
                               a);
        }
        if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;
    }
    return LPSIFT_OK;
}

}  // namespace

int launch_detect(const lpsift_image* imgs, int n, const Geometry& g,
                  const lpsift_keypoints* out, hipStream_t stream)
{
    if (!nested_small(g)) return launch_window_detect(imgs, n, g, out, stream);
    const int Lmax = g.L[g.n_scales - 1];
    const int T = Lmax * (Lmax < 128 ? 128 / Lmax : 1);   // ~128 px per tile side
    DetectArgs a{};
    a.n_scales = g.n_scales;
    a.T = T;
    a.Tp = (int)align_up((size_t)T, 4);
    int words = 0;
    for (int s = 0; s < g.n_scales; ++s) {
        a.L[s] = g.L[s];
        a.lvl_off[s] = words;
        const int ns = T / g.L[s];
        words += 3 * ns * ns;
    }
    a.tile_words = (words + 3) & ~3;   // the pixel tile 16-byte aligned in LDS
    const size_t lds = (size_t)a.tile_words * 4 + (size_t)a.Tp * T;
    for (int b0 = 0; b0 < n; b0 += kMaxBatch) {
        const int nb = (n - b0 < kMaxBatch) ? n - b0 : kMaxBatch;
        a.n_images = nb;
        int tiles = 0;
        for (int i = 0; i < nb; ++i) {
            const lpsift_image& im = imgs[b0 + i];
            const lpsift_keypoints& kp = out[b0 + i];
            DetectImg& d = a.img[i];
            d.data = im.data;
            d.pitch = im.pitch;
            d.h = im.height;
            d.w = im.width;
            d.tiles_x = (int)n_windows(im.width, T);
            d.tile_begin = tiles;
            tiles += d.tiles_x * (int)n_windows(im.height, T);
            d.x = kp.x;
            d.y = kp.y;
            d.scale = kp.scale;
            d.type = kp.type;
            d.value = kp.value;
            d.contrast = kp.contrast;
            int64_t base = 0;
            for (int s = 0; s < g.n_scales; ++s) {
                d.base[s] = base;
                base += 2 * n_windows(im.height, g.L[s]) * n_windows(im.width, g.L[s]);
            }
        }
        {
            TimedScope ts(LPSIFT_KERNEL_DETECT, stream);
            hipLaunchKernelGGL(detect_kernel, dim3(tiles), dim3(kThreads), lds, stream, a);
        }
        if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;
    }
    return LPSIFT_OK;
}

}  // namespace lpsift
