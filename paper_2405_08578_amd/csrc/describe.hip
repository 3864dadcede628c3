// Orientation assignment and SIFT description at the detected window extrema
// (Sec. 2.3, Eq. 3-5).
//
// Three kernels, all enqueued by launch_describe:
//  1. disc tables (built by the first polar_field_kernel launch): for every
//     scale, the offsets of the orientation disc (radius round(1.5 w_s)),
//     row-major, and of the descriptor disc (radius w_s sqrt(2) (d+1)/2,
//     which circumscribes the rotated d+1 cell square where trilinear weights
//     can be non-zero), once per bucket of 64 orientation buckets, keeping
//     the entries that the rotated square can reach for an angle of the bucket.
//  2. polar_field_kernel: the Eq. 5 gradient of every pixel once, as
//     (magnitude, angle in turns in [0, 1)); border pixels get magnitude 0.
//     Each image pixel is visited by ~10 keypoint supports, so the angle and
//     the square root are paid once per pixel instead of once per visit.
//  3. orient_describe_kernel: one wavefront per keypoint, four per workgroup.
//     Lane l takes table entries l, l + 64, l + 128, ... (four at a time, all
//     their loads issued before any is used), so one load instruction reads
//     consecutive table entries and mostly neighbouring pixels of the field;
//     lanes of even and odd index vote into two copies of the histogram, which
//     halves the collisions of neighbouring pixels on one bin. Votes are
//     accumulated in LDS as fixed point with integer atomics: ds_add_u64
//     runs at close to full rate where ds_add_f32 does not, and integer sums
//     do not depend on the order of the votes, so the result is bit-identical
//     from run to run. Orientation votes (at most 255 sqrt 2 < 362, all
//     weights <= 1) are scaled by 2^23, truncated to 32 bits by one
//     v_cvt_u32_f32 and added to 64-bit bins. Descriptor votes are scaled per
//     scale so that no bin can reach 2^32 (the bound is derived with the
//     geometry) and rounded to nearest; a descriptor visit's two direction
//     bins o and o + 1 (mod 8) of a cell then go out as one 64-bit atomic,
//     the low word to bin o and the high word to bin o + 1 (no carry crosses
//     the words), which halves the LDS atomics of the descriptor.
//     Orientation (36 bins, smoothing, argmax,
//     parabola), then the 128-bin descriptor, normalisation, clipping at 0.2
//     and renormalisation happen in the same wave; the descriptor row is
//     stored with two coalesced 256-byte writes. orient_describe_half_kernel
//     does the same for the smallest scale with one keypoint per 32-lane half
//     of a wavefront, bit for bit.
#include "internal.h"

namespace lpsift {
namespace {

// Images per launch (keeps the by-value kernel arguments small).
constexpr int kDescBatch = kMaxBatch;
// Gradient-field bytes per launch group: half of MI355X's 256 MB last-level
// (Infinity) cache, where the describe kernel's repeated field reads then hit.
constexpr size_t kFieldGroupBytes = 128u << 20;

// ---------------------------------------------------------------- tables --

struct TableArgs {
    int32_t n_scales;
    int32_t r2_orient[LPSIFT_MAX_SCALES];
    int32_t off_orient[LPSIFT_MAX_SCALES];
    float k_orient[LPSIFT_MAX_SCALES];     // Gaussian exponent factor of the table
    int32_t r2_desc[LPSIFT_MAX_SCALES];
    int32_t off_desc[LPSIFT_MAX_SCALES];
    int32_t cap_desc[LPSIFT_MAX_SCALES];
    int32_t n_buckets[LPSIFT_MAX_SCALES];
    float k_desc[LPSIFT_MAX_SCALES];
    float dscale[LPSIFT_MAX_SCALES];       // descriptor vote scale (folded into the weights)
    double inv_ws[LPSIFT_MAX_SCALES];
};

__device__ inline int32_t pack_offset(int dx, int dy)
{
    return (int32_t)((uint32_t)(dx & 0xFFFF) | ((uint32_t)dy << 16));
}

// One disc entry: the offset as floats (for the rotation), its Gaussian
// weight exp2((dx^2 + dy^2) k) times the votes' fixed-point scale (computed
// once here), and the packed integer offset (for the field address) -- one
// 16-byte load per visit.
__device__ inline float4 disc_entry(int dx, int dy, float k, float scale)
{
    return make_float4((float)dx, (float)dy,
                       __builtin_amdgcn_exp2f((float)(dx * dx + dy * dy) * k) * scale,
                       __int_as_float(pack_offset(dx, dy)));
}

// Whether offset (dx, dy) can fall in the square |u|, |v| < 2.5 of reachable
// subregions for some angle of an orientation bucket of nb (angles in
// [b, b + 1) / nb turns). (c, s) = (cos, sin) of the bucket's centre angle,
// divided by w_s: the offset rotates there to (u, v), in subregions; within
// the bucket the angle differs by at most pi / nb, which moves each
// coordinate by at most r pi / nb (r = the offset's length in subregions).
// The margin takes 1 % more and 1e-3 subregions for the rounding of this test
// and of the visit's own rotation, so the bucket keeps every entry that a
// visit's test can accept.
__device__ inline bool in_bucket(int dx, int dy, float c, float s, float inv_ws, float slack)
{
    const float fx = (float)dx, fy = (float)dy;
    const float u = fmaf(c, fx, s * fy), v = fmaf(c, fy, -(s * fx));
    const float m = fmaf(sqrtf(fmaf(fx, fx, fy * fy)) * inv_ws, slack, 2.5f + 1e-3f);
    return fabsf(u) < m && fabsf(v) < m;
}

constexpr int kTabThreads = 256;
constexpr int kTabMaxRows = 4001;   // 2 R + 1 rows, R <= 2000 (support radius limit)
static_assert(kBucketMaxEntries <= 32 * kTabThreads, "a thread's run of a bucketed disc fits a 32-bit mask");

// Inclusive scan of one value per thread over the workgroup (Hillis-Steele).
__device__ inline int block_scan(int* scan, int v)
{
    const int tid = threadIdx.x;
    scan[tid] = v;
    __syncthreads();
    for (int off = 1; off < kTabThreads; off <<= 1) {
        const int u = (tid >= off) ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += u;
        __syncthreads();
    }
    const int r = scan[tid];
    __syncthreads();
    return r;
}

// Table job (j, s) of one workgroup: j = 0 the orientation disc of scale s,
// j = 1 + b bucket b of its descriptor disc. The disc's entries, in row-major order, are split
// into 256 contiguous runs, one per thread (at most 32 entries each when the
// disc is bucketed); a thread marks the entries of its run that the bucket
// keeps, and a block scan of the marked counts gives every run its output
// start, so the list stays in row-major order. The entry count of each
// descriptor bucket goes to counts[s kDescBuckets + b].
__device__ void build_table(const TableArgs& a, float4* tables, int32_t* counts, int j, int s,
                            int* scan, int* row_start)
{
    const int tid = threadIdx.x;
    const bool orient = j == 0;
    const int b = j - 1;
    if (!orient && b >= a.n_buckets[s]) return;
    const int r2 = orient ? a.r2_orient[s] : a.r2_desc[s];
    const int nb = orient ? 1 : a.n_buckets[s];
    const int R = isqrt_floor(r2);
    const int rows = 2 * R + 1;

    // row starts: thread t sums a contiguous run of rows, a block scan places them
    {
        const int per = (rows + kTabThreads - 1) / kTabThreads;
        const int i0 = tid * per, i1 = min(i0 + per, rows);
        int c = 0;
        for (int i = i0; i < i1; ++i) c += 2 * isqrt_floor(r2 - (i - R) * (i - R)) + 1;
        int at = block_scan(scan, c) - c;
        for (int i = i0; i < i1; ++i) {
            row_start[i] = at;
            at += 2 * isqrt_floor(r2 - (i - R) * (i - R)) + 1;
        }
        if (tid == kTabThreads - 1) row_start[rows] = at;
        __syncthreads();
    }
    const int n = row_start[rows];
    const int per = (n + kTabThreads - 1) / kTabThreads;
    const int j0 = min(tid * per, n), j1 = min(j0 + per, n);
    // the row of entry j0: the last row starting at or before it
    int lo = 0, hi = rows - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_start[mid] <= j0) lo = mid; else hi = mid - 1;
    }
    const int i_first = lo;
    const int dy_first = i_first - R;
    const int hw_first = isqrt_floor(r2 - dy_first * dy_first);
    const int dx_first = -hw_first + (j0 - row_start[i_first]);

    // (cos, sin) of the bucket's centre angle over w_s, and the slack
    // (single precision: its error is far inside the 1e-3 margin)
    const float th = 6.2831853f * ((float)b + 0.5f) / (float)nb;
    const float inv_ws = (float)a.inv_ws[s];
    float sn, c;
    sincosf(th, &sn, &c);
    c *= inv_ws;
    sn *= inv_ws;
    const float slack = (float)(3.141592653589793 / nb * 1.01);
    const bool filter = nb > 1;   // bucketed discs have at most 8,192 entries: per <= 32

    unsigned keep = 0u;
    int cnt = j1 - j0;
    if (filter) {
        int dx = dx_first, dy = dy_first, hw = hw_first;
        for (int k = 0; k < j1 - j0; ++k) {
            if (in_bucket(dx, dy, c, sn, inv_ws, slack)) keep |= 1u << k;
            if (++dx > hw) {
                ++dy;
                hw = isqrt_floor(r2 - dy * dy);
                dx = -hw;
            }
        }
        cnt = __popc(keep);
    }
    const int total = block_scan(scan, cnt);
    int at = total - cnt;
    float4* out = tables + (orient ? (int64_t)a.off_orient[s]
                                   : (int64_t)a.off_desc[s] + (int64_t)b * a.cap_desc[s]);
    const float k = orient ? a.k_orient[s] : a.k_desc[s];
    const float vscale = orient ? kOrientVoteScale : a.dscale[s];
    {
        int dx = dx_first, dy = dy_first, hw = hw_first;
        for (int e = 0; e < j1 - j0; ++e) {
            if (!filter || ((keep >> e) & 1u)) out[at++] = disc_entry(dx, dy, k, vscale);
            if (++dx > hw) {
                ++dy;
                hw = isqrt_floor(r2 - dy * dy);
                dx = -hw;
            }
        }
    }
    if (!orient && tid == kTabThreads - 1) counts[s * kDescBuckets + b] = total;
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

// Direction of the integer gradient (x, y) = (bv, av), (x, y) != (0, 0), in
// turns in [0, 1): atan2(y, x) / (2 pi), wrapped. The octant is reduced to
// a = min / max in [0, 1] (v_rcp_f32), and atan(a) / (2 pi) = a P(a^2) with
// P of degree 7 fitted to atan(sqrt(s)) / (2 pi sqrt(s)) on s in [0, 1]
// (least squares on Chebyshev nodes, reweighted toward the minimax error);
// over all gradients of 8-bit images (|x|, |y| <= 255) the result is within
// 7e-8 turns of the exact angle with the reciprocal off by up to one ulp,
// as close as a correctly rounded atan2f scaled to turns.
// POLAR_COEFFS_BEGIN
constexpr float kPolarP[8] = {1.591548324e-01f, -5.304612219e-02f, 3.174594417e-02f,
                              -2.213625796e-02f, 1.534599904e-02f, -8.898677304e-03f,
                              3.479566891e-03f, -6.452961243e-04f};
// POLAR_COEFFS_END
__device__ inline float polar_turns(int y, int x)
{
    const float ax = fabsf((float)x), ay = fabsf((float)y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float a = mn * __builtin_amdgcn_rcpf(mx);
    const float s = a * a;
    float p = kPolarP[7];
#pragma unroll
    for (int k = 6; k >= 0; --k) p = fmaf(p, s, kPolarP[k]);
    // [0, 1/8], or 1/4 minus it (one rounding) past the diagonal: [0, 1/4]
    float r = (ay > ax) ? fmaf(-a, p, 0.25f) : a * p;
    if (x < 0) r = 0.5f - r;                // [0, 1/2]
    if (y < 0) r = 1.0f - r;                // (1/2, 1]
    return r >= 1.0f ? r - 1.0f : r;
}

// One launch builds the disc tables and the gradient fields: workgroups
// 0 .. n_table - 1 take the table jobs (dispatched first, so the few long
// table jobs run beside the many short field rows instead of after them);
// workgroup n_table + (z gy + y) gx + x then takes the row segment of
// 256 kFieldPx pixels at column 256 kFieldPx x of row y of image z, thread t
// the pixels t + 256 k (coalesced; a few pixels per thread keep the waves
// fewer than one per 64 pixels, whose launch rate bounded the field).
constexpr int kFieldPx = 4;
__global__ __launch_bounds__(256) void polar_field_kernel(FieldArgs a, TableArgs ta,
                                                          float4* tables, int32_t* counts,
                                                          int n_table, int gx, int gy)
{
    static_assert(kTabThreads == 256, "table jobs run on the field kernel's workgroups");
    __shared__ int scan[kTabThreads];
    __shared__ int row_start[kTabMaxRows + 1];
    const int blk = (int)blockIdx.x;
    if (blk < n_table) {
        build_table(ta, tables, counts, blk % (1 + kDescBuckets), blk / (1 + kDescBuckets), scan,
                    row_start);
        return;
    }
    const int f = blk - n_table;
    const int z = f / (gx * gy), rem = f - z * (gx * gy);
    const FieldImg& I = a.img[z];
    const int r = rem / gx;
    if (r >= I.h) return;
    const int c0 = (rem - r * gx) * (256 * kFieldPx) + threadIdx.x;
    const bool row_in = r >= 1 && r <= I.h - 2;
    const uint8_t* prow = I.data + (int64_t)r * I.pitch;
    float2* frow = I.field + (int64_t)r * I.w;
#pragma unroll
    for (int k = 0; k < kFieldPx; ++k) {
        const int c = c0 + 256 * k;
        if (c >= I.w) break;
        float2 out = make_float2(0.0f, 0.0f);
        if (row_in && c >= 1 && c <= I.w - 2) {
            const uint8_t* p = prow + c;
            const int av = (int)p[I.pitch] - (int)p[-I.pitch];   // along rows
            const int bv = (int)p[1] - (int)p[-1];               // along columns
            const int n2 = av * av + bv * bv;
            // v_sqrt_f32 (within 1 ulp) of the integer sum, the angle above
            if (n2 > 0) out = make_float2(__builtin_amdgcn_sqrtf((float)n2), polar_turns(av, bv));
        }
        frow[c] = out;
    }
}

// ------------------------------------------------------ orient + describe --

struct DescImg {
    const float2* field;
    int32_t h, w;
    const int32_t* x;
    const int32_t* y;
    float* theta;
    float* desc;
    const int32_t* sel;    // list mode: slots to describe, outputs compacted
    int64_t n_sel;
    int64_t n_kp;          // slots of the image
    // multi-orientation variant
    float* obuf;           // [n_kp][kMaxOrient] angles in turns
    int32_t* count;        // [n_kp] orientations per slot
    int64_t* offset;       // [n_kp] first output row of each slot
    int32_t* rows;         // output: slot of every row
};

struct DescArgs {   // passed by value: keep well under 4 KB
    int32_t n_images;
    int32_t n_scales;
    int32_t list;          // 1: describe img[i].sel[0 .. n_sel) only
    int32_t max_orient;    // multi-orientation variant: 1 .. kMaxOrient
    int32_t first_scale;   // orient_describe_kernel: scales first_scale .. n_scales - 1
    int32_t half_scales;   // orient_describe_half_kernel: scales 0 .. half_scales - 1
    float peak_ratio;      // and its secondary-peak threshold
    const int32_t* bcount; // entries of descriptor bucket b of scale s at [s kDescBuckets + b]
    ScaleGeom geom[LPSIFT_MAX_SCALES];
    int32_t L[LPSIFT_MAX_SCALES];
    // first slot of scale s in image i
    int64_t slot_base[LPSIFT_MAX_SCALES][kDescBatch];
    DescImg img[kDescBatch];
};

// Workgroup i runs on XCD i % 8 (round-robin dispatch). XCD x takes band x of
// eight horizontal bands of window rows of every scale and image, largest
// scale first: its L2 then holds one band of the gradient field, and every
// XCD gets the same mix of scales.
constexpr int kXcds = 8;

__host__ __device__ inline int64_t band_items(int x, int64_t nby, int64_t nbx)
{
    const int64_t r0 = (x * nby) / kXcds, r1 = ((x + 1) * nby) / kXcds;
    return 2 * (r1 - r0) * nbx;
}

constexpr int kWaves = 4;          // keypoints per workgroup
constexpr int kUnroll = 4;         // visits per lane per step
constexpr int kBins = 128 + 36;    // descriptor bins, then orientation bins
// Bins before the first histogram of a workgroup's LDS: a descriptor vote
// addresses its four cells from one base at a cell index clamped to >= -5,
// which may lie up to 5 cells before the histogram (only in-range cells are
// written).
constexpr int kCellPad = 40;
constexpr int kMaxOrient = 4;      // orientations per keypoint (multi-orientation variant)
// Scales whose descriptor disc has at most this many entries take the
// half-wavefront kernel (L = 16 with the default geometry; measured: 2 % faster
// than whole wavefronts there, slower once L = 32 is included).
constexpr int kHalfMaxVisits = 700;
// Histogram copies per half wavefront (even and odd lanes, as in the whole-
// wavefront kernel), of 128 bins each: the orientation histogram takes the
// first 36 bins of each copy and is cleared after it is read, which keeps
// the workgroup's LDS within 1/8 of the CU's (8 workgroups per CU).
constexpr int kHalfCopies = 2;
constexpr int kHalfWords = 128;
// Histogram copies per wave: lane l votes into copy l mod kCopies, so the
// neighbouring pixels that neighbouring lanes visit rarely hit one address
// at once; the copies are summed when read (integer sums: order-free). With
// a cell's two direction bins in one atomic, 2 copies measured faster than 4
// in the whole-wavefront kernel (4 leave room for 7 workgroups per CU, 2 for
// 8), and 1 slower than 2 in the half-wavefront kernel.
constexpr int kCopies = 2;

__device__ inline float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

constexpr float kOrientVoteInv = 1.0f / kOrientVoteScale;

// Orientation vote, pre-scaled: truncated to an integer, added to a 64-bit bin.
__device__ inline void vote(unsigned long long* h, float w_scaled)
{
    atomicAdd(h, (unsigned long long)(uint32_t)w_scaled);
}

// floor(x) as an integer in one instruction (|x| well inside the int range).
__device__ inline int floor_int(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Descriptor bin b (cell b / 8, direction b % 8) over kC histogram copies
// of kW words, in vote units before the scale: the votes of visits whose
// lower direction bin is o sit in 64-bit word (cell, o), for bin o in its
// low and for bin o + 1 (mod 8) in its high 32-bit word. Each word converts
// to float exactly to 24 bits and the 2 kC parts add in this fixed order, so
// every kernel reads the same value (within 3e-7 relative of the integer
// total).
template <int kC, int kW>
__device__ inline float desc_bin(const unsigned long long* h, int b)
{
    const uint32_t* w = reinterpret_cast<const uint32_t*>(h);
    const int prev = (b & ~7) | ((b + 7) & 7);
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kC; ++c) {
        s += (float)w[2 * (c * kW + b)];
        s += (float)w[2 * (c * kW + prev) + 1];
    }
    return s;
}

// Makes a wave's LDS writes visible to its own later reads. Enough where each
// wave owns its LDS region (no other wave reads it), and lets the waves of a
// workgroup run different numbers of passes.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool kWaveOnly>
__device__ inline void hist_sync()
{
    if (kWaveOnly)
        wave_sync();
    else
        __syncthreads();
}

// Kernel modes: one orientation and its descriptor per keypoint; the
// orientation pass of the multi-orientation variant (counts and angles per
// slot); descriptors at the angles that pass stored, rows compacted.
enum { kModeFull = 0, kModeOrient = 1, kModeGiven = 2 };


// Smoothed 36-bin orientation histogram of one keypoint; lane k < 36 returns
// bin k, other lanes -1. Ends with the votes visible to the whole wave.
// [1 4 6 4 1] / 16 smoothing of five neighbouring bins, written with explicit
// FMAs so that every kernel rounds it the same way.
__device__ inline float smooth5(float h2m, float h1m, float h0, float h1p, float h2p)
{
    float s = fmaf(4.0f, h1m, h2m);
    s = fmaf(6.0f, h0, s);
    s = fmaf(4.0f, h1p, s);
    return (s + h2p) * 0.0625f;
}

// Parabolic offset of the peak at a bin of height h0 between hm and hp.
__device__ inline float parabola_offset(float hm, float h0, float hp)
{
    const float den = fmaf(-2.0f, h0, hm) + hp;
    return (den != 0.0f) ? 0.5f * (hm - hp) * __builtin_amdgcn_rcpf(den) : 0.0f;
}

// Angle in turns of orientation bin k refined by the parabola offset.
__device__ inline float bin_turns(int k, float hm, float h0, float hp)
{
    return ((float)k + parabola_offset(hm, h0, hp)) * (1.0f / 36.0f);
}

// Orientation votes of one keypoint into ho[0..36) of each histogram copy;
// its kStride lanes (sub = 0 .. kStride - 1) take table entries sub,
// sub + kStride, ...
template <int kStride, int kC = kCopies, int kW = kBins>
__device__ __forceinline__ void orient_votes(unsigned long long* ho, int sub, bool live, int kx,
                                             int ky, const float2* field, int W, int H,
                                             const ScaleGeom& G, const float4* tables)
{
    const int n = live ? G.n_orient : 0;
    const int per = (n + kStride - 1) / kStride;
    const float4* tab = tables + G.off_orient;
    unsigned long long* hv = ho + (sub % kC) * kW;   // this lane's copy
    for (int it0 = 0; it0 < per; it0 += kUnroll) {
        int dx[kUnroll], dy[kUnroll];
        bool ok[kUnroll];
        float2 ft[kUnroll];
        float gw[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            // branch-free loads, as in desc_votes
            const int j = (it0 + u) * kStride + sub;
            ok[u] = j < n;
            const float4 e = tab[ok[u] ? (uint32_t)j : 0u];
            const int32_t pk = __float_as_int(e.w);
            dx[u] = (int)(int16_t)(pk & 0xFFFF);
            dy[u] = pk >> 16;
            gw[u] = e.z;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int px = kx + dx[u], py = ky + dy[u];
            const bool in = ok[u] & ((unsigned)px < (unsigned)W) & ((unsigned)py < (unsigned)H);
            const uint32_t at = (uint32_t)(__mul24(py, W) + px);
            ft[u] = field[in ? at : 0u];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (ft[u].x == 0.0f) continue;
            // Gaussian weight times 2^23 from the table (its exponent is above
            // -7 for every geometry, far from the denormal range: v_exp_f32
            // alone)
            const float wt = ft[u].x * gw[u];
            // the product is rounded before fract and floor take it (neither
            // can fuse with it), so every kernel gets the same bins
            const float t = ft[u].y * 36.0f;
            const float fr = __builtin_amdgcn_fractf(t);
            int k0 = floor_int(t);
            if (k0 >= 36) k0 -= 36;
            const int k1 = (k0 == 35) ? 0 : k0 + 1;
            vote(hv + k0, (1.0f - fr) * wt);
            vote(hv + k1, fr * wt);
        }
    }
}

template <int kC>
__device__ __forceinline__ float orient_hist(unsigned long long* ho, int lane, bool live, int kx,
                                             int ky, const float2* field, int W, int H,
                                             const ScaleGeom& G, const float4* tables)
{
    orient_votes<64, kC>(ho, lane, live, kx, ky, field, W, H, G, tables);
    wave_sync();
    const float inv = kOrientVoteInv;
    // lane k < 36 converts bin k once; its neighbours come by shuffles
    float h0 = 0.0f;
    if (lane < 36) {
        unsigned long long v = 0ull;
#pragma unroll
        for (int c = 0; c < kC; ++c) v += ho[c * kBins + lane];
        h0 = (float)v * inv;
    }
    const int l = lane < 36 ? lane : 0;
    const float h2m = __shfl(h0, (l + 34) % 36), h1m = __shfl(h0, (l + 35) % 36);
    const float h1p = __shfl(h0, (l + 1) % 36), h2p = __shfl(h0, (l + 2) % 36);
    return lane < 36 ? smooth5(h2m, h1m, h0, h1p, h2p) : -1.0f;
}

// Highest value over the wave with its lane (lowest lane on ties).
__device__ inline void wave_argmax(float& v, int& k)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(v, off);
        const int okk = __shfl_xor(k, off);
        if (ov > v || (ov == v && okk < k)) {
            v = ov;
            k = okk;
        }
    }
}

// Peak angle in turns: bin k refined by the parabola through its neighbours.
__device__ inline float peak_turns(float sm, int k, float h0)
{
    const float hm = __shfl(sm, (k + 35) % 36);
    const float hp = __shfl(sm, (k + 1) % 36);
    return bin_turns(k, hm, h0, hp);
}

// Descriptor of one keypoint at angle th_turns: votes into hist[0..128),
// normalise, clip at 0.2, renormalise; lane l returns elements l and l + 64.
// kWaveOnly: the wave synchronises alone (the caller's waves may diverge).
// Descriptor votes of one keypoint at angle th_turns into hist[0..128) of
// each histogram copy (the packed layout read by desc_bin); lanes as in
// orient_votes.
template <int kStride, int kC = kCopies, int kW = kBins>
__device__ __forceinline__ void desc_votes(unsigned long long* hist, int sub, bool live, int kx,
                                           int ky, const float2* field, int W, int H,
                                           const ScaleGeom& G, const float4* tables,
                                           const int32_t* bcount, float th_turns)
{
    float sn, cs;
    sn = __builtin_amdgcn_sinf(th_turns);   // v_sin_f32 / v_cos_f32 take revolutions
    cs = __builtin_amdgcn_cosf(th_turns);
    const float ca = cs * G.inv_ws, sa = sn * G.inv_ws;   // rotation by -theta, in cells
    const float th8 = th_turns * 8.0f;
    // the bucket of theta (any angle, wrapped to [0, 1) turns by the mask)
    const int bk = G.n_buckets > 1 ? ((int)floorf(th_turns * (float)kDescBuckets) & (kDescBuckets - 1)) : 0;
    const int nd = live ? bcount[bk] : 0;
    const int perd = (nd + kStride - 1) / kStride;
    const float4* tabd = tables + G.off_desc + (int64_t)bk * G.cap_desc;
    unsigned long long* hv = hist + (sub % kC) * kW;   // this lane's copy
    for (int it0 = 0; it0 < perd; it0 += kUnroll) {
        int dx[kUnroll], dy[kUnroll];
        bool ok[kUnroll];
        float2 ft[kUnroll];
        float fdx[kUnroll], fdy[kUnroll], gw[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            // loads without branches: a lane past the list reads entry 0, and
            // its visit, like one outside the image, reads field pixel 0 (a
            // border pixel, so of magnitude 0: it casts no vote)
            const int j = (it0 + u) * kStride + sub;
            ok[u] = j < nd;
            const float4 e = tabd[ok[u] ? (uint32_t)j : 0u];
            const int32_t pk = __float_as_int(e.w);
            dx[u] = (int)(int16_t)(pk & 0xFFFF);
            dy[u] = pk >> 16;
            fdx[u] = e.x;
            fdy[u] = e.y;
            gw[u] = e.z;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int px = kx + dx[u], py = ky + dy[u];
            const bool in = ok[u] & ((unsigned)px < (unsigned)W) & ((unsigned)py < (unsigned)H);
            const uint32_t at = (uint32_t)(__mul24(py, W) + px);   // 24-bit multiply: full rate
            ft[u] = field[in ? at : 0u];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (ft[u].x == 0.0f) continue;
            // offset rotated by -theta, in subregion units, shifted by 1.5 so
            // that cell i covers [i, i + 1); offsets outside the square of
            // reachable cells find no cell in range below
            const float cu = fmaf(ca, fdx[u], fmaf(sa, fdy[u], 1.5f));
            const float cv = fmaf(ca, fdy[u], fmaf(-sa, fdx[u], 1.5f));
            // Gaussian weight and vote scale from the table
            const float m = ft[u].x * gw[u];
            // direction bins o0 and o0 + 1 (mod 8) of the angle relative to theta
            const float t = fmaf(ft[u].y, 8.0f, -th8);   // (-8, 8)
            const int o0 = floor_int(t) & 7;
            const float fo = __builtin_amdgcn_fractf(t);
            const float m1 = m * fo;
            const float m0 = fmaf(ft[u].x, gw[u], -m1);   // explicit: the same rounding in every kernel
            const int ix0 = floor_int(cu), iy0 = floor_int(cv);
            const float fx = __builtin_amdgcn_fractf(cu), fy = __builtin_amdgcn_fractf(cv);
            // word (cell, o0) of the four cells at constant offsets from one
            // base at cell 4 iy0 + ix0, clamped to -5 .. 15 so that the base
            // stays within the histogram and the pad before it (an index
            // that needs the clamp has no cell in range)
            unsigned long long* b0 = hv + min(max(iy0 * 4 + ix0, -5), 15) * 8 + o0;
#pragma unroll
            for (int jy = 0; jy < 2; ++jy) {
                if ((unsigned)(iy0 + jy) > 3u) continue;
                const float wy = jy ? fy : 1.0f - fy;
#pragma unroll
                for (int jx = 0; jx < 2; ++jx) {
                    if ((unsigned)(ix0 + jx) > 3u) continue;
                    const float wxy = (jx ? fx : 1.0f - fx) * wy;
                    // round to nearest: non-negative values, + 1/2, truncate
                    const uint32_t lo = (uint32_t)fmaf(m0, wxy, 0.5f);
                    const uint32_t hi = (uint32_t)fmaf(m1, wxy, 0.5f);
                    atomicAdd(b0 + (jy * 4 + jx) * 8, ((unsigned long long)hi << 32) | lo);
                }
            }
        }
    }
}

template <bool kWaveOnly, int kC>
__device__ __forceinline__ void describe_at(unsigned long long* hist, int lane, bool live, int kx,
                                            int ky, const float2* field, int W, int H,
                                            const ScaleGeom& G, const float4* tables,
                                            const int32_t* bcount, float th_turns, float& r0,
                                            float& r1)
{
    desc_votes<64, kC>(hist, lane, live, kx, ky, field, W, H, G, tables, bcount, th_turns);
    hist_sync<kWaveOnly>();
    const float dinv = G.dinv;
    float d0 = desc_bin<kC, kBins>(hist, lane) * dinv;
    float d1 = desc_bin<kC, kBins>(hist, lane + 64) * dinv;
    float inv = __builtin_amdgcn_rcpf(fmaxf(sqrtf(wave_sum(fmaf(d0, d0, d1 * d1))), 1e-12f));
    d0 = fminf(d0 * inv, 0.2f);
    d1 = fminf(d1 * inv, 0.2f);
    inv = __builtin_amdgcn_rcpf(fmaxf(sqrtf(wave_sum(fmaf(d0, d0, d1 * d1))), 1e-12f));
    r0 = d0 * inv;
    r1 = d1 * inv;
}

template <int kMode>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void orient_describe_kernel(DescArgs a, const float4* tables)
{
    constexpr int kC = kCopies;
    __shared__ unsigned long long hist_mem[kCellPad + kWaves * kC * kBins];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long* hist = hist_mem + kCellPad + wave * kC * kBins;

    bool live = false, has_out = false;
    int sc = 0, im = 0;
    int64_t slot = 0, out_at = 0;
    if (kMode == kModeFull && a.list) {
        // list mode: entries of every image in turn, each list from its end
        // (largest slots, i.e. largest scale, first); output at the entry
        int64_t j = (int64_t)blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(wave);
        for (int i = 0; i < a.n_images; ++i) {
            if (j < a.img[i].n_sel) {
                im = i;
                has_out = true;
                out_at = a.img[i].n_sel - 1 - j;
                slot = a.img[i].sel[out_at];
                live = slot >= 0 && slot < a.img[i].n_kp;
                for (int s = a.n_scales - 1; s >= 0; --s)
                    if (slot >= a.slot_base[s][i]) {
                        sc = s;
                        break;
                    }
                break;
            }
            j -= a.img[i].n_sel;
        }
    } else {
        // locate (scale, image, slot) of this wave's keypoint in its XCD's band list
        // (32-bit arithmetic: window counts and slots of one image are < 2^31)
        const int xcd = blockIdx.x % kXcds;
        int64_t j = (int64_t)(blockIdx.x / kXcds) * kWaves + __builtin_amdgcn_readfirstlane(wave);
        for (int so = 0; so < a.n_scales - a.first_scale && !live; ++so) {
            const int s = a.n_scales - 1 - so;
            const uint32_t L = (uint32_t)a.L[s];
            for (int i = 0; i < a.n_images; ++i) {
                const uint32_t nby = ((uint32_t)a.img[i].h + L - 1u) / L;
                const uint32_t nbx = ((uint32_t)a.img[i].w + L - 1u) / L;
                const uint32_t r0 = (uint32_t)xcd * nby / kXcds;
                const uint32_t r1 = (uint32_t)(xcd + 1) * nby / kXcds;
                const int64_t cnt = 2 * (int64_t)(r1 - r0) * nbx;
                if (j < cnt) {
                    live = true;
                    sc = s;
                    im = i;
                    slot = a.slot_base[s][i] + 2 * (int64_t)r0 * nbx + j;
                    break;
                }
                j -= cnt;
            }
        }
        has_out = live;
        out_at = slot;
    }
    if (!live) slot = 0;
    const DescImg& I = a.img[im];
    const ScaleGeom G = a.geom[sc];   // a copy: its fields stay in registers through the visit loops
    const int kx = I.x[slot], ky = I.y[slot];
    const float2* field = I.field;
    const int W = I.w, H = I.h;

    for (int b = lane; b < kC * kBins; b += 64) hist[b] = 0ull;
    wave_sync();

    if (kMode != kModeGiven) {
        // ---- orientation: smoothing, argmax (lowest bin on ties), parabola ----
        const float sm = orient_hist<kC>(hist + 128, lane, live, kx, ky, field, W, H, G, tables);
        float bv = sm;
        int bk = lane;
        wave_argmax(bv, bk);
        const float th_turns = peak_turns(sm, bk, bv);
        if (kMode == kModeFull) {
            if (live && lane == 0) I.theta[out_at] = th_turns * 6.283185307179586f;
            // ---- descriptor histogram: 4 x 4 cells x 8 directions ----
            float r0, r1;
            describe_at<true, kC>(hist, lane, live, kx, ky, field, W, H, G, tables,
                                  a.bcount + sc * kDescBuckets, th_turns, r0, r1);
            if (live) {
                float* out = I.desc + out_at * 128;
                out[lane] = r0;
                out[lane + 64] = r1;
            } else if (has_out) {   // list entry naming no slot of the image
                float* out = I.desc + out_at * 128;
                out[lane] = 0.0f;
                out[lane + 64] = 0.0f;
                if (lane == 0) I.theta[out_at] = __builtin_nanf("");
            }
        } else {
            // secondary peaks: strict local maxima other than the dominant bin
            // with height >= peak_ratio x the maximum, highest first
            const float smm = __shfl(sm, (lane + 35) % 36), smp = __shfl(sm, (lane + 1) % 36);
            float cv = (lane < 36 && lane != bk && sm > smm && sm > smp && sm >= a.peak_ratio * bv)
                           ? sm : -1.0f;
            int cnt = 1;
            if (live && lane == 0) I.obuf[slot * kMaxOrient] = th_turns;
#pragma unroll
            for (int m = 1; m < kMaxOrient; ++m) {
                if (m >= a.max_orient) break;
                float v = cv;
                int k = lane;
                wave_argmax(v, k);
                if (v < 0.0f) break;
                const float t = peak_turns(sm, k, v);
                if (live && lane == 0) I.obuf[slot * kMaxOrient + m] = t;
                if (lane == k) cv = -1.0f;
                ++cnt;
            }
            if (live && lane == 0) I.count[slot] = cnt;
        }
        return;
    }

    // ---- given orientations: one descriptor row per (slot, orientation) ----
    // Each wave loops over its own slot's orientations and synchronises alone.
    const int cnt = live ? I.count[slot] : 0;
    const int64_t row0 = live ? I.offset[slot] : 0;
    for (int m = 0; m < cnt; ++m) {
        if (m > 0) {
#pragma unroll
            for (int c = 0; c < kC; ++c)
                for (int b = lane; b < 128; b += 64) hist[c * kBins + b] = 0ull;
            wave_sync();
        }
        const float th = I.obuf[slot * kMaxOrient + m];
        float r0, r1;
        describe_at<true, kC>(hist, lane, true, kx, ky, field, W, H, G, tables,
                              a.bcount + sc * kDescBuckets, th, r0, r1);
        const int64_t row = row0 + m;
        float* out = I.desc + row * 128;
        out[lane] = r0;
        out[lane + 64] = r1;
        if (lane == 0) {
            I.theta[row] = th * 6.283185307179586f;
            I.rows[row] = (int32_t)slot;
        }
        wave_sync();   // the next pass clears this pass's histogram
    }
}

// Single-orientation path for the small scales (s < a.half_scales): each
// 32-lane half of a wavefront describes its own keypoint (lanes take table
// entries sub, sub + 32, ...), so the per-keypoint steps -- smoothing,
// arg-max, rotation, normalisation -- serve two keypoints per instruction.
// Same arithmetic as orient_describe_kernel<kModeFull>, except that the
// normalisation sums add over 32 lanes in a different order.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8)))
void orient_describe_half_kernel(DescArgs a, const float4* tables)
{
    __shared__ unsigned long long hist_mem[kCellPad + kWaves * 2 * kHalfCopies * kHalfWords];
    __shared__ float smv[kWaves][2][36];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int hf = lane >> 5, sub = lane & 31;
    unsigned long long* hist = hist_mem + kCellPad + (wave * 2 + hf) * kHalfCopies * kHalfWords;
    float* sv = smv[wave][hf];

    // this half's keypoint in its XCD's band list of the small scales. The
    // wave's two halves take entries 2 m and 2 m + 1 of the list, and every
    // (scale, image) band holds an even number of entries (a max and a min
    // per window), so both halves fall in one band: the search runs once
    // per wave, in scalar registers, and the halves differ by their slot.
    bool live = false;
    int sc = 0, im = 0;
    int64_t slot = 0;
    {
        const int xcd = blockIdx.x % kXcds;
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        int64_t j = (int64_t)(blockIdx.x / kXcds) * (2 * kWaves) + 2 * wv;
        for (int so = 0; so < a.half_scales && !live; ++so) {
            const int s = a.half_scales - 1 - so;
            const uint32_t L = (uint32_t)a.L[s];
            for (int i = 0; i < a.n_images; ++i) {
                const uint32_t nby = ((uint32_t)a.img[i].h + L - 1u) / L;
                const uint32_t nbx = ((uint32_t)a.img[i].w + L - 1u) / L;
                const uint32_t r0 = (uint32_t)xcd * nby / kXcds;
                const uint32_t r1 = (uint32_t)(xcd + 1) * nby / kXcds;
                const int64_t cnt = 2 * (int64_t)(r1 - r0) * nbx;
                if (j < cnt) {
                    live = true;
                    sc = s;
                    im = i;
                    slot = a.slot_base[s][i] + 2 * (int64_t)r0 * nbx + j;
                    break;
                }
                j -= cnt;
            }
        }
    }
    slot = live ? slot + hf : 0;
    const DescImg& I = a.img[im];
    const ScaleGeom G = a.geom[sc];   // a copy: its fields stay in registers through the visit loops
    const int kx = I.x[slot], ky = I.y[slot];
    const float2* field = I.field;
    const int W = I.w, H = I.h;

    for (int b = sub; b < kHalfCopies * kHalfWords; b += 32) hist[b] = 0ull;
    wave_sync();

    // ---- orientation ----
    orient_votes<32, kHalfCopies, kHalfWords>(hist, sub, live, kx, ky, field, W, H, G, tables);
    wave_sync();
    auto bin = [&](int k) {
        unsigned long long v = 0ull;
#pragma unroll
        for (int c = 0; c < kHalfCopies; ++c) v += hist[c * kHalfWords + k];
        return (float)v * kOrientVoteInv;
    };
    // each bin converted once: lane sub holds bin sub (ha) and, for sub < 4,
    // bin 32 + sub (hb); a neighbour bin comes from the lane that holds it
    const float ha = bin(sub);
    const float hb = sub < 4 ? bin(32 + sub) : 0.0f;
    // each lane clears the orientation bins it read (the descriptor votes
    // come after the next wave_sync)
#pragma unroll
    for (int c = 0; c < kHalfCopies; ++c) {
        hist[c * kHalfWords + sub] = 0ull;
        if (sub < 4) hist[c * kHalfWords + 32 + sub] = 0ull;
    }
    auto at = [&](int b) {           // bin b (0 .. 35) of this half's histogram
        const float va = __shfl(ha, b & 31, 32);
        const float vb = __shfl(hb, (b - 32) & 31, 32);
        return b < 32 ? va : vb;
    };
    auto smooth = [&](int k, float h0) {
        return smooth5(at((k + 34) % 36), at((k + 35) % 36), h0, at((k + 1) % 36),
                       at((k + 2) % 36));
    };
    // lane sub holds bin sub and, for sub < 4, bin 32 + sub
    const float s1 = smooth(sub, ha);
    const float s2t = smooth(32 + (sub & 3), hb);   // every lane joins the shuffles
    const float s2 = sub < 4 ? s2t : -1.0f;
    sv[sub] = s1;
    if (sub < 4) sv[32 + sub] = s2;
    float bv = s1;
    int bk = sub;
    if (s2 > bv) {            // bin 32 + sub above bin sub (ties keep the lower bin)
        bv = s2;
        bk = 32 + sub;
    }
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
        const float ov = __shfl_xor(bv, off, 32);
        const int okk = __shfl_xor(bk, off, 32);
        if (ov > bv || (ov == bv && okk < bk)) {
            bv = ov;
            bk = okk;
        }
    }
    wave_sync();
    const float hm = sv[(bk + 35) % 36], hp = sv[(bk + 1) % 36];
    const float th_turns = bin_turns(bk, hm, bv, hp);
    if (live && sub == 0) I.theta[slot] = th_turns * 6.283185307179586f;

    // ---- descriptor: lane sub holds elements sub + 32 q ----
    // The norms add (e, e + 64) pairs first, then the halves, then butterflies
    // over 32 lanes: the summation tree of wave_sum in the whole-wave kernel,
    // so both kernels give bit-identical descriptors.
    desc_votes<32, kHalfCopies, kHalfWords>(hist, sub, live, kx, ky, field, W, H, G, tables,
                                a.bcount + sc * kDescBuckets, th_turns);
    wave_sync();
    float d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = desc_bin<kHalfCopies, kHalfWords>(hist, sub + 32 * q) * G.dinv;
    auto half_norm = [&]() {
        float ss = fmaf(d[0], d[0], d[2] * d[2]) + fmaf(d[1], d[1], d[3] * d[3]);
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 32);
        return __builtin_amdgcn_rcpf(fmaxf(sqrtf(ss), 1e-12f));
    };
    float inv = half_norm();
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = fminf(d[q] * inv, 0.2f);
    inv = half_norm();
    if (live) {
        float* out = I.desc + slot * 128;
#pragma unroll
        for (int q = 0; q < 4; ++q) out[sub + 32 * q] = d[q] * inv;
    }
}

// Exclusive prefix of the per-slot orientation counts of each image (one
// 1024-thread workgroup per image): row offset of every slot and the total.
struct ScanImg {
    const int32_t* count;
    int64_t* offset;
    int64_t n;
    int64_t* total;
};
struct ScanArgs {
    int32_t n_images;
    ScanImg img[kDescBatch];
};

constexpr int kScanThreads = 1024;
constexpr int kScanTile = 4 * kScanThreads;   // counts per pass: four per thread

// Passes over tiles of 4,096 counts: thread t sums counts 4t .. 4t + 3 of the
// tile (one 16-byte load), a shuffle scan within each wavefront and a scan of
// the 16 wavefront totals give its exclusive prefix, and the tile total
// carries into the next pass. Loads and stores are coalesced.
__global__ __launch_bounds__(kScanThreads) void orient_scan_kernel(ScanArgs a)
{
    __shared__ int64_t wsum[kScanThreads / 64];
    const ScanImg& I = a.img[blockIdx.x];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int64_t carry = 0;
    for (int64_t base = 0; base < I.n; base += kScanTile) {
        const int64_t i0 = base + 4 * t;
        int c[4] = {0, 0, 0, 0};
        if (i0 + 3 < I.n) {
            const int4 v = *reinterpret_cast<const int4*>(I.count + i0);
            c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
        } else {
            for (int k = 0; k < 4; ++k)
                if (i0 + k < I.n) c[k] = I.count[i0 + k];
        }
        const int sum = c[0] + c[1] + c[2] + c[3];
        int x = sum;                                   // inclusive scan in the wavefront
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        if (w == 0) {                                  // inclusive scan of the 16 totals
            int64_t v = lane < kScanThreads / 64 ? wsum[lane] : 0;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const int64_t y = __shfl_up(v, off);
                if (lane >= off) v += y;
            }
            if (lane < kScanThreads / 64) wsum[lane] = v;
        }
        __syncthreads();
        int64_t run = carry + (w > 0 ? wsum[w - 1] : 0) + (x - sum);
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < I.n) I.offset[i0 + k] = run;
            run += c[k];
        }
        carry += wsum[kScanThreads / 64 - 1];
        __syncthreads();                               // wsum is rewritten by the next pass
    }
    if (t == 0) *I.total = carry;
}

// Workspace: disc tables, then the bucket entry counts, then the fields.
size_t counts_offset(const Geometry& g)
{
    return align_up((size_t)g.table_entries * sizeof(float4), 256);
}

size_t field_offset(const Geometry& g)
{
    return counts_offset(g) + align_up((size_t)LPSIFT_MAX_SCALES * kDescBuckets * 4, 256);
}

}  // namespace

size_t describe_workspace_bytes(const lpsift_image* imgs, int n, const Geometry& g)
{
    size_t b = field_offset(g);
    for (int i = 0; i < n; ++i)
        b += align_up((size_t)imgs[i].height * (size_t)imgs[i].width * sizeof(float2), 256);
    return b;
}

namespace {

int64_t slots_of(const lpsift_image& im, const Geometry& g)
{
    int64_t n_kp = 0;
    for (int s = 0; s < g.n_scales; ++s)
        n_kp += 2 * n_windows(im.height, g.L[s]) * n_windows(im.width, g.L[s]);
    return n_kp;
}

// Per-image buffers of the multi-orientation variant, after the fields:
// angles [n_kp][kMaxOrient] f32, counts [n_kp] i32, row offsets [n_kp] i64.
size_t multi_bytes(int64_t n_kp)
{
    return align_up((size_t)n_kp * kMaxOrient * 4, 256) + align_up((size_t)n_kp * 4, 256) +
           align_up((size_t)n_kp * 8, 256);
}

int run_describe(const lpsift_image* imgs, int n, const lpsift_keypoints* kps, const Geometry& g,
                 void* ws, float* const* theta, float* const* desc, const int32_t* const* sel,
                 const int64_t* n_sel, const MultiSpec* ms, hipStream_t stream)
{
    char* base = static_cast<char*>(ws);
    float4* tables = reinterpret_cast<float4*>(base);

    int32_t* bcount = reinterpret_cast<int32_t*>(base + counts_offset(g));
    TableArgs ta{};
    ta.n_scales = g.n_scales;
    for (int s = 0; s < g.n_scales; ++s) {
        const ScaleGeom& G = g.s[s];
        ta.r2_orient[s] = G.r2_orient;
        ta.off_orient[s] = G.off_orient;
        ta.k_orient[s] = G.k_orient;
        ta.r2_desc[s] = G.r2_desc;
        ta.off_desc[s] = G.off_desc;
        ta.cap_desc[s] = G.cap_desc;
        ta.n_buckets[s] = G.n_buckets;
        ta.k_desc[s] = G.k_desc;
        ta.dscale[s] = G.dscale;
        ta.inv_ws[s] = 1.0 / (double)G.ws;
    }
    // the tables are built by the first field launch (n_table workgroups)
    int n_table = (1 + kDescBuckets) * g.n_scales;

    size_t foff = field_offset(g);
    size_t moff = describe_workspace_bytes(imgs, n, g);   // multi buffers follow the fields
    for (int b0 = 0, nb = 0; b0 < n; b0 += nb) {
        // images per launch pair (field + describe): at most kDescBatch, and
        // gradient fields of at most kFieldGroupBytes together so that they
        // stay in the last-level cache while the describe kernel reads them
        size_t group = 0;
        nb = 0;
        while (b0 + nb < n && nb < kDescBatch) {
            const size_t fb = (size_t)imgs[b0 + nb].height * (size_t)imgs[b0 + nb].width * sizeof(float2);
            if (nb > 0 && group + fb > kFieldGroupBytes) break;
            group += fb;
            ++nb;
        }
        FieldArgs fa{};
        DescArgs da{};
        ScanArgs sa{};
        fa.n_images = nb;
        da.n_images = nb;
        da.n_scales = g.n_scales;
        sa.n_images = nb;
        int maxw = 0, maxh = 0;
        for (int i = 0; i < nb; ++i) {
            const lpsift_image& im = imgs[b0 + i];
            float2* field = reinterpret_cast<float2*>(base + foff);
            foff += align_up((size_t)im.height * (size_t)im.width * sizeof(float2), 256);
            fa.img[i] = FieldImg{im.data, im.pitch, im.height, im.width, field};
            maxw = im.width > maxw ? im.width : maxw;
            maxh = im.height > maxh ? im.height : maxh;
            const lpsift_keypoints& kp = kps[b0 + i];
            const int64_t n_kp = slots_of(im, g);
            da.img[i] = DescImg{field, im.height, im.width, kp.x, kp.y, theta[b0 + i], desc[b0 + i],
                                sel ? sel[b0 + i] : nullptr, sel ? n_sel[b0 + i] : 0, n_kp,
                                nullptr, nullptr, nullptr, nullptr};
            if (ms) {
                char* m = base + moff;
                da.img[i].obuf = reinterpret_cast<float*>(m);
                m += align_up((size_t)n_kp * kMaxOrient * 4, 256);
                da.img[i].count = reinterpret_cast<int32_t*>(m);
                m += align_up((size_t)n_kp * 4, 256);
                da.img[i].offset = reinterpret_cast<int64_t*>(m);
                da.img[i].rows = ms->rows[b0 + i];
                moff += multi_bytes(n_kp);
                sa.img[i] = ScanImg{da.img[i].count, da.img[i].offset, n_kp, ms->n_rows + b0 + i};
            }
        }
        {
            TimedScope ts(LPSIFT_KERNEL_GRADIENT, stream);
            const int gx = (maxw + 256 * kFieldPx - 1) / (256 * kFieldPx);
            const int64_t blocks = (int64_t)n_table + (int64_t)gx * maxh * nb;
            hipLaunchKernelGGL(polar_field_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, fa,
                               ta, tables, bcount, n_table, gx, maxh);
            n_table = 0;
        }
        if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;

        da.list = sel ? 1 : 0;
        da.max_orient = ms ? ms->max_orient : 1;
        da.peak_ratio = ms ? ms->peak_ratio : 1.0f;
        da.bcount = bcount;
        // per-XCD band lists; the grid covers the longest one
        int64_t longest = 0;
        for (int s = 0; s < g.n_scales; ++s) {
            da.geom[s] = g.s[s];
            da.L[s] = g.L[s];
        }
        for (int i = 0; i < nb; ++i) {
            const lpsift_image& im = imgs[b0 + i];
            int64_t slot = 0;
            for (int s = 0; s < g.n_scales; ++s) {
                da.slot_base[s][i] = slot;
                slot += 2 * n_windows(im.height, g.L[s]) * n_windows(im.width, g.L[s]);
            }
        }
        for (int x = 0; x < kXcds; ++x) {
            int64_t items = 0;
            for (int s = 0; s < g.n_scales; ++s)
                for (int i = 0; i < nb; ++i)
                    items += band_items(x, n_windows(imgs[b0 + i].height, g.L[s]),
                                        n_windows(imgs[b0 + i].width, g.L[s]));
            longest = items > longest ? items : longest;
        }
        const dim3 grid((unsigned)(((longest + kWaves - 1) / kWaves) * kXcds));
        if (sel) {
            int64_t entries = 0;
            for (int i = 0; i < nb; ++i) entries += n_sel[b0 + i];
            if (entries > 0) {
                TimedScope ts(LPSIFT_KERNEL_DESCRIBE, stream);
                hipLaunchKernelGGL(orient_describe_kernel<kModeFull>,
                                   dim3((unsigned)((entries + kWaves - 1) / kWaves)),
                                   dim3(64 * kWaves), 0, stream, da, tables);
                if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;
            }
        } else if (ms) {
            {
                TimedScope ts(LPSIFT_KERNEL_ORIENT_MULTI, stream);
                if (longest > 0)
                    hipLaunchKernelGGL(orient_describe_kernel<kModeOrient>, grid, dim3(64 * kWaves),
                                       0, stream, da, tables);
                hipLaunchKernelGGL(orient_scan_kernel, dim3(nb), dim3(kScanThreads), 0, stream, sa);
                if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;
            }
            if (longest > 0) {
                TimedScope ts(LPSIFT_KERNEL_DESCRIBE, stream);
                hipLaunchKernelGGL(orient_describe_kernel<kModeGiven>, grid, dim3(64 * kWaves), 0,
                                   stream, da, tables);
                if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;
            }
        } else if (longest > 0) {
            // small scales on half wavefronts, the others on whole ones
            int hs = 0;
            while (hs < g.n_scales && g.s[hs].n_desc <= kHalfMaxVisits) ++hs;
            int64_t half_longest = 0, full_longest = 0;
            for (int x = 0; x < kXcds; ++x) {
                int64_t ih = 0, ifu = 0;
                for (int s = 0; s < g.n_scales; ++s)
                    for (int i = 0; i < nb; ++i) {
                        const int64_t it = band_items(x, n_windows(imgs[b0 + i].height, g.L[s]),
                                                      n_windows(imgs[b0 + i].width, g.L[s]));
                        (s < hs ? ih : ifu) += it;
                    }
                half_longest = ih > half_longest ? ih : half_longest;
                full_longest = ifu > full_longest ? ifu : full_longest;
            }
            da.half_scales = hs;
            da.first_scale = hs;
            TimedScope ts(LPSIFT_KERNEL_DESCRIBE, stream);
            if (full_longest > 0) {
                const dim3 gf((unsigned)(((full_longest + kWaves - 1) / kWaves) * kXcds));
                hipLaunchKernelGGL(orient_describe_kernel<kModeFull>, gf, dim3(64 * kWaves), 0,
                                   stream, da, tables);
            }
            if (half_longest > 0) {
                const dim3 gh((unsigned)(((half_longest + 2 * kWaves - 1) / (2 * kWaves)) * kXcds));
                hipLaunchKernelGGL(orient_describe_half_kernel, gh, dim3(64 * kWaves), 0, stream, da,
                                   tables);
            }
            if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;
        }
    }
    return LPSIFT_OK;
}

}  // namespace

int launch_describe(const lpsift_image* imgs, int n, const lpsift_keypoints* kps,
                    const Geometry& g, void* ws, float* const* theta, float* const* desc,
                    const int32_t* const* sel, const int64_t* n_sel, hipStream_t stream)
{
    return run_describe(imgs, n, kps, g, ws, theta, desc, sel, n_sel, nullptr, stream);
}

size_t describe_multi_workspace_bytes(const lpsift_image* imgs, int n, const Geometry& g)
{
    size_t b = describe_workspace_bytes(imgs, n, g);
    for (int i = 0; i < n; ++i) b += multi_bytes(slots_of(imgs[i], g));
    return b;
}

int launch_describe_multi(const lpsift_image* imgs, int n, const lpsift_keypoints* kps,
                          const Geometry& g, void* ws, const MultiSpec& ms, float* const* theta,
                          float* const* desc, hipStream_t stream)
{
    return run_describe(imgs, n, kps, g, ws, theta, desc, nullptr, nullptr, &ms, stream);
}

}  // namespace lpsift
