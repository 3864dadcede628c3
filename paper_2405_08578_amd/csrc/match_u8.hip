// uint8 descriptors: quantisation and an exact matcher on the int8 matrix
// cores (Sec. 2.4, Eq. 6, on the stored form SIFT implementations use).
//
// q = min(255, rint(512 d)) per element. With queries a and candidates b in
// 0..255, a_hat = 127 - a and b' = b - 128 are int8 (bytes a ^ 0x7F, b ^ 0x80)
// and, with P = a_hat . b' from v_mfma_i32_32x32x32_i8 (exact in int32),
//     D - |a - 128|^2 = C_b + 2 P,   C_b = |b - 128|^2 + 2 sum(b - 128),
// where D = |a - b|^2 is the exact squared distance. C_b depends on the
// candidate only, so for each query the candidates rank by C_b + 2 P; shifted
// by 2^21 that value lies in [0, 2^24) for any uint8 input. Candidates are
// taken in chunks of 256, and each output becomes the exact 32-bit key
//     ((C_b + 2^21) << 8 | chunk-local index) + (P << 9)
// in one shift-add (unsigned order = (distance, index)); each lane keeps a
// top-2 with one min and one med3. At the end of a chunk the two keys are
// widened to 64 bits (value << 32 | global index) and folded into the lane's
// running top-2. A wavefront holds 4 x 32 queries in registers (16 per set);
// a 256-thread workgroup (512 queries) streams a range of chunks through LDS,
// 32 candidates per tile, the next tile's loads in flight during the current
// tile. A merge kernel (one thread per query) takes the two smallest keys over
// the ranges, adds |a - 128|^2 back and applies the ratio test on sqrt(D) in
// double; no rescoring is needed.
#include "internal.h"

namespace lpsift {
namespace {

typedef int intx4 __attribute__((ext_vector_type(4)));
typedef int intx16 __attribute__((ext_vector_type(16)));

constexpr int kU8Sets = 4;                   // 32-query sets per wavefront
constexpr int kU8QB = 4 * 32 * kU8Sets;      // queries per workgroup (512)
constexpr int kU8CT = 32;                    // candidates per LDS tile
constexpr int kU8Row = 128 + 16;             // LDS bytes per candidate row
constexpr int kU8Chunk = 256;                // candidates per chunk (8 index bits)
constexpr uint32_t kEmpty = 0xFFFFFFFFu;     // above every real key (value < 2^24 - 1)
constexpr int kOff = 1 << 21;                // |a - 128|^2 <= 2^21
constexpr uint64_t kNone = ~0ull;

__global__ __launch_bounds__(256) void quantize_u8_kernel(const float* __restrict__ d, int64_t n,
                                                          uint8_t* __restrict__ q)
{
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i >= n * 128) return;
    const float4 v = *reinterpret_cast<const float4*>(d + i);
    const float f[4] = {v.x, v.y, v.z, v.w};
    uint32_t w = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float r = fminf(fmaxf(rintf(512.0f * f[k]), 0.0f), 255.0f);   // 512 d is exact
        w |= (uint32_t)r << (8 * k);
    }
    *reinterpret_cast<uint32_t*>(q + i) = w;
}

// Candidate term of every row, as the low half of its key:
// ((|b - 128|^2 + 2 sum(b - 128) + 2^21) << 8) | (row mod 256). 16 lanes per row.
__global__ __launch_bounds__(256) void cterm_u8_kernel(const uint8_t* __restrict__ B, int64_t n,
                                                       uint32_t* __restrict__ cterm)
{
    const int64_t row = (int64_t)blockIdx.x * 16 + threadIdx.x / 16;
    const int part = threadIdx.x % 16;
    int s = 0;
    if (row < n) {
        const uint2 v = *reinterpret_cast<const uint2*>(B + row * 128 + part * 8);
        const uint32_t w[2] = {v.x, v.y};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = (int)((w[k >> 2] >> (8 * (k & 3))) & 255u) - 128;
            s += c * c + 2 * c;
        }
    }
    for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
    if (row < n && part == 0) cterm[row] = ((uint32_t)(s + kOff) << 8) | (uint32_t)(row & 255);
}

__device__ inline intx4 xor_bytes(uint4 u, uint32_t m)
{
    return intx4{(int)(u.x ^ m), (int)(u.y ^ m), (int)(u.z ^ m), (int)(u.w ^ m)};
}

// median of three unsigned values (v_med3_u32, no builtin exists for it)
__device__ inline uint32_t umed3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ inline void top2_u64(uint64_t x, uint64_t& a, uint64_t& b)
{
    const uint64_t lo = x < a ? x : a, hi = x < a ? a : x;
    a = lo;
    b = hi < b ? hi : b;
}

__device__ inline void fold_key(uint32_t k, int64_t chunk, uint64_t& a, uint64_t& b)
{
    if (k == kEmpty) return;
    top2_u64(((uint64_t)(k >> 8) << 32) | (uint64_t)(chunk * kU8Chunk + (k & 255u)), a, b);
}

// Grid: x = query blocks of 512, y = chunk ranges of `per` chunks.
// part[(y * nA + q) * 2 + {0, 1}] = the two smallest 64-bit keys of query q
// over range y (kNone where there are fewer candidates).
__global__ __launch_bounds__(256, 2) void match_topk_u8_kernel(
    const uint8_t* __restrict__ A, int64_t nA, const uint8_t* __restrict__ B, int64_t nB,
    const uint32_t* __restrict__ cterm, int per, uint64_t* __restrict__ part)
{
    __shared__ __attribute__((aligned(16))) uint8_t tile[kU8CT * kU8Row];
    __shared__ __attribute__((aligned(16))) uint32_t tc[kU8CT];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int64_t c0 = (int64_t)blockIdx.y * per;
    const int64_t nchunks = (nB + kU8Chunk - 1) / kU8Chunk;
    const int64_t c1 = (c0 + per < nchunks) ? c0 + per : nchunks;

    // queries: set t, K-step s holds bytes [32 s + 16 h, +16) of query q_t
    intx4 qv[kU8Sets][4];
    int64_t qi[kU8Sets];
#pragma unroll
    for (int t = 0; t < kU8Sets; ++t) {
        const int64_t q = (int64_t)blockIdx.x * kU8QB + wave * (32 * kU8Sets) + t * 32 + col;
        qi[t] = q;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const uint4 u = (q < nA) ? *reinterpret_cast<const uint4*>(A + q * 128 + 32 * s + 16 * h)
                                     : make_uint4(0u, 0u, 0u, 0u);
            qv[t][s] = xor_bytes(u, 0x7F7F7F7Fu);
        }
    }
    uint64_t K1[kU8Sets], K2[kU8Sets];
#pragma unroll
    for (int t = 0; t < kU8Sets; ++t) K1[t] = K2[t] = kNone;

    // staging: thread -> (row r, 16-byte piece c16) of a 32-row tile
    const int sr = tid >> 3, sc = tid & 7;
    const int64_t first = c0 * kU8Chunk;
    const int64_t last = (c1 * kU8Chunk < nB) ? c1 * kU8Chunk : nB;
    uint4 g = make_uint4(0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u);
    uint32_t gc = kEmpty;
    if (first + sr < last) g = *reinterpret_cast<const uint4*>(B + (first + sr) * 128 + sc * 16);
    if (tid < kU8CT && first + tid < last) gc = cterm[first + tid];
    for (int64_t chunk = c0; chunk < c1; ++chunk) {
        uint32_t k1[kU8Sets], k2[kU8Sets];
#pragma unroll
        for (int t = 0; t < kU8Sets; ++t) k1[t] = k2[t] = kEmpty;
        const int64_t cb = chunk * kU8Chunk;
        const int64_t ce = (cb + kU8Chunk < nB) ? cb + kU8Chunk : nB;
        for (int64_t t0 = cb; t0 < ce; t0 += kU8CT) {
            __syncthreads();
            *reinterpret_cast<intx4*>(&tile[sr * kU8Row + sc * 16]) = xor_bytes(g, 0x80808080u);
            if (tid < kU8CT) tc[tid] = gc;
            __syncthreads();
            {   // next tile of the range (padding rows: b = 128, key kEmpty)
                const int64_t n0 = t0 + kU8CT;
                g = make_uint4(0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u);
                gc = kEmpty;
                if (n0 + sr < last) g = *reinterpret_cast<const uint4*>(B + (n0 + sr) * 128 + sc * 16);
                if (tid < kU8CT && n0 + tid < last) gc = cterm[n0 + tid];
            }
            intx16 acc[kU8Sets];
#pragma unroll
            for (int t = 0; t < kU8Sets; ++t)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[t][r] = 0;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const intx4 b = *reinterpret_cast<const intx4*>(&tile[col * kU8Row + 32 * s + 16 * h]);
#pragma unroll
                for (int t = 0; t < kU8Sets; ++t)
                    acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(b, qv[t][s], acc[t], 0, 0, 0);
            }
            // accumulator r of the lane is candidate row 8 (r / 4) + 4 h + r % 4
            uint32_t cr[16];
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                const uint4 v = *reinterpret_cast<const uint4*>(&tc[8 * q4 + 4 * h]);
                cr[4 * q4 + 0] = v.x; cr[4 * q4 + 1] = v.y; cr[4 * q4 + 2] = v.z; cr[4 * q4 + 3] = v.w;
            }
            // two rows at a time: for k1 <= k2 and new keys x, y the two
            // smallest of all four are min3(k1, x, y) and min(k2, med3(k1, x, y))
#pragma unroll
            for (int r = 0; r < 16; r += 2) {
#pragma unroll
                for (int t = 0; t < kU8Sets; ++t) {
                    const uint32_t x = cr[r] + ((uint32_t)acc[t][r] << 9);
                    const uint32_t y = cr[r + 1] + ((uint32_t)acc[t][r + 1] << 9);
                    k2[t] = min(k2[t], umed3(k1[t], x, y));
                    k1[t] = min(k1[t], min(x, y));
                }
            }
        }
#pragma unroll
        for (int t = 0; t < kU8Sets; ++t) {
            fold_key(k1[t], chunk, K1[t], K2[t]);
            fold_key(k2[t], chunk, K1[t], K2[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < kU8Sets; ++t) {
        const uint64_t o1 = (uint64_t)__shfl_xor((long long)K1[t], 32);
        const uint64_t o2 = (uint64_t)__shfl_xor((long long)K2[t], 32);
        top2_u64(o1, K1[t], K2[t]);
        top2_u64(o2, K1[t], K2[t]);
        if (h == 0 && qi[t] < nA) {
            uint64_t* o = part + ((int64_t)blockIdx.y * nA + qi[t]) * 2;
            o[0] = K1[t];
            o[1] = K2[t];
        }
    }
}

// One thread per query: the two smallest keys over all ranges, D = value -
// 2^21 + |a - 128|^2, then Eq. 6 with the ratio test on sqrt(D).
__global__ __launch_bounds__(256) void merge_u8_kernel(
    const uint8_t* __restrict__ A, int64_t nA, int ranges, const uint64_t* __restrict__ part,
    double ratio, float abs_thresh, int32_t* __restrict__ match, float* __restrict__ d1out,
    float* __restrict__ d2out)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nA) return;
    uint64_t a = kNone, b = kNone;
    for (int y = 0; y < ranges; ++y) {
        const uint4 v = *reinterpret_cast<const uint4*>(part + ((int64_t)y * nA + q) * 2);
        const uint64_t x1 = ((uint64_t)v.y << 32) | v.x, x2 = ((uint64_t)v.w << 32) | v.z;
        top2_u64(x1, a, b);
        top2_u64(x2, a, b);
    }
    if (a == kNone) {
        match[q] = -1;
        d1out[q] = INFINITY;
        d2out[q] = INFINITY;
        return;
    }
    int na = 0;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const uint4 u = *reinterpret_cast<const uint4*>(A + q * 128 + 16 * p);
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int c = (int)((w[k >> 2] >> (8 * (k & 3))) & 255u) - 128;
            na += c * c;
        }
    }
    const int64_t D1 = (int64_t)(a >> 32) - kOff + na;
    const double s1 = sqrt((double)D1);
    const double s2 = (b == kNone) ? INFINITY : sqrt((double)((int64_t)(b >> 32) - kOff + na));
    const bool ratio_ok = __builtin_isinf(ratio) || s1 < ratio * s2;
    const bool keep = ratio_ok && s1 / 512.0 < (double)abs_thresh;
    match[q] = keep ? (int32_t)(a & 0xFFFFFFFFu) : -1;
    d1out[q] = (float)(s1 / 512.0);
    d2out[q] = (float)(s2 / 512.0);
}

struct U8Plan {
    int64_t qblocks, chunks, per, ranges;
};

U8Plan plan_u8(int64_t nA, int64_t nB)
{
    U8Plan p;
    p.qblocks = (nA + kU8QB - 1) / kU8QB;
    p.chunks = (nB + kU8Chunk - 1) / kU8Chunk;
    // about 2048 workgroups (8 per compute unit) when the product allows
    const int64_t want = p.qblocks > 0 ? (2048 + p.qblocks - 1) / p.qblocks : 1;
    const int64_t ranges = want < p.chunks ? want : p.chunks;
    p.per = ranges > 0 ? (p.chunks + ranges - 1) / ranges : 1;
    p.ranges = (p.chunks + p.per - 1) / p.per;
    return p;
}

}  // namespace

int launch_quantize_u8(const float* desc, int64_t n, uint8_t* out, hipStream_t stream)
{
    if (n == 0) return LPSIFT_OK;
    const int64_t quads = n * 32;
    hipLaunchKernelGGL(quantize_u8_kernel, dim3((unsigned)((quads + 255) / 256)), dim3(256), 0,
                       stream, desc, n, out);
    return hipGetLastError() == hipSuccess ? LPSIFT_OK : LPSIFT_EHIP;
}

size_t match_u8_workspace_bytes(int64_t nA, int64_t nB)
{
    const U8Plan p = plan_u8(nA, nB);
    return align_up((size_t)nB * 4, 256) + align_up((size_t)(p.ranges * nA) * 16, 256);
}

int launch_match_u8(const uint8_t* A, int64_t nA, const uint8_t* B, int64_t nB, double ratio,
                    float abs_thresh, void* ws, int32_t* match, float* d1, float* d2,
                    hipStream_t stream)
{
    if (nA == 0) return LPSIFT_OK;
    const U8Plan p = plan_u8(nA, nB);
    uint32_t* cterm = static_cast<uint32_t*>(ws);
    uint64_t* part = reinterpret_cast<uint64_t*>(static_cast<char*>(ws) +
                                                 align_up((size_t)nB * 4, 256));
    if (nB > 0) {
        {
            TimedScope ts(LPSIFT_KERNEL_MATCH_U8_AUX, stream);
            hipLaunchKernelGGL(cterm_u8_kernel, dim3((unsigned)((nB + 15) / 16)), dim3(256), 0,
                               stream, B, nB, cterm);
        }
        TimedScope ts(LPSIFT_KERNEL_MATCH_U8, stream);
        hipLaunchKernelGGL(match_topk_u8_kernel, dim3((unsigned)p.qblocks, (unsigned)p.ranges),
                           dim3(256), 0, stream, A, nA, B, nB, cterm, (int)p.per, part);
    }
    TimedScope ts(LPSIFT_KERNEL_MATCH_U8_AUX, stream);
    hipLaunchKernelGGL(merge_u8_kernel, dim3((unsigned)((nA + 255) / 256)), dim3(256), 0, stream,
                       A, nA, (int)p.ranges, part, ratio, abs_thresh, match, d1, d2);
    return hipGetLastError() == hipSuccess ? LPSIFT_OK : LPSIFT_EHIP;
}

}  // namespace lpsift
