// Descriptor matching (Sec. 2.4, Eq. 6) with the ratio test.
//
// |a - b|^2 = |a|^2 + |b|^2 - 2 a.b, and |a|^2 is constant per query, so the
// nearest candidates of a query are those with the smallest |b|^2 - 2 a.b.
// The a.b contraction is a GEMM of the two descriptor sets and runs on the
// matrix cores; the N_A x N_B score matrix is never stored.
//
// FP32 path (precision 0), v_mfma_f32_32x32x2_f32:
//  * the MFMA's A operand is a 32-candidate tile (rows) and its B operand 32
//    queries (columns), so lane l of the 32x32 result holds 16 candidates of
//    one query (l % 32): the top-2 bookkeeping is private to each lane;
//  * a wavefront keeps 2 x 32 queries in registers for the whole sweep (the K
//    dimension split in halves: lanes 0-31 carry k = 0..63, lanes 32-63 carry
//    k = 64..127 -- any permutation of K shared by both operands leaves the
//    dot products unchanged);
//  * a 256-thread workgroup (4 wavefronts, 256 queries) streams the candidates
//    of its chunk through LDS, 32 at a time, the next tile prefetched into
//    registers while the current one is contracted; the candidate range is
//    split into chunks so that the grid fills the chip.
//  Each lane's top-2 of each chunk survives (4 candidates per query and
//  chunk). The queries are negated and the accumulator starts at |b|^2 / 2
//  of its row, so it ends at |b|^2 / 2 - a.b = (|a - b|^2 - |a|^2) / 2, which
//  orders a query's candidates like their squared distances; a lane keeps
//  32-bit keys (its bits with the low 4 replaced by the accumulator row)
//  with float min3 and med3, about 2.5 VALU instructions per score against
//  ~9 for (score, index) compare-selects -- VALU and MFMA work do not
//  overlap on this part. The 4-bit truncation moves a key by at most 15
//  units in the last place, below the FP32 contraction's own rounding. The rescore kernel keeps the 4 best by contraction score,
//  recomputes their squared distances directly in FP32, takes the two
//  smallest (lowest index on ties) and applies d1 < ratio * d2 in double.
//
// Quantised paths (approximate): BF16 (precision 1, v_mfma_f32_32x32x16_bf16)
// and FP8 E4M3 with one scale per descriptor (precision 2,
// v_mfma_f32_32x32x64_f8f6f4), FP32 accumulation, 4 x 32 queries per wavefront.
// At these rates the VALU can afford ~4 instructions per contraction output, so
// each output becomes one 32-bit key -- the score's float bits with the low
// bits replaced by the candidate's index in its chunk -- and a lane's top-2 is
// kept with an unsigned min and med3 (the score carries an offset C that makes
// it positive, so float bits order like values). The 8 best kept candidates of
// a query are rescored in FP32; a true nearest neighbour can be missed.
//
// Split path (precision 3, exact): each FP32 value is split into two BF16
// parts, a.b ~ hi.hi + hi.lo + lo.hi (three BF16 MFMAs, FP32 accumulation),
// which is ~5x cheaper than the FP32 contraction and accurate to ~1e-4. Each
// lane keeps float keys (the score with its low 4 bits replaced by the
// accumulator row, within 15 units in the last place of the score): the two
// largest, whose candidates are recovered, and the third largest as the bound
// of everything left behind. From the split errors and that truncation a
// per-query bound E on every score error follows; if
// everything a lane did not keep scores above the kept second best by more
// than 2E, the true two nearest are among the kept ones and FP32 rescoring of
// those is exact. Other queries go to a device-side list matched by the FP32
// path. The lists equal the FP32 path's.
#include <vector>

#include "internal.h"

namespace lpsift {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

constexpr int kDefaultWaves = 4; // FP32: wavefronts (64 queries each) per workgroup
constexpr int kCT = 32;         // FP32: candidates per LDS tile
constexpr int kRow = 128 + 4;   // FP32: padded LDS row (floats)
constexpr int kKeep = 4;        // FP32: candidates kept per (query, chunk)

// Relative bound on the BF16 contraction error per unit |a||b|: 2u + u^2 +
// 128 x 2^-24 with u = 2^-8 (used to keep the quantised paths' scores positive).
constexpr float kBf16DotErr = 0.00785f;

// ------------------------------------------------------------------ common --

// Zeroes the per-call counters (used instead of a memset so the whole call
// can be captured in a graph).
__global__ void init_counters_kernel(uint32_t* c, int n)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
}

// Maximum of v over the 256-thread workgroup, merged into *dst with one
// atomic per workgroup (v: bits of non-negative floats, which order like
// unsigned integers).
__device__ inline void block_max_atomic(uint32_t* dst, uint32_t v)
{
    __shared__ uint32_t red[4];
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(dst, max(max(red[0], red[1]), max(red[2], red[3])));
    __syncthreads();
}

// Rows per workgroup of the row passes: 16 blocks of 16 rows, so that the
// maxima over rows cost one atomic per 256 rows.
constexpr int kRowBlocks = 16;
constexpr int kRowsPerWg = 16 * kRowBlocks;

// |x|^2 of row blk * 16 + threadIdx.x / 16 (written to out if given), 16 lanes
// per row; returns it (0 beyond n).
__device__ inline float sqnorm_rows(const float* __restrict__ X, int64_t n, int64_t blk,
                                    float* __restrict__ out)
{
    const int64_t row = blk * 16 + threadIdx.x / 16;
    const int part = threadIdx.x % 16;
    float s = 0.0f;
    if (row < n) {
        const float4* p = reinterpret_cast<const float4*>(X + row * 128 + part * 8);
        const float4 a = p[0], b = p[1];
        s = a.x * a.x + a.y * a.y + a.z * a.z + a.w * a.w + b.x * b.x + b.y * b.y + b.z * b.z + b.w * b.w;
    }
    for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
    if (row < n && part == 0 && out) out[row] = s;
    return s;
}

// |x|^2 of every row (optional output) and the maximum over rows, as the bit
// pattern of a non-negative float (bits order like values); kRowsPerWg rows
// per workgroup.
__global__ __launch_bounds__(256) void sqnorm_kernel(const float* __restrict__ X, int64_t n,
                                                     float* __restrict__ out,
                                                     uint32_t* __restrict__ maxbits)
{
    float m = 0.0f;
    for (int k = 0; k < kRowBlocks; ++k)
        m = fmaxf(m, sqnorm_rows(X, n, (int64_t)blockIdx.x * kRowBlocks + k, out));
    if (maxbits) block_max_atomic(maxbits, __float_as_uint(m));
}

// ---------------------------------------------------------------- FP32 path --

// Median of three unsigned integers (one VALU instruction; the compiler
// does not form it from min/max).
__device__ inline uint32_t umed3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Minimum and median of three finite floats given as their bits (the
// compiler's float min / med3 would first quiet each operand, rebuilt from
// integer bits, as a possible NaN: one more instruction per operand).
__device__ inline int fmin3_bits(int a, int b, int c)
{
    int r;
    asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ inline int fmed3_bits(int a, int b, int c)
{
    int r;
    asm("v_med3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// |b|^2 standing in for padded tile rows: finite, so their keys stay
// ordinary floats, and above every real squared distance.
constexpr float kPadNorm = 3.0e38f;

// One (query block, chunk) work item of the FP32 contraction, kW wavefronts
// of 64 queries each (a block of 64 kW queries). nq: number of queries;
// qlist (optional) maps list entry i to its query row, results for entry i
// are stored at position i.
template <int kW>
__device__ inline void topk_f32_item(const float* __restrict__ A, int64_t nq,
                                     const int32_t* __restrict__ qlist,
                                     const float* __restrict__ B, int64_t nB,
                                     const float* __restrict__ nrmB, int64_t chunk_len, int chunks,
                                     int32_t* __restrict__ cidx, float* __restrict__ cscore,
                                     int64_t qblk, int chunk)
{
    __shared__ __attribute__((aligned(16))) float tile[kCT * kRow];
    __shared__ __attribute__((aligned(16))) float tnrm[kCT];   // |b|^2 / 2 of the tile rows
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int64_t i0 = qblk * (64 * kW) + wave * 64 + col;
    const int64_t i1 = i0 + 32;
    const int64_t q0 = (i0 < nq) ? (qlist ? qlist[i0] : i0) : -1;
    const int64_t q1 = (i1 < nq) ? (qlist ? qlist[i1] : i1) : -1;
    // candidate rows cb .. ce - 1 (nB < 2^31: unsigned tile positions cannot wrap)
    const uint32_t cb = (uint32_t)((int64_t)chunk * chunk_len);
    const uint32_t ce = (uint32_t)(((int64_t)cb + chunk_len < nB) ? (int64_t)cb + chunk_len : nB);

    // queries in registers, negated: qa[i] = -A[q0][h*64 + i], qb[i] =
    // -A[q1][h*64 + i]; na, nb: |a|^2 of the two queries
    float qa[64], qb[64];
    float na, nb;
    {
        const float4* pa = reinterpret_cast<const float4*>(A + q0 * 128 + h * 64);
        const float4* pb = reinterpret_cast<const float4*>(A + q1 * 128 + h * 64);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float4 va = (q0 >= 0) ? pa[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 vb = (q1 >= 0) ? pb[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            qa[4 * i + 0] = -va.x; qa[4 * i + 1] = -va.y; qa[4 * i + 2] = -va.z; qa[4 * i + 3] = -va.w;
            qb[4 * i + 0] = -vb.x; qb[4 * i + 1] = -vb.y; qb[4 * i + 2] = -vb.z; qb[4 * i + 3] = -vb.w;
        }
        float sa = 0.0f, sb = 0.0f;
#pragma unroll
        for (int i = 0; i < 64; ++i) {
            // opaque from here on: the compiler would otherwise keep the
            // loaded values and negate them again in every tile
            asm volatile("" : "+v"(qa[i]), "+v"(qb[i]));
            sa = fmaf(qa[i], qa[i], sa);
            sb = fmaf(qb[i], qb[i], sb);
        }
        na = sa + __shfl_xor(sa, 32);
        nb = sb + __shfl_xor(sb, 32);
    }

    // Every accumulator starts at |b|^2 / 2 of its row (the same registers for
    // both queries: the first MFMA takes them as its addend) and ends at
    // |b|^2 / 2 - a.b = (|a - b|^2 - |a|^2) / 2, which orders the candidates
    // of a query like their squared distances, with no epilogue arithmetic.
    // Each lane keeps the top-2 of its candidates as 32-bit keys: that float
    // with its low 4 bits replaced by the accumulator row r, compared as
    // floats. A key is kept with min3 and med3; the tile of each kept key is
    // recovered once per tile by comparing the keys with their values before
    // the tile.
    constexpr int kNoKey = 0x7F800000;   // +inf
    int ka1 = kNoKey, ka2 = kNoKey, kb1 = kNoKey, kb2 = kNoKey;
    int ta1 = -1, ta2 = -1, tb1 = -1, tb2 = -1;

    // prefetch: thread t moves float4 number t + nt k (nt = 64 kW threads,
    // k < kF) of a 32 x 128 tile (row (t + nt k) / 32), threads t < 32 also
    // the norm of row t; the base address is uniform, so a whole tile needs no
    // per-lane address or bounds arithmetic
    constexpr int nt = 64 * kW;
    constexpr int kF = kCT * 32 / nt;   // float4 per thread per tile
    static_assert(kF * nt == kCT * 32, "the workgroup moves whole tiles");
    float4 pf[kF];
    float pn = kPadNorm;
    auto fetch = [&](uint32_t t0) {
        const float4* base = reinterpret_cast<const float4*>(B + (int64_t)t0 * 128);
        if (ce - t0 >= (uint32_t)kCT) {
#pragma unroll
            for (int k = 0; k < kF; ++k) pf[k] = base[tid + nt * k];
            if (tid < kCT) pn = nrmB[t0 + tid];
        } else {
#pragma unroll
            for (int k = 0; k < kF; ++k)
                pf[k] = ((uint32_t)((tid + nt * k) >> 5) < ce - t0) ? base[tid + nt * k]
                                                                    : make_float4(0.f, 0.f, 0.f, 0.f);
            if (tid < kCT) pn = ((uint32_t)tid < ce - t0) ? nrmB[t0 + tid] : kPadNorm;
        }
    };
    if (cb < ce) fetch(cb);

    for (uint32_t t0 = cb; t0 < ce; t0 += kCT) {
        __syncthreads();   // the previous tile is no longer read
#pragma unroll
        for (int k = 0; k < kF; ++k) {
            const int f = tid + nt * k;
            const int r = f >> 5, c4 = f & 31;
            *reinterpret_cast<float4*>(&tile[r * kRow + c4 * 4]) = pf[k];
        }
        if (tid < kCT) tnrm[tid] = 0.5f * pn;
        __syncthreads();
        if (ce - t0 > (uint32_t)kCT) fetch(t0 + kCT);

        // rows of accumulator r in this lane: 8 (r / 4) + 4 h + r % 4
        floatx16 acc0, acc1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float4 v = *reinterpret_cast<const float4*>(&tnrm[8 * i + 4 * h]);
            acc0[4 * i] = v.x;
            acc0[4 * i + 1] = v.y;
            acc0[4 * i + 2] = v.z;
            acc0[4 * i + 3] = v.w;
        }
        acc1 = acc0;
        const float* trow = &tile[col * kRow + h * 64];
#pragma unroll
        for (int i4 = 0; i4 < 16; ++i4) {
            const float4 a4 = *reinterpret_cast<const float4*>(trow + 4 * i4);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, qa[4 * i4 + 0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, qb[4 * i4 + 0], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, qa[4 * i4 + 1], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, qb[4 * i4 + 1], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, qa[4 * i4 + 2], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, qb[4 * i4 + 2], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, qa[4 * i4 + 3], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, qb[4 * i4 + 3], acc1, 0, 0, 0);
        }
        const int pa1 = ka1, pa2 = ka2, pb1 = kb1, pb2 = kb2;
        // four rows at a time: for k1 <= k2 and new keys x, y the two smallest
        // of all four are min3(k1, x, y) and min(k2, med3(k1, x, y)); two such
        // steps share one min3 for k2 -- five instructions for four keys
#pragma unroll
        for (int r = 0; r < 16; r += 4) {
            const int xa = (__float_as_int(acc0[r]) & -16) | r;
            const int ya = (__float_as_int(acc0[r + 1]) & -16) | (r + 1);
            const int za = (__float_as_int(acc0[r + 2]) & -16) | (r + 2);
            const int wa = (__float_as_int(acc0[r + 3]) & -16) | (r + 3);
            const int xb = (__float_as_int(acc1[r]) & -16) | r;
            const int yb = (__float_as_int(acc1[r + 1]) & -16) | (r + 1);
            const int zb = (__float_as_int(acc1[r + 2]) & -16) | (r + 2);
            const int wb = (__float_as_int(acc1[r + 3]) & -16) | (r + 3);
            const int ma = fmed3_bits(ka1, xa, ya);
            ka1 = fmin3_bits(ka1, xa, ya);
            ka2 = fmin3_bits(ka2, ma, fmed3_bits(ka1, za, wa));
            ka1 = fmin3_bits(ka1, za, wa);
            const int mb = fmed3_bits(kb1, xb, yb);
            kb1 = fmin3_bits(kb1, xb, yb);
            kb2 = fmin3_bits(kb2, mb, fmed3_bits(kb1, zb, wb));
            kb1 = fmin3_bits(kb1, zb, wb);
        }
        // A kept key equal to its value before the tile is that candidate; the
        // second key equal to the old first one is the old first candidate,
        // unless the first key kept that value too: then this tile produced a
        // key identical to it (same truncated distance and row) and the
        // second slot takes the tile's candidate. Else the key is new.
        const int tt = (int)(t0 - cb);   // chunk-relative tile start
        ta2 = (ka2 == pa2) ? ta2 : ((ka2 == pa1 && ka1 != pa1) ? ta1 : tt);
        ta1 = (ka1 == pa1) ? ta1 : tt;
        tb2 = (kb2 == pb2) ? tb2 : ((kb2 == pb1 && kb1 != pb1) ? tb1 : tt);
        tb1 = (kb1 == pb1) ? tb1 : tt;
    }

    // key -> (candidate index, approximate squared distance |a|^2 + 2 key);
    // padded rows (keys near kPadNorm / 2) and empty slots give index -1
    auto unpack = [&](int k, int t, float nq2, int& j, float& sc) {
        const float v = __int_as_float(k & -16);
        const int r = k & 15;
        const bool real = t >= 0 && v < 0.25f * kPadNorm;
        j = real ? (int)cb + t + 8 * (r >> 2) + 4 * h + (r & 3) : -1;
        sc = real ? fmaf(2.0f, v, nq2) : INFINITY;
    };
    if (q0 >= 0) {
        const int64_t o = (i0 * chunks + chunk) * kKeep + 2 * h;
        int j1, j2;
        float s1, s2;
        unpack(ka1, ta1, na, j1, s1);
        unpack(ka2, ta2, na, j2, s2);
        cidx[o] = j1; cidx[o + 1] = j2;
        cscore[o] = s1; cscore[o + 1] = s2;
    }
    if (q1 >= 0) {
        const int64_t o = (i1 * chunks + chunk) * kKeep + 2 * h;
        int j1, j2;
        float s1, s2;
        unpack(kb1, tb1, nb, j1, s1);
        unpack(kb2, tb2, nb, j2, s2);
        cidx[o] = j1; cidx[o + 1] = j2;
        cscore[o] = s1; cscore[o + 1] = s2;
    }
}

__device__ inline float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Direct FP32 squared distance of query row a (lanes hold a0 = a[lane],
// a1 = a[64 + lane]) to candidate j, summed across the wavefront.
__device__ inline float sqdist(float a0, float a1, const float* __restrict__ B, int64_t j, int lane)
{
    const float x0 = a0 - B[j * 128 + lane], x1 = a1 - B[j * 128 + 64 + lane];
    return wave_sum(fmaf(x0, x0, x1 * x1));
}

// ordered insert by (squared distance, index)
__device__ inline void best2_insert(float s, int j, float& e1, int& j1, float& e2, int& j2)
{
    if (s < e1 || (s == e1 && j < j1)) {
        e2 = e1; j2 = j1;
        e1 = s; j1 = j;
    } else if (s < e2 || (s == e2 && j < j2)) {
        e2 = s; j2 = j;
    }
}

__device__ inline void write_result(int64_t q, float e1, int j1, float e2, double ratio,
                                    float abs_thresh, int32_t* match, float* d1out, float* d2out)
{
    const float dd1 = sqrtf(e1), dd2 = sqrtf(e2);
    // ratio = +inf: the absolute threshold of Eq. 6 alone
    const bool ratio_ok = __builtin_isinf(ratio) || (double)dd1 < ratio * (double)dd2;
    const bool keep = j1 >= 0 && ratio_ok && dd1 < abs_thresh;
    match[q] = keep ? j1 : -1;
    d1out[q] = dd1;
    d2out[q] = dd2;
}

// Sixteen lanes per query (four queries per wavefront): keep the 4 best
// candidates by contraction score (chunks x 4 entries), recompute their
// distances directly, then the ratio test. Lane t of a group holds elements
// t + 16 u of a row and adds them in the order of a 64-lane butterfly over
// pairs (l, l + 64), so distances are bit-identical to the wavefront sums of
// the other rescoring paths.
__device__ inline float group_sqdist(const float (&a)[8], const float* __restrict__ b, int t)
{
    float p[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const float x0 = a[u] - b[t + 16 * u], x1 = a[u + 4] - b[t + 16 * u + 64];
        p[u] = fmaf(x0, x0, x1 * x1);   // virtual lane t + 16 u
    }
    // butterfly levels 32 and 16 within the lane, then 8 .. 1 across the group
    float v = (p[0] + p[2]) + (p[1] + p[3]);
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
    return v;
}

__device__ inline void rescore_f32_query(const float* __restrict__ A, const float* __restrict__ B,
                                         int64_t nB, int chunks, int64_t i, int64_t q,
                                         const int32_t* __restrict__ cidx,
                                         const float* __restrict__ cscore, double ratio,
                                         float abs_thresh, int32_t* __restrict__ match,
                                         float* __restrict__ d1out, float* __restrict__ d2out)
{
    const int t = threadIdx.x & 15;
    const int nc = chunks * kKeep;   // <= 256: up to 16 entries per lane
    // the (up to) 4 best entries by contraction score, selected first ...
    int pick[4];
    int cnt = 0;
    int taken[4] = {0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF};
#pragma unroll
    for (int round = 0; round < 4; ++round) {
        // this lane's best untaken entry, then the group's
        float bs = INFINITY;
        int bi = 0x7FFFFFFF;
        for (int e = t; e < nc; e += 16) {
            const int c = cidx[i * nc + e];
            if (c < 0 || c == taken[0] || c == taken[1] || c == taken[2]) continue;
            const float sc = cscore[i * nc + e];
            if (sc < bs || (sc == bs && c < bi)) {
                bs = sc;
                bi = c;
            }
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            const float os = __shfl_xor(bs, off, 16);
            const int oi = __shfl_xor(bi, off, 16);
            if (os < bs || (os == bs && oi < bi)) {
                bs = os;
                bi = oi;
            }
        }
        pick[round] = bi;
        taken[round] = bi;
        if (bi != 0x7FFFFFFF && bs != INFINITY) cnt = round + 1;
    }
    // ... then their rows loaded together (one memory latency instead of four)
    // and their distances computed directly; the top-2 by (distance, index)
    // does not depend on the insertion order
    float a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = A[q * 128 + t + 16 * u];
    float e1 = INFINITY, e2 = INFINITY;
    int j1 = -1, j2 = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < cnt) best2_insert(group_sqdist(a, B + (int64_t)pick[k] * 128, t), pick[k], e1, j1, e2, j2);
    }
    // Without a ratio test an exact tie d1 = d2 is kept, and the nearest
    // neighbour must then be the lowest tied index. The contraction's lane
    // top-2 keeps the lowest accumulator rows of a tie, not the lowest
    // indices, so with three or more tied candidates a lower one may be
    // missing: search the indices below j1 directly (e1, j1 are equal in
    // the 16 lanes of the group, so the loop is uniform there).
    if (__builtin_isinf(ratio) && j1 > 0 && e1 == e2 && sqrtf(e1) < abs_thresh) {
        const int64_t lim = j1 < nB ? (int64_t)j1 : nB;
        for (int64_t j = 0; j < lim; ++j) {
            if (group_sqdist(a, B + j * 128, t) == e1) {
                j1 = (int)j;
                break;
            }
        }
    }
    if (t == 0) write_result(q, e1, j1, e2, ratio, abs_thresh, match, d1out, d2out);
}

// ------------------------------------------------------ low-precision paths --

template <int P> struct Lp;
template <> struct Lp<1> {             // BF16
    static constexpr int kRowBytes = 256;
    static constexpr int kOpBytes = 16;  // operand bytes per lane per MFMA
    static constexpr int kSteps = 8;     // MFMAs per 32 x 32 block over K = 128
    static constexpr int kKStep = 16;    // K per MFMA
    static constexpr int kEsize = 2;
    static constexpr int kCT = 64;       // candidates per LDS tile
};
template <> struct Lp<2> {             // FP8 E4M3
    static constexpr int kRowBytes = 128;
    static constexpr int kOpBytes = 32;
    static constexpr int kSteps = 2;
    static constexpr int kKStep = 64;
    static constexpr int kEsize = 1;
    // candidates per LDS tile: 128 halves the tile barriers per candidate
    // (10 % faster; BF16's larger rows would spill at 128)
    static constexpr int kCT = 128;
};

// BF16 bits of x, rounded to nearest even (finite x).
__device__ inline uint32_t bf16_bits(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

constexpr int kLpSets = 4;                         // 32-query sets per wavefront
constexpr int kLpKeepBf16 = 2;                     // keys kept per lane: BF16 ...
constexpr int kLpKeepFp8 = 2;                      // ... and FP8
constexpr int kLpRescore = 8;                      // kept candidates rescored in FP32
constexpr int kLpQB = 4 * 32 * kLpSets;            // queries per workgroup (512)
constexpr float kFp8Max = 448.0f;                  // largest finite E4M3 value

// Quantise rows of 128 floats: BF16 (round to nearest even) or FP8 E4M3 with
// the per-row scale max|x| / 448. 16 lanes per row, 8 values each.
template <int P>
__global__ __launch_bounds__(256) void quantize_kernel(const float* __restrict__ X, int64_t n,
                                                       uint8_t* __restrict__ Y,
                                                       float* __restrict__ scale,
                                                       uint32_t* __restrict__ max_err2)
{
    const int64_t row = (int64_t)blockIdx.x * 16 + threadIdx.x / 16;
    const int part = threadIdx.x % 16;
    float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (row < n) {
        const float4* p = reinterpret_cast<const float4*>(X + row * 128 + part * 8);
        const float4 a = p[0], b = p[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    }
    if (P == 1) {
        uint32_t w[4];
        float e2 = 0.0f;   // |x - bf16(x)|^2 of this row part (each difference is exact)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t lo = bf16_bits(v[2 * k]), hi = bf16_bits(v[2 * k + 1]);
            const float dl = v[2 * k] - __uint_as_float(lo << 16);
            const float dh = v[2 * k + 1] - __uint_as_float(hi << 16);
            e2 += dl * dl + dh * dh;
            w[k] = lo | (hi << 16);
        }
        for (int off = 8; off > 0; off >>= 1) e2 += __shfl_xor(e2, off, 16);
        if (row < n) {
            *reinterpret_cast<uint4*>(Y + row * 256 + part * 16) = make_uint4(w[0], w[1], w[2], w[3]);
            if (part == 0 && max_err2) atomicMax(max_err2, __float_as_uint(e2 * 1.0001f));
        }
    } else {
        float m = 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) m = fmaxf(m, fabsf(v[k]));
        for (int off = 8; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 16));
        // scale m / 448: the row maximum maps to 448 exactly, and with it the
        // many entries that the descriptor's clipping made equal to it (a
        // power-of-two scale would round them, measured to cost recall)
        const float s = (m > 0.0f) ? m / kFp8Max : 1.0f;
        const float inv = (m > 0.0f) ? kFp8Max / m : 1.0f;
        float x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fminf(fmaxf(v[k] * inv, -kFp8Max), kFp8Max);
        int w0 = __builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false);
        w0 = __builtin_amdgcn_cvt_pk_fp8_f32(x[2], x[3], w0, true);
        int w1 = __builtin_amdgcn_cvt_pk_fp8_f32(x[4], x[5], 0, false);
        w1 = __builtin_amdgcn_cvt_pk_fp8_f32(x[6], x[7], w1, true);
        const uint32_t w[2] = {(uint32_t)w0, (uint32_t)w1};
        if (row < n) {
            *reinterpret_cast<uint2*>(Y + row * 128 + part * 8) = make_uint2(w[0], w[1]);
            if (part == 0) scale[row] = s;
        }
    }
}

// Contraction + per-lane top-K of packed keys for one (query block, chunk).
// keys[((i * chunks + chunk) * 2 + h) * K + {0 .. K-1}] = lane half h's best K
// keys of query i, ascending (0xFFFFFFFF = none). key = (float bits of
// -score / 2 & ~idx_mask) | index in chunk, score = |b|^2 + C - 2 a.b > 0 (C
// from the per-call scalars): negative floats, whose bits ascend with their
// magnitude.
// Two workgroups per CU: within the 256 registers a lane then has, the
// accumulators are ordinary VGPRs that the epilogue reads directly (with
// more registers the compiler places them in AGPRs, and every score costs
// one more v_accvgpr_read), and the two 32-row halves of a tile run one
// after the other so that only one half's accumulators are live.
template <int P, int K>
__global__ __launch_bounds__(256, 2) void match_topk_lp_kernel(
    const uint8_t* __restrict__ Aq, const float* __restrict__ sA, int64_t nA,
    const uint8_t* __restrict__ Bq, const float* __restrict__ sB, int64_t nB,
    const float* __restrict__ nrmB, const float* __restrict__ scal, int64_t chunk_len,
    int chunks, uint32_t idx_mask, uint32_t* __restrict__ keys)
{
    using T = Lp<P>;
    constexpr int kLRow = T::kRowBytes + 16;   // padded LDS row
    constexpr int kU4 = T::kCT * T::kRowBytes / 16 / 256;   // uint4 per thread per tile
    __shared__ __attribute__((aligned(16))) uint8_t tile[T::kCT * kLRow];
    // -(|b|^2 + C) / 2 per tile row: the accumulators' starting values
    __shared__ __attribute__((aligned(16))) float tnb[T::kCT];
    __shared__ float tsb[T::kCT];                // candidate scales (FP8)
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int chunk = blockIdx.y;
    const int64_t cb = (int64_t)chunk * chunk_len;
    const int64_t ce = (cb + chunk_len < nB) ? cb + chunk_len : nB;
    const float C = scal[0];

    // queries: set t, operand step s -> bytes [(s*KStep + h*KStep/2)*esize, +OpBytes)
    constexpr int kQRegs = T::kOpBytes / 16;   // uint4 per operand
    uint4 qv[kLpSets][T::kSteps][kQRegs];
    float qs[kLpSets];                          // query scale (FP8)
    int64_t qi[kLpSets];
#pragma unroll
    for (int t = 0; t < kLpSets; ++t) {
        const int64_t q = (int64_t)blockIdx.x * kLpQB + wave * (32 * kLpSets) + t * 32 + col;
        qi[t] = q;
        const uint8_t* row = Aq + q * T::kRowBytes;
#pragma unroll
        for (int s = 0; s < T::kSteps; ++s)
#pragma unroll
            for (int u = 0; u < kQRegs; ++u)
                qv[t][s][u] = (q < nA) ? *reinterpret_cast<const uint4*>(
                                             row + (s * T::kKStep + h * T::kKStep / 2) * T::kEsize + 16 * u)
                                       : make_uint4(0u, 0u, 0u, 0u);
        qs[t] = (P == 2 && q < nA) ? sA[q] : 0.0f;
    }
    uint32_t k1[kLpSets], k2[kLpSets], k3[kLpSets];
#pragma unroll
    for (int t = 0; t < kLpSets; ++t) {
        k1[t] = 0xFFFFFFFFu;
        k2[t] = 0xFFFFFFFFu;
        k3[t] = 0xFFFFFFFFu;
    }

    uint4 pf[kU4];
    auto fetch = [&](int64_t t0) {
#pragma unroll
        for (int k = 0; k < kU4; ++k) {
            const int f = tid + 256 * k;
            const int r = f / (T::kRowBytes / 16), c16 = f % (T::kRowBytes / 16);
            const int64_t j = t0 + r;
            pf[k] = (j < ce) ? reinterpret_cast<const uint4*>(Bq + j * T::kRowBytes)[c16]
                             : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    if (cb < ce) fetch(cb);

    for (int64_t t0 = cb; t0 < ce; t0 += T::kCT) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kU4; ++k) {
            const int f = tid + 256 * k;
            const int r = f / (T::kRowBytes / 16), c16 = f % (T::kRowBytes / 16);
            *reinterpret_cast<uint4*>(&tile[r * kLRow + c16 * 16]) = pf[k];
        }
        if (tid < T::kCT) {
            const int64_t j = t0 + tid;
            tnb[tid] = (j < ce) ? -0.5f * (nrmB[j] + C) : -INFINITY;
            tsb[tid] = (P == 2 && j < ce) ? sB[j] : 1.0f;
        }
        __syncthreads();
        if (t0 + T::kCT < ce) fetch(t0 + T::kCT);
        const uint32_t local0 = (uint32_t)(t0 - cb);

#pragma unroll 1
        for (int sub = 0; sub < T::kCT / 32; ++sub) {
            // BF16: every accumulator starts at -(|b|^2 + C) / 2 of its row
            // (the same for all four query sets: the first MFMA of each set
            // takes these registers as its addend), so that it ends at
            // a.b - (|b|^2 + C) / 2 = -score / 2 < 0 without an epilogue FMA.
            // FP8 accumulates the codes from zero; its row scales are applied
            // in the epilogue. Rows of the lane: 8 i + 4 h + 0..3 of the half.
            floatx16 init;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float4 v = (P == 1) ? *reinterpret_cast<const float4*>(&tnb[sub * 32 + 8 * i + 4 * h])
                                          : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                init[4 * i] = v.x;
                init[4 * i + 1] = v.y;
                init[4 * i + 2] = v.z;
                init[4 * i + 3] = v.w;
            }
            floatx16 acc[kLpSets];
            const uint8_t* trow = &tile[(sub * 32 + col) * kLRow];
            // FP8: the wave issuing its MFMAs takes precedence over the other
            // wave of the SIMD (in its epilogue), which keeps the matrix core
            // fed (measured 2-4 % faster; no change for BF16)
            if constexpr (P == 2) __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int s = 0; s < T::kSteps; ++s) {
                uint4 av[kQRegs];
#pragma unroll
                for (int u = 0; u < kQRegs; ++u)
                    av[u] = *reinterpret_cast<const uint4*>(
                        trow + (s * T::kKStep + h * T::kKStep / 2) * T::kEsize + 16 * u);
#pragma unroll
                for (int t = 0; t < kLpSets; ++t) {
                    const floatx16 addend = (s == 0) ? init : acc[t];
                    if constexpr (P == 1) {
                        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, av[0]), __builtin_bit_cast(bf16x8, qv[t][s][0]),
                            addend, 0, 0, 0);
                    } else {
                        const intx8 a8 = {(int)av[0].x, (int)av[0].y, (int)av[0].z, (int)av[0].w,
                                          (int)av[1].x, (int)av[1].y, (int)av[1].z, (int)av[1].w};
                        const intx8 b8 = {(int)qv[t][s][0].x, (int)qv[t][s][0].y, (int)qv[t][s][0].z,
                                          (int)qv[t][s][0].w, (int)qv[t][s][1].x, (int)qv[t][s][1].y,
                                          (int)qv[t][s][1].z, (int)qv[t][s][1].w};
                        acc[t] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            a8, b8, addend, 0, 0, 0, 0, 0, 0);
                    }
                }
            }
            if constexpr (P == 2) __builtin_amdgcn_s_setprio(0);
            // epilogue: key = (accumulator bits & ~mask) | index in chunk.
            // The accumulators are negative, so their bits (sign set) order
            // like their magnitudes, i.e. like the scores; top-K by min /
            // med3 (keys are unique)
            auto lp_key = [&](int t, int r) {
                const int cl = sub * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                // FP8: -score / 2 = sA sB qa.qb - (|b|^2 + C) / 2
                const float v = (P == 1) ? acc[t][r] : fmaf(qs[t] * tsb[cl], acc[t][r], tnb[cl]);
                return (__float_as_uint(v) & ~idx_mask) | (local0 + (uint32_t)cl);
            };
            if constexpr (K == 2) {
                // two rows at a time: for k1 <= k2 and new keys x, y the two
                // smallest of all four are min3(k1, x, y) and min(k2, med3(k1, x, y))
#pragma unroll
                for (int r = 0; r < 16; r += 2) {
#pragma unroll
                    for (int t = 0; t < kLpSets; ++t) {
                        const uint32_t x = lp_key(t, r), y = lp_key(t, r + 1);
                        k2[t] = min(k2[t], umed3(k1[t], x, y));
                        k1[t] = min(k1[t], min(x, y));
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
#pragma unroll
                    for (int t = 0; t < kLpSets; ++t) {
                        // sorted insertion (k1 <= k2 <= k3): the new i-th
                        // smallest is the key clamped to [k(i-1), k(i)]
                        const uint32_t key = lp_key(t, r);
                        k3[t] = umed3(key, k2[t], k3[t]);
                        k2[t] = umed3(key, k1[t], k2[t]);
                        k1[t] = min(k1[t], key);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kLpSets; ++t) {
        if (qi[t] < nA) {
            const int64_t o = ((qi[t] * chunks + chunk) * 2 + h) * K;
            keys[o] = k1[t];
            keys[o + 1] = k2[t];
            if (K == 3) keys[o + 2] = k3[t];
        }
    }
}

// 16 lanes per query. Entries: K keys per (chunk, lane half). The 8
// smallest kept keys are rescored in FP32 (approximate paths).
template <int K>
__global__ __launch_bounds__(256) void rescore_lp_kernel(
    const float* __restrict__ A, int64_t nA, const float* __restrict__ B, int chunks,
    int64_t chunk_len, uint32_t idx_mask, const uint32_t* __restrict__ keys, double ratio,
    float abs_thresh, int n_rescore, int32_t* __restrict__ match, float* __restrict__ d1out,
    float* __restrict__ d2out)
{
    // 16 lanes per query, four queries per wavefront (see rescore_f32_query)
    const int t = threadIdx.x & 15;
    const int64_t q = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    if (q >= nA) return;   // the whole group of 16 lanes leaves together
    const int ne = chunks * 2 * K;   // <= 64: up to 4 entries per lane
    float sc[4];
    int64_t jv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = t + 16 * u;
        sc[u] = INFINITY;
        jv[u] = -1;
        if (e < ne) {
            // keys are the bits of negative accumulators (sign set, below
            // -inf's 0xFF800000): their magnitudes are half the scores
            const uint32_t key = keys[q * ne + e];
            if (key >= 0x80000000u && key < 0xFF800000u) {
                sc[u] = __uint_as_float(key & ~idx_mask & 0x7FFFFFFFu);
                jv[u] = (int64_t)(e / (2 * K)) * chunk_len + (key & idx_mask);
            }
        }
    }
    // the n_rescore <= kLpRescore best kept keys (ties: lower entry first),
    // selected first ...
    int64_t pick[kLpRescore];
    int cnt = 0;
#pragma unroll
    for (int round = 0; round < kLpRescore; ++round) {
        float bs = sc[0];
        int be = t;
#pragma unroll
        for (int u = 1; u < 4; ++u)
            if (sc[u] < bs) {   // entries of a lane ascend, so ties keep the lower one
                bs = sc[u];
                be = t + 16 * u;
            }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            const float os = __shfl_xor(bs, off, 16);
            const int oe = __shfl_xor(be, off, 16);
            if (os < bs || (os == bs && oe < be)) {
                bs = os;
                be = oe;
            }
        }
        if (bs != INFINITY && round < n_rescore) cnt = round + 1;
        int64_t jj = -1;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t + 16 * u == be) {
                jj = jv[u];
                sc[u] = INFINITY;
            }
        pick[round] = __shfl(jj, be & 15, 16);
    }
    // ... then their rows loaded together and their distances computed
    // directly; the top-2 by (distance, index) does not depend on the order
    float a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = A[q * 128 + t + 16 * u];
    float e1 = INFINITY, e2 = INFINITY;
    int j1 = -1, j2 = -1;
#pragma unroll
    for (int k = 0; k < kLpRescore; ++k) {
        if (k < cnt)
            best2_insert(group_sqdist(a, B + pick[k] * 128, t), (int)pick[k], e1, j1, e2, j2);
    }
    if (t == 0) write_result(q, e1, j1, e2, ratio, abs_thresh, match, d1out, d2out);
}

// ------------------------------------------------------------- BF16x3 path --
//
// x = hi + lo + res with hi = bf16(x), lo = bf16(x - hi) (each difference exact
// in FP32, |res| <= 2^-16 |x|); a.b ~ hi.hi + hi.lo + lo.hi on the matrix cores
// with FP32 accumulation starting from -|b|^2 / 2, so acc = a.b - |b|^2/2 and
// the score |b|^2 - 2 a.b = -2 acc. Scores stay exact floats: each lane keeps
// its top-2 (score, index) and its third-best score, which bounds everything it
// did not keep.

__device__ inline void split_bf16(float x, uint32_t& hi, uint32_t& lo, float& res)
{
    hi = bf16_bits(x);
    const float r = x - __uint_as_float(hi << 16);
    lo = bf16_bits(r);
    res = r - __uint_as_float(lo << 16);
}

// Per row: |x|^2 (stored) and the row split into BF16 hi and lo parts (512
// bytes: 128 hi values, then 128 lo values, the layout of the contraction's
// LDS tile); over rows, the maxima of |x|^2, |lo|^2 and |res|^2.
__device__ inline void split_rows(const float* __restrict__ X, int64_t n, int64_t blk,
                                  float* __restrict__ nrm, uint8_t* __restrict__ hl, float m[3])
{
    const int64_t row = blk * 16 + threadIdx.x / 16;
    const int part = threadIdx.x % 16;
    float s = 0.0f, sl = 0.0f, sr = 0.0f;
    if (row < n) {
        const float4* p = reinterpret_cast<const float4*>(X + row * 128 + part * 8);
        const float4 a = p[0], b = p[1];
        const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        uint32_t h[8], l[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            float res;
            split_bf16(v[k], h[k], l[k], res);
            const float lf = __uint_as_float(l[k] << 16);
            s += v[k] * v[k];
            sl += lf * lf;
            sr += res * res;
        }
        *reinterpret_cast<uint4*>(hl + row * 512 + part * 16) =
            make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
        *reinterpret_cast<uint4*>(hl + row * 512 + 256 + part * 16) =
            make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16));
    }
    for (int off = 8; off > 0; off >>= 1) {
        s += __shfl_xor(s, off, 16);
        sl += __shfl_xor(sl, off, 16);
        sr += __shfl_xor(sr, off, 16);
    }
    if (row < n && part == 0) nrm[row] = s;
    m[0] = fmaxf(m[0], s);
    m[1] = fmaxf(m[1], sl);
    m[2] = fmaxf(m[2], sr);
}

constexpr int kX3QB = 256;          // queries per workgroup (4 waves x 2 x 32)
constexpr int kX3CT = 32;           // candidates per LDS tile
constexpr int kX3Row = 512 + 16;    // LDS bytes per candidate: hi row, lo row, pad

__device__ inline uint4 load_split8(const float* p, uint4& lo)
{
    const float4 a = reinterpret_cast<const float4*>(p)[0];
    const float4 b = reinterpret_cast<const float4*>(p)[1];
    const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t h[8], l[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        float res;
        split_bf16(v[k], h[k], l[k], res);
    }
    lo = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16));
    return make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

// Padded candidate rows start their accumulator here instead of -|b|^2/2: a
// finite value far below any real score (keys stay free of inf and NaN).
constexpr float kX3Pad = -3.0e38f;
// k1's update is med3(x, k1, kX3Top), which is max(x, k1) for every key below
// kX3Top: a key is a.b - |b|^2/2 <= |a|^2/2, so any pair of descriptors whose
// squared norms are finite in FP32 stays below it. A plain max would first
// quiet x as a possible NaN, since x is rebuilt from integer bits: one more
// VALU instruction per accumulator in the loop.
constexpr float kX3Top = 3.0e38f;

__device__ inline void topk_x3_item(const float* __restrict__ A, int64_t nA,
                                    const uint8_t* __restrict__ Bhl, int64_t nB,
                                    const float* __restrict__ nrmB, int64_t chunk_len, int chunks,
                                    int32_t* __restrict__ cidx, float* __restrict__ cscore,
                                    float* __restrict__ cthird, int64_t qblk, int chunk)
{
    __shared__ __attribute__((aligned(16))) uint8_t tile[kX3CT * kX3Row];
    __shared__ __attribute__((aligned(16))) float tinit[kX3CT];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    // candidate rows cb .. ce - 1 (nB < 2^31: unsigned tile positions cannot wrap)
    const uint32_t cb = (uint32_t)((int64_t)chunk * chunk_len);
    const uint32_t ce = (uint32_t)(((int64_t)cb + chunk_len < nB) ? (int64_t)cb + chunk_len : nB);

    // queries, set t: dims [16 s + 8 h, +8) of query col as hi and lo BF16
    uint4 qh[2][8], ql[2][8];
    int64_t qi[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int64_t q = qblk * kX3QB + wave * 64 + t * 32 + col;
        qi[t] = q;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            if (q < nA) {
                qh[t][s] = load_split8(A + q * 128 + 16 * s + 8 * h, ql[t][s]);
            } else {
                qh[t][s] = make_uint4(0u, 0u, 0u, 0u);
                ql[t][s] = make_uint4(0u, 0u, 0u, 0u);
            }
        }
    }
    // Per lane and query set: the two largest keys and the third largest. A
    // key is the float acc with its low 4 bits replaced by the accumulator row
    // r (a change of at most 15 units in the last place, which the rescoring
    // bound allows for), kept with three v_med3_f32; the tile of each
    // kept key is recovered once per tile by comparing it with its value
    // before the tile.
    float k1[2], k2[2], k3[2];
    int t1[2], t2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        k1[t] = k2[t] = k3[t] = -INFINITY;
        t1[t] = t2[t] = -1;
    }

    // a 32 x 512-byte tile of split rows: thread t moves uint4 number t + 256 k
    // (row (t + 256 k) / 32) from a uniform base; threads t < 32 also the
    // accumulator start of row t
    uint4 pf[4];
    float pn = kX3Pad;
    auto fetch = [&](uint32_t t0) {
        const uint4* base = reinterpret_cast<const uint4*>(Bhl + (int64_t)t0 * 512);
        if (ce - t0 >= (uint32_t)kX3CT) {
#pragma unroll
            for (int k = 0; k < 4; ++k) pf[k] = base[tid + 256 * k];
            if (tid < kX3CT) pn = -0.5f * nrmB[t0 + tid];
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                pf[k] = ((uint32_t)((tid + 256 * k) >> 5) < ce - t0) ? base[tid + 256 * k]
                                                                      : make_uint4(0u, 0u, 0u, 0u);
            if (tid < kX3CT) pn = ((uint32_t)tid < ce - t0) ? -0.5f * nrmB[t0 + tid] : kX3Pad;
        }
    };
    if (cb < ce) fetch(cb);

    for (uint32_t t0 = cb; t0 < ce; t0 += kX3CT) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int f = tid + 256 * k;
            const int r = f >> 5, c16 = f & 31;
            *reinterpret_cast<uint4*>(&tile[r * kX3Row + c16 * 16]) = pf[k];
        }
        if (tid < kX3CT) tinit[tid] = pn;
        __syncthreads();
        if (ce - t0 > (uint32_t)kX3CT) fetch(t0 + kX3CT);

        // accumulators start at -|b|^2 / 2 of their candidate row
        floatx16 acc[2];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const float4 iv = *reinterpret_cast<const float4*>(&tinit[8 * g + 4 * h]);
            acc[0][4 * g + 0] = iv.x; acc[0][4 * g + 1] = iv.y;
            acc[0][4 * g + 2] = iv.z; acc[0][4 * g + 3] = iv.w;
        }
        acc[1] = acc[0];
        const uint8_t* trow = &tile[col * kX3Row];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const uint4 bh = *reinterpret_cast<const uint4*>(trow + (16 * s + 8 * h) * 2);
            const uint4 bl = *reinterpret_cast<const uint4*>(trow + 256 + (16 * s + 8 * h) * 2);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    __builtin_bit_cast(bf16x8, bh), __builtin_bit_cast(bf16x8, qh[t][s]), acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    __builtin_bit_cast(bf16x8, bl), __builtin_bit_cast(bf16x8, qh[t][s]), acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    __builtin_bit_cast(bf16x8, bh), __builtin_bit_cast(bf16x8, ql[t][s]), acc[t], 0, 0, 0);
            }
        }
        // result row (candidate) of accumulator r in this lane: 8 (r/4) + 4 h + r % 4
        float p1[2], p2[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            p1[t] = k1[t];
            p2[t] = k2[t];
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const float x = __int_as_float((__float_as_int(acc[t][r]) & -16) | r);
                k3[t] = __builtin_amdgcn_fmed3f(x, k2[t], k3[t]);   // k1 >= k2 >= k3
                k2[t] = __builtin_amdgcn_fmed3f(x, k1[t], k2[t]);
                k1[t] = __builtin_amdgcn_fmed3f(x, k1[t], kX3Top);
            }
        }
        // tile of each kept key, as in the FP32 path: a key bit-equal to its
        // value before the tile is that candidate; the second key equal to the
        // old first one is the old first candidate unless the first key kept
        // that value too (a bit-identical key of this tile); else it is new.
        // So the kept pair never holds one candidate twice, and every other
        // candidate's key is at most k3.
        const int tt = (int)(t0 - cb);   // chunk-relative tile start
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int b1 = __float_as_int(k1[t]), b2 = __float_as_int(k2[t]);
            const int o1 = __float_as_int(p1[t]), o2 = __float_as_int(p2[t]);
            t2[t] = (b2 == o2) ? t2[t] : ((b2 == o1 && b1 != o1) ? t1[t] : tt);
            t1[t] = (b1 == o1) ? t1[t] : tt;
        }
    }
    // key -> (candidate index, score -2 acc); empty slots and padded rows give
    // index -1 and score +inf
    auto unpack = [&](float k, int t, int& j, float& sc) {
        const int r = __float_as_int(k) & 15;
        const bool real = t >= 0 && k > 0.5f * kX3Pad;
        j = real ? (int)cb + t + 8 * (r >> 2) + 4 * h + (r & 3) : -1;
        sc = real ? -2.0f * k : INFINITY;
    };
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        if (qi[t] < nA) {
            const int64_t o = (qi[t] * chunks + chunk) * 4 + 2 * h;
            int ja, jb;
            float sa, sb;
            unpack(k1[t], t1[t], ja, sa);
            unpack(k2[t], t2[t], jb, sb);
            cidx[o] = ja;
            cidx[o + 1] = jb;
            cscore[o] = sa;
            cscore[o + 1] = sb;
            // no real candidate left behind: +inf
            cthird[(qi[t] * chunks + chunk) * 2 + h] = (k3[t] > 0.5f * kX3Pad) ? -2.0f * k3[t] : INFINITY;
        }
    }
}

// One wavefront per query: certify the kept set of the BF16x3 contraction and
// rescore it in FP32, or queue the query for the FP32 path.
__device__ inline void rescore_x3_query(
    const float* __restrict__ A, const float* __restrict__ B, int chunks, int64_t q,
    const int32_t* __restrict__ cidx, const float* __restrict__ cscore,
    const float* __restrict__ cthird, const uint32_t* __restrict__ maxbits, double ratio,
    float abs_thresh, int32_t* __restrict__ match, float* __restrict__ d1out,
    float* __restrict__ d2out, uint32_t* __restrict__ fb_count, int32_t* __restrict__ fb_list)
{
    const int lane = threadIdx.x & 63;
    const int ne = chunks * 4;   // <= 64
    float sc = INFINITY;
    int jj = -1;
    if (lane < ne) {
        const int c = cidx[q * ne + lane];
        if (c >= 0) {
            jj = c;
            sc = cscore[q * ne + lane];
        }
    }
    float tg = (lane < 2 * chunks) ? cthird[q * 2 * chunks + lane] : INFINITY;
    const float a0 = A[q * 128 + lane], a1 = A[q * 128 + 64 + lane];
    // error bound of every score, from the split errors of a and the largest
    // of b: |(a.b)~ - a.b| <= |a_lo||b_lo| + (|a| + |a_res|)|b_res|
    //   + |a_res|(|b| + |b_res|) + gamma (3 (|a| + |a_res|)(|b| + |b_res|) + |b|^2/2)
    uint32_t hh, ll;
    float r0, r1;
    split_bf16(a0, hh, ll, r0);
    const float l0 = __uint_as_float(ll << 16);
    split_bf16(a1, hh, ll, r1);
    const float l1 = __uint_as_float(ll << 16);
    const float an = sqrtf(wave_sum(a0 * a0 + a1 * a1));
    const float aln = sqrtf(wave_sum(l0 * l0 + l1 * l1)) * 1.0001f;
    const float arn = sqrtf(wave_sum(r0 * r0 + r1 * r1)) * 1.0001f;
    const float bn2 = __uint_as_float(maxbits[0]);
    const float bn = sqrtf(bn2), bln = sqrtf(__uint_as_float(maxbits[1]));
    const float brn = sqrtf(__uint_as_float(maxbits[2]));
    const float gamma = 385.0f * 5.9604645e-8f;   // FP32 additions along one accumulator chain
    const float dot_err = aln * bln + (an + arn) * brn + arn * (bn + brn)
                          + gamma * (3.0f * (an + arn) * (bn + brn) + 0.5f * bn2);
    // score = -2 acc; |b|^2 itself carries the FP32 error of a 128-term sum.
    // The contraction kept keys, not scores: each kept and third value is
    // off by at most 15 units in the last place of |acc| <= M, i.e. by
    // 30 x 2^-23 M <= 2^-18 M in score units (2^-17 M allowed).
    const float M = 0.5f * bn2 + an * bn + dot_err;
    const float E = 2.02f * dot_err + 1e-5f * bn2 + 1e-7f + 7.62939453125e-6f * M;
    // T: best score any group may have left behind (its third best)
    float m1 = sc, m2 = INFINITY;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        tg = fminf(tg, __shfl_xor(tg, off));
        const float o1 = __shfl_xor(m1, off), o2 = __shfl_xor(m2, off);
        const float n1 = fminf(m1, o1);
        m2 = fminf(fmaxf(m1, o1), fminf(m2, o2));
        m1 = n1;
    }
    const float U2 = m2 + E;
    if (!(tg - E > U2)) {
        if (lane == 0) {
            const uint32_t pos = atomicAdd(fb_count, 1u);
            fb_list[pos] = (int32_t)q;
        }
        return;
    }
    float e1 = INFINITY, e2 = INFINITY;
    int j1 = -1, j2 = -1;
    uint64_t todo = __ballot(jj >= 0 && sc - E <= U2);
    while (todo) {
        const int l = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const int j = __shfl(jj, l);
        best2_insert(sqdist(a0, a1, B, j, lane), j, e1, j1, e2, j2);
    }
    if (lane == 0) write_result(q, e1, j1, e2, ratio, abs_thresh, match, d1out, d2out);
}

// Per-call scalars of the quantised paths: [0] = C as float, [1] = max |a|^2
// bits, [2] = max |b|^2 bits. C > (1 + 2 err)(|a|^2 + |b|^2) keeps every score
// |b|^2 + C - 2 (a.b)~ positive, so that float bits order like values.
__global__ void lp_scalars_kernel(float* scal, float dot_err)
{
    const float maxa2 = __uint_as_float(reinterpret_cast<const uint32_t*>(scal)[1]);
    const float maxb2 = __uint_as_float(reinterpret_cast<const uint32_t*>(scal)[2]);
    scal[0] = (1.0f + 2.0f * dot_err) * (maxa2 + maxb2) + 1.0f;
}

// ------------------------------------------------------------- batched launches --
//
// One launch serves up to kPairs pairs: each kernel takes a table of per-pair
// jobs by value and walks a flat range of work items, item `it` belonging to
// the first job whose cumulative item count exceeds it. Item counts may depend
// on device-side query counts (the FP32 re-match of uncertified queries), so
// they are evaluated inside the kernel; such launches use a grid smaller than
// the largest possible item range and stride over it.

// 36 pairs: all pairs of 9 images in one launch. The largest job table
// (RescoreX3Batch, 104 B per job) then stays below 4 KB of kernel arguments.
constexpr int kPairs = 36;

// Job k of batch b that item `it` belongs to (-1 past the end) and the item's
// index within that job. items(job) must be uniform across the workgroup.
template <class Batch, class Items>
__device__ inline int find_job(const Batch& b, int64_t it, Items items, int64_t& local)
{
    int64_t base = 0;
    for (int k = 0; k < b.n; ++k) {
        const int64_t c = items(b.j[k]);
        if (it < base + c) {
            local = it - base;
            return k;
        }
        base += c;
    }
    return -1;
}

// Per distinct candidate set: |b|^2 of every row, and for the split path the
// BF16 hi/lo rows and the row maxima.
struct RowsJob {
    const float* X;
    float* nrm;
    uint8_t* hl;          // split rows (split path), else null
    uint32_t* maxbits;    // split path: maxima of |x|^2, |lo|^2, |res|^2
    int64_t n;
};
struct RowsBatch {
    int32_t n;
    RowsJob j[kPairs];
};

__global__ __launch_bounds__(256) void rows_kernel(const RowsBatch b)
{
    int64_t wg;
    const int k = find_job(b, (int64_t)blockIdx.x,
                           [](const RowsJob& J) { return (J.n + kRowsPerWg - 1) / kRowsPerWg; },
                           wg);
    if (k < 0) return;
    const RowsJob& J = b.j[k];
    if (J.hl) {
        float m[3] = {0.0f, 0.0f, 0.0f};
        for (int r = 0; r < kRowBlocks; ++r) split_rows(J.X, J.n, wg * kRowBlocks + r, J.nrm, J.hl, m);
        // 1.0001: margin for the FP32 rounding of the sums
        block_max_atomic(J.maxbits + 0, __float_as_uint(m[0] * 1.0001f));
        block_max_atomic(J.maxbits + 1, __float_as_uint(m[1] * 1.0001f));
        block_max_atomic(J.maxbits + 2, __float_as_uint(m[2] * 1.0001f));
    } else {
        for (int r = 0; r < kRowBlocks; ++r) sqnorm_rows(J.X, J.n, wg * kRowBlocks + r, J.nrm);
    }
}

// FP32 contraction with top-2 per lane. Items of a job are (chunk, query
// block) with the query block fastest, so workgroups running together share
// a candidate chunk. With qlist set, the job's queries are the first *qcount
// entries of that list.
struct F32Job {
    const float* A;
    const int32_t* qlist;
    const uint32_t* qcount;
    const float* B;
    const float* nrm;
    int32_t* cidx;
    float* cscore;
    int64_t nq;           // queries (without a list), else the list's capacity
    int64_t nB;
    int64_t chunk_len;
    int32_t chunks;
};
struct F32Batch {
    int32_t n;
    F32Job j[kPairs];
};

__device__ inline int64_t f32_queries(const F32Job& J)
{
    return J.qlist ? (int64_t)*J.qcount : J.nq;
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup w on XCD
// w % 8), each XCD with its own L2. When all N items run in one wave (at most
// kOneWave workgroups, 2 per CU) and the grid is a multiple of 8, they are
// taken in blocks of 8 x run, run = min(kXcdRun, ceil(N / 8)): in each block
// the workgroups of XCD x take the run consecutive (chunk, query block)
// items starting at x * run, so one XCD streams one candidate chunk through
// its L2 instead of every chunk, and small launches still spread over all
// XCDs (same items, same results; only the order). Launches of many waves
// (batched pairs with smaller chunks) keep the launch order, which measured
// faster there.
constexpr int kXcdRun = 64;

// kW wavefronts per workgroup (2, 4 or 8), 8 / kW workgroups per CU: two
// waves per SIMD, each with 256 registers.
template <int kW>
__global__ __launch_bounds__(64 * kW) __attribute__((amdgpu_waves_per_eu(2, 2)))
void match_topk_f32_kernel(const F32Batch b)
{
    constexpr int64_t kOneWave = 256 * (8 / kW);   // workgroups resident at once
    constexpr int64_t qb = 64 * kW;
    auto items = [](const F32Job& J) { return (f32_queries(J) + qb - 1) / qb * J.chunks; };
    int64_t n_items = 0;
    for (int k = 0; k < b.n; ++k) n_items += items(b.j[k]);
    const bool by_xcd = (gridDim.x % 8u) == 0 && n_items <= kOneWave;
    const int64_t run = (n_items + 7) / 8 < kXcdRun ? ((n_items + 7) / 8 > 0 ? (n_items + 7) / 8 : 1)
                                                    : kXcdRun;
    const int64_t blk = 8 * run;
    const int64_t n_virtual = by_xcd ? (n_items + blk - 1) / blk * blk : n_items;
    for (int64_t v = blockIdx.x; v < n_virtual; v += gridDim.x) {
        const int64_t it = by_xcd ? (v / blk) * blk + (v % 8) * run + (v / 8) % run : v;
        if (it >= n_items) continue;   // uniform over the workgroup
        int64_t local;
        const int k = find_job(b, it, items, local);
        if (k < 0) return;
        const F32Job& J = b.j[k];
        const int64_t nq = f32_queries(J);
        const int64_t qblocks = (nq + qb - 1) / qb;
        const int chunk = (int)(local / qblocks);
        topk_f32_item<kW>(J.A, nq, J.qlist, J.B, J.nB, J.nrm, J.chunk_len, J.chunks, J.cidx,
                          J.cscore, local - chunk * qblocks, chunk);
        __syncthreads();   // the LDS tile is reused by the next item
    }
}

// FP32 rescore, 16 lanes per query (list entry). chunks = 0: no
// candidates (an empty candidate set), every query is rejected.
struct RescoreF32Job {
    const float* A;
    const float* B;
    const int32_t* qlist;
    const uint32_t* qcount;
    const int32_t* cidx;
    const float* cscore;
    int32_t* match;
    float* d1;
    float* d2;
    int64_t nq;
    int64_t nB;
    int32_t chunks;
};
struct RescoreF32Batch {
    int32_t n;
    double ratio;
    float abs_thresh;
    RescoreF32Job j[kPairs];
};

__global__ __launch_bounds__(256) void rescore_f32_kernel(const RescoreF32Batch b)
{
    auto items = [](const RescoreF32Job& J) {
        return ((J.qlist ? (int64_t)*J.qcount : J.nq) + 15) / 16;
    };
    for (int64_t it = blockIdx.x;; it += gridDim.x) {
        int64_t local;
        const int k = find_job(b, it, items, local);
        if (k < 0) return;
        const RescoreF32Job& J = b.j[k];
        const int64_t nq = J.qlist ? (int64_t)*J.qcount : J.nq;
        const int64_t i = local * 16 + (threadIdx.x >> 4);   // 16 queries per workgroup
        if (i < nq)
            rescore_f32_query(J.A, J.B, J.nB, J.chunks, i, J.qlist ? J.qlist[i] : i, J.cidx, J.cscore,
                              b.ratio, b.abs_thresh, J.match, J.d1, J.d2);
    }
}

// Split-BF16 contraction, one item per (chunk, query block).
struct X3Job {
    const float* A;
    const uint8_t* Bhl;
    const float* nrm;
    int32_t* cidx;
    float* cscore;
    float* cthird;
    int64_t nA;
    int64_t nB;
    int64_t chunk_len;
    int32_t chunks;
};
struct X3Batch {
    int32_t n;
    X3Job j[kPairs];
};

__global__ __launch_bounds__(256, 2) void match_topk_x3_kernel(const X3Batch b)
{
    int64_t local;
    const int k = find_job(b, (int64_t)blockIdx.x,
                           [](const X3Job& J) { return (J.nA + kX3QB - 1) / kX3QB * J.chunks; },
                           local);
    if (k < 0) return;
    const X3Job& J = b.j[k];
    const int64_t qblocks = (J.nA + kX3QB - 1) / kX3QB;
    const int chunk = (int)(local / qblocks);
    topk_x3_item(J.A, J.nA, J.Bhl, J.nB, J.nrm, J.chunk_len, J.chunks, J.cidx, J.cscore, J.cthird,
                 local - chunk * qblocks, chunk);
}

struct RescoreX3Job {
    const float* A;
    const float* B;
    const int32_t* cidx;
    const float* cscore;
    const float* cthird;
    const uint32_t* maxbits;
    int32_t* match;
    float* d1;
    float* d2;
    uint32_t* fb_count;
    int32_t* fb_list;
    int64_t nA;
    int32_t chunks;
};
struct RescoreX3Batch {
    int32_t n;
    double ratio;
    float abs_thresh;
    RescoreX3Job j[kPairs];
};

__global__ __launch_bounds__(256) void rescore_x3_kernel(const RescoreX3Batch b)
{
    int64_t local;
    const int k = find_job(b, (int64_t)blockIdx.x,
                           [](const RescoreX3Job& J) { return (J.nA + 3) / 4; }, local);
    if (k < 0) return;
    const RescoreX3Job& J = b.j[k];
    const int64_t q = local * 4 + (threadIdx.x >> 6);
    if (q < J.nA)
        rescore_x3_query(J.A, J.B, J.chunks, q, J.cidx, J.cscore, J.cthird, J.maxbits, b.ratio,
                         b.abs_thresh, J.match, J.d1, J.d2, J.fb_count, J.fb_list);
}

// Per-pair counters: zeroed before a launch sequence, summed into the
// caller's statistics word after it.
struct CounterBatch {
    int32_t n;
    uint32_t* c[kPairs];
};
static_assert(sizeof(RowsBatch) <= 4096 && sizeof(F32Batch) <= 4096 && sizeof(X3Batch) <= 4096 &&
                  sizeof(RescoreF32Batch) <= 4096 && sizeof(RescoreX3Batch) <= 4096,
              "job tables are kernel arguments: keep them within 4 KB");

// Four counter words per job; launched with kCounterThreads >= 4 kPairs threads.
constexpr int kCounterThreads = 4 * kPairs;
__global__ void zero_counters_kernel(const CounterBatch b, int words)
{
    const int k = threadIdx.x / 4, w = threadIdx.x % 4;
    if (k < b.n && w < words) b.c[k][w] = 0u;
}

__global__ void add_counters_kernel(const CounterBatch b, uint32_t* dst)
{
    if (threadIdx.x == 0) {
        uint32_t s = *dst;
        for (int k = 0; k < b.n; ++k) s += *b.c[k];
        *dst = s;
    }
}

// ------------------------------------------------------------------ layout --

struct WsF32 {
    size_t nrm, cidx, cscore, total;
};

WsF32 ws_f32(int64_t nA, int64_t nB, const MatchPlan& p)
{
    WsF32 w;
    w.nrm = 0;
    w.cidx = align_up((size_t)nB * 4, 256);
    const size_t nc = (size_t)nA * (size_t)p.chunks * kKeep;
    w.cscore = w.cidx + align_up(nc * 4, 256);
    w.total = w.cscore + align_up(nc * 4, 256);
    return w;
}

// quantised paths (precision 1, 2)
struct WsLp {
    size_t scal, aq, bq, sa, sb, keys, nrm, total;
};

WsLp ws_lp(int64_t nA, int64_t nB, int precision, const MatchPlan& p)
{
    const size_t rb = (precision == 1) ? 256 : 128;
    const int keep = (precision == 1) ? kLpKeepBf16 : kLpKeepFp8;
    WsLp w;
    w.scal = 0;
    w.aq = 256;
    w.bq = w.aq + align_up((size_t)nA * rb, 256);
    w.sa = w.bq + align_up((size_t)nB * rb, 256);
    w.sb = w.sa + align_up((size_t)nA * 4, 256);
    w.keys = w.sb + align_up((size_t)nB * 4, 256);
    w.nrm = w.keys + align_up((size_t)nA * p.chunks * 2 * keep * 4, 256);
    w.total = w.nrm + align_up((size_t)nB * 4, 256);
    return w;
}

// split path (precision 3): counters, candidate lists, thirds, fallback list,
// then the FP32 path's own workspace for the fallback
struct WsX3 {
    size_t cnt, bhl, cidx, cscore, cthird, fb, f32, total;
};

WsX3 ws_x3(int64_t nA, int64_t nB, const MatchPlan& p, const MatchPlan& pf)
{
    WsX3 w;
    w.cnt = 0;
    const size_t nc = (size_t)nA * (size_t)p.chunks * 4;
    w.bhl = 256;
    w.cidx = w.bhl + align_up((size_t)nB * 512, 256);
    w.cscore = w.cidx + align_up(nc * 4, 256);
    w.cthird = w.cscore + align_up(nc * 4, 256);
    w.fb = w.cthird + align_up((size_t)nA * p.chunks * 2 * 4, 256);
    w.f32 = w.fb + align_up((size_t)nA * 4, 256);
    w.total = w.f32 + ws_f32(nA, nB, pf).total;
    return w;
}


MatchPlan plan_chunks(int64_t nA, int64_t nB, int qb_size, int tile, int max_chunks, int req,
                      int resident = 512)
{
    MatchPlan p;
    int chunks = req;
    if (chunks <= 0) {
        // `resident` workgroups run at once (two per compute unit for 4-wave
        // workgroups): pick the chunk count whose grid comes closest to a
        // whole number of rounds
        const int64_t qblocks = (nA + qb_size - 1) / qb_size;
        chunks = 1;
        double best = -1.0;
        for (int c = 1; c <= max_chunks; ++c) {
            const double rounds = (double)qblocks * c / (double)resident;
            const double eff = rounds / std::ceil(rounds);
            if (eff > best + 0.02) {   // prefer full rounds, then fewer chunks
                best = eff;
                chunks = c;
            }
        }
    }
    if (chunks > max_chunks) chunks = max_chunks;
    const int64_t tiles = (nB + tile - 1) / tile;
    if (tiles > 0 && chunks > tiles) chunks = (int)tiles;
    if (chunks < 1) chunks = 1;
    p.chunks = chunks;
    p.chunk_len = ((tiles + chunks - 1) / chunks) * tile;
    return p;
}

uint32_t idx_mask_for(int64_t chunk_len)
{
    uint32_t m = 1;
    while ((int64_t)m < chunk_len) m <<= 1;
    return m - 1;
}

// Wavefronts per workgroup of the FP32 contraction (0 = the default).
int f32_waves(const lpsift_match_params* mp)
{
    return mp->qblock_waves > 0 ? mp->qblock_waves : kDefaultWaves;
}

void launch_f32(int waves, dim3 grid, const F32Batch& b, hipStream_t stream)
{
    if (waves == 2)
        hipLaunchKernelGGL(match_topk_f32_kernel<2>, grid, dim3(128), 0, stream, b);
    else if (waves == 8)
        hipLaunchKernelGGL(match_topk_f32_kernel<8>, grid, dim3(512), 0, stream, b);
    else
        hipLaunchKernelGGL(match_topk_f32_kernel<4>, grid, dim3(256), 0, stream, b);
}

// waves: wavefronts per workgroup of the FP32 contraction (2, 4 or 8).
MatchPlan plan_fp32(int64_t nA, int64_t nB, int req, int waves)
{
    return plan_chunks(nA, nB, 64 * waves, kCT, 16, req, 256 * (8 / waves));
}

// The FP32 re-match of uncertified queries: usually few queries, so the
// candidate range is split finely (the rescore merges up to 256 entries).
MatchPlan plan_fallback(int64_t nA, int64_t nB, int waves)
{
    return plan_chunks(nA, nB, 64 * waves, kCT, 64, 64, 256 * (8 / waves));
}

}  // namespace

int launch_quantize_lowp(const float* desc, int64_t n, int precision, void* q, float* scale,
                         hipStream_t stream)
{
    if (n == 0) return LPSIFT_OK;
    const dim3 grid((unsigned)((n + 15) / 16));
    uint8_t* y = static_cast<uint8_t*>(q);
    if (precision == 1)
        hipLaunchKernelGGL(quantize_kernel<1>, grid, dim3(256), 0, stream, desc, n, y, scale,
                           (uint32_t*)nullptr);
    else
        hipLaunchKernelGGL(quantize_kernel<2>, grid, dim3(256), 0, stream, desc, n, y, scale,
                           (uint32_t*)nullptr);
    return hipGetLastError() == hipSuccess ? LPSIFT_OK : LPSIFT_EHIP;
}

MatchPlan plan_match(int64_t nA, int64_t nB, const lpsift_match_params* mp)
{
    switch (mp->precision) {
    case 0: return plan_fp32(nA, nB, mp->b_chunks, f32_waves(mp));
    case 3: return plan_chunks(nA, nB, kX3QB, kX3CT, 16, mp->b_chunks);
    default: {
        // the rescore wavefront holds chunks x 2 lane halves x K keys
        const int keep = (mp->precision == 1) ? kLpKeepBf16 : kLpKeepFp8;
        return plan_chunks(nA, nB, kLpQB, mp->precision == 2 ? Lp<2>::kCT : Lp<1>::kCT, 64 / (2 * keep),
                           mp->b_chunks);
    }
    }
}

size_t match_workspace_bytes(int64_t nA, int64_t nB, const lpsift_match_params* mp)
{
    const MatchPlan p = plan_match(nA, nB, mp);
    switch (mp->precision) {
    case 0: return ws_f32(nA, nB, p).total;
    case 3: return ws_x3(nA, nB, p, plan_fallback(nA, nB, f32_waves(mp))).total;
    default: {
        // an empty candidate set is handled by the FP32 kernels
        const size_t a = ws_lp(nA, nB, mp->precision, p).total;
        const size_t b = ws_f32(nA, nB, plan_fp32(nA, nB, 0, f32_waves(mp))).total;
        return a > b ? a : b;
    }
    }
}

namespace {

// Quantised approximate paths (precision 1, 2), one pair with nA, nB > 0.
int launch_lp_pair(const MatchPairIO& io, const lpsift_match_params* mp, hipStream_t stream)
{
    const int64_t nA = io.nA, nB = io.nB;
    const float* A = io.A;
    const float* B = io.B;
    char* base = static_cast<char*>(io.ws);
    const MatchPlan p = plan_match(nA, nB, mp);
    const dim3 gr((unsigned)((nA + 15) / 16));   // rescore: 16 queries per workgroup
    const WsLp L = ws_lp(nA, nB, mp->precision, p);
    float* scal = reinterpret_cast<float*>(base + L.scal);
    uint32_t* counters = reinterpret_cast<uint32_t*>(scal);   // [1], [2] max bits
    uint8_t* aq = reinterpret_cast<uint8_t*>(base + L.aq);
    uint8_t* bq = reinterpret_cast<uint8_t*>(base + L.bq);
    float* sa = reinterpret_cast<float*>(base + L.sa);
    float* sb = reinterpret_cast<float*>(base + L.sb);
    uint32_t* keys = reinterpret_cast<uint32_t*>(base + L.keys);
    float* nrm = reinterpret_cast<float*>(base + L.nrm);
    const uint32_t mask = idx_mask_for(p.chunk_len);
    const dim3 grid((unsigned)((nA + kLpQB - 1) / kLpQB), (unsigned)p.chunks);
    const dim3 gq((unsigned)((nA + 15) / 16)), gqb((unsigned)((nB + 15) / 16));
    const dim3 gn((unsigned)((nA + kRowsPerWg - 1) / kRowsPerWg));
    const dim3 gnb((unsigned)((nB + kRowsPerWg - 1) / kRowsPerWg));

    hipLaunchKernelGGL(init_counters_kernel, dim3(1), dim3(64), 0, stream, counters, 4);
    hipLaunchKernelGGL(sqnorm_kernel, gn, dim3(256), 0, stream, A, nA, (float*)nullptr, counters + 1);
    hipLaunchKernelGGL(sqnorm_kernel, gnb, dim3(256), 0, stream, B, nB, nrm, counters + 2);
    if (mp->precision == 1) {
        hipLaunchKernelGGL(quantize_kernel<1>, gq, dim3(256), 0, stream, A, nA, aq, sa,
                           (uint32_t*)nullptr);
        hipLaunchKernelGGL(quantize_kernel<1>, gqb, dim3(256), 0, stream, B, nB, bq, sb,
                           (uint32_t*)nullptr);
        hipLaunchKernelGGL(lp_scalars_kernel, dim3(1), dim3(1), 0, stream, scal, kBf16DotErr);
        {
            TimedScope ts(LPSIFT_KERNEL_MATCH_LOWP, stream);
            hipLaunchKernelGGL((match_topk_lp_kernel<1, kLpKeepBf16>), grid, dim3(256), 0, stream,
                               aq, sa, nA, bq, sb, nB, nrm, scal, p.chunk_len, p.chunks, mask, keys);
        }
        TimedScope ts(LPSIFT_KERNEL_MATCH_RESCORE, stream);
        hipLaunchKernelGGL((rescore_lp_kernel<kLpKeepBf16>), gr, dim3(256), 0, stream, A, nA, B,
                           p.chunks, p.chunk_len, mask, keys, mp->ratio, mp->abs_thresh,
                           mp->topk ? mp->topk : kLpRescore, io.match, io.d1, io.d2);
    } else {
        hipLaunchKernelGGL(quantize_kernel<2>, gq, dim3(256), 0, stream, A, nA, aq, sa,
                           (uint32_t*)nullptr);
        hipLaunchKernelGGL(quantize_kernel<2>, gqb, dim3(256), 0, stream, B, nB, bq, sb,
                           (uint32_t*)nullptr);
        hipLaunchKernelGGL(lp_scalars_kernel, dim3(1), dim3(1), 0, stream, scal, 0.13f);
        {
            TimedScope ts(LPSIFT_KERNEL_MATCH_LOWP, stream);
            hipLaunchKernelGGL((match_topk_lp_kernel<2, kLpKeepFp8>), grid, dim3(256), 0, stream,
                               aq, sa, nA, bq, sb, nB, nrm, scal, p.chunk_len, p.chunks, mask, keys);
        }
        TimedScope ts(LPSIFT_KERNEL_MATCH_RESCORE, stream);
        hipLaunchKernelGGL((rescore_lp_kernel<kLpKeepFp8>), gr, dim3(256), 0, stream, A, nA, B,
                           p.chunks, p.chunk_len, mask, keys, mp->ratio, mp->abs_thresh,
                           mp->topk ? mp->topk : kLpRescore, io.match, io.d1, io.d2);
    }
    return hipGetLastError() == hipSuccess ? LPSIFT_OK : LPSIFT_EHIP;
}

// Grid of a launch whose item count is only known on the device: at most
// `cap` workgroups stride over at most `most` items.
unsigned strided_grid(int64_t most, int64_t cap)
{
    return (unsigned)((most < cap) ? (most > 0 ? most : 1) : cap);
}

// Per-pair workspace pointers of the FP32 and split paths. The norms (and
// split rows) of a candidate set shared by several pairs of the call live in
// the workspace of the first pair that uses it (its owner).
struct PairPtrs {
    MatchPlan p, pf;
    float* nrm;
    uint8_t* bhl;
    uint32_t* cnt;         // split: [0] re-matched queries, [1..3] row maxima of B
    int32_t* cidx;
    float* cscore;
    float* cthird;
    int32_t* fb;
    int32_t* fidx;
    float* fscore;
};

PairPtrs pair_ptrs(const MatchPairIO& io, const lpsift_match_params* mp)
{
    PairPtrs r{};
    char* base = static_cast<char*>(io.ws);
    if (mp->precision == 3) {
        r.p = plan_match(io.nA, io.nB, mp);
        r.pf = plan_fallback(io.nA, io.nB, f32_waves(mp));
        const WsX3 L = ws_x3(io.nA, io.nB, r.p, r.pf);
        const WsF32 F = ws_f32(io.nA, io.nB, r.pf);
        char* fbase = base + L.f32;
        r.cnt = reinterpret_cast<uint32_t*>(base + L.cnt);
        r.bhl = reinterpret_cast<uint8_t*>(base + L.bhl);
        r.cidx = reinterpret_cast<int32_t*>(base + L.cidx);
        r.cscore = reinterpret_cast<float*>(base + L.cscore);
        r.cthird = reinterpret_cast<float*>(base + L.cthird);
        r.fb = reinterpret_cast<int32_t*>(base + L.fb);
        r.nrm = reinterpret_cast<float*>(fbase + F.nrm);
        r.fidx = reinterpret_cast<int32_t*>(fbase + F.cidx);
        r.fscore = reinterpret_cast<float*>(fbase + F.cscore);
    } else {
        r.pf = plan_fp32(io.nA, io.nB, mp->precision == 0 ? mp->b_chunks : 0, f32_waves(mp));
        const WsF32 F = ws_f32(io.nA, io.nB, r.pf);
        r.nrm = reinterpret_cast<float*>(base + F.nrm);
        r.fidx = reinterpret_cast<int32_t*>(base + F.cidx);
        r.fscore = reinterpret_cast<float*>(base + F.cscore);
    }
    return r;
}

}  // namespace

int launch_match_pairs(const MatchPairIO* io, int n, const lpsift_match_params* mp,
                       hipStream_t stream)
{
    uint32_t* stats = static_cast<uint32_t*>(mp->stats);
    if (stats) hipLaunchKernelGGL(init_counters_kernel, dim3(1), dim3(64), 0, stream, stats, 1);

    // pairs with queries; of those, the ones with candidates
    std::vector<int> act;
    for (int i = 0; i < n; ++i)
        if (io[i].nA > 0) act.push_back(i);
    std::vector<PairPtrs> pp(n);
    std::vector<int> owner(n, -1);
    for (int i : act) {
        pp[i] = pair_ptrs(io[i], mp);
        if (io[i].nB == 0) continue;
        owner[i] = i;
        for (int k : act) {
            if (k >= i) break;
            if (io[k].nB == io[i].nB && io[k].B == io[i].B) {
                owner[i] = owner[k];
                break;
            }
        }
    }
    const bool lp = (mp->precision == 1 || mp->precision == 2);
    const int waves = f32_waves(mp);
    const int64_t qb = 64 * waves;   // queries per FP32 workgroup

    for (size_t b0 = 0; b0 < act.size(); b0 += kPairs) {
        const size_t b1 = (b0 + kPairs < act.size()) ? b0 + kPairs : act.size();
        RowsBatch rows{};
        F32Batch main{}, fall{};
        X3Batch x3{};
        RescoreX3Batch rx3{};
        RescoreF32Batch rf{};
        CounterBatch cnt{};
        rx3.ratio = rf.ratio = mp->ratio;
        rx3.abs_thresh = rf.abs_thresh = mp->abs_thresh;
        int64_t rows_wg = 0, main_wg = 0, x3_wg = 0, rx3_wg = 0, fall_most = 0, rf_most = 0;
        for (size_t a = b0; a < b1; ++a) {
            const int i = act[a];
            const MatchPairIO& P = io[i];
            const PairPtrs& Q = pp[i];
            if (P.nB == 0) {            // no candidates: every query rejected
                rf.j[rf.n++] = RescoreF32Job{P.A, P.B, nullptr, nullptr, nullptr, nullptr,
                                             P.match, P.d1, P.d2, P.nA, P.nB, 0};
                rf_most += (P.nA + 15) / 16;
                continue;
            }
            if (lp) {
                const int st = launch_lp_pair(P, mp, stream);
                if (st != LPSIFT_OK) return st;
                continue;
            }
            const PairPtrs& O = pp[owner[i]];
            if (owner[i] == i) {
                rows.j[rows.n++] = RowsJob{P.B, Q.nrm, mp->precision == 3 ? Q.bhl : nullptr,
                                           Q.cnt ? Q.cnt + 1 : nullptr, P.nB};
                rows_wg += (P.nB + kRowsPerWg - 1) / kRowsPerWg;
            }
            if (mp->precision == 0) {
                main.j[main.n++] = F32Job{P.A, nullptr, nullptr, P.B, O.nrm, Q.fidx, Q.fscore,
                                          P.nA, P.nB, Q.pf.chunk_len, Q.pf.chunks};
                main_wg += (P.nA + qb - 1) / qb * Q.pf.chunks;
                rf.j[rf.n++] = RescoreF32Job{P.A, P.B, nullptr, nullptr, Q.fidx, Q.fscore,
                                             P.match, P.d1, P.d2, P.nA, P.nB, Q.pf.chunks};
                rf_most += (P.nA + 15) / 16;
                continue;
            }
            // split path, then the FP32 re-match of the queries it did not certify
            cnt.c[cnt.n++] = Q.cnt;
            x3.j[x3.n++] = X3Job{P.A, O.bhl, O.nrm, Q.cidx, Q.cscore, Q.cthird, P.nA, P.nB,
                                 Q.p.chunk_len, Q.p.chunks};
            x3_wg += (P.nA + kX3QB - 1) / kX3QB * Q.p.chunks;
            rx3.j[rx3.n++] = RescoreX3Job{P.A, P.B, Q.cidx, Q.cscore, Q.cthird, O.cnt + 1,
                                          P.match, P.d1, P.d2, Q.cnt, Q.fb, P.nA, Q.p.chunks};
            rx3_wg += (P.nA + 3) / 4;
            fall.j[fall.n++] = F32Job{P.A, Q.fb, Q.cnt, P.B, O.nrm, Q.fidx, Q.fscore, P.nA, P.nB,
                                      Q.pf.chunk_len, Q.pf.chunks};
            fall_most += (P.nA + qb - 1) / qb * Q.pf.chunks;
            rf.j[rf.n++] = RescoreF32Job{P.A, P.B, Q.fb, Q.cnt, Q.fidx, Q.fscore, P.match, P.d1,
                                         P.d2, P.nA, P.nB, Q.pf.chunks};
            rf_most += (P.nA + 15) / 16;
        }
        // the split rows' maxima are accumulated with atomics: zero them first
        if (cnt.n > 0)
            hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(kCounterThreads), 0, stream, cnt, 4);
        if (rows.n > 0) {
            TimedScope ts(LPSIFT_KERNEL_MATCH_NORMS, stream);
            hipLaunchKernelGGL(rows_kernel, dim3((unsigned)rows_wg), dim3(256), 0, stream, rows);
        }
        if (main.n > 0) {
            TimedScope ts(LPSIFT_KERNEL_MATCH_FP32, stream);
            // a multiple of 8 workgroups: the XCD-ordered item mapping
            launch_f32(waves, dim3((unsigned)((main_wg + 7) / 8 * 8)), main, stream);
        }
        if (x3.n > 0) {
            {
                TimedScope ts(LPSIFT_KERNEL_MATCH_SPLIT, stream);
                hipLaunchKernelGGL(match_topk_x3_kernel, dim3((unsigned)x3_wg), dim3(256), 0,
                                   stream, x3);
            }
            {
                TimedScope ts(LPSIFT_KERNEL_MATCH_RESCORE, stream);
                hipLaunchKernelGGL(rescore_x3_kernel, dim3((unsigned)rx3_wg), dim3(256), 0,
                                   stream, rx3);
            }
            TimedScope ts(LPSIFT_KERNEL_MATCH_REMATCH, stream);
            launch_f32(waves, dim3(strided_grid(fall_most, 1024)), fall, stream);
        }
        if (rf.n > 0) {
            TimedScope ts(LPSIFT_KERNEL_MATCH_RESCORE, stream);
            hipLaunchKernelGGL(rescore_f32_kernel, dim3(strided_grid(rf_most, 8192)), dim3(256), 0,
                               stream, rf);
        }
        if (stats && cnt.n > 0)
            hipLaunchKernelGGL(add_counters_kernel, dim3(1), dim3(64), 0, stream, cnt, stats);
        if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;
    }
    return LPSIFT_OK;
}

}  // namespace lpsift
