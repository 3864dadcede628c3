// Descriptor matching (Sec. 2.4, Eq. 6) with the ratio test.
//
// |a - b|^2 = |a|^2 + |b|^2 - 2 a.b, and |a|^2 is constant per query, so the
// nearest candidates of a query are those with the smallest |b|^2 - 2 a.b.
// The a.b contraction is a GEMM of the two descriptor sets and runs on the
// matrix cores (v_mfma_f32_32x32x2_f32, FP32 in and out):
//
//  * the MFMA's A operand is a 32-candidate tile (rows) and its B operand 32
//    queries (columns), so lane l of the 32x32 result holds 16 candidates of
//    one query (l % 32): the top-2 bookkeeping is private to each lane and the
//    N_A x N_B score matrix is never stored;
//  * a wavefront keeps 2 x 32 queries in registers for the whole sweep (the K
//    dimension split in halves: lanes 0-31 carry k = 0..63, lanes 32-63 carry
//    k = 64..127 -- any permutation of K shared by both operands leaves the
//    dot products unchanged);
//  * a 256-thread workgroup (4 wavefronts, 256 queries) streams the candidates
//    of its chunk through LDS, 32 at a time, with the next tile prefetched into
//    registers while the current one is contracted;
//  * the candidate range is split into chunks so that the grid fills the chip.
//
// Each lane's top-2 of each chunk survives (4 candidates per query and chunk).
// The rescore kernel keeps the 4 best by contraction score, recomputes their
// squared distances directly in FP32, takes the two smallest (lowest index on
// ties) and applies d1 < ratio * d2 in double precision.
#include "internal.h"

namespace lpsift {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kQB = 256;        // queries per workgroup
constexpr int kCT = 32;         // candidates per LDS tile
constexpr int kRow = 128 + 4;   // padded LDS row (floats)
constexpr int kKeep = 4;        // candidates kept per (query, chunk)

__global__ __launch_bounds__(256) void sqnorm_kernel(const float* __restrict__ B, int64_t n,
                                                     float* __restrict__ out)
{
    // 16 lanes per row, 8 floats each
    const int64_t row = (int64_t)blockIdx.x * 16 + threadIdx.x / 16;
    const int part = threadIdx.x % 16;
    float s = 0.0f;
    if (row < n) {
        const float4* p = reinterpret_cast<const float4*>(B + row * 128 + part * 8);
        const float4 a = p[0], b = p[1];
        s = a.x * a.x + a.y * a.y + a.z * a.z + a.w * a.w + b.x * b.x + b.y * b.y + b.z * b.z + b.w * b.w;
    }
    for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
    if (row < n && part == 0) out[row] = s;
}

// Branch-free insertion into a (score, index) top-2; on equal scores the
// earlier (lower) index stays first because candidates arrive in index order.
__device__ inline void top2_push(float s, int j, float& s1, int& j1, float& s2, int& j2)
{
    const bool lt1 = s < s1;
    const bool lt2 = s < s2;
    s2 = lt1 ? s1 : (lt2 ? s : s2);
    j2 = lt1 ? j1 : (lt2 ? j : j2);
    s1 = lt1 ? s : s1;
    j1 = lt1 ? j : j1;
}

__global__ __launch_bounds__(256, 2) void match_topk_f32_kernel(
    const float* __restrict__ A, int64_t nA, const float* __restrict__ B, int64_t nB,
    const float* __restrict__ nrmB, int64_t chunk_len, int chunks,
    int32_t* __restrict__ cidx, float* __restrict__ cscore)
{
    __shared__ __attribute__((aligned(16))) float tile[kCT * kRow];
    __shared__ float tnrm[kCT];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int64_t q0 = (int64_t)blockIdx.x * kQB + wave * 64 + col;
    const int64_t q1 = q0 + 32;
    const int chunk = blockIdx.y;
    const int64_t cb = (int64_t)chunk * chunk_len;
    const int64_t ce = (cb + chunk_len < nB) ? cb + chunk_len : nB;

    // queries in registers: qa[i] = A[q0][h*64 + i], qb[i] = A[q1][h*64 + i]
    float qa[64], qb[64];
    {
        const float4* pa = reinterpret_cast<const float4*>(A + q0 * 128 + h * 64);
        const float4* pb = reinterpret_cast<const float4*>(A + q1 * 128 + h * 64);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float4 va = (q0 < nA) ? pa[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 vb = (q1 < nA) ? pb[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            qa[4 * i + 0] = va.x; qa[4 * i + 1] = va.y; qa[4 * i + 2] = va.z; qa[4 * i + 3] = va.w;
            qb[4 * i + 0] = vb.x; qb[4 * i + 1] = vb.y; qb[4 * i + 2] = vb.z; qb[4 * i + 3] = vb.w;
        }
    }

    float sa1 = INFINITY, sa2 = INFINITY, sb1 = INFINITY, sb2 = INFINITY;
    int ja1 = -1, ja2 = -1, jb1 = -1, jb2 = -1;

    // prefetch: thread t moves float4 number t + 256 k (k < 4) of a 32 x 128 tile
    float4 pf[4];
    auto fetch = [&](int64_t t0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int f = tid + 256 * k;
            const int r = f >> 5, c4 = f & 31;
            const int64_t j = t0 + r;
            pf[k] = (j < ce) ? reinterpret_cast<const float4*>(B + j * 128)[c4]
                             : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    if (cb < ce) fetch(cb);

    for (int64_t t0 = cb; t0 < ce; t0 += kCT) {
        __syncthreads();   // the previous tile is no longer read
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int f = tid + 256 * k;
            const int r = f >> 5, c4 = f & 31;
            *reinterpret_cast<float4*>(&tile[r * kRow + c4 * 4]) = pf[k];
        }
        if (tid < kCT) tnrm[tid] = (t0 + tid < ce) ? nrmB[t0 + tid] : INFINITY;
        __syncthreads();
        if (t0 + kCT < ce) fetch(t0 + kCT);

        floatx16 acc0, acc1;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            acc0[r] = 0.0f;
            acc1[r] = 0.0f;
        }
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
        // result row (candidate) of accumulator r in this lane: 8 (r/4) + 4 h + r % 4
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int cl = 8 * (r >> 2) + 4 * h + (r & 3);
            const float nb = tnrm[cl];
            const int j = (int)(t0 + cl);
            top2_push(fmaf(-2.0f, acc0[r], nb), j, sa1, ja1, sa2, ja2);
            top2_push(fmaf(-2.0f, acc1[r], nb), j, sb1, jb1, sb2, jb2);
        }
    }

    // candidates of padded rows carry score +inf and are never pushed
    if (q0 < nA) {
        const int64_t o = (q0 * chunks + chunk) * kKeep + 2 * h;
        cidx[o] = ja1; cidx[o + 1] = ja2;
        cscore[o] = sa1; cscore[o + 1] = sa2;
    }
    if (q1 < nA) {
        const int64_t o = (q1 * chunks + chunk) * kKeep + 2 * h;
        cidx[o] = jb1; cidx[o + 1] = jb2;
        cscore[o] = sb1; cscore[o + 1] = sb2;
    }
}

// One wavefront per query: keep the 4 best candidates by contraction score,
// recompute their distances directly, then the ratio test.
__global__ __launch_bounds__(256) void rescore_kernel(
    const float* __restrict__ A, int64_t nA, const float* __restrict__ B, int chunks,
    const int32_t* __restrict__ cidx, const float* __restrict__ cscore, double ratio,
    float abs_thresh, int32_t* __restrict__ match, float* __restrict__ d1out,
    float* __restrict__ d2out)
{
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= nA) return;
    const int nc = chunks * kKeep;   // <= 64
    float sc = INFINITY;
    int id = -1;
    if (lane < nc) {
        id = cidx[q * nc + lane];
        sc = (id >= 0) ? cscore[q * nc + lane] : INFINITY;
        if (id < 0) id = 0x7FFFFFFF;
    } else {
        id = 0x7FFFFFFF;
    }
    const float a0 = A[q * 128 + lane], a1 = A[q * 128 + 64 + lane];
    float e1 = INFINITY, e2 = INFINITY;
    int j1 = -1, j2 = -1;
    for (int round = 0; round < 4; ++round) {
        float bs = sc;
        int bi = id;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float os = __shfl_xor(bs, off);
            const int oi = __shfl_xor(bi, off);
            if (os < bs || (os == bs && oi < bi)) {
                bs = os;
                bi = oi;
            }
        }
        if (bi == 0x7FFFFFFF || bs == INFINITY) break;
        if (id == bi) sc = INFINITY, id = 0x7FFFFFFF;   // taken
        const float b0 = B[(int64_t)bi * 128 + lane], b1 = B[(int64_t)bi * 128 + 64 + lane];
        const float x0 = a0 - b0, x1 = a1 - b1;
        float s = x0 * x0 + x1 * x1;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        // ordered insert by (squared distance, index)
        if (s < e1 || (s == e1 && bi < j1)) {
            e2 = e1; j2 = j1;
            e1 = s; j1 = bi;
        } else if (s < e2 || (s == e2 && bi < j2)) {
            e2 = s; j2 = bi;
        }
    }
    if (lane == 0) {
        const float dd1 = sqrtf(e1), dd2 = sqrtf(e2);
        const bool keep = j1 >= 0 && (double)dd1 < ratio * (double)dd2 && dd1 < abs_thresh;
        match[q] = keep ? j1 : -1;
        d1out[q] = dd1;
        d2out[q] = dd2;
    }
}

struct WsLayout {
    size_t nrm, cidx, cscore, total;
};

WsLayout ws_layout(int64_t nA, int64_t nB, const MatchPlan& p)
{
    WsLayout w;
    w.nrm = 0;
    w.cidx = align_up((size_t)nB * 4, 256);
    const size_t nc = (size_t)nA * (size_t)p.chunks * kKeep;
    w.cscore = w.cidx + align_up(nc * 4, 256);
    w.total = w.cscore + align_up(nc * 4, 256);
    return w;
}

}  // namespace

MatchPlan plan_match(int64_t nA, int64_t nB, const lpsift_match_params* mp)
{
    MatchPlan p;
    int chunks = mp->b_chunks;
    if (chunks <= 0) {
        // aim for about two resident workgroups per compute unit (256 CUs)
        const int64_t qblocks = (nA + kQB - 1) / kQB;
        chunks = (int)((512 + qblocks - 1) / (qblocks > 0 ? qblocks : 1));
        if (chunks < 1) chunks = 1;
    }
    if (chunks > 16) chunks = 16;
    const int64_t tiles = (nB + kCT - 1) / kCT;
    if (tiles > 0 && chunks > tiles) chunks = (int)tiles;
    if (chunks < 1) chunks = 1;
    p.chunks = chunks;
    p.chunk_len = ((tiles + chunks - 1) / chunks) * kCT;
    return p;
}

size_t match_workspace_bytes(int64_t nA, int64_t nB, const lpsift_match_params* mp)
{
    return ws_layout(nA, nB, plan_match(nA, nB, mp)).total;
}

int launch_match(const float* A, int64_t nA, const float* B, int64_t nB,
                 const lpsift_match_params* mp, void* ws, int32_t* match, float* d1, float* d2,
                 hipStream_t stream)
{
    if (nA == 0) return LPSIFT_OK;
    const MatchPlan p = plan_match(nA, nB, mp);
    const WsLayout L = ws_layout(nA, nB, p);
    char* base = static_cast<char*>(ws);
    float* nrm = reinterpret_cast<float*>(base + L.nrm);
    int32_t* cidx = reinterpret_cast<int32_t*>(base + L.cidx);
    float* cscore = reinterpret_cast<float*>(base + L.cscore);
    if (nB > 0) {
        hipLaunchKernelGGL(sqnorm_kernel, dim3((unsigned)((nB + 15) / 16)), dim3(256), 0, stream,
                           B, nB, nrm);
        if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;
        const dim3 grid((unsigned)((nA + kQB - 1) / kQB), (unsigned)p.chunks);
        hipLaunchKernelGGL(match_topk_f32_kernel, grid, dim3(256), 0, stream, A, nA, B, nB, nrm,
                           p.chunk_len, p.chunks, cidx, cscore);
        if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;
    }
    const int chunks = (nB > 0) ? p.chunks : 0;
    hipLaunchKernelGGL(rescore_kernel, dim3((unsigned)((nA + 3) / 4)), dim3(256), 0, stream, A, nA,
                       B, chunks, cidx, cscore, mp->ratio, mp->abs_thresh, match, d1, d2);
    if (hipGetLastError() != hipSuccess) return LPSIFT_EHIP;
    return LPSIFT_OK;
}

}  // namespace lpsift
