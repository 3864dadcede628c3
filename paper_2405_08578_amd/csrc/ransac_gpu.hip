// Batched RANSAC homography on the GPU (Sec. 2.5, Eq. 7), FP64.
//
// Per pair of a batch:
//  1. ransac_points_kernel compacts the accepted matches of a match list into
//     point arrays (query order) and their count, on the device, so that no
//     host round trip is needed before sampling;
//  2. ransac_hyp_kernel: one thread per hypothesis. Its 4 indices come from
//     caller-supplied uniforms (slot s takes the first try whose floor(u n) is
//     new); samples with 3 nearly collinear points in either image are
//     skipped; the homography through the 4 pairs is the closed-form
//     projective-basis solution in Hartley coordinates (each side's 4 points
//     mapped to the canonical basis, then composed). Every hypothesis scores
//     all matches, staged through LDS 1,024 at a time; each workgroup keeps
//     its best (most inliers, earliest hypothesis) and that hypothesis' H;
//  3. ransac_refit_kernel: one workgroup per pair picks the best hypothesis,
//     refits H by linear least squares over its inliers (normal equations,
//     8 unknowns, Hartley coordinates of the inlier set, fixed-order
//     reductions) and writes the final inlier mask and counts.
// A pair is an inlier when the one-way reprojection error |H a - b| is below
// the threshold (points mapped to w ~ 0 are outliers).
#include "internal.h"

namespace lpsift {
namespace {

constexpr int kCompactThreads = 1024;
constexpr int kCompactPer = 8;
constexpr int kHypThreads = 256;
constexpr int kPointTile = 1024;
constexpr int kRefitThreads = 256;

// ------------------------------------------------------------- compaction --

__device__ inline uint32_t compact_scan(uint32_t v, uint32_t* total, uint32_t* sh)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int nw = kCompactThreads / 64;
        uint32_t w = (lane < nw) ? sh[lane] : 0u;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(w, off);
            if (lane >= off) w += y;
        }
        if (lane < nw) sh[64 + lane] = w;
    }
    __syncthreads();
    const uint32_t before = (wave > 0) ? sh[64 + wave - 1] : 0u;
    *total = sh[64 + kCompactThreads / 64 - 1];
    __syncthreads();
    return before + x - v;
}

__global__ __launch_bounds__(kCompactThreads) void ransac_points_kernel(RansacBatch b)
{
    __shared__ uint32_t sh[128];
    const RansacPair& P = b.p[blockIdx.x];
    uint32_t base = 0u;
    for (int64_t i0 = 0; i0 < P.nq; i0 += (int64_t)kCompactThreads * kCompactPer) {
        const int64_t i = i0 + (int64_t)kCompactPer * threadIdx.x;
        int32_t m[kCompactPer];
        uint32_t cnt = 0u;
#pragma unroll
        for (int e = 0; e < kCompactPer; ++e) {
            m[e] = (i + e < P.nq) ? P.match[i + e] : -1;
            cnt += (m[e] >= 0) ? 1u : 0u;
        }
        uint32_t tot;
        uint32_t pos = base + compact_scan(cnt, &tot, sh);
#pragma unroll
        for (int e = 0; e < kCompactPer; ++e) {
            if (m[e] < 0) continue;
            const int32_t sa = P.selA ? P.selA[i + e] : (int32_t)(i + e);
            const int32_t sb = P.selB ? P.selB[m[e]] : m[e];
            P.slotA[pos] = sa;
            P.slotB[pos] = sb;
            P.pa[2 * pos] = (double)P.ax[sa];
            P.pa[2 * pos + 1] = (double)P.ay[sa];
            P.pb[2 * pos] = (double)P.bx[sb];
            P.pb[2 * pos + 1] = (double)P.by[sb];
            ++pos;
        }
        base += tot;
    }
    if (threadIdx.x == 0) *P.count = (int32_t)base;
}

// ------------------------------------------------------------- hypotheses --

__device__ inline bool degenerate4(const double x[4], const double y[4])
{
    double x0 = x[0], x1 = x[0], y0 = y[0], y1 = y[0];
    for (int k = 1; k < 4; ++k) {
        x0 = fmin(x0, x[k]);
        x1 = fmax(x1, x[k]);
        y0 = fmin(y0, y[k]);
        y1 = fmax(y1, y[k]);
    }
    const double ext = fmax(x1 - x0, y1 - y0);
    const double tol = 1e-6 * ext * ext;
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j)
            for (int k = j + 1; k < 4; ++k) {
                const double ex = x[j] - x[i], ey = y[j] - y[i];
                const double fx = x[k] - x[i], fy = y[k] - y[i];
                if (fabs(ex * fy - ey * fx) <= tol) return true;
            }
    return false;
}

struct Norm2 {
    double s, cx, cy;
};

__device__ inline Norm2 hartley4(const double x[4], const double y[4])
{
    const double cx = (x[0] + x[1] + x[2] + x[3]) / 4.0;
    const double cy = (y[0] + y[1] + y[2] + y[3]) / 4.0;
    double d = 0.0;
    for (int k = 0; k < 4; ++k) d += sqrt((x[k] - cx) * (x[k] - cx) + (y[k] - cy) * (y[k] - cy));
    d /= 4.0;
    return Norm2{d > 0.0 ? sqrt(2.0) / d : 1.0, cx, cy};
}

// 3x3 adjugate (row-major) and determinant
__device__ inline double adj3(const double m[9], double a[9])
{
    a[0] = m[4] * m[8] - m[5] * m[7];
    a[1] = m[2] * m[7] - m[1] * m[8];
    a[2] = m[1] * m[5] - m[2] * m[4];
    a[3] = m[5] * m[6] - m[3] * m[8];
    a[4] = m[0] * m[8] - m[2] * m[6];
    a[5] = m[2] * m[3] - m[0] * m[5];
    a[6] = m[3] * m[7] - m[4] * m[6];
    a[7] = m[1] * m[6] - m[0] * m[7];
    a[8] = m[0] * m[4] - m[1] * m[3];
    return m[0] * a[0] + m[1] * a[3] + m[2] * a[6];
}

__device__ inline void mul3(const double a[9], const double b[9], double c[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            c[i * 3 + j] = a[i * 3] * b[j] + a[i * 3 + 1] * b[3 + j] + a[i * 3 + 2] * b[6 + j];
}

// Matrix mapping the canonical projective basis e1, e2, e3, (1,1,1) to the
// 4 normalised points (columns p1..p3 scaled by M^-1 p4); false if singular.
__device__ inline bool basis4(const double x[4], const double y[4], const Norm2& n, double A[9])
{
    double u[4], v[4];
    for (int k = 0; k < 4; ++k) {
        u[k] = n.s * (x[k] - n.cx);
        v[k] = n.s * (y[k] - n.cy);
    }
    const double M[9] = {u[0], u[1], u[2], v[0], v[1], v[2], 1.0, 1.0, 1.0};
    double J[9];
    const double det = adj3(M, J);
    if (!(fabs(det) > 1e-300)) return false;
    double lam[3];
    for (int i = 0; i < 3; ++i) lam[i] = (J[i * 3] * u[3] + J[i * 3 + 1] * v[3] + J[i * 3 + 2]) / det;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i * 3 + j] = M[i * 3 + j] * lam[j];
    return true;
}

// Homography (h33 = 1) through the 4 pairs (xa, ya) -> (xb, yb).
__device__ inline bool homography4(const double xa[4], const double ya[4], const double xb[4],
                                   const double yb[4], double H[9])
{
    const Norm2 na = hartley4(xa, ya), nb = hartley4(xb, yb);
    double A[9], B[9], Ai[9], Hn[9], T[9], G[9];
    if (!basis4(xa, ya, na, A) || !basis4(xb, yb, nb, B)) return false;
    adj3(A, Ai);                                  // A^-1 up to scale
    mul3(B, Ai, Hn);
    const double Ta[9] = {na.s, 0.0, -na.s * na.cx, 0.0, na.s, -na.s * na.cy, 0.0, 0.0, 1.0};
    const double Tbi[9] = {1.0 / nb.s, 0.0, nb.cx, 0.0, 1.0 / nb.s, nb.cy, 0.0, 0.0, 1.0};
    mul3(Hn, Ta, T);
    mul3(Tbi, T, G);
    if (!(fabs(G[8]) > 1e-300)) return false;
    for (int i = 0; i < 9; ++i) {
        H[i] = G[i] / G[8];
        if (!isfinite(H[i])) return false;
    }
    return true;
}

__device__ inline bool is_inlier(const double H[9], double x, double y, double bx, double by,
                                 double thresh2)
{
    const double w = H[6] * x + H[7] * y + H[8];
    if (!(fabs(w) > 1e-12)) return false;
    const double ex = (H[0] * x + H[1] * y + H[2]) / w - bx;
    const double ey = (H[3] * x + H[4] * y + H[5]) / w - by;
    return ex * ex + ey * ey < thresh2;
}

__device__ inline uint64_t max_u64(uint64_t a, uint64_t b) { return a > b ? a : b; }

__global__ __launch_bounds__(kHypThreads) void ransac_hyp_kernel(RansacBatch b)
{
    __shared__ double spa[2 * kPointTile], spb[2 * kPointTile];
    __shared__ uint64_t sbest[kHypThreads / 64];
    const int pair = blockIdx.x / b.n_blocks, blk = blockIdx.x % b.n_blocks;
    const RansacPair& P = b.p[pair];
    const int n = *P.count;
    if (n < 4) {
        if (threadIdx.x == 0) {
            P.bestc[2 * blk] = -1;
            P.bestc[2 * blk + 1] = b.n_iter;
        }
        return;
    }
    const int it = blk * kHypThreads + threadIdx.x;
    bool valid = it < b.n_iter;
    int idx[4] = {0, 0, 0, 0};
    if (valid) {
        for (int s = 0; s < 4 && valid; ++s) {
            bool found = false;
            for (int t = 0; t < b.tries && !found; ++t) {
                int i = (int)floor(b.u[((int64_t)it * 4 + s) * b.tries + t] * (double)n);
                i = i < n - 1 ? i : n - 1;
                bool fresh = true;
                for (int r = 0; r < s; ++r) fresh = fresh && (idx[r] != i);
                if (fresh) {
                    idx[s] = i;
                    found = true;
                }
            }
            valid = found;
        }
    }
    double H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (valid) {
        double xa[4], ya[4], xb[4], yb[4];
        for (int k = 0; k < 4; ++k) {
            xa[k] = P.pa[2 * idx[k]];
            ya[k] = P.pa[2 * idx[k] + 1];
            xb[k] = P.pb[2 * idx[k]];
            yb[k] = P.pb[2 * idx[k] + 1];
        }
        valid = !degenerate4(xa, ya) && !degenerate4(xb, yb) && homography4(xa, ya, xb, yb, H);
    }
    int cnt = 0;
    for (int k0 = 0; k0 < n; k0 += kPointTile) {
        const int m = (n - k0 < kPointTile) ? n - k0 : kPointTile;
        __syncthreads();
        for (int e = threadIdx.x; e < 2 * m; e += kHypThreads) {
            spa[e] = P.pa[2 * (int64_t)k0 + e];
            spb[e] = P.pb[2 * (int64_t)k0 + e];
        }
        __syncthreads();
        if (valid)
            for (int k = 0; k < m; ++k)
                cnt += is_inlier(H, spa[2 * k], spa[2 * k + 1], spb[2 * k], spb[2 * k + 1], b.thresh2)
                           ? 1 : 0;
    }
    // best of the workgroup: most inliers, then the earliest hypothesis
    const uint64_t key = valid ? ((uint64_t)(cnt + 1) << 32) | (uint32_t)(~(uint32_t)it) : 0ull;
    uint64_t best = key;
    for (int off = 32; off > 0; off >>= 1) best = max_u64(best, (uint64_t)__shfl_xor((long long)best, off));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sbest[wave] = best;
    __syncthreads();
    best = sbest[0];
    for (int w = 1; w < kHypThreads / 64; ++w) best = max_u64(best, sbest[w]);
    if (best == 0ull) {
        if (threadIdx.x == 0) {
            P.bestc[2 * blk] = -1;
            P.bestc[2 * blk + 1] = b.n_iter;
        }
        return;
    }
    if (key == best) {   // unique: hypothesis indices differ
        P.bestc[2 * blk] = cnt;
        P.bestc[2 * blk + 1] = it;
        for (int i = 0; i < 9; ++i) P.bestH[9 * blk + i] = H[i];
    }
}

// ------------------------------------------------------------------ refit --

// Sum of K per-thread values over the workgroup in a fixed order; every
// thread receives the totals.
template <int K>
__device__ inline void block_sum(double v[K], double* sh)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = v[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        v[k] = x;
    }
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < K; ++k) sh[wave * K + k] = v[k];
    __syncthreads();
    for (int k = 0; k < K; ++k) {
        double s = sh[k];
        for (int w = 1; w < kRefitThreads / 64; ++w) s += sh[w * K + k];
        v[k] = s;
    }
}

// n x n solve with partial pivoting (row-major, in place); false if singular
__device__ inline bool solve8(double* A, double* r)
{
    constexpr int n = 8;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int q = c + 1; q < n; ++q)
            if (fabs(A[q * n + c]) > fabs(A[p * n + c])) p = q;
        if (!(fabs(A[p * n + c]) > 1e-300)) return false;
        if (p != c) {
            for (int k = 0; k < n; ++k) {
                const double t = A[p * n + k];
                A[p * n + k] = A[c * n + k];
                A[c * n + k] = t;
            }
            const double t = r[p];
            r[p] = r[c];
            r[c] = t;
        }
        for (int q = c + 1; q < n; ++q) {
            const double f = A[q * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[q * n + k] -= f * A[c * n + k];
            r[q] -= f * r[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double s = r[c];
        for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * r[k];
        r[c] = s / A[c * n + c];
    }
    for (int c = 0; c < n; ++c)
        if (!isfinite(r[c])) return false;
    return true;
}

__global__ __launch_bounds__(kRefitThreads) void ransac_refit_kernel(RansacBatch b)
{
    __shared__ double sh[(kRefitThreads / 64) * 44];
    __shared__ double sH[9];
    __shared__ int sbest;
    const RansacPair& P = b.p[blockIdx.x];
    const int n = *P.count;
    const int tid = threadIdx.x;

    if (tid == 0) {
        int bc = -1, bi = b.n_iter, bb = -1;
        if (n >= 4)
            for (int k = 0; k < b.n_blocks; ++k) {
                const int c = P.bestc[2 * k], i = P.bestc[2 * k + 1];
                if (c > bc || (c == bc && c >= 0 && i < bi)) {
                    bc = c;
                    bi = i;
                    bb = k;
                }
            }
        sbest = (bc >= 0) ? bb : -1;
        P.stats[0] = n;
        P.stats[2] = (bc >= 0) ? bi : -1;
        if (bc >= 0)
            for (int i = 0; i < 9; ++i) sH[i] = P.bestH[9 * bb + i];
    }
    __syncthreads();
    if (sbest < 0) {
        for (int k = tid; k < n; k += kRefitThreads) P.inlier[k] = 0;
        if (tid < 9) P.H[tid] = 0.0;
        if (tid == 0) P.stats[1] = 0;
        return;
    }
    double H0[9];
    for (int i = 0; i < 9; ++i) H0[i] = sH[i];

    // inliers of the best hypothesis: count and centroids
    double c5[5] = {0, 0, 0, 0, 0};
    for (int k = tid; k < n; k += kRefitThreads) {
        const double x = P.pa[2 * k], y = P.pa[2 * k + 1], u = P.pb[2 * k], v = P.pb[2 * k + 1];
        if (is_inlier(H0, x, y, u, v, b.thresh2)) {
            c5[0] += 1.0;
            c5[1] += x;
            c5[2] += y;
            c5[3] += u;
            c5[4] += v;
        }
    }
    block_sum<5>(c5, sh);
    double F[9];
    for (int i = 0; i < 9; ++i) F[i] = H0[i];
    if (c5[0] >= 4.0) {
        const double m = c5[0];
        const double cxa = c5[1] / m, cya = c5[2] / m, cxb = c5[3] / m, cyb = c5[4] / m;
        double d2[2] = {0, 0};
        for (int k = tid; k < n; k += kRefitThreads) {
            const double x = P.pa[2 * k], y = P.pa[2 * k + 1], u = P.pb[2 * k], v = P.pb[2 * k + 1];
            if (is_inlier(H0, x, y, u, v, b.thresh2)) {
                d2[0] += sqrt((x - cxa) * (x - cxa) + (y - cya) * (y - cya));
                d2[1] += sqrt((u - cxb) * (u - cxb) + (v - cyb) * (v - cyb));
            }
        }
        block_sum<2>(d2, sh);
        const double sa = (d2[0] > 0.0) ? sqrt(2.0) / (d2[0] / m) : 1.0;
        const double sb = (d2[1] > 0.0) ? sqrt(2.0) / (d2[1] / m) : 1.0;
        // normal equations: upper triangle of N (36) and N^T r (8)
        double acc[44];
        for (int e = 0; e < 44; ++e) acc[e] = 0.0;
        for (int k = tid; k < n; k += kRefitThreads) {
            const double X = P.pa[2 * k], Y = P.pa[2 * k + 1], U = P.pb[2 * k], V = P.pb[2 * k + 1];
            if (!is_inlier(H0, X, Y, U, V, b.thresh2)) continue;
            const double x = sa * (X - cxa), y = sa * (Y - cya);
            const double u = sb * (U - cxb), v = sb * (V - cyb);
            const double r0[8] = {x, y, 1.0, 0.0, 0.0, 0.0, -u * x, -u * y};
            const double r1[8] = {0.0, 0.0, 0.0, x, y, 1.0, -v * x, -v * y};
            int e = 0;
            for (int i = 0; i < 8; ++i)
                for (int j = i; j < 8; ++j) acc[e++] += r0[i] * r0[j] + r1[i] * r1[j];
            for (int i = 0; i < 8; ++i) acc[36 + i] += r0[i] * u + r1[i] * v;
        }
        block_sum<44>(acc, sh);
        if (tid == 0) {
            double N[64], r[8];
            int e = 0;
            for (int i = 0; i < 8; ++i)
                for (int j = i; j < 8; ++j) {
                    N[i * 8 + j] = acc[e];
                    N[j * 8 + i] = acc[e];
                    ++e;
                }
            for (int i = 0; i < 8; ++i) r[i] = acc[36 + i];
            bool ok = solve8(N, r);
            double G[9];
            if (ok) {
                const double Hn[9] = {r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7], 1.0};
                const double Ta[9] = {sa, 0.0, -sa * cxa, 0.0, sa, -sa * cya, 0.0, 0.0, 1.0};
                const double Tbi[9] = {1.0 / sb, 0.0, cxb, 0.0, 1.0 / sb, cyb, 0.0, 0.0, 1.0};
                double T[9];
                mul3(Hn, Ta, T);
                mul3(Tbi, T, G);
                ok = fabs(G[8]) > 1e-300;
                for (int i = 0; i < 9 && ok; ++i) {
                    G[i] /= G[8];
                    ok = isfinite(G[i]);
                }
            }
            for (int i = 0; i < 9; ++i) sH[i] = ok ? G[i] : H0[i];
        }
        __syncthreads();
        for (int i = 0; i < 9; ++i) F[i] = sH[i];
    }
    double c1[1] = {0.0};
    for (int k = tid; k < n; k += kRefitThreads) {
        const bool in = is_inlier(F, P.pa[2 * k], P.pa[2 * k + 1], P.pb[2 * k], P.pb[2 * k + 1],
                                  b.thresh2);
        P.inlier[k] = in ? 1 : 0;
        c1[0] += in ? 1.0 : 0.0;
    }
    block_sum<1>(c1, sh);
    if (tid < 9) P.H[tid] = F[tid];
    if (tid == 0) P.stats[1] = (int32_t)c1[0];
}

}  // namespace

size_t ransac_workspace_bytes(int64_t nq, int32_t n_iter)
{
    const int64_t blocks = (n_iter + kHypThreads - 1) / kHypThreads;
    return align_up((size_t)nq * 16, 256) * 2 + 256 + align_up((size_t)blocks * 8, 256) +
           align_up((size_t)blocks * 72, 256);
}

void ransac_layout(void* ws, int64_t nq, int32_t n_iter, RansacPair& p)
{
    const int64_t blocks = (n_iter + kHypThreads - 1) / kHypThreads;
    char* c = static_cast<char*>(ws);
    p.pa = reinterpret_cast<double*>(c);
    c += align_up((size_t)nq * 16, 256);
    p.pb = reinterpret_cast<double*>(c);
    c += align_up((size_t)nq * 16, 256);
    p.count = reinterpret_cast<int32_t*>(c);
    c += 256;
    p.bestc = reinterpret_cast<int32_t*>(c);
    c += align_up((size_t)blocks * 8, 256);
    p.bestH = reinterpret_cast<double*>(c);
}

int launch_ransac(RansacBatch& b, hipStream_t stream)
{
    b.n_blocks = (b.n_iter + kHypThreads - 1) / kHypThreads;
    TimedScope ts(LPSIFT_KERNEL_RANSAC, stream);
    hipLaunchKernelGGL(ransac_points_kernel, dim3((unsigned)b.n), dim3(kCompactThreads), 0, stream, b);
    if (b.n_blocks > 0)
        hipLaunchKernelGGL(ransac_hyp_kernel, dim3((unsigned)(b.n * b.n_blocks)), dim3(kHypThreads), 0,
                           stream, b);
    hipLaunchKernelGGL(ransac_refit_kernel, dim3((unsigned)b.n), dim3(kRefitThreads), 0, stream, b);
    return hipGetLastError() == hipSuccess ? LPSIFT_OK : LPSIFT_EHIP;
}

}  // namespace lpsift
