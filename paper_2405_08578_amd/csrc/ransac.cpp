// Host RANSAC homography (Sec. 2.5, Eq. 7) over matched pairs, FP64.
//
// Hypotheses are exact homographies (h33 = 1) through 4 sampled pairs, solved
// in Hartley coordinates by 8x8 Gaussian elimination with partial pivoting;
// samples with 3 nearly collinear points in either image are skipped. The
// hypothesis with the most inliers (one-way reprojection error below the
// threshold; earliest on ties) is refined by linear least squares over its
// inliers (normal equations, 8 unknowns, Hartley coordinates) and the final
// mask is the inlier set of the refined H. The random draws are an input
// (an [n_iter][4] index array) so that runs are reproducible.
//
// lpsift_refine_host repeats that least-squares step from a given H until the
// inlier set stops changing (a local optimisation of the estimate, so that the
// final inliers depend on the data rather than on which sample won).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "lpsift.h"

namespace {

struct Norm {
    double s, cx, cy;   // p' = s (p - c)
};

Norm hartley(const double* xy, const int64_t* idx, int64_t m)
{
    double cx = 0, cy = 0;
    for (int64_t k = 0; k < m; ++k) {
        cx += xy[2 * idx[k]];
        cy += xy[2 * idx[k] + 1];
    }
    cx /= (double)m;
    cy /= (double)m;
    double d = 0;
    for (int64_t k = 0; k < m; ++k) {
        const double dx = xy[2 * idx[k]] - cx, dy = xy[2 * idx[k] + 1] - cy;
        d += std::sqrt(dx * dx + dy * dy);
    }
    d /= (double)m;
    return Norm{d > 0 ? std::sqrt(2.0) / d : 1.0, cx, cy};
}

// Solves the n x n system A x = b in place (row-major); false if singular.
bool solve(double* A, double* b, int n)
{
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
        if (!(std::fabs(A[p * n + c]) > 1e-300)) return false;
        if (p != c) {
            for (int k = 0; k < n; ++k) std::swap(A[p * n + k], A[c * n + k]);
            std::swap(b[p], b[c]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double s = b[c];
        for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * b[k];
        b[c] = s / A[c * n + c];
    }
    for (int c = 0; c < n; ++c)
        if (!std::isfinite(b[c])) return false;
    return true;
}

// Homography through the listed pairs, least squares in Hartley coordinates.
bool dlt(const double* A, const double* B, const int64_t* idx, int64_t m, double H[9])
{
    const Norm na = hartley(A, idx, m), nb = hartley(B, idx, m);
    double N[64] = {0}, r[8] = {0};
    for (int64_t k = 0; k < m; ++k) {
        const double x = na.s * (A[2 * idx[k]] - na.cx), y = na.s * (A[2 * idx[k] + 1] - na.cy);
        const double u = nb.s * (B[2 * idx[k]] - nb.cx), v = nb.s * (B[2 * idx[k] + 1] - nb.cy);
        const double rows[2][8] = {{x, y, 1, 0, 0, 0, -u * x, -u * y},
                                   {0, 0, 0, x, y, 1, -v * x, -v * y}};
        const double rhs[2] = {u, v};
        for (int q = 0; q < 2; ++q)
            for (int i = 0; i < 8; ++i) {
                r[i] += rows[q][i] * rhs[q];
                for (int j = 0; j < 8; ++j) N[i * 8 + j] += rows[q][i] * rows[q][j];
            }
    }
    if (!solve(N, r, 8)) return false;
    // H = Tb^-1 Hn Ta
    const double Hn[9] = {r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7], 1.0};
    const double Ta[9] = {na.s, 0, -na.s * na.cx, 0, na.s, -na.s * na.cy, 0, 0, 1};
    const double Tbi[9] = {1 / nb.s, 0, nb.cx, 0, 1 / nb.s, nb.cy, 0, 0, 1};
    double T[9], G[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            T[i * 3 + j] = 0;
            for (int k = 0; k < 3; ++k) T[i * 3 + j] += Hn[i * 3 + k] * Ta[k * 3 + j];
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            G[i * 3 + j] = 0;
            for (int k = 0; k < 3; ++k) G[i * 3 + j] += Tbi[i * 3 + k] * T[k * 3 + j];
        }
    if (!(std::fabs(G[8]) > 1e-300)) return false;
    for (int i = 0; i < 9; ++i) H[i] = G[i] / G[8];
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(H[i])) return false;
    return true;
}

bool degenerate(const double* P, const int64_t* idx)
{
    double x0 = P[2 * idx[0]], x1 = x0, y0 = P[2 * idx[0] + 1], y1 = y0;
    for (int k = 1; k < 4; ++k) {
        x0 = std::fmin(x0, P[2 * idx[k]]);
        x1 = std::fmax(x1, P[2 * idx[k]]);
        y0 = std::fmin(y0, P[2 * idx[k] + 1]);
        y1 = std::fmax(y1, P[2 * idx[k] + 1]);
    }
    const double ext = std::fmax(x1 - x0, y1 - y0);
    const double tol = 1e-6 * ext * ext;
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j)
            for (int k = j + 1; k < 4; ++k) {
                const double ex = P[2 * idx[j]] - P[2 * idx[i]], ey = P[2 * idx[j] + 1] - P[2 * idx[i] + 1];
                const double fx = P[2 * idx[k]] - P[2 * idx[i]], fy = P[2 * idx[k] + 1] - P[2 * idx[i] + 1];
                if (std::fabs(ex * fy - ey * fx) <= tol) return true;
            }
    return false;
}

bool inlier(const double H[9], const double* A, const double* B, int64_t i, double thresh)
{
    const double x = A[2 * i], y = A[2 * i + 1];
    const double w = H[6] * x + H[7] * y + H[8];
    if (!(std::fabs(w) > 1e-12)) return false;
    const double ex = (H[0] * x + H[1] * y + H[2]) / w - B[2 * i];
    const double ey = (H[3] * x + H[4] * y + H[5]) / w - B[2 * i + 1];
    return std::sqrt(ex * ex + ey * ey) < thresh;
}

}  // namespace

extern "C" int lpsift_ransac_host(const double* xyA, const double* xyB, int64_t n,
                                  const int32_t* samples, int32_t n_iter, double thresh,
                                  double* H, uint8_t* mask, int64_t* n_inliers, int32_t* best_iter)
{
    if (n < 0 || n_iter < 0 || !H || !n_inliers || !best_iter) return LPSIFT_EINVAL;
    if (!(thresh > 0.0) || !std::isfinite(thresh)) return LPSIFT_EINVAL;
    if (n > 0 && (!xyA || !xyB || !mask)) return LPSIFT_EINVAL;
    if (n_iter > 0 && !samples) return LPSIFT_EINVAL;
    if (n >= 4)
        for (int64_t k = 0; k < 4 * (int64_t)n_iter; ++k)
            if (samples[k] < 0 || (int64_t)samples[k] >= n) return LPSIFT_EINVAL;

    std::memset(H, 0, 9 * sizeof(double));
    if (n > 0) std::memset(mask, 0, (size_t)n);
    *n_inliers = 0;
    *best_iter = -1;
    if (n < 4) return LPSIFT_OK;

    int64_t best_cnt = -1;
    double best_H[9];
    for (int32_t it = 0; it < n_iter; ++it) {
        int64_t idx[4];
        for (int k = 0; k < 4; ++k) idx[k] = samples[4 * it + k];
        if (degenerate(xyA, idx) || degenerate(xyB, idx)) continue;
        double G[9];
        if (!dlt(xyA, xyB, idx, 4, G)) continue;
        int64_t cnt = 0;
        for (int64_t i = 0; i < n; ++i) cnt += inlier(G, xyA, xyB, i, thresh);
        if (cnt > best_cnt) {
            best_cnt = cnt;
            *best_iter = it;
            std::memcpy(best_H, G, sizeof G);
        }
    }
    if (*best_iter < 0) return LPSIFT_OK;

    std::vector<int64_t> in;
    for (int64_t i = 0; i < n; ++i)
        if (inlier(best_H, xyA, xyB, i, thresh)) in.push_back(i);
    double F[9];
    if (!(in.size() >= 4 && dlt(xyA, xyB, in.data(), (int64_t)in.size(), F)))
        std::memcpy(F, best_H, sizeof F);
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        mask[i] = inlier(F, xyA, xyB, i, thresh) ? 1 : 0;
        cnt += mask[i];
    }
    std::memcpy(H, F, sizeof F);
    *n_inliers = cnt;
    return LPSIFT_OK;
}

extern "C" int lpsift_refine_host(const double* xyA, const double* xyB, int64_t n, double thresh,
                                  int32_t max_rounds, double* H, uint8_t* mask,
                                  int64_t* n_inliers, int32_t* rounds)
{
    if (n < 0 || !H || !n_inliers || !rounds) return LPSIFT_EINVAL;
    if (!(thresh > 0.0) || !std::isfinite(thresh)) return LPSIFT_EINVAL;
    if (max_rounds < 0 || max_rounds > 1000) return LPSIFT_EINVAL;
    if (n > 0 && (!xyA || !xyB || !mask)) return LPSIFT_EINVAL;
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(H[i])) return LPSIFT_EINVAL;

    // inliers of the starting H
    std::vector<int64_t> in;
    for (int64_t i = 0; i < n; ++i) {
        mask[i] = inlier(H, xyA, xyB, i, thresh) ? 1 : 0;
        if (mask[i]) in.push_back(i);
    }
    int32_t r = 0;
    while (r < max_rounds && in.size() >= 4) {
        double F[9];
        if (!dlt(xyA, xyB, in.data(), (int64_t)in.size(), F)) break;
        ++r;
        std::memcpy(H, F, sizeof F);
        // the inlier set of the new H; stop once it equals the one it was fitted to
        std::vector<int64_t> next;
        bool same = true;
        for (int64_t i = 0; i < n; ++i) {
            const uint8_t m = inlier(H, xyA, xyB, i, thresh) ? 1 : 0;
            same = same && (m == mask[i]);
            mask[i] = m;
            if (m) next.push_back(i);
        }
        in.swap(next);
        if (same) break;
    }
    *n_inliers = (int64_t)in.size();
    *rounds = r;
    return LPSIFT_OK;
}
