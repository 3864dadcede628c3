/*
 * FP64 CPU oracle of the LP-SIFT hot path (Li, Wang, Zhao, Zhao:
 * "Local-peak scale-invariant feature transform for fast and random image
 * stitching").
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes or
 * calls this file; only the tests, the smoke check and the CPU baseline of the
 * benchmark load it. It is deliberately plain: every window is scanned pixel by
 * pixel, every descriptor is accumulated visit by visit, every query is
 * compared with every candidate. Outer loops over independent outputs carry an
 * OpenMP pragma; nothing else is reordered.
 *
 * Readings of passages the paper leaves open (each is listed in the design
 * notes of the repository with its justification):
 *  - Eq. 1 ramp: alpha is taken as infinitesimal, so the ramp only breaks ties
 *    between equal intensities, in favour of the larger raster index for a
 *    maximum and the smaller one for a minimum. Gradients use the raw image.
 *  - Eq. 2 windows: L x L tiles from the origin, partial tiles at the right and
 *    bottom edges clipped and kept; one maximum and one minimum per tile.
 *  - Eq. 3-4: beta = beta0 (L/Lmax)^(-1/2), w_s = beta L, w = d w_s; the sign of
 *    the exponent in Eq. 4 is read as +1/2 (so that w <= L for every L), which
 *    makes beta0 = (1/d) sqrt(Lmin/Lmax) the largest admissible value.
 *  - Eq. 5: a is the row difference, b the column difference (no 1/2 factor);
 *    the orientation is the full-circle angle atan2(a, b).
 *  - Orientation (not given in the method text; rotation invariance is claimed
 *    in Sec. 3.5): a 36-bin histogram of Gaussian-weighted magnitudes over a
 *    disc of radius round(1.5 w_s), sigma w_s/2, linear votes between the two
 *    nearest bins (bin k centred at 10k degrees), one circular [1 4 6 4 1]/16
 *    smoothing, argmax (lowest bin on ties), parabolic peak refinement.
 *  - Descriptor (Sec. 2.3, d x d cells x 8 directions): offsets rotated by
 *    -theta0 and divided by w_s, cell centres at -(d-1)/2 .. (d-1)/2, Gaussian
 *    weight with sigma d/2 cells, trilinear votes over two cells per axis and
 *    two of 8 direction bins (bin o centred at 45 o degrees relative to
 *    theta0), normalise, clip at 0.2, normalise again; element index
 *    (cy d + cx) 8 + o.
 *  - Eq. 6 matching: each reference descriptor takes its nearest registered
 *    descriptor (lowest index on ties); it is kept when d1 < ratio * d2 (the
 *    product rounded in FP64, a tie d1 == d2 rejected) and d1 < Delta_s.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static int64_t n_windows(int64_t n, int64_t L) { return (n + L - 1) / L; }

/* Number of keypoints: one maximum and one minimum per window, all scales. */
int64_t oracle_num_keypoints(int32_t h, int32_t w, int32_t n_scales, const int32_t* L)
{
    int64_t n = 0;
    for (int s = 0; s < n_scales; ++s) n += 2 * n_windows(h, L[s]) * n_windows(w, L[s]);
    return n;
}

/* Window extrema (Sec. 2.2, Eq. 2, with the Eq. 1 ramp as a tie-break).
 * Output slot of window (by, bx) at scale s: base_s + 2 (by nbx + bx) for the
 * maximum, +1 for the minimum. contrast = |v - window mean| / 255. */
void oracle_detect(const uint8_t* img, int32_t h, int32_t w, int64_t pitch,
                   int32_t n_scales, const int32_t* L,
                   int32_t* kx, int32_t* ky, int32_t* kscale, int32_t* ktype,
                   int32_t* kvalue, double* kcontrast)
{
    int64_t base = 0;
    for (int s = 0; s < n_scales; ++s) {
        const int64_t Ls = L[s];
        const int64_t nby = n_windows(h, Ls), nbx = n_windows(w, Ls);
#pragma omp parallel for schedule(static)
        for (int64_t wi = 0; wi < nby * nbx; ++wi) {
            const int64_t by = wi / nbx, bx = wi % nbx;
            const int64_t r0 = by * Ls, r1 = (r0 + Ls < h) ? r0 + Ls : h;
            const int64_t c0 = bx * Ls, c1 = (c0 + Ls < w) ? c0 + Ls : w;
            int vmax = -1, vmin = 256;
            int64_t imax = -1, imin = -1, sum = 0;
            for (int64_t r = r0; r < r1; ++r) {
                for (int64_t c = c0; c < c1; ++c) {
                    const int v = img[r * pitch + c];
                    const int64_t idx = r * (int64_t)w + c; /* raster index */
                    sum += v;
                    if (v > vmax || (v == vmax && idx > imax)) { vmax = v; imax = idx; }
                    if (v < vmin || (v == vmin && idx < imin)) { vmin = v; imin = idx; }
                }
            }
            const double n = (double)((r1 - r0) * (c1 - c0));
            const double mean = (double)sum / n;
            const int64_t smax = base + 2 * wi, smin = smax + 1;
            kx[smax] = (int32_t)(imax % w); ky[smax] = (int32_t)(imax / w);
            kscale[smax] = s; ktype[smax] = +1; kvalue[smax] = vmax;
            kcontrast[smax] = fabs((double)vmax - mean) / 255.0;
            kx[smin] = (int32_t)(imin % w); ky[smin] = (int32_t)(imin / w);
            kscale[smin] = s; ktype[smin] = -1; kvalue[smin] = vmin;
            kcontrast[smin] = fabs((double)vmin - mean) / 255.0;
        }
        base += 2 * nby * nbx;
    }
}

/* Subregion side w_s = beta L with beta = beta0 (L/Lmax)^(-1/2)  (Eq. 3). */
double oracle_subregion_side(int32_t L, int32_t Lmax, double beta0)
{
    const double beta = beta0 * pow((double)L / (double)Lmax, -0.5);
    return beta * (double)L;
}

/* Largest beta0 that keeps w = d w_s <= L for every L of the set (Eq. 4). */
double oracle_default_beta0(int32_t d, int32_t Lmin, int32_t Lmax)
{
    return (1.0 / (double)d) * sqrt((double)Lmin / (double)Lmax);
}

/* Image gradient at an interior pixel (Eq. 5): a along rows, b along columns. */
static void gradient(const uint8_t* img, int64_t pitch, int64_t r, int64_t c,
                     double* mag, double* ang)
{
    const double a = (double)img[(r + 1) * pitch + c] - (double)img[(r - 1) * pitch + c];
    const double b = (double)img[r * pitch + c + 1] - (double)img[r * pitch + c - 1];
    *mag = sqrt(a * a + b * b);
    *ang = atan2(a, b); /* (-pi, pi] */
}

static int interior(int64_t r, int64_t c, int32_t h, int32_t w)
{
    return r >= 1 && r <= h - 2 && c >= 1 && c <= w - 2;
}

/* Dominant gradient orientation of each keypoint, in radians.
 * hist_out (optional, [n][36]) receives the smoothed histogram. */
void oracle_orientation(const uint8_t* img, int32_t h, int32_t w, int64_t pitch,
                        int64_t n, const int32_t* kx, const int32_t* ky,
                        const double* ws, double* theta0, double* hist_out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        double hist[36], sm[36];
        memset(hist, 0, sizeof hist);
        const int64_t R = (int64_t)floor(1.5 * ws[k] + 0.5);
        const double sigma = 0.5 * ws[k];
        for (int64_t dy = -R; dy <= R; ++dy) {
            for (int64_t dx = -R; dx <= R; ++dx) {
                if (dx * dx + dy * dy > R * R) continue;
                const int64_t r = ky[k] + dy, c = kx[k] + dx;
                if (!interior(r, c, h, w)) continue;
                double f, th;
                gradient(img, pitch, r, c, &f, &th);
                const double wt = f * exp(-(double)(dx * dx + dy * dy) / (2.0 * sigma * sigma));
                double deg = th * 180.0 / M_PI;
                if (deg < 0.0) deg += 360.0;
                const double t = deg / 10.0;
                const double k0f = floor(t);
                const double fr = t - k0f;
                const int k0 = ((int)k0f) % 36;
                hist[k0] += (1.0 - fr) * wt;
                hist[(k0 + 1) % 36] += fr * wt;
            }
        }
        for (int b = 0; b < 36; ++b) {
            sm[b] = (hist[(b + 34) % 36] + 4.0 * hist[(b + 35) % 36] + 6.0 * hist[b]
                     + 4.0 * hist[(b + 1) % 36] + hist[(b + 2) % 36]) / 16.0;
        }
        int best = 0;
        for (int b = 1; b < 36; ++b)
            if (sm[b] > sm[best]) best = b;
        const double hm = sm[(best + 35) % 36], h0 = sm[best], hp = sm[(best + 1) % 36];
        const double den = hm - 2.0 * h0 + hp;
        const double off = (den != 0.0) ? 0.5 * (hm - hp) / den : 0.0;
        theta0[k] = ((double)best + off) * 10.0 * M_PI / 180.0;
        if (hist_out) memcpy(hist_out + 36 * k, sm, sizeof sm);
    }
}

/* d x d x 8 descriptor of each keypoint at orientation theta0 (Sec. 2.3). */
void oracle_describe(const uint8_t* img, int32_t h, int32_t w, int64_t pitch,
                     int64_t n, const int32_t* kx, const int32_t* ky,
                     const double* ws, const double* theta0, int32_t d,
                     double* desc)
{
    const int nb = d * d * 8;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        double* D = desc + (int64_t)nb * k;
        for (int i = 0; i < nb; ++i) D[i] = 0.0;
        const double half = 0.5 * (double)(d + 1) * ws[k];
        const double R2 = 2.0 * half * half; /* (w_s sqrt(2) (d+1)/2)^2 */
        const int64_t R = (int64_t)floor(sqrt(R2));
        const double ct = cos(theta0[k]), st = sin(theta0[k]);
        const double centre = 0.5 * (double)(d - 1);
        const double sig = 0.5 * (double)d;
        for (int64_t dy = -R; dy <= R; ++dy) {
            for (int64_t dx = -R; dx <= R; ++dx) {
                if ((double)(dx * dx + dy * dy) > R2) continue;
                const int64_t r = ky[k] + dy, c = kx[k] + dx;
                if (!interior(r, c, h, w)) continue;
                double f, th;
                gradient(img, pitch, r, c, &f, &th);
                /* offset rotated by -theta0, in subregion units */
                const double u = (ct * (double)dx + st * (double)dy) / ws[k];
                const double v = (-st * (double)dx + ct * (double)dy) / ws[k];
                const double m = f * exp(-(u * u + v * v) / (2.0 * sig * sig));
                double rel = fmod(th - theta0[k], 2.0 * M_PI);
                if (rel < 0.0) rel += 2.0 * M_PI;
                const double t = rel * 8.0 / (2.0 * M_PI);
                const double cu = u + centre, cv = v + centre;
                const double ix0 = floor(cu), iy0 = floor(cv), io0 = floor(t);
                const double fx = cu - ix0, fy = cv - iy0, fo = t - io0;
                for (int jy = 0; jy < 2; ++jy) {
                    const int iy = (int)iy0 + jy;
                    if (iy < 0 || iy >= d) continue;
                    const double wy = jy ? fy : 1.0 - fy;
                    for (int jx = 0; jx < 2; ++jx) {
                        const int ix = (int)ix0 + jx;
                        if (ix < 0 || ix >= d) continue;
                        const double wx = jx ? fx : 1.0 - fx;
                        for (int jo = 0; jo < 2; ++jo) {
                            const int io = (((int)io0 + jo) % 8 + 8) % 8;
                            const double wo = jo ? fo : 1.0 - fo;
                            D[(iy * d + ix) * 8 + io] += m * wx * wy * wo;
                        }
                    }
                }
            }
        }
        double nrm = 0.0;
        for (int i = 0; i < nb; ++i) nrm += D[i] * D[i];
        nrm = sqrt(nrm);
        if (nrm < 1e-12) nrm = 1e-12;
        for (int i = 0; i < nb; ++i) {
            D[i] /= nrm;
            if (D[i] > 0.2) D[i] = 0.2;
        }
        nrm = 0.0;
        for (int i = 0; i < nb; ++i) nrm += D[i] * D[i];
        nrm = sqrt(nrm);
        if (nrm < 1e-12) nrm = 1e-12;
        for (int i = 0; i < nb; ++i) D[i] /= nrm;
    }
}

/* Nearest-neighbour matching with the distance of Eq. 6 and a ratio test.
 * For every reference row i: j1[i] = argmin_j |A_i - B_j| (lowest j on ties),
 * d1 = that distance, d2 = the second smallest distance over j != j1 (+inf when
 * nB < 2), match[i] = j1 if d1 < ratio * d2 and d1 < abs_thresh, else -1.
 * ratio = +inf leaves the absolute threshold of Eq. 6 alone (no ratio test,
 * so equal d1 and d2 are not rejected). */
void oracle_match(const double* A, int64_t nA, const double* B, int64_t nB, int32_t dim,
                  double ratio, double abs_thresh,
                  int32_t* j1, double* d1, double* d2, int32_t* match)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < nA; ++i) {
        const double* a = A + (int64_t)dim * i;
        double b1 = INFINITY, b2 = INFINITY;
        int64_t jb = -1;
        for (int64_t j = 0; j < nB; ++j) {
            const double* b = B + (int64_t)dim * j;
            double s = 0.0;
            for (int c = 0; c < dim; ++c) {
                const double e = a[c] - b[c];
                s += e * e;
            }
            if (s < b1) { b2 = b1; b1 = s; jb = j; }
            else if (s < b2) { b2 = s; }
        }
        const double e1 = sqrt(b1), e2 = sqrt(b2);
        j1[i] = (int32_t)jb;
        d1[i] = e1;
        d2[i] = e2;
        const int ratio_ok = isinf(ratio) || e1 < ratio * e2;
        match[i] = (jb >= 0 && ratio_ok && e1 < abs_thresh) ? (int32_t)jb : -1;
    }
}

/* Convenience for tests: gradient magnitude and angle at one pixel. */
int oracle_gradient_at(const uint8_t* img, int32_t h, int32_t w, int64_t pitch,
                       int32_t r, int32_t c, double* mag, double* ang)
{
    if (!interior(r, c, h, w)) return -1;
    gradient(img, pitch, r, c, mag, ang);
    return 0;
}
