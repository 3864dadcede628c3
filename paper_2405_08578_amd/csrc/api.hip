// C-ABI entry points of liblpsift: argument validation on the host, then the
// launchers of detect.hip, describe.hip and match.hip. No call allocates device
// memory, synchronises, throws or aborts.
#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "internal.h"

namespace lpsift {

int make_geometry(const lpsift_params* p, Geometry* g)
{
    if (!p || !g) return LPSIFT_EINVAL;
    if (p->n_scales < 1 || p->n_scales > LPSIFT_MAX_SCALES) return LPSIFT_EINVAL;
    if (p->d < 1 || p->d > 16) return LPSIFT_EINVAL;
    if (!(p->beta0 <= 0.0f || std::isfinite(p->beta0))) return LPSIFT_EINVAL;
    if (std::isnan(p->beta0)) return LPSIFT_EINVAL;
    for (int s = 0; s < p->n_scales; ++s) {
        if (p->L[s] < 4 || p->L[s] > 65536) return LPSIFT_EINVAL;
        if (s > 0 && p->L[s] <= p->L[s - 1]) return LPSIFT_EINVAL;
    }
    if (p->d != 4) return LPSIFT_EUNSUPPORTED;
    const int Lmin = p->L[0], Lmax = p->L[p->n_scales - 1];

    // Eq. 3-4: beta = beta0 (L/Lmax)^(-1/2), w_s = beta L; default beta0 is the
    // largest value with w = d w_s <= L at every scale
    const double beta0 = (p->beta0 > 0.0f) ? (double)p->beta0
                                            : (1.0 / p->d) * std::sqrt((double)Lmin / (double)Lmax);
    const double log2e = 1.4426950408889634;
    g->n_scales = p->n_scales;
    int entries = 0;
    for (int s = 0; s < p->n_scales; ++s) {
        const double L = p->L[s];
        const double ws = beta0 * std::pow(L / (double)Lmax, -0.5) * L;
        const double half = 0.5 * (p->d + 1) * ws;
        const double r2d = 2.0 * half * half;
        const double ro = std::floor(1.5 * ws + 0.5);
        if (!(ws > 0.0) || r2d > 4.0e6) return LPSIFT_EINVAL;   // support radius <= 2000 px
        ScaleGeom& G = g->s[s];
        g->L[s] = p->L[s];
        G.ws = (float)ws;
        G.inv_ws = (float)(1.0 / ws);
        G.k_orient = (float)(-log2e / (2.0 * (0.5 * ws) * (0.5 * ws)));
        G.k_desc = (float)(-log2e / (2.0 * (0.5 * p->d) * (0.5 * p->d) * ws * ws));
        G.r2_orient = (int)(ro * ro);
        G.r2_desc = (int)std::floor(r2d);
        G.off_orient = entries;
        G.n_orient = disc_count(G.r2_orient);
        entries += G.n_orient;
        G.off_desc = entries;
        G.n_desc = disc_count(G.r2_desc);
        G.n_buckets = G.n_desc <= kBucketMaxEntries ? kDescBuckets : 1;
        G.cap_desc = G.n_desc;
        // Descriptor votes are 32-bit fixed point. A bin takes from every
        // pixel of its cell's support (a square of side 2 w_s) at most
        // 362 (> 255 sqrt 2, the largest gradient) times the bilinear cell
        // weight (the Gaussian and direction weights are <= 1); over the
        // integer pixels the bilinear weights of one cell sum to less than
        // w_s^2 + 4.5 w_s + 1 at any angle and position (the weight is
        // log-concave, so each row and then the rows sum to at most their
        // integral plus their largest term: w_s^2 + 3 sqrt 2 w_s + 1). Rounding adds at most 1/2 per
        // vote, one vote per support pixel, < (2 sqrt 2 w_s + 2)^2 of them.
        // The scale keeps the bound below 0.98 of 2^32.
        const double cell_sum = ws * ws + 4.5 * ws + 1.0;
        const double n_votes = (2.0 * std::sqrt(2.0) * ws + 2.0) * (2.0 * std::sqrt(2.0) * ws + 2.0);
        const double dscale = (0.98 * 4294967296.0 - 0.5 * n_votes) / (362.0 * cell_sum);
        G.dscale = (float)dscale;
        G.dinv = (float)(1.0 / (double)G.dscale);
        entries += G.n_buckets * G.cap_desc;
    }
    g->table_entries = entries;
    return LPSIFT_OK;
}

}  // namespace lpsift

using namespace lpsift;

namespace {

int check_images(const lpsift_image* imgs, int32_t n)
{
    if (!imgs || n < 1) return LPSIFT_EINVAL;
    for (int i = 0; i < n; ++i) {
        const lpsift_image& im = imgs[i];
        if (!im.data || im.height < 1 || im.width < 1 || im.pitch < im.width) return LPSIFT_EINVAL;
        if (im.height > 32767 || im.width > 32767) return LPSIFT_EINVAL;
    }
    return LPSIFT_OK;
}

int check_keypoints(const lpsift_image* imgs, int32_t n, const lpsift_keypoints* kps,
                    const lpsift_params* p)
{
    if (!kps) return LPSIFT_EINVAL;
    for (int i = 0; i < n; ++i) {
        const lpsift_keypoints& k = kps[i];
        if (!k.x || !k.y || !k.scale || !k.type || !k.value || !k.contrast) return LPSIFT_EINVAL;
        if (k.capacity < lpsift_num_keypoints(imgs[i].height, imgs[i].width, p))
            return LPSIFT_ECAPACITY;
    }
    return LPSIFT_OK;
}

}  // namespace

extern "C" {

int lpsift_version(void) { return 100; }

const char* lpsift_status_string(int status)
{
    switch (status) {
    case LPSIFT_OK: return "ok";
    case LPSIFT_EINVAL: return "invalid argument";
    case LPSIFT_ECAPACITY: return "buffer too small";
    case LPSIFT_EHIP: return "HIP runtime or launch failure";
    case LPSIFT_EUNSUPPORTED: return "not supported on the GPU path";
    default: return "unknown status";
    }
}

int64_t lpsift_num_keypoints(int32_t height, int32_t width, const lpsift_params* p)
{
    if (!p || height < 1 || width < 1 || p->n_scales < 1 || p->n_scales > LPSIFT_MAX_SCALES)
        return -1;
    int64_t n = 0;
    for (int s = 0; s < p->n_scales; ++s) {
        if (p->L[s] < 1) return -1;
        n += 2 * n_windows(height, p->L[s]) * n_windows(width, p->L[s]);
    }
    return n;
}

int lpsift_detect(const lpsift_image* imgs, int32_t n, const lpsift_params* p,
                  const lpsift_keypoints* out, void* stream)
{
    Geometry g;
    int st = make_geometry(p, &g);
    if (st == LPSIFT_EINVAL) return st;
    const int sti = check_images(imgs, n);
    if (sti != LPSIFT_OK) return sti;
    const int stk = check_keypoints(imgs, n, out, p);
    if (stk != LPSIFT_OK) return stk;
    if (st != LPSIFT_OK) return st;
    return launch_detect(imgs, n, g, out, static_cast<hipStream_t>(stream));
}

size_t lpsift_describe_workspace_size(const lpsift_image* imgs, int32_t n, const lpsift_params* p)
{
    Geometry g;
    if (make_geometry(p, &g) != LPSIFT_OK || check_images(imgs, n) != LPSIFT_OK) return 0;
    return describe_workspace_bytes(imgs, n, g);
}

int lpsift_describe(const lpsift_image* imgs, int32_t n, const lpsift_keypoints* kps,
                    const lpsift_params* p, void* workspace, size_t ws_bytes,
                    float* const* theta, float* const* desc, void* stream)
{
    Geometry g;
    int st = make_geometry(p, &g);
    if (st == LPSIFT_EINVAL) return st;
    const int sti = check_images(imgs, n);
    if (sti != LPSIFT_OK) return sti;
    if (!theta || !desc || !workspace) return LPSIFT_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!theta[i] || !desc[i]) return LPSIFT_EINVAL;
    const int stk = check_keypoints(imgs, n, kps, p);
    if (stk != LPSIFT_OK) return stk;
    if (st != LPSIFT_OK) return st;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return LPSIFT_EINVAL;
    if (ws_bytes < describe_workspace_bytes(imgs, n, g)) return LPSIFT_ECAPACITY;
    return launch_describe(imgs, n, kps, g, workspace, theta, desc, nullptr, nullptr,
                           static_cast<hipStream_t>(stream));
}

int lpsift_describe_selected(const lpsift_image* imgs, int32_t n, const lpsift_keypoints* kps,
                             const lpsift_params* p, const int32_t* const* sel,
                             const int64_t* n_sel, void* workspace, size_t ws_bytes,
                             float* const* theta, float* const* desc, void* stream)
{
    Geometry g;
    int st = make_geometry(p, &g);
    if (st == LPSIFT_EINVAL) return st;
    const int sti = check_images(imgs, n);
    if (sti != LPSIFT_OK) return sti;
    if (!theta || !desc || !workspace || !sel || !n_sel) return LPSIFT_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (n_sel[i] < 0 || n_sel[i] > INT32_MAX) return LPSIFT_EINVAL;
        if (n_sel[i] > 0 && (!sel[i] || !theta[i] || !desc[i])) return LPSIFT_EINVAL;
    }
    const int stk = check_keypoints(imgs, n, kps, p);
    if (stk != LPSIFT_OK) return stk;
    if (st != LPSIFT_OK) return st;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return LPSIFT_EINVAL;
    if (ws_bytes < describe_workspace_bytes(imgs, n, g)) return LPSIFT_ECAPACITY;
    return launch_describe(imgs, n, kps, g, workspace, theta, desc, sel, n_sel,
                           static_cast<hipStream_t>(stream));
}

size_t lpsift_describe_multi_workspace_size(const lpsift_image* imgs, int32_t n,
                                            const lpsift_params* p)
{
    Geometry g;
    if (make_geometry(p, &g) != LPSIFT_OK || check_images(imgs, n) != LPSIFT_OK) return 0;
    return describe_multi_workspace_bytes(imgs, n, g);
}

int lpsift_describe_multi(const lpsift_image* imgs, int32_t n, const lpsift_keypoints* kps,
                          const lpsift_params* p, int32_t max_orient, float peak_ratio,
                          void* workspace, size_t ws_bytes, int32_t* const* rows,
                          float* const* theta, float* const* desc, int64_t* n_rows, void* stream)
{
    Geometry g;
    int st = make_geometry(p, &g);
    if (st == LPSIFT_EINVAL) return st;
    const int sti = check_images(imgs, n);
    if (sti != LPSIFT_OK) return sti;
    if (max_orient < 1 || max_orient > 4 || !(peak_ratio > 0.0f) || !(peak_ratio <= 1.0f))
        return LPSIFT_EINVAL;
    if (!rows || !theta || !desc || !n_rows || !workspace) return LPSIFT_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!rows[i] || !theta[i] || !desc[i]) return LPSIFT_EINVAL;
    if (reinterpret_cast<uintptr_t>(n_rows) & 7u) return LPSIFT_EINVAL;
    const int stk = check_keypoints(imgs, n, kps, p);
    if (stk != LPSIFT_OK) return stk;
    if (st != LPSIFT_OK) return st;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return LPSIFT_EINVAL;
    if (ws_bytes < describe_multi_workspace_bytes(imgs, n, g)) return LPSIFT_ECAPACITY;
    const MultiSpec ms{max_orient, peak_ratio, rows, n_rows};
    return launch_describe_multi(imgs, n, kps, g, workspace, ms, theta, desc,
                                 static_cast<hipStream_t>(stream));
}

// normalised log2 window size per scale (feature 256 of the scorer)
static void scale_features(const lpsift_params* p, float* out)
{
    const double l0 = std::log2((double)p->L[0]);
    const double l1 = std::log2((double)p->L[p->n_scales - 1]);
    for (int s = 0; s < LPSIFT_MAX_SCALES; ++s) {
        out[s] = 0.0f;
        if (s < p->n_scales && p->n_scales > 1)
            out[s] = (float)((std::log2((double)p->L[s]) - l0) / (l1 - l0));
    }
}

int lpsift_score(const lpsift_image* imgs, int32_t n, const lpsift_keypoints* kps,
                 const lpsift_params* p, const float* weights, float* const* scores, void* stream)
{
    Geometry g;
    int st = make_geometry(p, &g);
    if (st == LPSIFT_EINVAL) return st;
    const int sti = check_images(imgs, n);
    if (sti != LPSIFT_OK) return sti;
    if (!weights || !scores) return LPSIFT_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!scores[i]) return LPSIFT_EINVAL;
    const int stk = check_keypoints(imgs, n, kps, p);
    if (stk != LPSIFT_OK) return stk;
    if (st != LPSIFT_OK) return st;
    for (int b0 = 0; b0 < n; b0 += kMaxBatch) {
        const int nb = (n - b0 < kMaxBatch) ? n - b0 : kMaxBatch;
        ScoreArgs a{};
        a.n_images = nb;
        scale_features(p, a.sfeat);
        for (int i = 0; i < nb; ++i) {
            const lpsift_image& im = imgs[b0 + i];
            const lpsift_keypoints& k = kps[b0 + i];
            a.img[i] = ScoreImg{im.data, im.pitch, im.height, im.width, k.x, k.y, k.scale,
                                k.contrast, scores[b0 + i],
                                lpsift_num_keypoints(im.height, im.width, p)};
        }
        const int r = launch_score(a, weights, static_cast<hipStream_t>(stream));
        if (r != LPSIFT_OK) return r;
    }
    return LPSIFT_OK;
}

int lpsift_prune(const float* const* scores, const int64_t* n, const int64_t* k,
                 int32_t n_images, int32_t* const* sel, void* stream)
{
    if (!scores || !n || !k || !sel || n_images < 1) return LPSIFT_EINVAL;
    for (int i = 0; i < n_images; ++i) {
        if (n[i] < 0 || n[i] > INT32_MAX || k[i] < 0 || k[i] > n[i]) return LPSIFT_EINVAL;
        if (n[i] > 0 && !scores[i]) return LPSIFT_EINVAL;
        if ((reinterpret_cast<uintptr_t>(scores[i]) & 15u) != 0) return LPSIFT_EINVAL;
        if (k[i] > 0 && !sel[i]) return LPSIFT_EINVAL;
    }
    for (int b0 = 0; b0 < n_images; b0 += kMaxBatch) {
        const int nb = (n_images - b0 < kMaxBatch) ? n_images - b0 : kMaxBatch;
        PruneArgs a{};
        a.n_images = nb;
        for (int i = 0; i < nb; ++i)
            a.img[i] = PruneImg{scores[b0 + i], n[b0 + i], k[b0 + i], sel[b0 + i]};
        const int r = launch_prune(a, static_cast<hipStream_t>(stream));
        if (r != LPSIFT_OK) return r;
    }
    return LPSIFT_OK;
}

int lpsift_scorer_gather(const lpsift_image* imgs, int32_t n, const lpsift_keypoints* kps,
                         const lpsift_params* p, const int32_t* const* sel, const int64_t* n_sel,
                         uint8_t* const* patches, float* const* extra, void* stream)
{
    Geometry g;
    const int st = make_geometry(p, &g);
    if (st == LPSIFT_EINVAL) return st;
    const int sti = check_images(imgs, n);
    if (sti != LPSIFT_OK) return sti;
    if (!patches || !extra) return LPSIFT_EINVAL;
    const int stk = check_keypoints(imgs, n, kps, p);
    if (stk != LPSIFT_OK) return stk;
    for (int i = 0; i < n; ++i) {
        const int64_t cnt = sel ? (n_sel ? n_sel[i] : -1)
                                : lpsift_num_keypoints(imgs[i].height, imgs[i].width, p);
        if (cnt < 0 || cnt > INT32_MAX) return LPSIFT_EINVAL;
        if (cnt > 0 && (!patches[i] || !extra[i] || (sel && !sel[i]))) return LPSIFT_EINVAL;
        if ((reinterpret_cast<uintptr_t>(patches[i]) & 3u) != 0) return LPSIFT_EINVAL;
    }
    for (int b0 = 0; b0 < n; b0 += kMaxBatch) {
        const int nb = (n - b0 < kMaxBatch) ? n - b0 : kMaxBatch;
        GatherArgs a{};
        a.n_images = nb;
        scale_features(p, a.sfeat);
        for (int i = 0; i < nb; ++i) {
            const lpsift_image& im = imgs[b0 + i];
            const lpsift_keypoints& k = kps[b0 + i];
            const int64_t nkp = lpsift_num_keypoints(im.height, im.width, p);
            a.img[i] = GatherImg{im.data, im.pitch, im.height, im.width, k.x, k.y, k.scale,
                                 k.contrast, sel ? sel[b0 + i] : nullptr,
                                 sel ? n_sel[b0 + i] : nkp, nkp, patches[b0 + i], extra[b0 + i]};
        }
        const int r = launch_gather(a, static_cast<hipStream_t>(stream));
        if (r != LPSIFT_OK) return r;
    }
    return LPSIFT_OK;
}

size_t lpsift_scorer_train_workspace_size(int64_t batch)
{
    return batch < 1 ? 0 : train_workspace_bytes(batch);
}

int lpsift_scorer_train_step(const uint8_t* patches, const float* extra, const float* labels,
                             const float* cweight, int64_t batch, float* weights, float* adam_m,
                             float* adam_v, int64_t step, float lr, void* workspace,
                             size_t ws_bytes, float* loss, void* stream)
{
    if (!patches || !extra || !labels || !cweight || !weights || !adam_m || !adam_v ||
        !workspace || batch < 1 || batch > (int64_t)1 << 26 || step < 1 ||
        !(lr > 0.0f) || !std::isfinite(lr))
        return LPSIFT_EINVAL;
    if (ws_bytes < train_workspace_bytes(batch)) return LPSIFT_ECAPACITY;
    TrainArgs a{patches, extra, labels, cweight, batch, weights, adam_m, adam_v,
                static_cast<float*>(workspace), loss, step, lr};
    return launch_train(a, static_cast<hipStream_t>(stream));
}

static int check_match_params(const lpsift_match_params* mp)
{
    if (!mp) return LPSIFT_EINVAL;
    if (!(mp->ratio > 0.0)) return LPSIFT_EINVAL;      // +inf: no ratio test (Eq. 6 alone)
    if (std::isnan(mp->abs_thresh) || !(mp->abs_thresh > 0.0f)) return LPSIFT_EINVAL;
    if (mp->b_chunks < 0 || mp->b_chunks > 16) return LPSIFT_EINVAL;
    if (mp->qblock_waves != 0 && mp->qblock_waves != 2 && mp->qblock_waves != 4 &&
        mp->qblock_waves != 8)
        return LPSIFT_EINVAL;
    if (mp->precision < 0 || mp->precision > 3) return LPSIFT_EINVAL;
    // the ratio test needs a second rescored candidate: topk 2 .. 8
    if (mp->topk != 0 && (mp->topk < 2 || mp->topk > 8)) return LPSIFT_EINVAL;
    if (mp->topk != 0 && (mp->precision == 0 || mp->precision == 3)) return LPSIFT_EINVAL;
    return LPSIFT_OK;
}

size_t lpsift_match_workspace_size(const int64_t* nA, const int64_t* nB, int32_t n_pairs,
                                   const lpsift_match_params* mp)
{
    if (!nA || !nB || n_pairs < 1 || check_match_params(mp) != LPSIFT_OK) return 0;
    size_t b = 0;
    for (int i = 0; i < n_pairs; ++i) {
        if (nA[i] < 0 || nB[i] < 0) return 0;
        b += align_up(match_workspace_bytes(nA[i], nB[i], mp), 256);
    }
    return b;
}

}  // extern "C"

// Everything lpsift_match checks except the workspace size.
static int check_match_call(const float* const* descA, const int64_t* nA,
                            const float* const* descB, const int64_t* nB, int32_t n_pairs,
                            const lpsift_match_params* mp, int32_t* const* match,
                            float* const* d1, float* const* d2)
{
    const int sp = check_match_params(mp);
    if (sp != LPSIFT_OK) return sp;
    if (!descA || !nA || !descB || !nB || n_pairs < 1 || !match || !d1 || !d2)
        return LPSIFT_EINVAL;
    for (int i = 0; i < n_pairs; ++i) {
        if (nA[i] < 0 || nB[i] < 0 || nA[i] > INT32_MAX || nB[i] > INT32_MAX) return LPSIFT_EINVAL;
        if (nA[i] > 0 && (!descA[i] || !match[i] || !d1[i] || !d2[i])) return LPSIFT_EINVAL;
        if (nB[i] > 0 && !descB[i]) return LPSIFT_EINVAL;
        if ((reinterpret_cast<uintptr_t>(descA[i]) | reinterpret_cast<uintptr_t>(descB[i])) & 15u)
            return LPSIFT_EINVAL;
    }
    return LPSIFT_OK;
}

// Splits a validated call's workspace into per-pair slices and launches.
static int launch_match_call(const float* const* descA, const int64_t* nA,
                             const float* const* descB, const int64_t* nB, int32_t n_pairs,
                             const lpsift_match_params* mp, char* ws, int32_t* const* match,
                             float* const* d1, float* const* d2, hipStream_t stream)
{
    std::vector<MatchPairIO> io(n_pairs);
    for (int i = 0; i < n_pairs; ++i) {
        io[i] = MatchPairIO{descA[i], nA[i], descB[i], nB[i], ws, match[i], d1[i], d2[i]};
        ws += align_up(match_workspace_bytes(nA[i], nB[i], mp), 256);
    }
    return launch_match_pairs(io.data(), n_pairs, mp, stream);
}

// The fixed device scratch of lpsift_match_noalloc. Each device holds its own
// copy (placed when this code object is loaded there) until the process
// ends. In host code `scratch` names a host-side stand-in, never device
// memory: the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[LPSIFT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

// Device address of the scratch array on the current device, looked up on the
// first call made with that device current.
static int scratch_address(hipStream_t stream, char** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LPSIFT_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return LPSIFT_EUNSUPPORTED;
    if (stream) {      // the array used is the current device's: the stream must be on it
        hipDevice_t sd = -1;
        if (hipStreamGetDevice(stream, &sd) != hipSuccess) return LPSIFT_EHIP;
        if (sd != dev) return LPSIFT_EINVAL;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LPSIFT_EHIP;
        g_scratch_dev[dev] = p;
    }
    *out = static_cast<char*>(g_scratch_dev[dev]);
    return LPSIFT_OK;
}

extern "C" {

int lpsift_match(const float* const* descA, const int64_t* nA, const float* const* descB,
                 const int64_t* nB, int32_t n_pairs, const lpsift_match_params* mp,
                 void* workspace, size_t ws_bytes, int32_t* const* match, float* const* d1,
                 float* const* d2, void* stream)
{
    const int sc = check_match_call(descA, nA, descB, nB, n_pairs, mp, match, d1, d2);
    if (sc != LPSIFT_OK) return sc;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return LPSIFT_EINVAL;
    if (ws_bytes < lpsift_match_workspace_size(nA, nB, n_pairs, mp)) return LPSIFT_ECAPACITY;
    return launch_match_call(descA, nA, descB, nB, n_pairs, mp, static_cast<char*>(workspace),
                             match, d1, d2, static_cast<hipStream_t>(stream));
}

int lpsift_match_noalloc(const float* const* descA, const int64_t* nA, const float* const* descB,
                         const int64_t* nB, int32_t n_pairs, const lpsift_match_params* mp,
                         int32_t* const* match, float* const* d1, float* const* d2, void* stream)
{
    const int sc = check_match_call(descA, nA, descB, nB, n_pairs, mp, match, d1, d2);
    if (sc != LPSIFT_OK) return sc;
    if (lpsift_match_workspace_size(nA, nB, n_pairs, mp) > (size_t)LPSIFT_NOALLOC_SCRATCH_BYTES)
        return LPSIFT_ECAPACITY;
    char* ws = nullptr;
    const int sa = scratch_address(static_cast<hipStream_t>(stream), &ws);
    if (sa != LPSIFT_OK) return sa;
    // every kernel of the call initialises the workspace words it reads
    // (counters by a fill kernel), so the previous call's contents do not matter
    return launch_match_call(descA, nA, descB, nB, n_pairs, mp, ws, match, d1, d2,
                             static_cast<hipStream_t>(stream));
}

int lpsift_quantize_lowp(const float* desc, int64_t n, int32_t precision, void* q, float* scale,
                        void* stream)
{
    if (n < 0 || n > INT32_MAX) return LPSIFT_EINVAL;
    if (precision != 1 && precision != 2) return LPSIFT_EINVAL;
    if (n > 0 && (!desc || !q || (precision == 2 && !scale))) return LPSIFT_EINVAL;
    const uintptr_t qa = reinterpret_cast<uintptr_t>(q);
    if ((reinterpret_cast<uintptr_t>(desc) & 15u) || (qa & (precision == 1 ? 15u : 7u)) ||
        (reinterpret_cast<uintptr_t>(scale) & 3u))
        return LPSIFT_EINVAL;
    return launch_quantize_lowp(desc, n, precision, q, scale, static_cast<hipStream_t>(stream));
}

int lpsift_quantize_u8(const float* desc, int64_t n, uint8_t* q, void* stream)
{
    if (n < 0 || n > INT32_MAX) return LPSIFT_EINVAL;
    if (n > 0 && (!desc || !q)) return LPSIFT_EINVAL;
    if ((reinterpret_cast<uintptr_t>(desc) & 15u) || (reinterpret_cast<uintptr_t>(q) & 3u))
        return LPSIFT_EINVAL;
    return launch_quantize_u8(desc, n, q, static_cast<hipStream_t>(stream));
}

size_t lpsift_match_u8_workspace_size(int64_t nA, int64_t nB)
{
    if (nA < 0 || nB < 0 || nA > INT32_MAX || nB > INT32_MAX) return 0;
    return match_u8_workspace_bytes(nA, nB);
}

int lpsift_match_u8(const uint8_t* qA, int64_t nA, const uint8_t* qB, int64_t nB, double ratio,
                    float abs_thresh, void* workspace, size_t ws_bytes, int32_t* match,
                    float* d1, float* d2, void* stream)
{
    if (nA < 0 || nB < 0 || nA > INT32_MAX || nB > INT32_MAX) return LPSIFT_EINVAL;
    if (!(ratio > 0.0) || std::isnan(abs_thresh) || !(abs_thresh > 0.0f)) return LPSIFT_EINVAL;
    if (nA > 0 && (!qA || !match || !d1 || !d2)) return LPSIFT_EINVAL;
    if (nB > 0 && !qB) return LPSIFT_EINVAL;
    if ((reinterpret_cast<uintptr_t>(qA) | reinterpret_cast<uintptr_t>(qB)) & 15u)
        return LPSIFT_EINVAL;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return LPSIFT_EINVAL;
    if (ws_bytes < match_u8_workspace_bytes(nA, nB)) return LPSIFT_ECAPACITY;
    return launch_match_u8(qA, nA, qB, nB, ratio, abs_thresh, workspace, match, d1, d2,
                           static_cast<hipStream_t>(stream));
}

int64_t lpsift_probe_out_size(void)
{
    return probe_out_floats();
}

double lpsift_probe_ops(int32_t kind, int64_t iters)
{
    if (kind < LPSIFT_PROBE_MFMA_F32 || kind > LPSIFT_PROBE_MFMA_I8 || iters < 1) return 0.0;
    return probe_ops(kind, iters);
}

int lpsift_probe(int32_t kind, int64_t iters, float* out, void* stream)
{
    if (kind < LPSIFT_PROBE_MFMA_F32 || kind > LPSIFT_PROBE_MFMA_I8) return LPSIFT_EINVAL;
    if (iters < 1 || iters > (1 << 24) || !out) return LPSIFT_EINVAL;
    return launch_probe(kind, iters, out, static_cast<hipStream_t>(stream));
}

int lpsift_warp_blend(const lpsift_image* imgs, int32_t n, const double* G, double x0,
                      double y0, int32_t out_w, int32_t out_h, float* canvas, uint8_t* count,
                      void* stream)
{
    if (n < 1 || n > kWarpMax || !G) return LPSIFT_EINVAL;
    const int sti = check_images(imgs, n);
    if (sti != LPSIFT_OK) return sti;
    if (out_w < 0 || out_h < 0 || (int64_t)out_w * out_h >= ((int64_t)1 << 31)) return LPSIFT_EINVAL;
    if (!std::isfinite(x0) || !std::isfinite(y0)) return LPSIFT_EINVAL;
    if ((int64_t)out_w * out_h > 0 && !canvas) return LPSIFT_EINVAL;
    WarpArgs a{};
    a.n = n;
    a.W = out_w;
    a.H = out_h;
    a.x0 = x0;
    a.y0 = y0;
    a.canvas = canvas;
    a.count = count;
    for (int k = 0; k < n; ++k) {
        const double* g = G + 9 * k;
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(g[i])) return LPSIFT_EINVAL;
        // inverse by the adjugate
        const double c00 = g[4] * g[8] - g[5] * g[7], c01 = g[5] * g[6] - g[3] * g[8],
                     c02 = g[3] * g[7] - g[4] * g[6];
        const double det = g[0] * c00 + g[1] * c01 + g[2] * c02;
        double scale = 0.0;
        for (int i = 0; i < 9; ++i) scale = std::fmax(scale, std::fabs(g[i]));
        if (!(std::fabs(det) > 1e-12 * scale * scale * scale)) return LPSIFT_EINVAL;
        const double id = 1.0 / det;
        WarpImg& w = a.img[k];
        w.hi[0] = c00 * id;
        w.hi[1] = (g[2] * g[7] - g[1] * g[8]) * id;
        w.hi[2] = (g[1] * g[5] - g[2] * g[4]) * id;
        w.hi[3] = c01 * id;
        w.hi[4] = (g[0] * g[8] - g[2] * g[6]) * id;
        w.hi[5] = (g[2] * g[3] - g[0] * g[5]) * id;
        w.hi[6] = c02 * id;
        w.hi[7] = (g[1] * g[6] - g[0] * g[7]) * id;
        w.hi[8] = (g[0] * g[4] - g[1] * g[3]) * id;
        w.data = static_cast<const uint8_t*>(imgs[k].data);
        w.pitch = imgs[k].pitch;
        w.h = imgs[k].height;
        w.w = imgs[k].width;
        // canvas box of the mapped corners; the whole canvas when the map's
        // denominator changes sign over the image (the image then reaches the
        // line at infinity and its footprint is not bounded by the corners)
        const double cx[4] = {0.0, (double)(w.w - 1), (double)(w.w - 1), 0.0};
        const double cy[4] = {0.0, 0.0, (double)(w.h - 1), (double)(w.h - 1)};
        double lo_x = INFINITY, hi_x = -INFINITY, lo_y = INFINITY, hi_y = -INFINITY;
        int pos = 0, neg = 0;
        for (int c = 0; c < 4; ++c) {
            const double z = g[6] * cx[c] + g[7] * cy[c] + g[8];
            pos += z > 0.0;
            neg += z < 0.0;
            const double X = (g[0] * cx[c] + g[1] * cy[c] + g[2]) / z;
            const double Y = (g[3] * cx[c] + g[4] * cy[c] + g[5]) / z;
            lo_x = std::fmin(lo_x, X);
            hi_x = std::fmax(hi_x, X);
            lo_y = std::fmin(lo_y, Y);
            hi_y = std::fmax(hi_y, Y);
        }
        if (pos == 4 || neg == 4) {
            const double bx0 = std::floor(lo_x - x0) - 1.0, bx1 = std::floor(hi_x - x0) + 2.0;
            const double by0 = std::floor(lo_y - y0) - 1.0, by1 = std::floor(hi_y - y0) + 2.0;
            w.bx0 = (int32_t)std::fmax(0.0, std::fmin((double)out_w, bx0));
            w.bx1 = (int32_t)std::fmax(0.0, std::fmin((double)out_w, bx1));
            w.by0 = (int32_t)std::fmax(0.0, std::fmin((double)out_h, by0));
            w.by1 = (int32_t)std::fmax(0.0, std::fmin((double)out_h, by1));
        } else {
            w.bx0 = 0;
            w.by0 = 0;
            w.bx1 = out_w;
            w.by1 = out_h;
        }
    }
    return launch_warp_blend(a, static_cast<hipStream_t>(stream));
}

size_t lpsift_ransac_workspace_size(const int64_t* nq, int32_t n_pairs, int32_t n_iter)
{
    if (!nq || n_pairs < 1 || n_iter < 0 || n_iter > (1 << 20)) return 0;
    size_t b = 0;
    for (int i = 0; i < n_pairs; ++i) {
        if (nq[i] < 0 || nq[i] > INT32_MAX) return 0;
        b += align_up(ransac_workspace_bytes(nq[i], n_iter), 256);
    }
    return b;
}

int lpsift_ransac(const lpsift_keypoints* kpA, const lpsift_keypoints* kpB,
                  const int32_t* const* selA, const int32_t* const* selB,
                  const int32_t* const* match, const int64_t* nq, int32_t n_pairs,
                  const lpsift_ransac_params* rp, void* workspace, size_t ws_bytes,
                  int32_t* const* slotA, int32_t* const* slotB, uint8_t* const* inlier,
                  double* H, int32_t* stats, void* stream)
{
    if (!kpA || !kpB || !match || !nq || n_pairs < 1 || !rp || !slotA || !slotB || !inlier ||
        !H || !stats || !workspace)
        return LPSIFT_EINVAL;
    if (rp->n_iter < 0 || rp->n_iter > (1 << 20) || rp->tries < 1 || rp->tries > 64 ||
        !(rp->thresh > 0.0) || !std::isfinite(rp->thresh) || (rp->n_iter > 0 && !rp->uniforms))
        return LPSIFT_EINVAL;
    for (int i = 0; i < n_pairs; ++i) {
        if (nq[i] < 0 || nq[i] > INT32_MAX) return LPSIFT_EINVAL;
        if (nq[i] > 0 && (!kpA[i].x || !kpA[i].y || !kpB[i].x || !kpB[i].y || !match[i] ||
                          !slotA[i] || !slotB[i] || !inlier[i]))
            return LPSIFT_EINVAL;
        if (selA && nq[i] > 0 && !selA[i]) return LPSIFT_EINVAL;
        if (selB && !selB[i]) return LPSIFT_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return LPSIFT_EINVAL;
    if (ws_bytes < lpsift_ransac_workspace_size(nq, n_pairs, rp->n_iter)) return LPSIFT_ECAPACITY;
    char* ws = static_cast<char*>(workspace);
    for (int b0 = 0; b0 < n_pairs; b0 += kRansacPairs) {
        const int nb = (n_pairs - b0 < kRansacPairs) ? n_pairs - b0 : kRansacPairs;
        RansacBatch b{};
        b.n = nb;
        b.n_iter = rp->n_iter;
        b.tries = rp->tries;
        b.thresh2 = rp->thresh * rp->thresh;
        b.u = rp->uniforms;
        for (int k = 0; k < nb; ++k) {
            const int i = b0 + k;
            RansacPair& P = b.p[k];
            P.ax = kpA[i].x;
            P.ay = kpA[i].y;
            P.bx = kpB[i].x;
            P.by = kpB[i].y;
            P.selA = selA ? selA[i] : nullptr;
            P.selB = selB ? selB[i] : nullptr;
            P.match = match[i];
            P.nq = nq[i];
            ransac_layout(ws, nq[i], rp->n_iter, P);
            ws += align_up(ransac_workspace_bytes(nq[i], rp->n_iter), 256);
            P.slotA = slotA[i];
            P.slotB = slotB[i];
            P.inlier = inlier[i];
            P.H = H + 9 * (int64_t)i;
            P.stats = stats + 3 * (int64_t)i;
        }
        const int st = launch_ransac(b, static_cast<hipStream_t>(stream));
        if (st != LPSIFT_OK) return st;
    }
    return LPSIFT_OK;
}

int lpsift_match_tune(const float* const* descA, const int64_t* nA, const float* const* descB,
                      const int64_t* nB, int32_t n_pairs, const lpsift_match_params* mp,
                      const int32_t* candidates, int32_t n_candidates, const int32_t* waves,
                      int32_t n_waves, int32_t reps, void* workspace, size_t ws_bytes,
                      int32_t* const* match, float* const* d1, float* const* d2, float* ms,
                      int32_t* best, int32_t* best_waves, void* stream)
{
    const int sc = check_match_call(descA, nA, descB, nB, n_pairs, mp, match, d1, d2);
    if (sc != LPSIFT_OK) return sc;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return LPSIFT_EINVAL;
    if (!candidates || n_candidates < 1 || reps < 1 || reps > 1000 || !ms || !best)
        return LPSIFT_EINVAL;
    if (n_waves < 0 || (n_waves > 0 && (!waves || !best_waves))) return LPSIFT_EINVAL;
    const int nw = n_waves > 0 ? n_waves : 1;
    lpsift_match_params m = *mp;
    for (int w = 0; w < nw; ++w) {
        if (n_waves > 0) m.qblock_waves = waves[w];
        for (int c = 0; c < n_candidates; ++c) {
            if (candidates[c] < 1 || candidates[c] > 16) return LPSIFT_EINVAL;
            m.b_chunks = candidates[c];
            const size_t need = lpsift_match_workspace_size(nA, nB, n_pairs, &m);
            if (need == 0) return LPSIFT_EINVAL;   // also a bad wave count
            if (ws_bytes < need) return LPSIFT_ECAPACITY;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LPSIFT_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);   // cleanup on the error path: its status adds nothing
        return LPSIFT_EHIP;
    }
    int st = LPSIFT_OK;
    float best_ms = 0.0f;
    bool first = true;
    for (int w = 0; w < nw && st == LPSIFT_OK; ++w) {
        if (n_waves > 0) m.qblock_waves = waves[w];
        for (int c = 0; c < n_candidates && st == LPSIFT_OK; ++c) {
            m.b_chunks = candidates[c];
            // one untimed run, then reps timed runs
            st = lpsift_match(descA, nA, descB, nB, n_pairs, &m, workspace, ws_bytes, match, d1,
                              d2, stream);
            if (st != LPSIFT_OK) break;
            if (hipEventRecord(e0, s) != hipSuccess) { st = LPSIFT_EHIP; break; }
            for (int r = 0; r < reps && st == LPSIFT_OK; ++r)
                st = lpsift_match(descA, nA, descB, nB, n_pairs, &m, workspace, ws_bytes, match,
                                  d1, d2, stream);
            if (st != LPSIFT_OK) break;
            float t = 0.0f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
                st = LPSIFT_EHIP;
                break;
            }
            const float v = t / (float)reps;
            ms[w * n_candidates + c] = v;
            if (first || v < best_ms) {
                first = false;
                best_ms = v;
                *best = candidates[c];
                if (n_waves > 0) *best_waves = waves[w];
            }
        }
    }
    // the timing events are released whatever the outcome; a failure to
    // release them does not change the measured result
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // extern "C"
