// Internal declarations of liblpsift: launch descriptors passed by value to the
// kernels and the host launchers each kernel file provides to the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lpsift.h"

namespace lpsift {

// Images per kernel launch; larger batches are split into several launches.
constexpr int kMaxBatch = 16;

__host__ __device__ inline int64_t n_windows(int64_t n, int64_t L) { return (n + L - 1) / L; }

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// floor(sqrt(v)) for v >= 0, exact for every int32 value.
__host__ __device__ inline int isqrt_floor(int v)
{
    int r = (int)sqrtf((float)v);
    while (r > 0 && r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

// Number of integer offsets (dx, dy) with dx^2 + dy^2 <= r2 (r2 >= 0).
__host__ __device__ inline int disc_count(int r2)
{
    const int R = isqrt_floor(r2);
    int n = 0;
    for (int dy = -R; dy <= R; ++dy) n += 2 * isqrt_floor(r2 - dy * dy) + 1;
    return n;
}

// Per-scale geometry of orientation and description (Eq. 3).
struct ScaleGeom {
    float ws;          // subregion side w_s = beta L
    float inv_ws;      // 1 / w_s
    float k_orient;    // -log2(e) / (2 sigma_o^2), sigma_o = w_s / 2
    float k_desc;      // -log2(e) / (2 (d/2)^2 w_s^2), Gaussian of sigma d/2 cells
    int r2_orient;     // round(1.5 w_s)^2
    int r2_desc;       // floor((w_s sqrt(2) (d+1)/2)^2)
    int off_orient;    // entry offset of the orientation disc table
    int n_orient;      // entries of that table
    int off_desc;      // entry offset of the descriptor tables (bucket b at off_desc + b cap_desc)
    int n_desc;        // entries of the whole descriptor disc
    int n_buckets;     // orientation buckets of the descriptor table: kDescBuckets or 1
    int cap_desc;      // entries reserved per bucket (n_desc)
    float dscale;      // fixed-point scale of the descriptor votes (a bin stays below 2^32)
    float dinv;        // 1 / dscale
};

// Fixed-point scale of the orientation votes (64-bit bins).
constexpr float kOrientVoteScale = 8388608.0f;   // 2^23

// The descriptor disc is stored once per orientation bucket, keeping only the
// entries that the square of reachable subregions can cover for some angle of
// the bucket (about 27 % fewer visits than the whole disc); discs above
// kBucketMaxEntries entries are stored whole, as one bucket.
constexpr int kDescBuckets = 64;
constexpr int kBucketMaxEntries = 8192;

struct Geometry {
    int n_scales;
    int L[LPSIFT_MAX_SCALES];
    ScaleGeom s[LPSIFT_MAX_SCALES];
    int table_entries;  // total 16-byte entries of all disc tables
};

// Validated, derived view of lpsift_params. Returns LPSIFT_OK or an error.
int make_geometry(const lpsift_params* p, Geometry* g);

// While lpsift_timing_enable(1) is in force, brackets the launches made in
// its lifetime with HIP events on `stream`, booked under `kernel`
// (LPSIFT_KERNEL_*); otherwise does nothing.
class TimedScope {
public:
    TimedScope(int kernel, hipStream_t stream);
    ~TimedScope();
    TimedScope(const TimedScope&) = delete;
    TimedScope& operator=(const TimedScope&) = delete;

private:
    int kernel_;
    hipStream_t stream_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

// ---- launchers (enqueue only; return LPSIFT_OK or LPSIFT_EHIP) ----

int launch_detect(const lpsift_image* imgs, int n, const Geometry& g,
                  const lpsift_keypoints* out, hipStream_t s);

// Workspace layout of describe: disc tables, then one float2 gradient field
// per image (8 bytes per pixel), each 256-byte aligned.
size_t describe_workspace_bytes(const lpsift_image* imgs, int n, const Geometry& g);
// sel / n_sel (host arrays, or null for every slot): describe only the listed
// slots of each image, outputs compacted in list order.
int launch_describe(const lpsift_image* imgs, int n, const lpsift_keypoints* kps,
                    const Geometry& g, void* ws, float* const* theta, float* const* desc,
                    const int32_t* const* sel, const int64_t* n_sel, hipStream_t s);

// Multi-orientation variant: up to max_orient orientations per slot
// (secondary peaks >= peak_ratio x the highest), one descriptor row each,
// rows compacted in slot order; n_rows: device int64 [n].
struct MultiSpec {
    int32_t max_orient;
    float peak_ratio;
    int32_t* const* rows;
    int64_t* n_rows;
};
size_t describe_multi_workspace_bytes(const lpsift_image* imgs, int n, const Geometry& g);
int launch_describe_multi(const lpsift_image* imgs, int n, const lpsift_keypoints* kps,
                          const Geometry& g, void* ws, const MultiSpec& ms, float* const* theta,
                          float* const* desc, hipStream_t stream);

struct MatchPlan {
    int chunks;          // candidate-range split
    int64_t chunk_len;   // candidates per chunk, a multiple of 32
};
MatchPlan plan_match(int64_t nA, int64_t nB, const lpsift_match_params* mp);
size_t match_workspace_bytes(int64_t nA, int64_t nB, const lpsift_match_params* mp);
// The quantised forms the precision 1 / 2 contractions read (the same kernel):
// BF16 bits [n][128] (precision 1) or E4M3 bytes [n][128] and scales [n] (2).
int launch_quantize_lowp(const float* desc, int64_t n, int precision, void* q, float* scale,
                         hipStream_t stream);

// One pair of a match call: descriptor sets, its 256-byte aligned workspace
// slice of match_workspace_bytes(nA, nB), and its outputs.
struct MatchPairIO {
    const float* A;
    int64_t nA;
    const float* B;
    int64_t nB;
    void* ws;
    int32_t* match;
    float* d1;
    float* d2;
};
// All pairs of a call; the FP32 and split paths batch up to 16 pairs per
// launch and compute the norms of a candidate set shared by several pairs once.
int launch_match_pairs(const MatchPairIO* pairs, int n, const lpsift_match_params* mp,
                       hipStream_t s);

// ---- learned keypoint scorer ----

struct ScoreImg {
    const uint8_t* data;
    int64_t pitch;
    int32_t h, w;
    const int32_t* x;
    const int32_t* y;
    const uint8_t* scale;
    const float* contrast;
    float* score;
    int64_t n;             // keypoints (all slots)
};
struct ScoreArgs {
    int32_t n_images;
    float sfeat[LPSIFT_MAX_SCALES];   // normalised log2 window size per scale
    ScoreImg img[kMaxBatch];
};
int launch_score(const ScoreArgs& args, const float* weights, hipStream_t s);

struct PruneImg {
    const float* score;
    int64_t n;
    int64_t k;
    int32_t* sel;
};
struct PruneArgs {
    int32_t n_images;
    PruneImg img[kMaxBatch];
};
int launch_prune(const PruneArgs& args, hipStream_t s);

struct GatherImg {
    const uint8_t* data;
    int64_t pitch;
    int32_t h, w;
    const int32_t* x;
    const int32_t* y;
    const uint8_t* scale;
    const float* contrast;
    const int32_t* sel;    // slots to gather (null: all slots)
    int64_t n;             // entries
    int64_t n_kp;          // slots of the image (bound for sel)
    uint8_t* patches;      // [n][256]
    float* extra;          // [n][2]
};
struct GatherArgs {
    int32_t n_images;
    float sfeat[LPSIFT_MAX_SCALES];
    GatherImg img[kMaxBatch];
};
int launch_gather(const GatherArgs& args, hipStream_t s);

struct TrainArgs {
    const uint8_t* patches;   // [batch][256]
    const float* extra;       // [batch][2]
    const float* labels;      // [batch]
    const float* cweight;     // [batch]
    int64_t batch;
    float* weights;           // FP32 master, updated
    float* adam_m;
    float* adam_v;
    float* partials;          // workspace
    float* loss;              // optional
    int64_t step;
    float lr;
};
size_t train_workspace_bytes(int64_t batch);
int launch_train(TrainArgs args, hipStream_t s);

// ---- batched GPU RANSAC ----

constexpr int kRansacPairs = 16;

struct RansacPair {
    const int32_t* ax;        // keypoint coordinates of image A and image B
    const int32_t* ay;
    const int32_t* bx;
    const int32_t* by;
    const int32_t* selA;      // optional slot lists (descriptor row -> slot)
    const int32_t* selB;
    const int32_t* match;     // [nq]: registered row or -1
    int64_t nq;
    double* pa;               // workspace: compacted points [nq][2]
    double* pb;
    int32_t* count;           // workspace: number of accepted matches
    int32_t* bestc;           // workspace: per hypothesis block (inliers, hypothesis)
    double* bestH;            // workspace: per hypothesis block, its H
    int32_t* slotA;           // outputs [nq] (first count entries)
    int32_t* slotB;
    uint8_t* inlier;
    double* H;                // output [9]
    int32_t* stats;           // output [3]: matches, inliers, best hypothesis
};
struct RansacBatch {
    int32_t n;
    int32_t n_iter;
    int32_t n_blocks;
    int32_t tries;
    double thresh2;
    const double* u;          // [n_iter][4][tries]
    RansacPair p[kRansacPairs];
};
// Matrix-core probes (probe.hip)
int64_t probe_out_floats();
double probe_ops(int kind, int64_t iters);
int launch_probe(int kind, int64_t iters, float* out, hipStream_t s);

// Warp and blend (warp.hip)
constexpr int kWarpMax = 16;
struct WarpImg {
    const uint8_t* data;
    int64_t pitch;
    int32_t h, w;
    double hi[9];                  // inverse transform: reference pixel -> image pixel
    int32_t bx0, by0, bx1, by1;    // canvas box (half-open) outside which it covers nothing
};
struct WarpArgs {
    int32_t n;
    int32_t W, H;
    double x0, y0;                 // canvas pixel (0, 0) = reference point (x0, y0)
    float* canvas;
    uint8_t* count;
    WarpImg img[kWarpMax];
};
int launch_warp_blend(const WarpArgs& a, hipStream_t stream);

// uint8 descriptors (match_u8.hip)
int launch_quantize_u8(const float* desc, int64_t n, uint8_t* out, hipStream_t stream);
size_t match_u8_workspace_bytes(int64_t nA, int64_t nB);
int launch_match_u8(const uint8_t* A, int64_t nA, const uint8_t* B, int64_t nB, double ratio,
                    float abs_thresh, void* ws, int32_t* match, float* d1, float* d2,
                    hipStream_t stream);

size_t ransac_workspace_bytes(int64_t nq, int32_t n_iter);
void ransac_layout(void* ws, int64_t nq, int32_t n_iter, RansacPair& p);
int launch_ransac(RansacBatch& b, hipStream_t s);

}  // namespace lpsift
