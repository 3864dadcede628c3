/*
 * liblpsift: LP-SIFT feature front end on AMD Instinct MI355X (gfx950).
 *
 * The method is the local-peak scale-invariant feature transform of Li, Wang,
 * Zhao and Zhao ("Local-peak scale-invariant feature transform for fast and
 * random image stitching"): keypoints are the maximum and the minimum of every
 * L x L window at several window sizes L (Sec. 2.2), each is described by a
 * d x d x 8 SIFT histogram (Sec. 2.3), and descriptors of a reference image are
 * matched against those of a registered image by Euclidean distance (Sec. 2.4).
 *
 * Conventions shared by every call:
 *  - Pointers are DEVICE pointers unless the comment says "host".
 *  - The caller owns every buffer; the library never allocates device memory
 *    (the one fixed array of lpsift_match_noalloc is placed by the runtime
 *    when the library's code loads on a device).
 *  - Every call validates all arguments on the host first and returns
 *    LPSIFT_EINVAL / LPSIFT_ECAPACITY / LPSIFT_EUNSUPPORTED without touching the
 *    GPU. Valid calls enqueue kernels on `stream` (a hipStream_t; NULL is the
 *    null stream) and return without synchronising; a kernel launch failure
 *    returns LPSIFT_EHIP. Device faults surface at the caller's next sync.
 *  - No call aborts or throws. Calls on different streams may run concurrently
 *    as long as their output and workspace buffers do not overlap.
 *  - Images are 8-bit grayscale, row-major with a row pitch in bytes;
 *    x is the column and y the row.
 */
#ifndef LPSIFT_H
#define LPSIFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LPSIFT_OK = 0,
    LPSIFT_EINVAL = -1,       /* a null pointer, a bad size or parameter    */
    LPSIFT_ECAPACITY = -2,    /* an output or workspace buffer is too small */
    LPSIFT_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
    LPSIFT_EUNSUPPORTED = -4  /* valid for the method, not built on the GPU */
};

#define LPSIFT_MAX_SCALES 8
#define LPSIFT_DESC_DIM 128   /* d x d x 8 with d = 4 */

/* Kernels booked by the optional timing facility (lpsift_timing_*). */
enum lpsift_kernel {
    LPSIFT_KERNEL_DETECT = 0,          /* window extrema of every scale (Eq. 2) */
    LPSIFT_KERNEL_GRADIENT = 1,        /* gradient magnitude and angle field (Eq. 5) */
    LPSIFT_KERNEL_DESCRIBE = 2,        /* orientation + descriptor per keypoint */
    LPSIFT_KERNEL_MATCH_NORMS = 3,     /* |b|^2 (and split rows) of the registered sets */
    LPSIFT_KERNEL_MATCH_FP32 = 4,      /* FP32 matrix-core contraction with top-k */
    LPSIFT_KERNEL_MATCH_SPLIT = 5,     /* split-BF16 contraction with top-k */
    LPSIFT_KERNEL_MATCH_RESCORE = 6,   /* FP32 rescore + ratio test (all precisions) */
    LPSIFT_KERNEL_MATCH_REMATCH = 7,   /* FP32 re-match of uncertified split queries */
    LPSIFT_KERNEL_MATCH_LOWP = 8,      /* BF16 / FP8 contraction with top-k */
    LPSIFT_KERNEL_SCORE = 9,           /* learned scorer inference */
    LPSIFT_KERNEL_PRUNE = 10,          /* top-k selection of keypoint slots */
    LPSIFT_KERNEL_TRAIN = 11,          /* scorer training step (both kernels) */
    LPSIFT_KERNEL_RANSAC = 12,         /* batched GPU RANSAC (all three kernels) */
    LPSIFT_KERNEL_MATCH_U8 = 13,       /* uint8 int8-matrix-core contraction with top-2 */
    LPSIFT_KERNEL_MATCH_U8_AUX = 14,   /* uint8 candidate terms and final merge */
    LPSIFT_KERNEL_ORIENT_MULTI = 15,   /* multi-orientation pass and row scan */
    LPSIFT_KERNEL_WARP = 16,           /* warp and blend into the mosaic canvas */
    LPSIFT_KERNEL_COUNT = 17
};

/* Learned keypoint scorer: MLP 258 -> 64 -> 64 -> 1 (ReLU), parameters as one
 * FP32 vector in the order W1 [64][258], b1 [64], W2 [64][64], b2 [64],
 * w3 [64], b3 [1]. */
#define LPSIFT_SCORER_IN 258
#define LPSIFT_SCORER_HID 64
#define LPSIFT_SCORER_PARAMS 20801

/* Method parameters (Sec. 2.2-2.3).
 *  n_scales  number of window sizes, 1..LPSIFT_MAX_SCALES
 *  L         window sides, strictly ascending, 4 <= L <= 65536. Any set works;
 *            nested sets (each L divides the next) with the largest <= 128 use
 *            the tiled detect kernel, other sets (e.g. {32, 40}, {256, 512})
 *            one workgroup per window.
 *  d         subregions per side of the descriptor square; only 4 is built.
 *  beta0     Eq. 3-4 size factor; <= 0 selects the largest admissible value
 *            (1/d) sqrt(Lmin/Lmax), for which w = d w_s <= L at every scale. */
typedef struct lpsift_params {
    int32_t n_scales;
    int32_t L[LPSIFT_MAX_SCALES];
    int32_t d;
    float beta0;
} lpsift_params;

/* One 8-bit grayscale image in device memory: height rows of width bytes,
 * row r starting at data + r * pitch (pitch >= width). */
typedef struct lpsift_image {
    const uint8_t* data;
    int32_t height;
    int32_t width;
    int64_t pitch;
} lpsift_image;

/* Keypoints of one image, structure of arrays, `capacity` entries each.
 * Slot layout (fixed, no compaction): scales in the order of params.L; within
 * scale s, window (by, bx) of the ceil(H/L) x ceil(W/L) grid owns slots
 * base_s + 2 (by ceil(W/L) + bx) (its maximum) and that + 1 (its minimum),
 * base_s = sum over earlier scales of 2 ceil(H/L) ceil(W/L).
 *  x, y      pixel position of the extremum
 *  scale     index into params.L
 *  type      +1 maximum, -1 minimum
 *  value     intensity at the extremum
 *  contrast  |value - window mean| / 255, window mean over the clipped window */
typedef struct lpsift_keypoints {
    int32_t* x;
    int32_t* y;
    uint8_t* scale;
    int8_t* type;
    uint8_t* value;
    float* contrast;
    int64_t capacity;
} lpsift_keypoints;

/* Matching parameters (Sec. 2.4, Eq. 6).
 *  ratio       a query is kept when d1 < ratio * d2 (compared in double);
 *              +inf disables the ratio test (the absolute threshold alone)
 *  abs_thresh  ... and d1 < abs_thresh (the Delta_s of Eq. 6; +inf disables it)
 *  precision   contraction used to select candidates (d1 and d2 are always
 *              direct FP32 distances of the selected candidates):
 *              0 = FP32 matrix cores; exact up to FP32 rounding.
 *              1 = BF16 inputs, FP32 accumulation; the topk best kept
 *                  candidates per query are rescored: approximate (a true nearest
 *                  neighbour can be missed; ties are resolved to the lowest
 *                  index among the rescored candidates).
 *              2 = FP8 E4M3 inputs with one scale per descriptor, FP32
 *                  accumulation, topk candidates rescored: approximate.
 *              3 = FP32 split into two BF16 parts (three BF16 products per
 *                  term, FP32 accumulation), certified per query by an error
 *                  bound; queries it cannot certify are re-matched with
 *                  precision 0, so the lists equal precision 0's.
 *              Every precision expects descriptors whose squared norms are
 *              finite in FP32 (true of every row lpsift_describe writes);
 *              for other inputs the lists are unspecified.
 *  b_chunks   candidate-range split of the contraction (0 = automatic, <= 16)
 *  qblock_waves  wavefronts per workgroup of the FP32 contraction (precision 0
 *              and precision 3's re-match), each holding 64 queries: 0 =
 *              automatic (4), or 2, 4, 8; every value gives the same lists
 *  topk        precisions 1 and 2: the number of best candidates by the
 *              reduced-precision contraction that are rescored in FP32 per
 *              query, 2 .. 8 (0 = 8); fewer is faster to rescore and misses
 *              more true neighbours. Must be 0 at precisions 0 and 3, whose
 *              candidate selection is exact.
 *  stats       optional device pointer to one uint32: after the call (stream
 *              order) it holds the number of queries, summed over all pairs,
 *              that precision 3 re-matched with precision 0 (0 otherwise) */
typedef struct lpsift_match_params {
    double ratio;
    float abs_thresh;
    int32_t precision;
    int32_t b_chunks;
    int32_t qblock_waves;
    int32_t topk;
    void* stats;
} lpsift_match_params;

/* Library version as 10000*major + 100*minor + patch. Host only. */
int lpsift_version(void);

/* Human-readable name of a status code. Host only, static storage. */
const char* lpsift_status_string(int status);

/* Number of keypoints of an image (one maximum and one minimum per window of
 * every scale, partial windows at the right and bottom edges included):
 * 2 * sum_s ceil(height/L_s) ceil(width/L_s). Host only, pure.
 * Returns -1 for invalid arguments. */
int64_t lpsift_num_keypoints(int32_t height, int32_t width, const lpsift_params* params);

/* Feature point detection (Sec. 2.2, Eq. 2) with the linear background of
 * Eq. 1 taken as an infinitesimal tie-break: among equal intensities the
 * maximum of a window is the pixel with the largest raster index y*W + x and
 * the minimum the one with the smallest.
 *  imgs    host array of n_images image descriptors (device pixel data)
 *  out     host array of n_images keypoint buffers, each with capacity >=
 *          lpsift_num_keypoints(image); every slot is written.
 * Errors: EINVAL (null pointer, n_images < 1, empty image, pitch < width, bad
 * params), ECAPACITY (capacity too small), EUNSUPPORTED (d != 4), EHIP. */
int lpsift_detect(const lpsift_image* imgs, int32_t n_images, const lpsift_params* params,
                  const lpsift_keypoints* out, void* stream);

/* Device workspace, in bytes, that lpsift_describe needs for these images. */
size_t lpsift_describe_workspace_size(const lpsift_image* imgs, int32_t n_images,
                                      const lpsift_params* params);

/* Orientation assignment and description (Sec. 2.3, Eq. 3-5) of every keypoint
 * slot written by lpsift_detect for the same images and params.
 * Gradients (Eq. 5): a = I(y+1,x) - I(y-1,x), b = I(y,x+1) - I(y,x-1),
 * magnitude sqrt(a^2+b^2), angle atan2(a, b); pixels on the image border have
 * no gradient. With w_s = beta L (Eq. 3):
 *  theta   dominant orientation in radians: 36-bin histogram of magnitudes
 *          weighted by a Gaussian of sigma w_s/2 over the disc of radius
 *          round(1.5 w_s), linear votes between bins centred at multiples of
 *          10 degrees, one circular [1 4 6 4 1]/16 smoothing, argmax (lowest bin
 *          on ties) refined by a parabola through the peak and its neighbours.
 *  desc    [n_kp][128] row-major: offsets rotated by -theta and divided by w_s,
 *          cells centred at -1.5..1.5, Gaussian weight of sigma 2 cells,
 *          trilinear votes into 4 x 4 cells x 8 direction bins (bin o centred at
 *          45 o degrees from theta), element (cy*4 + cx)*8 + o; then normalised,
 *          clipped at 0.2 and normalised again (all zeros for a flat patch).
 * Arithmetic: FP32, histograms summed as fixed-point integers (results are
 * identical from run to run and do not depend on the order of the votes);
 * descriptors within 1e-4 relative L2 and theta within 1e-4 rad of an FP64
 * evaluation, except where the two highest smoothed orientation bins tie to
 * within 1e-5 relative.
 *  kps        host array of n_images keypoint buffers written by lpsift_detect
 *  workspace  device buffer of ws_bytes >= lpsift_describe_workspace_size()
 *  theta      host array of n_images device pointers to float[n_kp]
 *  desc       host array of n_images device pointers to float[n_kp * 128]
 * Errors: EINVAL, ECAPACITY (keypoint capacity or workspace), EUNSUPPORTED
 * (d != 4), EHIP. */
int lpsift_describe(const lpsift_image* imgs, int32_t n_images, const lpsift_keypoints* kps,
                    const lpsift_params* params, void* workspace, size_t ws_bytes,
                    float* const* theta, float* const* desc, void* stream);

/* lpsift_describe for listed keypoint slots only: for each image i, slots
 * sel[i][0 .. n_sel[i]) (device int32, each in [0, lpsift_num_keypoints)) are
 * described exactly as lpsift_describe does and written compacted:
 * theta[i][k], desc[i][k*128 ..] for list entry k. An entry naming no slot of
 * the image gets a zero descriptor and a NaN orientation. Same workspace as
 * lpsift_describe. Errors as lpsift_describe, plus EINVAL for a null or
 * negative list. */
int lpsift_describe_selected(const lpsift_image* imgs, int32_t n_images,
                             const lpsift_keypoints* kps, const lpsift_params* params,
                             const int32_t* const* sel, const int64_t* n_sel, void* workspace,
                             size_t ws_bytes, float* const* theta, float* const* desc,
                             void* stream);

/* Multi-orientation description (the secondary orientations of Lowe's SIFT,
 * which Sec. 2.3 builds on): each keypoint slot gets its dominant orientation
 * (exactly lpsift_describe's theta0) and, after it, up to max_orient - 1
 * further ones: the strict local maxima of the smoothed 36-bin orientation
 * histogram other than the dominant bin whose height is >= peak_ratio times
 * the highest (compared in FP32), highest first (lower bin on equal heights),
 * each refined by the parabola through its bin and the two neighbours. Every
 * (slot, orientation) gives one descriptor row; rows are compacted in slot
 * order, a slot's orientations in the order above:
 *  rows[i][r]   slot of row r (device int32, capacity n_kp[i] * max_orient)
 *  theta[i][r]  its orientation in radians (device float, same capacity)
 *  desc[i]      float [capacity][128]
 *  n_rows[i]    device int64 [n_images], 8-byte aligned: rows written for
 *               image i (rows beyond it are left untouched)
 * max_orient 1..4 (1 gives lpsift_describe's rows, one per slot), peak_ratio
 * in (0, 1] (Lowe: 0.8). Deterministic. Errors: as lpsift_describe, plus
 * EINVAL for bad max_orient / peak_ratio or a null or misaligned output. */
size_t lpsift_describe_multi_workspace_size(const lpsift_image* imgs, int32_t n_images,
                                            const lpsift_params* params);
int lpsift_describe_multi(const lpsift_image* imgs, int32_t n_images, const lpsift_keypoints* kps,
                          const lpsift_params* params, int32_t max_orient, float peak_ratio,
                          void* workspace, size_t ws_bytes, int32_t* const* rows,
                          float* const* theta, float* const* desc, int64_t* n_rows,
                          void* stream);

/* Learned keypoint scorer (not part of the paper's method; it ranks the
 * keypoints of Sec. 2.2 so that only the best share is described and matched).
 * Features of a keypoint at (x, y), 258 values: the 16 x 16 patch
 * I(y + r - 8, x + c - 8) / 255 at index 16 r + c (0 outside the image), then
 * (log2 L_s - log2 L_min) / (log2 L_max - log2 L_min) of its window size (0
 * with one scale), then its contrast. The score is the MLP's output logit
 * z = w3 . relu(W2 relu(W1 x + b1) + b2) + b3.
 *
 * lpsift_score: scores[i][slot] for every keypoint slot written by
 * lpsift_detect. weights: device FP32 [LPSIFT_SCORER_PARAMS]; W1 and W2 are
 * rounded to BF16 for the matrix cores (FP32 accumulation), and h1 to BF16 as
 * the second layer's input. Errors: EINVAL, ECAPACITY (keypoint capacity),
 * EUNSUPPORTED, EHIP. */
int lpsift_score(const lpsift_image* imgs, int32_t n_images, const lpsift_keypoints* kps,
                 const lpsift_params* params, const float* weights, float* const* scores,
                 void* stream);

/* Top-k prune: for each image i, the k[i] slots with the largest scores
 * scores[i][0 .. n[i]) (larger score first, lower slot on ties; NaN ranks
 * lowest), written to sel[i][0 .. k[i]) in ascending slot order. Host arrays
 * n, k, and of device pointers scores (16-byte aligned), sel. Errors: EINVAL
 * (k > n, negative counts, null or misaligned pointers), EHIP. */
int lpsift_prune(const float* const* scores, const int64_t* n, const int64_t* k,
                 int32_t n_images, int32_t* const* sel, void* stream);

/* Training records of keypoints: for list entry e of image i (sel null: every
 * slot), patches[i][e*256 ..] = the uint8 16 x 16 patch (0 outside the image)
 * and extra[i][2e], extra[i][2e+1] = the scale feature and the contrast.
 * patches must be 4-byte aligned. Errors: EINVAL, ECAPACITY, EHIP. */
int lpsift_scorer_gather(const lpsift_image* imgs, int32_t n_images, const lpsift_keypoints* kps,
                         const lpsift_params* params, const int32_t* const* sel,
                         const int64_t* n_sel, uint8_t* const* patches, float* const* extra,
                         void* stream);

/* Device workspace of lpsift_scorer_train_step for a batch (0 if batch < 1). */
size_t lpsift_scorer_train_workspace_size(int64_t batch);

/* One training step of the scorer on a batch of records: loss = sum_c
 * cweight[c] BCE(sigmoid(z_c), labels[c]) / sum_c cweight[c], gradients by
 * backpropagation in FP32 (deterministic: fixed-order sums), then Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with step t >= 1) on the
 * FP32 weights and moments adam_m, adam_v (device [LPSIFT_SCORER_PARAMS],
 * zero before the first step). loss: optional device float receiving the
 * batch loss at the weights before the step. Errors: EINVAL, ECAPACITY, EHIP. */
int lpsift_scorer_train_step(const uint8_t* patches, const float* extra, const float* labels,
                             const float* cweight, int64_t batch, float* weights, float* adam_m,
                             float* adam_v, int64_t step, float lr, void* workspace,
                             size_t ws_bytes, float* loss, void* stream);

/* Device workspace, in bytes, that lpsift_match needs. nA, nB: host arrays of
 * n_pairs descriptor counts. */
size_t lpsift_match_workspace_size(const int64_t* nA, const int64_t* nB, int32_t n_pairs,
                                   const lpsift_match_params* mp);

/* Descriptor matching (Sec. 2.4, Eq. 6) for n_pairs independent pairs. For each
 * reference descriptor i of pair p: j1 = the registered descriptor nearest in
 * Euclidean distance (lowest index on ties), d1 its distance and d2 the second
 * smallest distance over the other registered descriptors (+inf if there is
 * none). match[i] = j1 when d1 < ratio * d2 and d1 < abs_thresh, else -1.
 * d1 and d2 are FP32 distances sqrt(sum (a-b)^2) recomputed directly for the
 * best candidates of a matrix-core contraction (see precision).
 *  descA, descB  host arrays of n_pairs device pointers to float[n][128]
 *  nA, nB        host arrays of n_pairs counts (nA >= 0, nB >= 0)
 *  match, d1, d2 host arrays of n_pairs device pointers to int32/float[nA]
 * Precisions 0 and 3 run up to 36 pairs per kernel launch, and the norms of a
 * registered set that several pairs share (same pointer and count) are
 * computed once per call: all-pairs matching of N images costs a handful of
 * launches. Outputs must not overlap any input or each other.
 * Errors: EINVAL (null pointer, negative count, descriptor pointer not 16-byte
 * aligned, workspace not 256-byte aligned, bad ratio/abs_thresh/precision),
 * ECAPACITY (workspace), EHIP. */
int lpsift_match(const float* const* descA, const int64_t* nA, const float* const* descB,
                 const int64_t* nB, int32_t n_pairs, const lpsift_match_params* mp,
                 void* workspace, size_t ws_bytes, int32_t* const* match, float* const* d1,
                 float* const* d2, void* stream);

/* lpsift_match without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The workspace is a fixed array of
 * LPSIFT_NOALLOC_SCRATCH_BYTES inside the library, one per device: the
 * runtime places it when the library's code is loaded on a device and it
 * stays until the process ends. The call allocates nothing and calls no
 * allocating routine. Arguments, outputs and results are those of
 * lpsift_match with the same mp (its kernels run unchanged on the array).
 * Limit: lpsift_match_workspace_size(nA, nB, n_pairs, mp) must not exceed
 * LPSIFT_NOALLOC_SCRATCH_BYTES (for one pair of 43,396 x 43,396 descriptors
 * precision 0 needs ~4 MiB, 1 ~26 MiB, 2 ~15 MiB; 3 fits up to ~25,000).
 * The array is the one of the current device, so `stream` must belong to
 * it. Every call on a device shares that device's array and the array keeps
 * the last call's contents (each call initialises what it reads): calls
 * that can overlap on one device (different streams, host threads) race and
 * must be serialised by the caller.
 * Errors: those of lpsift_match, plus ECAPACITY (workspace need above the
 * array's size, checked before any GPU work), EINVAL (stream of a device
 * other than the current one), EUNSUPPORTED (device ordinal >= 64). */
#define LPSIFT_NOALLOC_SCRATCH_BYTES (64u << 20)
int lpsift_match_noalloc(const float* const* descA, const int64_t* nA,
                         const float* const* descB, const int64_t* nB, int32_t n_pairs,
                         const lpsift_match_params* mp, int32_t* const* match, float* const* d1,
                         float* const* d2, void* stream);

/* The reduced-precision forms of descriptors that lpsift_match contracts at
 * precision 1 and 2 (a precision variant of the Sec. 2.4 contraction; the
 * matcher runs this same quantisation on its inputs):
 *  precision 1  q = uint16 [n][128]: the BF16 bits of each FP32 element,
 *               rounded to nearest even; scale unused (may be null).
 *  precision 2  q = uint8 [n][128]: FP8 E4M3 (OCP: bias 7, largest finite
 *               448, subnormals kept) bytes of v * fl(448 / m), where
 *               m = max_k |desc[i][k]| in FP32 and the product is an FP32
 *               product clamped to [-448, 448] before rounding to nearest
 *               even; scale[i] = fl(m / 448) (FP32), or 1 for a zero row, so
 *               that desc[i] ~ scale[i] * q[i].
 * desc 16-byte aligned; q 16-byte (precision 1) or 8-byte (precision 2)
 * aligned; scale 4-byte aligned. Caller-owned buffers, written in stream
 * order. Errors: EINVAL (bad precision, n < 0, null or misaligned pointer),
 * EHIP. */
int lpsift_quantize_lowp(const float* desc, int64_t n, int32_t precision, void* q, float* scale,
                         void* stream);

/* Autotuner of lpsift_match's work split: the candidate-range split
 * (b_chunks) and, for the FP32 contraction, the wavefronts per workgroup
 * (qblock_waves; each wavefront holds 64 queries). For each of n_waves wave
 * counts (0, 2, 4 or 8; n_waves = 0 keeps mp->qblock_waves and ignores
 * waves / best_waves) and each of n_candidates split values (1..16) it runs
 * the call once untimed and reps times timed on `stream`, stores the mean
 * milliseconds per call in ms[w * n_candidates + c] (host array of
 * max(n_waves, 1) x n_candidates) and the fastest combination in *best and
 * *best_waves (host). Every combination gives the same lists. All other
 * arguments are those of lpsift_match; the workspace must satisfy every
 * combination (lpsift_match_workspace_size with both fields set). The outputs
 * hold the last run's lists. Synchronises the stream, so it cannot be
 * captured in a graph. Errors: EINVAL (bad candidate or wave count,
 * n_candidates < 1, n_waves < 0, reps outside 1..1000, null ms/best, null
 * waves/best_waves with n_waves > 0, or any lpsift_match argument error),
 * ECAPACITY, EHIP. */
int lpsift_match_tune(const float* const* descA, const int64_t* nA, const float* const* descB,
                      const int64_t* nB, int32_t n_pairs, const lpsift_match_params* mp,
                      const int32_t* candidates, int32_t n_candidates, const int32_t* waves,
                      int32_t n_waves, int32_t reps, void* workspace, size_t ws_bytes,
                      int32_t* const* match, float* const* d1, float* const* d2, float* ms,
                      int32_t* best, int32_t* best_waves, void* stream);

/* uint8 descriptors, the stored form of SIFT implementations (not fixed by the
 * paper; Sec. 2.3 descriptors are unit-norm FP32 vectors).
 * lpsift_quantize_u8: q[i][k] = min(255, rint(512 desc[i][k])) (round half to
 * even; negative values give 0) for n descriptors. desc 16-byte aligned, q
 * 4-byte aligned. Errors: EINVAL (null or misaligned pointer, n < 0), EHIP. */
int lpsift_quantize_u8(const float* desc, int64_t n, uint8_t* q, void* stream);

/* Device workspace, in bytes, of lpsift_match_u8 for nA queries and nB
 * registered descriptors (0 for negative counts). */
size_t lpsift_match_u8_workspace_size(int64_t nA, int64_t nB);

/* Exact matching of uint8 descriptors (Sec. 2.4, Eq. 6 on integer squared
 * distances D = sum (qa - qb)^2, computed exactly on the int8 matrix cores).
 * For each query i: j1 = the registered row with the smallest D (lowest index
 * on ties), D1 its distance, D2 the smallest over the other rows.
 * d1[i] = sqrt(D1) / 512, d2[i] = sqrt(D2) / 512 (+inf when nB < 2; both +inf
 * when nB = 0), rounded from double to float. match[i] = j1 when
 * (ratio = +inf or sqrt(D1) < ratio sqrt(D2)) and sqrt(D1) / 512 < abs_thresh
 * (the test is taken in double), else -1.
 *  qA, qB     device uint8 [n][128], 16-byte aligned
 *  nA, nB     0 .. 2^31 - 1
 *  workspace  device, 256-byte aligned, >= lpsift_match_u8_workspace_size
 *  match, d1, d2  device int32 / float [nA]
 * Errors: EINVAL (null or misaligned pointer, bad count, ratio or abs_thresh
 * not > 0), ECAPACITY (workspace), EHIP. */
int lpsift_match_u8(const uint8_t* qA, int64_t nA, const uint8_t* qB, int64_t nB, double ratio,
                    float abs_thresh, void* workspace, size_t ws_bytes, int32_t* match,
                    float* d1, float* d2, void* stream);

/* Batched RANSAC on the GPU (Sec. 2.5, Eq. 7), FP64, for match lists
 * written by lpsift_match. For pair p: the accepted matches of match[p]
 * (nq[p] queries; query i is slot selA[p][i] of image A, or slot i when selA
 * is null; registered row j is slot selB[p][j] of image B, or slot j) are
 * compacted in query order into slotA[p], slotB[p] (first stats[3p] entries);
 * hypotheses are homographies (h33 = 1) through 4 of them, drawn from the
 * uniforms: slot s of hypothesis h takes the first try t whose
 * floor(u[h][s][t] * n) is not yet taken (a hypothesis without 4 distinct
 * indices, or with 3 nearly collinear points in either image, is skipped);
 * the hypothesis with the most inliers (one-way reprojection error < thresh;
 * earliest on ties) is refitted by least squares over its inliers (Hartley
 * coordinates) and inlier[p][k] marks the inliers of that final H.
 *  kpA, kpB   host arrays of n_pairs keypoint buffers (x, y used)
 *  selA, selB host arrays of n_pairs device int32 pointers, or null
 *  match      host array of n_pairs device int32 pointers [nq[p]]
 *  H          device double [n_pairs][9] (zeros when no hypothesis is valid)
 *  stats      device int32 [n_pairs][3]: matches, inliers, best hypothesis (-1)
 *  uniforms   device double [n_iter][4][tries] in [0, 1), shared by all pairs
 * Match and slot lists must hold valid indices (as written by lpsift_match
 * and lpsift_prune). Errors: EINVAL, ECAPACITY (workspace), EHIP. */
typedef struct lpsift_ransac_params {
    int32_t n_iter;          /* hypotheses, 0 .. 1048576 */
    int32_t tries;           /* uniforms per slot, 1 .. 64 */
    double thresh;           /* inlier threshold in pixels, > 0 */
    const double* uniforms;
} lpsift_ransac_params;

size_t lpsift_ransac_workspace_size(const int64_t* nq, int32_t n_pairs, int32_t n_iter);

int lpsift_ransac(const lpsift_keypoints* kpA, const lpsift_keypoints* kpB,
                  const int32_t* const* selA, const int32_t* const* selB,
                  const int32_t* const* match, const int64_t* nq, int32_t n_pairs,
                  const lpsift_ransac_params* rp, void* workspace, size_t ws_bytes,
                  int32_t* const* slotA, int32_t* const* slotB, uint8_t* const* inlier,
                  double* H, int32_t* stats, void* stream);

/* Warp and blend: the stitched canvas of registered images (Sec. 4, Fig. 2(f),
 * Fig. 9; the paper fixes no blending rule, this one is feathering).
 * G: host double [n_images][9], row-major, image k pixels -> reference pixels
 * (the mosaic registration's transforms), each finite and invertible.
 * Canvas pixel (u, v) is the reference point p = (u + x0, v + y0). Image k
 * covers it when q = G_k^-1 p (divided by its third coordinate, in double)
 * lies in [0, w_k - 1] x [0, h_k - 1]; it then contributes the bilinear sample
 * of the image at q (neighbour index clamped at the last row / column) with
 * weight min(q.x + 1, w_k - q.x, q.y + 1, h_k - q.y).
 *  canvas  device float [out_h][out_w]: sum(weight x sample) / sum(weight),
 *          sums in double over images in order, 0 where no image covers
 *  count   device uint8 [out_h][out_w] (may be null): covering images
 * n_images 1..16; out_w, out_h >= 0 with out_w * out_h < 2^31. Every canvas
 * pixel is written. Errors: EINVAL (null pointer, bad sizes, a transform that
 * is not finite or not invertible), EHIP. */
int lpsift_warp_blend(const lpsift_image* imgs, int32_t n_images, const double* G, double x0,
                      double y0, int32_t out_w, int32_t out_h, float* canvas, uint8_t* count,
                      void* stream);

/* Kernel timing, a profiling aid. lpsift_timing_enable(1) resets the sums
 * and makes every later launch of the kernels listed in lpsift_kernel bracket
 * itself with two HIP events recorded on its stream (a few microseconds per
 * launch); lpsift_timing_enable(0) resets and stops. lpsift_timing_read waits
 * for every recorded event and returns, for one kernel, the summed device
 * milliseconds and the number of timed launches since the reset. Host-side
 * state shared by all streams and devices of the process; keep it disabled
 * while capturing a graph. Errors: EINVAL (bad kernel id or null pointer),
 * EHIP (an event could not be created, recorded or read; the sums then miss
 * those launches). */
int lpsift_timing_enable(int32_t on);
int lpsift_timing_read(int32_t kernel, double* ms, int64_t* launches);

/* Matrix-core throughput probes (a measurement aid, not part of the method):
 * lpsift_probe runs, on `stream`, 2048 workgroups of four wavefronts, each
 * wavefront `iters` rounds of four independent accumulator chains of one MFMA
 * shape, and writes one checksum per wavefront to out (device float
 * [lpsift_probe_out_size()]). lpsift_probe_ops gives the multiply-add count
 * x 2 of such a call, so ops / elapsed time is the achieved rate.
 * Errors: EINVAL (bad kind, iters outside 1 .. 2^24, null out), EHIP. */
enum lpsift_probe_kind {
    LPSIFT_PROBE_MFMA_F32 = 0,    /* v_mfma_f32_32x32x2_f32 */
    LPSIFT_PROBE_MFMA_BF16 = 1,   /* v_mfma_f32_32x32x16_bf16 */
    LPSIFT_PROBE_MFMA_FP8 = 2,    /* v_mfma_scale_f32_32x32x64_f8f6f4, E4M3 */
    LPSIFT_PROBE_MFMA_I8 = 3      /* v_mfma_i32_32x32x32_i8 */
};
int64_t lpsift_probe_out_size(void);
double lpsift_probe_ops(int32_t kind, int64_t iters);
int lpsift_probe(int32_t kind, int64_t iters, float* out, void* stream);

/* Homography between matched pairs by RANSAC (Sec. 2.5, Eq. 7), on the host in
 * FP64; no GPU involvement and no stream. Eq. 8's rigid transform is the special
 * case of a full homography (h33 = 1) fitted here.
 *  xyA, xyB   host arrays of n (x, y) pairs: pair i maps A point i to B point i
 *  samples    host [n_iter][4] indices into the pairs, the random draws of the
 *             sampling loop (given by the caller, so runs are reproducible)
 *  thresh     inlier iff the one-way reprojection error |H a - b| < thresh (px)
 * Each non-degenerate sample (no 3 of its points nearly collinear in A or B)
 * gives the exact homography through its 4 pairs (Hartley-normalised 8x8
 * solve); the one with the most inliers (earliest on ties) is refined by least
 * squares over its inliers. Outputs: H (host double[9], row-major, H[8] = 1;
 * all zeros when no hypothesis was valid or n < 4), mask (host uint8[n], the
 * inliers of the refined H), *n_inliers, *best_iter (-1 when none).
 * Errors: EINVAL (null pointer, negative size, thresh not positive, sample
 * index out of range when n >= 4). */
int lpsift_ransac_host(const double* xyA, const double* xyB, int64_t n, const int32_t* samples,
                       int32_t n_iter, double thresh, double* H, uint8_t* mask,
                       int64_t* n_inliers, int32_t* best_iter);

/* Local optimisation of a homography estimate (a reading: the paper fits
 * Eq. 7 by RANSAC and leaves the refinement of the winning model open; one
 * least-squares step over the inliers, as lpsift_ransac_host takes, still
 * depends on which sample won). On the host in FP64, no GPU involvement.
 *  xyA, xyB    host arrays of n (x, y) pairs, as for lpsift_ransac_host
 *  thresh      inlier iff |H a - b| < thresh (px), as for lpsift_ransac_host
 *  max_rounds  0 .. 1000 least-squares rounds at most
 *  H           host double[9], row-major: the start (finite), then the result
 * A round fits H by least squares (h33 = 1, Hartley coordinates, the same
 * solve as lpsift_ransac_host's refinement) to the inliers of the current H;
 * the rounds stop when a round leaves the inlier set unchanged, when fewer
 * than 4 inliers remain, when the solve is singular (H then stays the last
 * good one), or after max_rounds. Outputs: H, mask (host uint8[n], the
 * inliers of the final H), *n_inliers, *rounds (rounds taken; 0 leaves H
 * unchanged and gives its inliers). Errors: EINVAL (null pointer, negative
 * size, thresh not positive, max_rounds out of range, H not finite). */
int lpsift_refine_host(const double* xyA, const double* xyB, int64_t n, double thresh,
                       int32_t max_rounds, double* H, uint8_t* mask, int64_t* n_inliers,
                       int32_t* rounds);

#ifdef __cplusplus
}
#endif

#endif /* LPSIFT_H */
