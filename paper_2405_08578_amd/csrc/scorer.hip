// Learned keypoint scorer: inference, top-k prune and training.
//
// Not part of the paper's method: a small MLP ranks the keypoints of
// Sec. 2.2 so that only the best share is described and matched. Features of
// a keypoint at (x, y): the 16 x 16 patch I(y + r - 8, x + c - 8) / 255 (zero
// outside the image, index 16 r + c), then the normalised log2 window size and
// the keypoint's contrast. MLP 258 -> 64 -> 64 -> 1 with ReLU; the score is
// the output logit.
//
// Inference (score_kernel): the 256-wide patch part of layer 1 runs on
// v_mfma_f32_32x32x16_bf16 with the pixel values themselves as the B operand
// (integers 0..255 are exact in BF16) and W1 rounded to BF16 as the A operand,
// FP32 accumulation; the 1/255, the two scalar features and the bias are
// applied in FP32. Layer 2 takes h1 rounded to BF16 through LDS (the MFMA
// output and input layouts differ), layer 3 is a 64-term FP32 dot product
// across the accumulator lanes. One wavefront scores 32 keypoints.
//
// Prune (prune_kernel): one workgroup per image selects the k largest scores
// (ties: lower slot first) by an MSB-first radix select on order-preserving
// 32-bit keys, then compacts the selected slots in ascending order.
//
// Training (train_kernel + adam_kernel): FP32 on the vector units (the batch
// is small and off the hot path). A workgroup runs forward and backward for 64
// candidates and writes its partial gradient sums; the second kernel adds the
// partials in a fixed order (deterministic), divides by the batch's weight sum
// and applies Adam to the FP32 master weights.
#include "internal.h"

namespace lpsift {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kIn = LPSIFT_SCORER_IN;      // 258
constexpr int kHid = LPSIFT_SCORER_HID;    // 64
constexpr int kParams = LPSIFT_SCORER_PARAMS;
// offsets in the flat parameter vector
constexpr int kOffB1 = kHid * kIn;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid;

__device__ inline uint32_t bf16_rne(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// ------------------------------------------------------------ inference --

constexpr int kW1Row = 264;      // bf16 per LDS row of W1 (258 + pad, 16-byte rows)
constexpr int kW2Row = 72;       // bf16 per LDS row of W2
constexpr int kHRow = 72;        // bf16 per keypoint row of the h1 exchange
constexpr int kScoreWaves = 4;
constexpr int kScoreGroup = 32 * kScoreWaves;   // keypoints per workgroup step

__global__ __launch_bounds__(256) void score_kernel(ScoreArgs a, const float* __restrict__ wts)
{
    __shared__ __attribute__((aligned(16))) uint16_t w1[kHid * kW1Row];
    __shared__ __attribute__((aligned(16))) uint16_t w2[kHid * kW2Row];
    __shared__ __attribute__((aligned(16))) uint16_t hx[kScoreWaves][32 * kHRow];
    __shared__ float b1[kHid], b2[kHid], w3[kHid], w1x[kHid][2];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int c = lane & 31, hh = lane >> 5;

    // weights: W1 and W2 rounded to BF16, the rest FP32
    for (int e = tid; e < kHid * kIn; e += 256) {
        const int j = e / kIn, k = e - j * kIn;
        const uint32_t b = bf16_rne(wts[e]);
        w1[j * kW1Row + k] = (uint16_t)b;
        if (k >= 256) w1x[j][k - 256] = __uint_as_float(b << 16);
    }
    for (int e = tid; e < kHid * kHid; e += 256) {
        const int j = e / kHid, k = e - j * kHid;
        w2[j * kW2Row + k] = (uint16_t)bf16_rne(wts[kOffW2 + e]);
    }
    if (tid < kHid) {
        b1[tid] = wts[kOffB1 + tid];
        b2[tid] = wts[kOffB2 + tid];
        w3[tid] = wts[kOffW3 + tid];
    }
    const float b3 = wts[kOffB3];
    __syncthreads();

    int64_t total = 0;
    for (int i = 0; i < a.n_images; ++i) total += (a.img[i].n + kScoreGroup - 1) / kScoreGroup;

    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        // image and group of this step (uniform over the workgroup)
        int im = 0;
        int64_t g = it;
        for (int i = 0; i < a.n_images; ++i) {
            const int64_t cnt = (a.img[i].n + kScoreGroup - 1) / kScoreGroup;
            if (g < cnt) {
                im = i;
                break;
            }
            g -= cnt;
        }
        const ScoreImg& I = a.img[im];
        const int64_t idx = g * kScoreGroup + wave * 32 + c;
        const bool valid = idx < I.n;
        int kx = 0, ky = 0;
        float sf = 0.0f, ct = 0.0f;
        if (valid) {
            kx = I.x[idx];
            ky = I.y[idx];
            sf = a.sfeat[I.scale[idx]];
            ct = I.contrast[idx];
        }

        // layer 1, patch part: 16 patch rows = 16 K-steps of 16 pixels
        floatx16 acc0, acc1;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            acc0[r] = 0.0f;
            acc1[r] = 0.0f;
        }
        for (int r = 0; r < 16; ++r) {
            const int yy = ky + r - 8;
            const bool row_ok = valid && yy >= 0 && yy < I.h;
            const uint8_t* prow = I.data + (int64_t)(row_ok ? yy : 0) * I.pitch;
            uint32_t px[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int xx = kx - 8 + 8 * hh + e;
                const uint32_t v = (row_ok && xx >= 0 && xx < I.w) ? (uint32_t)prow[xx] : 0u;
                px[e] = __float_as_uint((float)v) >> 16;      // exact in BF16
            }
            const uint4 bq = make_uint4(px[0] | (px[1] << 16), px[2] | (px[3] << 16),
                                        px[4] | (px[5] << 16), px[6] | (px[7] << 16));
            const uint4 a0 = *reinterpret_cast<const uint4*>(&w1[c * kW1Row + 16 * r + 8 * hh]);
            const uint4 a1 = *reinterpret_cast<const uint4*>(&w1[(32 + c) * kW1Row + 16 * r + 8 * hh]);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a0),
                                                          __builtin_bit_cast(bf16x8, bq), acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a1),
                                                          __builtin_bit_cast(bf16x8, bq), acc1, 0, 0, 0);
        }
        // finish layer 1 in FP32; h1 as BF16 into this wave's exchange rows
        uint16_t* hrow = &hx[wave][c * kHRow];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int j0 = 8 * (r >> 2) + 4 * hh + (r & 3);
            const int j1 = 32 + j0;
            const float a10 = acc0[r] / 255.0f + w1x[j0][0] * sf + w1x[j0][1] * ct + b1[j0];
            const float a11 = acc1[r] / 255.0f + w1x[j1][0] * sf + w1x[j1][1] * ct + b1[j1];
            hrow[j0] = (uint16_t)bf16_rne(fmaxf(a10, 0.0f));
            hrow[j1] = (uint16_t)bf16_rne(fmaxf(a11, 0.0f));
        }
        __syncthreads();

        // layer 2: 4 K-steps of 16 hidden units
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            acc0[r] = 0.0f;
            acc1[r] = 0.0f;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const uint4 bq = *reinterpret_cast<const uint4*>(&hrow[16 * s + 8 * hh]);
            const uint4 a0 = *reinterpret_cast<const uint4*>(&w2[c * kW2Row + 16 * s + 8 * hh]);
            const uint4 a1 = *reinterpret_cast<const uint4*>(&w2[(32 + c) * kW2Row + 16 * s + 8 * hh]);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a0),
                                                          __builtin_bit_cast(bf16x8, bq), acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a1),
                                                          __builtin_bit_cast(bf16x8, bq), acc1, 0, 0, 0);
        }
        // layer 3: this lane's 32 hidden units, then its partner lane's
        float zp = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int j0 = 8 * (r >> 2) + 4 * hh + (r & 3);
            zp += w3[j0] * fmaxf(acc0[r] + b2[j0], 0.0f);
            zp += w3[32 + j0] * fmaxf(acc1[r] + b2[32 + j0], 0.0f);
        }
        const float z = zp + __shfl_xor(zp, 32) + b3;
        if (valid && hh == 0) I.score[idx] = z;
        __syncthreads();   // the exchange rows are rewritten by the next step
    }
}

// ---------------------------------------------------------------- prune --

constexpr int kPruneThreads = 1024;

// Order-preserving key of a float score (larger score, larger key); -0 and
// +0 share a key (they are equal scores), NaN ranks lowest.
__device__ inline uint32_t score_key(float s)
{
    if (s != s) return 0u;
    uint32_t u = __float_as_uint(s);
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Exclusive scan of one value per thread over the workgroup; returns the
// thread's prefix and writes the total.
__device__ inline uint32_t block_scan(uint32_t v, uint32_t* total, uint32_t* sh)
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
        const int nw = kPruneThreads / 64;
        uint32_t w = (lane < nw) ? sh[lane] : 0u;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(w, off);
            if (lane >= off) w += y;
        }
        if (lane < nw) sh[64 + lane] = w;   // inclusive per-wave totals
    }
    __syncthreads();
    const uint32_t before = (wave > 0) ? sh[64 + wave - 1] : 0u;
    *total = sh[64 + kPruneThreads / 64 - 1];
    __syncthreads();
    return before + x - v;
}

constexpr int kPer = 8;                          // scores per thread per tile
constexpr int kPruneTile = kPruneThreads * kPer;

// Keys of the 8 scores [i, i + 8) (i a multiple of 8; the scores are 16-byte
// aligned); entries at or beyond n get key 0 and valid = false.
__device__ inline void load_keys(const float* __restrict__ s, int64_t n, int64_t i,
                                 uint32_t key[kPer])
{
    if (i + kPer <= n) {
        const float4 a = *reinterpret_cast<const float4*>(s + i);
        const float4 b = *reinterpret_cast<const float4*>(s + i + 4);
        key[0] = score_key(a.x); key[1] = score_key(a.y); key[2] = score_key(a.z);
        key[3] = score_key(a.w); key[4] = score_key(b.x); key[5] = score_key(b.y);
        key[6] = score_key(b.z); key[7] = score_key(b.w);
    } else {
#pragma unroll
        for (int e = 0; e < kPer; ++e) key[e] = (i + e < n) ? score_key(s[i + e]) : 0u;
    }
}

__global__ __launch_bounds__(kPruneThreads) void prune_kernel(PruneArgs a)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t sh[128];
    __shared__ uint32_t sel_digit, sel_rank;
    const PruneImg& P = a.img[blockIdx.x];
    const int64_t n = P.n;
    const int64_t k = P.k;
    if (k <= 0) return;
    if (k >= n) {
        for (int64_t i = threadIdx.x; i < n; i += kPruneThreads) P.sel[i] = (int32_t)i;
        return;
    }
    // radix select of the k-th largest key, 8 bits at a time from the top;
    // thread t reads the run [tile + 8 t, tile + 8 t + 8) of every tile
    uint32_t prefix = 0u, mask = 0u;
    uint32_t need = (uint32_t)k;       // rank still to find among keys with this prefix
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = threadIdx.x; b < 256; b += kPruneThreads) hist[b] = 0u;
        __syncthreads();
        for (int64_t i0 = 0; i0 < n; i0 += kPruneTile) {
            const int64_t i = i0 + (int64_t)kPer * threadIdx.x;
            uint32_t key[kPer];
            load_keys(P.score, n, i, key);
#pragma unroll
            for (int e = 0; e < kPer; ++e)
                if (i + e < n && (key[e] & mask) == prefix)
                    atomicAdd(&hist[(key[e] >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t acc = 0u;
            int d = 255;
            for (; d > 0; --d) {
                if (acc + hist[d] >= need) break;
                acc += hist[d];
            }
            sel_digit = (uint32_t)d;
            sel_rank = need - acc;
        }
        __syncthreads();
        prefix |= sel_digit << shift;
        mask |= 255u << shift;
        need = sel_rank;
        __syncthreads();
    }
    // threshold key T = prefix; keys > T are all kept, `need` of the keys == T
    // (the lowest slots) complete the k
    const uint32_t T = prefix;
    uint32_t out_base = 0u, eq_base = 0u;
    for (int64_t i0 = 0; i0 < n; i0 += kPruneTile) {
        const int64_t i = i0 + (int64_t)kPer * threadIdx.x;
        uint32_t key[kPer];
        load_keys(P.score, n, i, key);
        uint32_t n_eq = 0u;
#pragma unroll
        for (int e = 0; e < kPer; ++e) n_eq += (i + e < n && key[e] == T) ? 1u : 0u;
        uint32_t eq_tot;
        uint32_t eq_rank = eq_base + block_scan(n_eq, &eq_tot, sh);
        uint32_t keep_mask = 0u, n_keep = 0u;
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            bool keep = false;
            if (i + e < n) {
                if (key[e] > T) keep = true;
                else if (key[e] == T) keep = (eq_rank++ < need);
            }
            keep_mask |= keep ? (1u << e) : 0u;
            n_keep += keep ? 1u : 0u;
        }
        uint32_t keep_tot;
        uint32_t pos = out_base + block_scan(n_keep, &keep_tot, sh);
#pragma unroll
        for (int e = 0; e < kPer; ++e)
            if (keep_mask & (1u << e)) P.sel[pos++] = (int32_t)(i + e);
        out_base += keep_tot;
        eq_base += eq_tot;
    }
}

// --------------------------------------------------------------- gather --

// Training records of listed keypoints: the 16 x 16 uint8 patch (zero
// outside the image) and the two scalar features. 64 threads per keypoint,
// 4 pixels each.
__global__ __launch_bounds__(256) void gather_kernel(GatherArgs a)
{
    int64_t g = blockIdx.x;
    int im = -1;
    for (int i = 0; i < a.n_images; ++i) {
        const int64_t cnt = (a.img[i].n + 3) / 4;
        if (g < cnt) {
            im = i;
            break;
        }
        g -= cnt;
    }
    if (im < 0) return;
    const GatherImg& I = a.img[im];
    const int q = threadIdx.x >> 6, t = threadIdx.x & 63;
    const int64_t e = g * 4 + q;
    if (e >= I.n) return;
    const int64_t slot = I.sel ? (int64_t)I.sel[e] : e;
    const bool ok = slot >= 0 && slot < I.n_kp;
    const int kx = ok ? I.x[slot] : 0, ky = ok ? I.y[slot] : 0;
    const int r = t >> 2, c0 = (t & 3) * 4;
    const int yy = ky + r - 8;
    uint32_t packed = 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int xx = kx + c0 + u - 8;
        const uint32_t v = (ok && yy >= 0 && yy < I.h && xx >= 0 && xx < I.w)
                               ? (uint32_t)I.data[(int64_t)yy * I.pitch + xx] : 0u;
        packed |= v << (8 * u);
    }
    *reinterpret_cast<uint32_t*>(I.patches + e * 256 + r * 16 + c0) = packed;
    if (t == 0) {
        I.extra[2 * e] = ok ? a.sfeat[I.scale[slot]] : 0.0f;
        I.extra[2 * e + 1] = ok ? I.contrast[slot] : 0.0f;
    }
}

// ------------------------------------------------------------- training --

constexpr int kTrainC = 64;       // candidates per workgroup
constexpr int kPad = kHid + 1;    // padded activation rows (no bank conflicts)

__global__ __launch_bounds__(256, 1) void train_kernel(TrainArgs a)
{
    __shared__ float w1[kHid * kIn];          // 66 KB
    __shared__ float w2[kHid * kHid];
    __shared__ float sb1[kHid], sb2[kHid], sw3[kHid];
    __shared__ uint8_t xs[256 * kTrainC];     // patch pixel k of candidate c at [k][c]
    __shared__ float ex[2][kTrainC];
    __shared__ float A1[kTrainC * kPad];      // a1, then d a1
    __shared__ float A2[kTrainC * kPad];      // a2, then d a2
    __shared__ float dz[kTrainC];
    __shared__ float red[2][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * kTrainC;
    const float* W = a.weights;

    for (int e = tid; e < kHid * kIn; e += 256) w1[e] = W[e];
    for (int e = tid; e < kHid * kHid; e += 256) w2[e] = W[kOffW2 + e];
    if (tid < kHid) {
        sb1[tid] = W[kOffB1 + tid];
        sb2[tid] = W[kOffB2 + tid];
        sw3[tid] = W[kOffW3 + tid];
    }
    for (int e = tid; e < 256 * kTrainC; e += 256) {
        const int c = e >> 8, k = e & 255;           // coalesced over k
        const int64_t cc = c0 + c;
        xs[k * kTrainC + c] = (cc < a.batch) ? a.patches[cc * 256 + k] : (uint8_t)0;
    }
    if (tid < 2 * kTrainC) {
        const int c = tid >> 1, f = tid & 1;
        const int64_t cc = c0 + c;
        ex[f][c] = (cc < a.batch) ? a.extra[cc * 2 + f] : 0.0f;
    }
    __syncthreads();

    // forward layer 1: wave q computes hidden units 16q .. 16q+15 of candidate `lane`
    const int c = lane;
    {
        float acc[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) acc[jj] = sb1[16 * wave + jj];
        for (int k = 0; k < 256; ++k) {
            const float xv = (float)xs[k * kTrainC + c] / 255.0f;
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) acc[jj] = fmaf(w1[(16 * wave + jj) * kIn + k], xv, acc[jj]);
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int j = 16 * wave + jj;
            acc[jj] = fmaf(w1[j * kIn + 256], ex[0][c], acc[jj]);
            acc[jj] = fmaf(w1[j * kIn + 257], ex[1][c], acc[jj]);
            A1[c * kPad + j] = acc[jj];
        }
    }
    __syncthreads();
    // forward layer 2
    {
        float acc[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) acc[jj] = sb2[16 * wave + jj];
        for (int k = 0; k < kHid; ++k) {
            const float h = fmaxf(A1[c * kPad + k], 0.0f);
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) acc[jj] = fmaf(w2[(16 * wave + jj) * kHid + k], h, acc[jj]);
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) A2[c * kPad + 16 * wave + jj] = acc[jj];
    }
    __syncthreads();
    // output, loss and d z (wave 0)
    if (wave == 0) {
        const int64_t cc = c0 + c;
        float z = a.weights[kOffB3];
        for (int j = 0; j < kHid; ++j) z = fmaf(sw3[j], fmaxf(A2[c * kPad + j], 0.0f), z);
        float m = 0.0f, y = 0.0f;
        if (cc < a.batch) {
            m = a.cweight[cc];
            y = a.labels[cc];
        }
        const float sg = 1.0f / (1.0f + expf(-z));
        dz[c] = m * (sg - y);                       // divided by the weight sum later
        float l = m * (fmaxf(z, 0.0f) - y * z + log1pf(expf(-fabsf(z))));
        float ms = m;
        for (int off = 32; off > 0; off >>= 1) {
            l += __shfl_xor(l, off);
            ms += __shfl_xor(ms, off);
        }
        if (lane == 0) {
            red[0][0] = l;
            red[1][0] = ms;
        }
    }
    __syncthreads();

    float* part = a.partials + (int64_t)blockIdx.x * (kParams + 2);
    // d w3, d b3, then d a2 in place
    if (tid < kHid) {
        const int j = tid;
        float s = 0.0f;
        for (int cc = 0; cc < kTrainC; ++cc) s = fmaf(dz[cc], fmaxf(A2[cc * kPad + j], 0.0f), s);
        part[kOffW3 + j] = s;
    }
    if (tid == kHid) {
        float s = 0.0f;
        for (int cc = 0; cc < kTrainC; ++cc) s += dz[cc];
        part[kOffB3] = s;
        part[kParams] = red[0][0];
        part[kParams + 1] = red[1][0];
    }
    __syncthreads();
    for (int e = tid; e < kTrainC * kHid; e += 256) {
        const int cc = e >> 6, j = e & 63;
        const float v = A2[cc * kPad + j];
        A2[cc * kPad + j] = (v > 0.0f) ? dz[cc] * sw3[j] : 0.0f;
    }
    __syncthreads();
    // d W2 [j][k] = sum_c d a2[c][j] h1[c][k]; d b2
    for (int e = tid; e < kHid * kHid; e += 256) {
        const int j = e >> 6, k = e & 63;
        float s = 0.0f;
        for (int cc = 0; cc < kTrainC; ++cc) s = fmaf(A2[cc * kPad + j], fmaxf(A1[cc * kPad + k], 0.0f), s);
        part[kOffW2 + e] = s;
    }
    if (tid < kHid) {
        float s = 0.0f;
        for (int cc = 0; cc < kTrainC; ++cc) s += A2[cc * kPad + tid];
        part[kOffB2 + tid] = s;
    }
    __syncthreads();
    // d a1 [c][k] = (sum_j W2[j][k] d a2[c][j]) [a1 > 0], in place
    {
        float g[16];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) g[kk] = 0.0f;
        for (int j = 0; j < kHid; ++j) {
            const float d = A2[c * kPad + j];
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) g[kk] = fmaf(w2[j * kHid + 16 * wave + kk], d, g[kk]);
        }
        __syncthreads();   // every read of A1 as h1 above is done
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int k = 16 * wave + kk;
            A1[c * kPad + k] = (A1[c * kPad + k] > 0.0f) ? g[kk] : 0.0f;
        }
    }
    __syncthreads();
    // d W1 [j][k] = sum_c d a1[c][j] x[c][k]; d b1
    for (int e = tid; e < kHid * kIn; e += 256) {
        const int j = e / kIn, k = e - j * kIn;
        float s = 0.0f;
        if (k < 256) {
            for (int cc = 0; cc < kTrainC; ++cc)
                s = fmaf(A1[cc * kPad + j], (float)xs[k * kTrainC + cc] / 255.0f, s);
        } else {
            for (int cc = 0; cc < kTrainC; ++cc) s = fmaf(A1[cc * kPad + j], ex[k - 256][cc], s);
        }
        part[e] = s;
    }
    if (tid < kHid) {
        float s = 0.0f;
        for (int cc = 0; cc < kTrainC; ++cc) s += A1[cc * kPad + tid];
        part[kOffB1 + tid] = s;
    }
}

// Sum of the partials in workgroup order, divided by the batch weight sum,
// then one Adam step per parameter (t = a.step >= 1).
__global__ __launch_bounds__(256) void adam_kernel(TrainArgs a, int n_parts)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > kParams) return;
    float msum = 0.0f;
    for (int b = 0; b < n_parts; ++b) msum += a.partials[(int64_t)b * (kParams + 2) + kParams + 1];
    const float inv = (msum > 0.0f) ? 1.0f / msum : 0.0f;
    if (p == kParams) {   // the loss
        float l = 0.0f;
        for (int b = 0; b < n_parts; ++b) l += a.partials[(int64_t)b * (kParams + 2) + kParams];
        if (a.loss) *a.loss = l * inv;
        return;
    }
    float g = 0.0f;
    for (int b = 0; b < n_parts; ++b) g += a.partials[(int64_t)b * (kParams + 2) + p];
    g *= inv;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float m = b1 * a.adam_m[p] + (1.0f - b1) * g;
    const float v = b2 * a.adam_v[p] + (1.0f - b2) * g * g;
    a.adam_m[p] = m;
    a.adam_v[p] = v;
    const float mh = m / (1.0f - powf(b1, (float)a.step));
    const float vh = v / (1.0f - powf(b2, (float)a.step));
    a.weights[p] -= a.lr * mh / (sqrtf(vh) + eps);
}

}  // namespace

int launch_score(const ScoreArgs& args, const float* weights, hipStream_t stream)
{
    int64_t total = 0;
    for (int i = 0; i < args.n_images; ++i) total += (args.img[i].n + kScoreGroup - 1) / kScoreGroup;
    if (total == 0) return LPSIFT_OK;
    const unsigned grid = (unsigned)(total < 1024 ? total : 1024);
    TimedScope ts(LPSIFT_KERNEL_SCORE, stream);
    hipLaunchKernelGGL(score_kernel, dim3(grid), dim3(256), 0, stream, args, weights);
    return hipGetLastError() == hipSuccess ? LPSIFT_OK : LPSIFT_EHIP;
}

int launch_prune(const PruneArgs& args, hipStream_t stream)
{
    TimedScope ts(LPSIFT_KERNEL_PRUNE, stream);
    hipLaunchKernelGGL(prune_kernel, dim3((unsigned)args.n_images), dim3(kPruneThreads), 0, stream,
                       args);
    return hipGetLastError() == hipSuccess ? LPSIFT_OK : LPSIFT_EHIP;
}

int launch_gather(const GatherArgs& args, hipStream_t stream)
{
    int64_t wg = 0;
    for (int i = 0; i < args.n_images; ++i) wg += (args.img[i].n + 3) / 4;
    if (wg == 0) return LPSIFT_OK;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)wg), dim3(256), 0, stream, args);
    return hipGetLastError() == hipSuccess ? LPSIFT_OK : LPSIFT_EHIP;
}

size_t train_workspace_bytes(int64_t batch)
{
    const int64_t parts = (batch + kTrainC - 1) / kTrainC;
    return (size_t)parts * (kParams + 2) * sizeof(float);
}

int launch_train(TrainArgs args, hipStream_t stream)
{
    const int64_t parts = (args.batch + kTrainC - 1) / kTrainC;
    TimedScope ts(LPSIFT_KERNEL_TRAIN, stream);
    hipLaunchKernelGGL(train_kernel, dim3((unsigned)parts), dim3(256), 0, stream, args);
    hipLaunchKernelGGL(adam_kernel, dim3((kParams + 1 + 255) / 256), dim3(256), 0, stream, args,
                       (int)parts);
    return hipGetLastError() == hipSuccess ? LPSIFT_OK : LPSIFT_EHIP;
}

}  // namespace lpsift
