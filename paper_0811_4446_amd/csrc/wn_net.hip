// Learned warm start: a 4-layer 3x3 convolutional network (7 -> 32 -> 32 ->
// 32 -> 3 channels, erf-form GELU after the first three layers, zero
// padding) that maps the prolonged coarse steady state (plus coordinate and
// parameter planes) to a correction of it on the fine grid.  Forward and
// input-gradient convolutions run on MFMA (v_mfma_f32_16x16x32_bf16: bf16
// operands, FP32 accumulation) as implicit GEMMs, and so does the weight
// gradient (a GEMM over pixels per tap, deterministic partial sums); Adam
// keeps FP32 master weights.
//
// Activations are NHWC bf16 with 32 channel slots (H = radial nodes, W =
// axial nodes, so a row is one radial line of the solver's fields).
#include <math.h>
#include <string.h>

#include <mutex>

#include "wn_net.h"

namespace mgf {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kC = 32;  // channel slots of every activation

struct LayerDims {
    int ci, co;
};
__constant__ LayerDims kLayers[4] = {{7, 32}, {32, 32}, {32, 32}, {32, 3}};
constexpr LayerDims kLayersH[4] = {{7, 32}, {32, 32}, {32, 32}, {32, 3}};

inline __host__ __device__ int64_t param_offset(int l) {
    int64_t off = 0;
    for (int q = 0; q < l; ++q) off += (int64_t)kLayersH[q].co * kLayersH[q].ci * 9 + kLayersH[q].co;
    return off;
}

// GELU with the exact normal CDF, Phi(z) = erfc(-z / sqrt 2) / 2.  erfc is
// the Chebyshev fit of Press et al. (Numerical Recipes, sec. 6.2): erfc(u) =
// t exp(-u^2 + P(t)), t = 1 / (1 + u/2), u >= 0, relative error below 1.2e-7
// for every u, and erfc(-u) = 2 - erfc(u).  One branch-free path of ~15
// vector instructions (hardware reciprocal and exp2), against ~40 with both
// branches of the library erff; with FP32 rounding the result stays within
// 2.4e-6 relative (|z| <= 5) and 4e-7 absolute of the exact GELU, far below
// the bf16 rounding of the stored activations.
__device__ inline float half_erfc_fit(float u) {  // erfc(u) / 2, u >= 0
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, u, 1.0f));
    float p = 0.17087277f;
    p = fmaf(p, t, -0.82215223f);
    p = fmaf(p, t, 1.48851587f);
    p = fmaf(p, t, -1.13520398f);
    p = fmaf(p, t, 0.27886807f);
    p = fmaf(p, t, -0.18628806f);
    p = fmaf(p, t, 0.09678418f);
    p = fmaf(p, t, 0.37409196f);
    p = fmaf(p, t, 1.00002368f);
    p = fmaf(p, t, -1.26551223f);
    return 0.5f * t * __builtin_amdgcn_exp2f(fmaf(-u, u, p) * 1.44269504088896341f);
}
__device__ inline float normal_cdf(float z) {
    const float h = half_erfc_fit(fabsf(z) * 0.70710678118654752f);
    return z >= 0.0f ? 1.0f - h : h;
}
__device__ inline float gelu(float z) { return z * normal_cdf(z); }
__device__ inline float gelu_grad(float z) {
    return normal_cdf(z) + z * __builtin_amdgcn_exp2f(-0.5f * 1.44269504088896341f * z * z) * 0.39894228040143268f;
}

// params (FP32, per layer W[co][ci][3][3] then b[co]) -> bf16 weight
// tiles: WB[l][tap][co][ci] for the forward pass and WT[l][tap'][ci][co]
// (taps mirrored) for the input gradient; biases copied to FP32 [l][32].
// WF0 (may be null): the first layer with its taps folded into K for the
// fused forward pass, [co][8 * tap + ci], 96 slots per row, zero for ci = 7
// and tap >= 9.
__global__ void k_pack_weights(const float *__restrict__ params, __bf16 *__restrict__ WB, __bf16 *__restrict__ WT,
                               float *__restrict__ bias, __bf16 *__restrict__ WF0) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;  // over 4 * 9 * 32 * 32
    if (WF0 && t < kC * 96) {
        int co = t / 96, tap = (t % 96) / 8, ci = t % 8;
        WF0[t] = (__bf16)((tap < 9 && ci < 7) ? params[((int64_t)co * 7 + ci) * 9 + tap] : 0.0f);
    }
    if (t >= 4 * 9 * kC * kC) return;
    int l = t / (9 * kC * kC), r = t % (9 * kC * kC);
    int tap = r / (kC * kC), co = (r / kC) % kC, ci = r % kC;
    LayerDims d = kLayers[l];
    const float *W = params + param_offset(l);
    float w = (co < d.co && ci < d.ci) ? W[((int64_t)co * d.ci + ci) * 9 + tap] : 0.0f;
    WB[(((int64_t)l * 9 + tap) * kC + co) * kC + ci] = (__bf16)w;
    int tapm = 8 - tap;  // (ky, kx) -> (2-ky, 2-kx)
    WT[(((int64_t)l * 9 + tapm) * kC + ci) * kC + co] = (__bf16)w;
    if (tap == 0 && ci == 0) bias[l * kC + co] = (co < d.co) ? W[(int64_t)d.co * d.ci * 9 + co] : 0.0f;
}

// FP32 NCHW [B][7][H][W] -> bf16 NHWC with 32 channel slots (zeros beyond
// 7): one thread per pixel and group of 8 slots, one 16-byte store each.
__global__ void k_pack_input(const float *__restrict__ in, __bf16 *__restrict__ x, int B, int H, int W) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over npix * 4
    const int64_t npix = (int64_t)B * H * W;
    if (t >= npix * (kC / 8)) return;
    const int c8 = (int)(t % (kC / 8));
    const int64_t pix = t / (kC / 8);
    const int64_t b = pix / ((int64_t)H * W), hw = pix % ((int64_t)H * W);
    bf16x8 v = {};
    if (c8 == 0)
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] = (__bf16)in[(b * 7 + c) * H * W + hw];
    *reinterpret_cast<bf16x8 *>(x + pix * kC + 8 * c8) = v;
}

// ---------------------------------------------------------------------------
// Fused forward pass (inference): one workgroup computes all four layers for
// a kFT x kFT tile of output pixels of one image and keeps every
// intermediate activation in LDS, so the only HBM traffic is the 7 input
// planes (with a 4-pixel halo) and the 3 output planes.  Layer l's region is
// the output tile grown by 3 - l pixels on each side; pixels of a region
// outside the image hold zero, which is the zero padding of every layer.
//
// The MFMA computes D (output channels x 16 pixels) = W (channels x K) *
// X (K x 16 pixels): lane (m, kg) supplies W[m][8kg..8kg+7] and the 8-channel
// chunk kg of pixel m, and receives channels 4kg..4kg+3 of pixel m.  The
// first layer (7 input channels) folds its nine taps into K: k = 8 * tap +
// ci, 96 slots, three MFMAs per 16 output channels instead of nine.
//
// LDS activations are chunk planes: plane j holds channels 8j..8j+7 of every
// pixel of the region as one 16-byte record, so the 16 lanes that read one
// chunk of 16 consecutive pixels touch 256 contiguous bytes.
// ---------------------------------------------------------------------------
constexpr int kFT = 16;            // output tile side
constexpr int kFIn = kFT + 8;      // input region side
constexpr int kFThreads = 256;     // four waves
constexpr int kFK0 = 96;           // folded K of the first layer (12 taps x 8 channel slots)
constexpr int kFBufA = 4 * (kFT + 6) * (kFT + 6);  // 16-byte records: layer-1 output, then layer-3 output
constexpr int kFBufB = 4 * (kFT + 4) * (kFT + 4);  // layer-2 output; the input planes before it
static_assert(kFIn * kFIn <= kFBufB, "input planes must fit in the layer-2 buffer");
static_assert(4 * (kFT + 2) * (kFT + 2) <= kFBufA, "layer-3 output must fit in the first buffer");

typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;

// Bias plus GELU (or zero outside the image) of the four channels a lane
// holds, packed for one 8-byte LDS store.
__device__ inline bf16x4 fused_act(f32x4 acc, const float *b4, bool inside) {
    bf16x4 o;
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = (__bf16)(inside ? gelu(acc[i] + b4[i]) : 0.0f);
    return o;
}

// Pixel p of a region of side S (clamped to the region's last pixel when p
// lies past it, so that every LDS address stays inside the region).
template <int S>
__device__ inline void region_rc(int p, int &r, int &c) {
    const int pc = p < S * S ? p : S * S - 1;
    r = pc / S;
    c = pc % S;
}

// One hidden 32 -> 32 layer over a region of side S (input region side
// S + 2, chunk-plane stride (S + 2)^2; output chunk-plane stride S^2).
// (oy, ox): image coordinates of the output region's first pixel.  A wave
// takes two blocks of 16 pixels at a time (blk and blk + 4), so four
// independent MFMA chains are in flight and one block's GELU overlaps the
// other's; a block past the region is computed but not stored.
template <int S>
__device__ inline void fused_hidden(const bf16x8 *__restrict__ src, bf16x4 *__restrict__ dst,
                                    const bf16x8 (&w)[9][2], const float (&b)[2][4], int oy, int ox, int H, int W,
                                    int wave, int m, int kg) {
    constexpr int SI = S + 2, NI = SI * SI, NO = S * S, NB = (NO + 15) / 16, NW = kFThreads / 64;
    for (int blk = wave; blk < NB; blk += 2 * NW) {
        const int p = blk * 16 + m, q = (blk + NW) * 16 + m;
        int rp, cp, rq, cq;
        region_rc<S>(p, rp, cp);
        region_rc<S>(q, rq, cq);
        const bf16x8 *sp = src + kg * NI + rp * SI + cp;
        const bf16x8 *sq = src + kg * NI + rq * SI + cq;
        f32x4 a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0}, e0 = {0, 0, 0, 0}, e1 = {0, 0, 0, 0};
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const bf16x8 x = sp[(tap / 3) * SI + tap % 3];
            const bf16x8 y = sq[(tap / 3) * SI + tap % 3];
            a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[tap][0], x, a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[tap][1], x, a1, 0, 0, 0);
            e0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[tap][0], y, e0, 0, 0, 0);
            e1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[tap][1], y, e1, 0, 0, 0);
        }
        // channels 4kg..4kg+3 (+16): plane (kg >> 1) (+2), half kg & 1
        if (p < NO) {
            const int gy = oy + rp, gx = ox + cp;
            const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
            dst[((kg >> 1) * NO + p) * 2 + (kg & 1)] = fused_act(a0, b[0], inside);
            dst[((2 + (kg >> 1)) * NO + p) * 2 + (kg & 1)] = fused_act(a1, b[1], inside);
        }
        if (q < NO) {
            const int gy = oy + rq, gx = ox + cq;
            const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
            dst[((kg >> 1) * NO + q) * 2 + (kg & 1)] = fused_act(e0, b[0], inside);
            dst[((2 + (kg >> 1)) * NO + q) * 2 + (kg & 1)] = fused_act(e1, b[1], inside);
        }
    }
}

__device__ inline void load_hidden_weights(const __bf16 *__restrict__ wl, int m, int kg, bf16x8 (&w)[9][2]) {
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int h = 0; h < 2; ++h)
            w[tap][h] = *reinterpret_cast<const bf16x8 *>(wl + ((int64_t)tap * kC + 16 * h + m) * kC + 8 * kg);
}

__device__ inline void load_bias(const float *__restrict__ bl, int kg, float (&b)[2][4]) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) b[h][i] = bl[16 * h + 4 * kg + i];
}

// in: FP32 NCHW [B][7][H][W]; WF0: first layer [32][96] bf16 (k = 8 * tap +
// ci); WB: [4][9][32][32] bf16 ([layer][tap][co][ci], layer 0 unused);
// bias: FP32 [4][32]; out: FP32 NCHW [B][3][H][W].  Tiles are numbered
// (image, tile row, tile column); workgroup g takes tiles g, g + gridDim.x,
// ...  Keeping the two hidden layers' weights resident across tiles would
// need 296 registers per lane, one wave per SIMD instead of two, so each
// layer's weights (up to 72 registers per lane) are reloaded per tile.
__global__ __launch_bounds__(kFThreads) void k_wn_forward_fused(const float *__restrict__ in,
                                                               const __bf16 *__restrict__ WF0,
                                                               const __bf16 *__restrict__ WB,
                                                               const float *__restrict__ bias, int B, int H, int W,
                                                               float *__restrict__ out) {
    __shared__ bf16x8 bufA[kFBufA];
    __shared__ bf16x8 bufB[kFBufB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int tiles_x = (W + kFT - 1) / kFT, tiles_y = (H + kFT - 1) / kFT;
    const int64_t ntiles = (int64_t)B * tiles_x * tiles_y;
    float bl[2][4];

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tx = (int)(tile % tiles_x);
        const int ty = (int)((tile / tiles_x) % tiles_y);
        const int b = (int)(tile / ((int64_t)tiles_x * tiles_y));
        const int y0 = ty * kFT, x0 = tx * kFT;
        // The weight pointer is made opaque per tile so that the compiler
        // does not hoist every layer's weight loads out of the tile loop
        // (all four layers' fragments at once would not fit two waves per
        // SIMD); each layer's are loaded while the layer before it runs.
        const __bf16 *wb = WB;
        asm volatile("" : "+s"(wb));

        // First-layer weights: A fragments of the folded K.
        bf16x8 w0[3][2];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                w0[j][h] = *reinterpret_cast<const bf16x8 *>(WF0 + (int64_t)(16 * h + m) * kFK0 + 32 * j + 8 * kg);
        load_bias(bias, kg, bl);
        bf16x8 w1[9][2];
        load_hidden_weights(wb + (int64_t)1 * 9 * kC * kC, m, kg, w1);

        // Input planes of the region (side kFIn, origin (y0 - 4, x0 - 4))
        // as bf16 records of 8 channel slots (the eighth is zero) in bufB.
        // The previous tile's last reads of bufB ended at its third barrier.
        for (int q = tid; q < kFIn * kFIn; q += kFThreads) {
            const int gy = y0 - 4 + q / kFIn, gx = x0 - 4 + q % kFIn;
            bf16x8 v = {};
            if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
                const float *src = in + ((int64_t)b * 7 * H + gy) * W + gx;
#pragma unroll
                for (int ci = 0; ci < 7; ++ci) v[ci] = (__bf16)src[(int64_t)ci * H * W];
            }
            bufB[q] = v;
        }
        __syncthreads();

        // Layer 1: 7 -> 32 over side kFT + 6, taps folded into K; two
        // blocks of 16 pixels per wave at a time, as in fused_hidden.
        {
            constexpr int S = kFT + 6, NO = S * S, NB = (NO + 15) / 16, NW = kFThreads / 64;
            bf16x4 *dst = reinterpret_cast<bf16x4 *>(bufA);
            const bf16x8 zero8 = {};
            for (int blk = wave; blk < NB; blk += 2 * NW) {
                const int p = blk * 16 + m, q = (blk + NW) * 16 + m;
                int rp, cp, rq, cq;
                region_rc<S>(p, rp, cp);
                region_rc<S>(q, rq, cq);
                f32x4 a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0}, e0 = {0, 0, 0, 0}, e1 = {0, 0, 0, 0};
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int tap = 4 * j + kg;
                    const int off = (tap / 3) * kFIn + tap % 3;
                    const bf16x8 x = tap < 9 ? bufB[rp * kFIn + cp + off] : zero8;
                    const bf16x8 y = tap < 9 ? bufB[rq * kFIn + cq + off] : zero8;
                    a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0[j][0], x, a0, 0, 0, 0);
                    a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0[j][1], x, a1, 0, 0, 0);
                    e0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0[j][0], y, e0, 0, 0, 0);
                    e1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0[j][1], y, e1, 0, 0, 0);
                }
                if (p < NO) {
                    const int gy = y0 - 3 + rp, gx = x0 - 3 + cp;
                    const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
                    dst[((kg >> 1) * NO + p) * 2 + (kg & 1)] = fused_act(a0, bl[0], inside);
                    dst[((2 + (kg >> 1)) * NO + p) * 2 + (kg & 1)] = fused_act(a1, bl[1], inside);
                }
                if (q < NO) {
                    const int gy = y0 - 3 + rq, gx = x0 - 3 + cq;
                    const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
                    dst[((kg >> 1) * NO + q) * 2 + (kg & 1)] = fused_act(e0, bl[0], inside);
                    dst[((2 + (kg >> 1)) * NO + q) * 2 + (kg & 1)] = fused_act(e1, bl[1], inside);
                }
            }
        }
        load_bias(bias + kC, kg, bl);
        bf16x8 w2[9][2];
        load_hidden_weights(wb + (int64_t)2 * 9 * kC * kC, m, kg, w2);
        __syncthreads();

        // Layer 2: bufA (side kFT + 6) -> bufB (side kFT + 4).
        fused_hidden<kFT + 4>(bufA, reinterpret_cast<bf16x4 *>(bufB), w1, bl, y0 - 2, x0 - 2, H, W, wave, m, kg);
        load_bias(bias + 2 * kC, kg, bl);
        bf16x8 w3[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
            w3[tap] = *reinterpret_cast<const bf16x8 *>(wb + (((int64_t)3 * 9 + tap) * kC + m) * kC + 8 * kg);
        __syncthreads();

        // Layer 3: bufB (side kFT + 4) -> bufA (side kFT + 2).
        fused_hidden<kFT + 2>(bufB, reinterpret_cast<bf16x4 *>(bufA), w2, bl, y0 - 1, x0 - 1, H, W, wave, m, kg);
        __syncthreads();

        // Layer 4: 32 -> 3 over the output tile; output channels 0..15 on
        // one MFMA (3 real), lanes kg == 0 hold channels 0..3.  The next
        // tile's first layer writes bufA only after its staging barrier,
        // which every wave reaches after these reads.
        {
            constexpr int S = kFT, SI = S + 2, NI = SI * SI, NB = S * S / 16;
            float b3[3];
#pragma unroll
            for (int co = 0; co < 3; ++co) b3[co] = bias[3 * kC + co];
            for (int blk = wave; blk < NB; blk += kFThreads / 64) {
                const int p = blk * 16 + m;
                const int r = p / S, c = p % S;
                const bf16x8 *s0 = bufA + kg * NI + r * SI + c;
                f32x4 a = {0, 0, 0, 0}, e = {0, 0, 0, 0};
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) {
                    if (tap < 5)
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3[tap], s0[(tap / 3) * SI + tap % 3], a, 0, 0, 0);
                    else
                        e = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3[tap], s0[(tap / 3) * SI + tap % 3], e, 0, 0, 0);
                }
                a += e;
                const int gy = y0 + r, gx = x0 + c;
                if (kg == 0 && gy < H && gx < W) {
#pragma unroll
                    for (int co = 0; co < 3; ++co) out[(((int64_t)b * 3 + co) * H + gy) * W + gx] = a[co] + b3[co];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// One 3x3 convolution layer for the training passes (every layer's
// activations are kept in HBM for the backward pass).  One workgroup per
// 16 x 16 output tile: the input tile with its one-pixel halo is staged once
// in LDS (8-channel planes of 16-byte records, as in the fused forward
// pass), the 32 x 32 weights of the nine taps stay in registers, and each
// wave takes rows of 16 pixels: D (output channels x pixels) = W X on
// v_mfma_f32_16x16x32_bf16, lanes (m, kg) receiving channels 4kg..4kg+3 (+16)
// of pixel m.  Activations are NHWC with 32 channel slots.
// MODE 0: hidden layer   -> z (FP32) and gelu(z) (bf16)
// MODE 1: last layer     -> FP32 NCHW output, channels < 3
// MODE 2: input gradient -> (sum) * gelu'(zprev), bf16 (w: the mirrored,
//         transposed weights, the same [tap][out][in] layout)
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(kFThreads) void k_conv3x3_tile(const __bf16 *__restrict__ in,
                                                            const __bf16 *__restrict__ w,
                                                            const float *__restrict__ bias, int B, int H, int W,
                                                            __bf16 *__restrict__ out_act, float *__restrict__ out_z,
                                                            float *__restrict__ out_f, const float *__restrict__ zprev) {
    constexpr int SI = kFT + 2, NI = SI * SI;
    __shared__ bf16x8 tile[4 * NI];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int tiles_x = (W + kFT - 1) / kFT, tiles_y = (H + kFT - 1) / kFT;
    const int tx = (int)(blockIdx.x % tiles_x);
    const int ty = (int)((blockIdx.x / tiles_x) % tiles_y);
    const int b = (int)(blockIdx.x / ((unsigned)tiles_x * tiles_y));
    if (b >= B) return;
    const int y0 = ty * kFT, x0 = tx * kFT;
    bf16x8 wr[9][2];
    load_hidden_weights(w, m, kg, wr);
    for (int q = tid; q < 4 * NI; q += kFThreads) {
        const int pix = q >> 2, c = q & 3;
        const int gy = y0 - 1 + pix / SI, gx = x0 - 1 + pix % SI;
        bf16x8 v = {};
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = *reinterpret_cast<const bf16x8 *>(in + (((int64_t)b * H + gy) * W + gx) * kC + 8 * c);
        tile[c * NI + pix] = v;
    }
    __syncthreads();
    for (int r = wave; r < kFT; r += kFThreads / 64) {
        const bf16x8 *s0 = tile + kg * NI + r * SI + m;
        f32x4 a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const bf16x8 x = s0[(tap / 3) * SI + tap % 3];
            a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[tap][0], x, a0, 0, 0, 0);
            if (MODE != 1) a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[tap][1], x, a1, 0, 0, 0);
        }
        const int gy = y0 + r, gx = x0 + m;
        if (gy >= H || gx >= W) continue;
        const int64_t pix = ((int64_t)b * H + gy) * W + gx;
        if (MODE == 1) {
            if (kg == 0) {
#pragma unroll
                for (int co = 0; co < 3; ++co) out_f[(((int64_t)b * 3 + co) * H + gy) * W + gx] = a0[co] + bias[co];
            }
            continue;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const f32x4 acc = h == 0 ? a0 : a1;
            const int c0 = 16 * h + 4 * kg;
            bf16x4 o;
            if (MODE == 0) {
                f32x4 z;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    z[i] = acc[i] + bias[c0 + i];
                    o[i] = (__bf16)gelu(z[i]);
                }
                *reinterpret_cast<f32x4 *>(out_z + pix * kC + c0) = z;
            } else {
                const f32x4 zp = *reinterpret_cast<const f32x4 *>(zprev + pix * kC + c0);
#pragma unroll
                for (int i = 0; i < 4; ++i) o[i] = (__bf16)(acc[i] * gelu_grad(zp[i]));
            }
            *reinterpret_cast<bf16x4 *>(out_act + pix * kC + c0) = o;
        }
    }
}

// MSE loss over B*3*H*W outputs: per-block partial sums of squared errors
// and the output gradient 2 (out - target) / count as bf16 NHWC (3 of the
// 32 channel slots).
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ out, const float *__restrict__ tgt, int B,
                                             int H, int W, __bf16 *__restrict__ dz, double *__restrict__ part) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t npix = (int64_t)B * H * W;
    double s = 0.0;
    if (t < npix) {
        int64_t b = t / ((int64_t)H * W), hw = t % ((int64_t)H * W);
        double inv = 2.0 / (3.0 * (double)npix);
        bf16x8 g8 = {};
        for (int c = 0; c < 3; ++c) {
            int64_t q = (b * 3 + c) * H * W + hw;
            float e = out[q] - tgt[q];
            s += (double)e * e;
            g8[c] = (__bf16)(float)(inv * e);
        }
        // slots 3..31 are zero: four 16-byte stores
        bf16x8 *d = reinterpret_cast<bf16x8 *>(dz + t * kC);
        const bf16x8 zero8 = {};
        d[0] = g8;
        d[1] = d[2] = d[3] = zero8;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Pixels per weight-gradient chunk: kWgSteps MFMA K steps of 32 pixels
// between two barriers.
constexpr int kWgSteps = 4;
constexpr int kWgChunk = 32 * kWgSteps;

// Weight and bias gradient of one layer on MFMA.  Per tap (dy, dx) the
// gradient is a GEMM over pixels: dW_tap[co][ci] = sum_p dz[p][co] *
// a[p + (dy, dx)][ci], i.e. D (co x ci) += A (co x 32 pixels) * B (32
// pixels x ci) per K step of 32 consecutive pixels of one image row, two by
// two 16x16x32 bf16 tiles with FP32 accumulators.  Wave `tap` of the
// 9-wave workgroup owns one tap.  The chunk's dz (transposed, [co][pixel])
// and the three input rows it reads (transposed, [row][ci][pixel], pixels
// x0-1..x0+kWgChunk, each value stored once) are staged in LDS; a tap's operand
// of 8 pixels starting dx pixels into the row is cut from two aligned
// 16-byte LDS reads (a shift by 0, 1 or 2 bf16 slots).  Wave 0 also sums dz
// for the bias gradient.  Every workgroup writes its partial sums in the
// layout k_wgrad_reduce adds in a fixed order.
constexpr int kWgPad = kWgChunk + 8;    // LDS row length (pixels) of the transposed dz
constexpr int kWgRow = kWgChunk + 16;   // LDS row length of the transposed input rows (kWgChunk + 2 used)
static_assert(kWgPad % 8 == 0 && kWgRow % 8 == 0, "16-byte LDS rows");
typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;
__global__ __launch_bounds__(576) void k_wgrad_mfma(const __bf16 *__restrict__ dz, const __bf16 *__restrict__ a,
                                                    int B, int H, int W, float *__restrict__ part) {
    __shared__ __attribute__((aligned(16))) __bf16 sdz[kC][kWgPad];
    __shared__ __attribute__((aligned(16))) __bf16 sa[3][kC][kWgRow];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int m = lane & 15, kg = lane >> 4;
    const int tap = wave, ky = tap / 3, kx = tap % 3;
    f32x4 acc[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) acc[h][h2] = f32x4{0, 0, 0, 0};
    float accb = 0.0f;
    // the slots past the kWgChunk + 2 staged pixels are read (and shifted out) only
    const __bf16 zero = (__bf16)0.0f;
    for (int q = t; q < 3 * kC * (kWgRow - (kWgChunk + 2)); q += blockDim.x) {
        const int w = kWgRow - (kWgChunk + 2);
        sa[q / (kC * w)][(q / w) % kC][kWgChunk + 2 + q % w] = zero;
    }
    const int chunks_x = (W + kWgChunk - 1) / kWgChunk;
    const int64_t nchunks = (int64_t)B * H * chunks_x;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int cx = (int)(ch % chunks_x);
        const int64_t by = ch / chunks_x;
        const int y = (int)(by % H), b = (int)(by / H);
        const int x0 = cx * kWgChunk;
        __syncthreads();
        // dz: kWgChunk pixels x 4 groups of 8 channels, one 16-byte load each
        for (int q = t; q < kWgChunk * (kC / 8); q += blockDim.x) {
            const int p = q / (kC / 8), c8 = (q % (kC / 8)) * 8, x = x0 + p;
            bf16x8 v = {};
            if (x < W) v = *reinterpret_cast<const bf16x8 *>(dz + (((int64_t)b * H + y) * W + x) * kC + c8);
#pragma unroll
            for (int u = 0; u < 8; ++u) sdz[c8 + u][p] = v[u];
        }
        // the three input rows y-1..y+1 over pixels x0-1..x0+kWgChunk
        for (int q = t; q < 3 * (kWgChunk + 2) * (kC / 8); q += blockDim.x) {
            const int r = q / ((kWgChunk + 2) * (kC / 8)), P = (q / (kC / 8)) % (kWgChunk + 2);
            const int c8 = (q % (kC / 8)) * 8;
            const int yy = y + r - 1, xx = x0 + P - 1;
            bf16x8 v = {};
            if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                v = *reinterpret_cast<const bf16x8 *>(a + (((int64_t)b * H + yy) * W + xx) * kC + c8);
#pragma unroll
            for (int u = 0; u < 8; ++u) sa[r][c8 + u][P] = v[u];
        }
        __syncthreads();
#pragma unroll
        for (int st = 0; st < kWgSteps; ++st) {
            if (x0 + 32 * st >= W) break;  // a step wholly past the row's end adds nothing
            const int o = 32 * st + 8 * kg;  // first pixel slot of this lane's K group
            bf16x8 A[2], Bm[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                A[h] = *reinterpret_cast<const bf16x8 *>(&sdz[h * 16 + m][o]);
                // slots o + kx .. o + kx + 7 of row ky (slot P holds pixel x0 - 1 + P)
                const u32x4 q0 = *reinterpret_cast<const u32x4 *>(&sa[ky][h * 16 + m][o]);
                const u32x4 q1 = *reinterpret_cast<const u32x4 *>(&sa[ky][h * 16 + m][o + 8]);
                u32x4 r;
                if (kx == 0) {
                    r = q0;
                } else if (kx == 2) {
                    r = u32x4{q0[1], q0[2], q0[3], q1[0]};
                } else {
                    r = u32x4{__builtin_amdgcn_alignbyte(q0[1], q0[0], 2), __builtin_amdgcn_alignbyte(q0[2], q0[1], 2),
                              __builtin_amdgcn_alignbyte(q0[3], q0[2], 2), __builtin_amdgcn_alignbyte(q1[0], q0[3], 2)};
                }
                Bm[h] = __builtin_bit_cast(bf16x8, r);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2)
                    acc[h][h2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[h], Bm[h2], acc[h][h2], 0, 0, 0);
        }
        if (wave == 0 && lane < kC)
            for (int p = 0; p < kWgChunk; ++p) accb += (float)sdz[lane][p];
    }
    float *o = part + (int64_t)blockIdx.x * (9 * kC * kC + kC);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = h * 16 + 4 * kg + i, ci = h2 * 16 + m;
                o[((int64_t)co * kC + ci) * 9 + tap] = acc[h][h2][i];
            }
    if (wave == 0 && lane < kC) o[9 * kC * kC + lane] = accb;
}

// grad (param layout of layer l) = sum over workgroups of the partials.  A
// workgroup owns 64 consecutive entries e; wave w adds the partials of
// workgroups w, w + 4, w + 8, ... in eight interleaved running sums, and the
// four waves' sums are combined in a fixed order, so the result does not
// depend on scheduling.  (One thread per entry over all partials used only
// 37 workgroups and ran at ~0.5 TB/s.)
constexpr int kWrEntries = 64;
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *__restrict__ part, int nwg, int ci_real,
                                                      int co_real, float *__restrict__ grad) {
    __shared__ float sums[4][kWrEntries];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int E = 9 * kC * kC + kC;
    const int e = blockIdx.x * kWrEntries + lane;
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (e < E) {
        int g = wave, k = 0;
        for (; g + 28 < nwg; g += 32)
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += part[(int64_t)(g + 4 * u) * E + e];
        for (; g < nwg; g += 4, k = (k + 1) & 7) acc[k] += part[(int64_t)g * E + e];
    }
    sums[wave][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    if (wave != 0 || e >= E) return;
    const float s = (sums[0][lane] + sums[1][lane]) + (sums[2][lane] + sums[3][lane]);
    if (e < 9 * kC * kC) {
        int co = e / (kC * 9), ci = (e / 9) % kC, tap = e % 9;
        if (co < co_real && ci < ci_real) grad[((int64_t)co * ci_real + ci) * 9 + tap] = s;
    } else {
        int co = e - 9 * kC * kC;
        if (co < co_real) grad[(int64_t)co_real * ci_real * 9 + co] = s;
    }
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float c1, float c2) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float gt = g[t];
    float mt = b1 * m[t] + (1.0f - b1) * gt;
    float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

__global__ void k_sum_double(const double *__restrict__ part, int n, double *__restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

struct Scratch {
    __bf16 *WB, *WT, *WF0, *X0, *A[3], *DZ[2];
    float *bias, *Z[3], *OUT, *part, *grad;
    double *lpart, *loss;
    int nwg;
};

constexpr int kWgradBlocks = 512;

Scratch carve_scratch(char *base, int B, int H, int W, int64_t *bytes) {
    Scratch s;
    int64_t off = 0;
    auto take = [&](int64_t n) {
        off = (off + 255) / 256 * 256;
        char *p = base ? base + off : nullptr;
        off += n;
        return p;
    };
    int64_t npix = (int64_t)B * H * W;
    s.WB = (__bf16 *)take(4 * 9 * kC * kC * 2);
    s.WT = (__bf16 *)take(4 * 9 * kC * kC * 2);
    s.bias = (float *)take(4 * kC * 4);
    s.WF0 = (__bf16 *)take(kC * kFK0 * 2);
    s.X0 = (__bf16 *)take(npix * kC * 2);
    for (int i = 0; i < 3; ++i) s.A[i] = (__bf16 *)take(npix * kC * 2);
    for (int i = 0; i < 3; ++i) s.Z[i] = (float *)take(npix * kC * 4);
    for (int i = 0; i < 2; ++i) s.DZ[i] = (__bf16 *)take(npix * kC * 2);
    s.OUT = (float *)take(npix * 3 * 4);
    s.nwg = kWgradBlocks;
    s.part = (float *)take((int64_t)kWgradBlocks * (9 * kC * kC + kC) * 4);
    s.grad = (float *)take(kWnParams * 4);
    s.lpart = (double *)take(((npix + 255) / 256 + 1) * 8);
    s.loss = (double *)take(8);
    if (bytes) *bytes = (off + 255) / 256 * 256;
    return s;
}

// Tiles of kFT x kFT output pixels of a batch (one workgroup each).
constexpr int64_t kFusedMaxTiles = (int64_t)1 << 24;

int64_t fused_tiles(int B, int H, int W) {
    return (int64_t)B * ((H + kFT - 1) / kFT) * ((W + kFT - 1) / kFT);
}

void forward_pass(const Scratch &s, const float *params, const float *in, int B, int H, int W, hipStream_t st) {
    int64_t npix = (int64_t)B * H * W;
    k_pack_weights<<<(4 * 9 * kC * kC + 255) / 256, 256, 0, st>>>(params, s.WB, s.WT, s.bias, nullptr);
    k_pack_input<<<(unsigned)((npix * (kC / 8) + 255) / 256), 256, 0, st>>>(in, s.X0, B, H, W);
    const unsigned g = (unsigned)fused_tiles(B, H, W);
    const __bf16 *x = s.X0;
    for (int l = 0; l < 3; ++l) {
        k_conv3x3_tile<0><<<g, kFThreads, 0, st>>>(x, s.WB + (int64_t)l * 9 * kC * kC, s.bias + l * kC, B, H, W,
                                                   s.A[l], s.Z[l], nullptr, nullptr);
        x = s.A[l];
    }
    k_conv3x3_tile<1><<<g, kFThreads, 0, st>>>(x, s.WB + (int64_t)3 * 9 * kC * kC, s.bias + 3 * kC, B, H, W, nullptr,
                                               nullptr, s.OUT, nullptr);
}

// Inference: weights packed into s (WB, bias, WF0), then the fused kernel
// from the caller's input planes to the caller's output planes.
// Compute units of the current device (looked up once per device).
int fused_cus() {
    static std::mutex mu;
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if (!cus[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

void forward_fused(const Scratch &s, const float *params, const float *in, float *out, int B, int H, int W,
                   hipStream_t st) {
    k_pack_weights<<<(4 * 9 * kC * kC + 255) / 256, 256, 0, st>>>(params, s.WB, s.WT, s.bias, s.WF0);
    const int64_t tiles = fused_tiles(B, H, W);
    const int64_t slots = 2 * (int64_t)fused_cus();  // two 56.6 KB LDS workgroups per compute unit
    k_wn_forward_fused<<<(unsigned)(tiles < slots ? tiles : slots), kFThreads, 0, st>>>(in, s.WF0, s.WB, s.bias, B,
                                                                                       H, W, out);
}

// Loss and gradient into s.grad (forward pass already run).
void backward_pass(const Scratch &s, const float *target, int B, int H, int W, hipStream_t st) {
    int64_t npix = (int64_t)B * H * W;
    unsigned nb = (unsigned)((npix + 255) / 256);
    k_mse<<<nb, 256, 0, st>>>(s.OUT, target, B, H, W, s.DZ[0], s.lpart);
    k_sum_double<<<1, 256, 0, st>>>(s.lpart, (int)nb, s.loss);
    const unsigned g = (unsigned)fused_tiles(B, H, W);
    int cur = 0;
    for (int l = 3; l >= 0; --l) {
        const __bf16 *aprev = (l == 0) ? s.X0 : s.A[l - 1];
        k_wgrad_mfma<<<s.nwg, 576, 0, st>>>(s.DZ[cur], aprev, B, H, W, s.part);
        const unsigned nred = (9 * kC * kC + kC + kWrEntries - 1) / kWrEntries;
        k_wgrad_reduce<<<nred, 256, 0, st>>>(s.part, s.nwg, kLayersH[l].ci, kLayersH[l].co,
                                             s.grad + param_offset(l));
        if (l > 0) {
            k_conv3x3_tile<2><<<g, kFThreads, 0, st>>>(s.DZ[cur], s.WT + (int64_t)l * 9 * kC * kC, nullptr, B, H,
                                                       W, s.DZ[cur ^ 1], nullptr, nullptr, s.Z[l - 1]);
            cur ^= 1;
        }
    }
}

// Build the seven input planes of one sample from solver fields on the fine
// grid: the prolonged coarse state (V, ne, np), r, z, V_top and the mobility
// ratio.  Normalisation: V / V_top, n / n_scale, r / R, z / d, V_top / 5,
// log10(ratio) / 3, where n_scale is the largest prolonged density.
__global__ void k_features(Geom g, const double *__restrict__ V, const double *__restrict__ ne,
                           const double *__restrict__ np, double R, double d, double vtop, double ratio,
                           const double *__restrict__ nscale, float *__restrict__ out) {
    int j = blockIdx.x * 64 + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    int64_t p = (int64_t)i * g.pitch + j;
    int64_t HW = (int64_t)(g.nr + 1) * (g.nz + 1), q = (int64_t)i * (g.nz + 1) + j;
    double ns = *nscale > 0 ? *nscale : 1.0;
    out[0 * HW + q] = (float)(V[p] / vtop);
    out[1 * HW + q] = (float)(ne[p] / ns);
    out[2 * HW + q] = (float)(np[p] / ns);
    out[3 * HW + q] = (float)(i * (g.dr) / R);
    out[4 * HW + q] = (float)(g.z[j] / d);
    out[5 * HW + q] = (float)(vtop / 5.0);
    out[6 * HW + q] = (float)(log10(ratio) / 3.0);
}

// Largest density of the prolonged state (single workgroup, fixed order).
__global__ void k_field_max(Geom g, const double *__restrict__ a, const double *__restrict__ b,
                            double *__restrict__ out) {
    __shared__ double sh[256];
    double m = 0.0;
    int64_t n = (int64_t)(g.nr + 1) * (g.nz + 1);
    for (int64_t t = threadIdx.x; t < n; t += 256) {
        int64_t p = (t / (g.nz + 1)) * g.pitch + t % (g.nz + 1);
        m = fmax(m, fmax(a[p], b[p]));
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// Targets: the correction from the prolonged to the fine steady state in the
// input's units, times kWnGain.  Apply: the inverse, with the densities
// clamped at zero and the electrode rows set from the boundary values.
__global__ void k_targets(Geom g, const double *__restrict__ Vu, const double *__restrict__ neu,
                          const double *__restrict__ npu, const double *__restrict__ Vf,
                          const double *__restrict__ nef, const double *__restrict__ npf, double vtop,
                          const double *__restrict__ nscale, float *__restrict__ out) {
    int j = blockIdx.x * 64 + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    int64_t p = (int64_t)i * g.pitch + j;
    int64_t HW = (int64_t)(g.nr + 1) * (g.nz + 1), q = (int64_t)i * (g.nz + 1) + j;
    double ns = *nscale > 0 ? *nscale : 1.0;
    out[0 * HW + q] = (float)(kWnGain * (Vf[p] - Vu[p]) / vtop);
    out[1 * HW + q] = (float)(kWnGain * (nef[p] - neu[p]) / ns);
    out[2 * HW + q] = (float)(kWnGain * (npf[p] - npu[p]) / ns);
}

__global__ void k_apply(Geom g, const double *__restrict__ Vu, const double *__restrict__ neu,
                        const double *__restrict__ npu, const float *__restrict__ corr, double vtop,
                        const double *__restrict__ nscale, double *__restrict__ V, double *__restrict__ ne,
                        double *__restrict__ np, double vb, double vt, double eb, double et, double pb, double pt) {
    int j = blockIdx.x * 64 + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    int64_t p = (int64_t)i * g.pitch + j;
    int64_t HW = (int64_t)(g.nr + 1) * (g.nz + 1), q = (int64_t)i * (g.nz + 1) + j;
    double ns = *nscale > 0 ? *nscale : 1.0;
    if (j == 0 || j == g.nz) {
        V[p] = (j == 0) ? vb : vt;
        ne[p] = (j == 0) ? eb : et;
        np[p] = (j == 0) ? pb : pt;
        return;
    }
    V[p] = Vu[p] + vtop * (double)corr[0 * HW + q] / kWnGain;
    ne[p] = fmax(0.0, neu[p] + ns * (double)corr[1 * HW + q] / kWnGain);
    np[p] = fmax(0.0, npu[p] + ns * (double)corr[2 * HW + q] / kWnGain);
}

}  // namespace

int64_t wn_scratch_size(int B, int H, int W) {
    int64_t bytes = 0;
    carve_scratch(nullptr, B, H, W, &bytes);
    return bytes;
}

int wn_forward_impl(const float *params, const float *in, float *out, int B, int H, int W, void *scratch,
                    hipStream_t st) {
    if (fused_tiles(B, H, W) > kFusedMaxTiles)
        return fail(MG_EINVAL, "image batch %d x %d x %d exceeds %lld tiles of %d x %d pixels", B, H, W,
                    (long long)kFusedMaxTiles, kFT, kFT);
    Scratch s = carve_scratch((char *)scratch, B, H, W, nullptr);
    forward_fused(s, params, in, out, B, H, W, st);
    HIP_OK(hipGetLastError());
    return MG_OK;
}

int wn_grad_impl(const float *params, const float *in, const float *target, int B, int H, int W, float *grad_out,
                 double *loss_host, void *scratch, hipStream_t st) {
    Scratch s = carve_scratch((char *)scratch, B, H, W, nullptr);
    forward_pass(s, params, in, B, H, W, st);
    backward_pass(s, target, B, H, W, st);
    if (grad_out) HIP_OK(hipMemcpyAsync(grad_out, s.grad, kWnParams * 4, hipMemcpyDeviceToDevice, st));
    if (loss_host) {
        HIP_OK(hipMemcpyAsync(loss_host, s.loss, 8, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        *loss_host /= 3.0 * (double)B * H * W;
    }
    HIP_OK(hipGetLastError());
    return MG_OK;
}

int wn_train_impl(float *params, float *m, float *v, int step, float lr, const float *in, const float *target,
                  int B, int H, int W, double *loss_host, void *scratch, hipStream_t st) {
    Scratch s = carve_scratch((char *)scratch, B, H, W, nullptr);
    forward_pass(s, params, in, B, H, W, st);
    backward_pass(s, target, B, H, W, st);
    float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
    k_adam<<<(kWnParams + 255) / 256, 256, 0, st>>>(params, m, v, s.grad, kWnParams, lr, c1, c2);
    if (loss_host) {
        HIP_OK(hipMemcpyAsync(loss_host, s.loss, 8, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        *loss_host /= 3.0 * (double)B * H * W;
    }
    HIP_OK(hipGetLastError());
    return MG_OK;
}

void launch_features(const Geom &g, const double *V, const double *ne, const double *np, double R, double d,
                     double vtop, double ratio, double *nscale, float *out, hipStream_t s) {
    k_field_max<<<1, 256, 0, s>>>(g, ne, np, nscale);
    dim3 grid((g.nz + 64) / 64, (g.nr + 4) / 4);
    k_features<<<grid, dim3(64, 4), 0, s>>>(g, V, ne, np, R, d, vtop, ratio, nscale, out);
}

void launch_targets(const Geom &g, const double *Vu, const double *neu, const double *npu, const double *Vf,
                    const double *nef, const double *npf, double vtop, const double *nscale, float *out,
                    hipStream_t s) {
    dim3 grid((g.nz + 64) / 64, (g.nr + 4) / 4);
    k_targets<<<grid, dim3(64, 4), 0, s>>>(g, Vu, neu, npu, Vf, nef, npf, vtop, nscale, out);
}

void launch_apply(const Geom &g, const double *Vu, const double *neu, const double *npu, const float *corr,
                  double vtop, const double *nscale, double *V, double *ne, double *np, const mg_physics &ph,
                  hipStream_t s) {
    dim3 grid((g.nz + 64) / 64, (g.nr + 4) / 4);
    k_apply<<<grid, dim3(64, 4), 0, s>>>(g, Vu, neu, npu, corr, vtop, nscale, V, ne, np, ph.V_bottom, ph.V_top,
                                         ph.ne_bottom, ph.ne_top, ph.np_bottom, ph.np_top);
}

}  // namespace mgf

// ---------------------------------------------------------------------------
// Allocation-free forward pass (wn_forward_noalloc): the same two kernels as
// wn_forward (weight packing, then the fused forward pass), with the packed
// weights in one file-scope device array per GPU instead of a caller-provided
// scratch buffer.  The fused kernel keeps every activation in LDS, so the
// array holds only the packed weights and biases (a fixed 155 KB whatever the
// image size) and the results are bitwise those of wn_forward.  Packing
// overwrites the whole array on every call, so nothing needs clearing; calls
// that overlap on one GPU race on it.
// ---------------------------------------------------------------------------
namespace mgf {
namespace {

constexpr int64_t round256(int64_t n) { return (n + 255) / 256 * 256; }
constexpr int64_t kStaticWeightBytes = 4 * 9 * kC * kC * 2;
constexpr int64_t kStaticScratchBytes =
    2 * round256(kStaticWeightBytes) + round256(4 * kC * 4) + round256(kC * kFK0 * 2);

}  // namespace
}  // namespace mgf

// The array itself: in host code this name is only a stand-in for the
// symbol; kernels receive the device address from hipGetSymbolAddress.
static __device__ __align__(256) char scratch[mgf::kStaticScratchBytes];

namespace mgf {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char *g_static_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int static_scratch(char **out) {
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MG_EINVAL, "device %d outside 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || reinterpret_cast<uintptr_t>(p) % 256) return fail(MG_EHIP, "scratch array address %p", p);
        g_static_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_static_ptr[dev];
    return MG_OK;
}

}  // namespace
}  // namespace mgf

extern "C" int wn_forward_noalloc(const float *params, const float *in, float *out, int32_t B, int32_t H, int32_t W,
                                  void *stream) {
    using namespace mgf;
    if (!params || !in || !out) return fail(MG_EINVAL, "null pointer");
    if (B < 1 || H < 1 || W < 1) return fail(MG_EINVAL, "bad image batch shape %d x %d x %d", B, H, W);
    if (fused_tiles(B, H, W) > kFusedMaxTiles)
        return fail(MG_EINVAL, "image batch %d x %d x %d exceeds %lld tiles of %d x %d pixels", B, H, W,
                    (long long)kFusedMaxTiles, kFT, kFT);
    char *base = nullptr;
    if (int e = static_scratch(&base)) return e;
    int64_t off = 0;
    auto take = [&](int64_t n) {
        char *p = base + off;
        off += round256(n);
        return p;
    };
    Scratch s;
    memset(&s, 0, sizeof s);
    s.WB = (__bf16 *)take(kStaticWeightBytes);
    s.WT = (__bf16 *)take(kStaticWeightBytes);
    s.bias = (float *)take(4 * kC * 4);
    s.WF0 = (__bf16 *)take(kC * kFK0 * 2);
    if (off > kStaticScratchBytes) return fail(MG_EINVAL, "static scratch layout overflow");
    forward_fused(s, params, in, out, B, H, W, reinterpret_cast<hipStream_t>(stream));
    HIP_OK(hipGetLastError());
    return MG_OK;
}
