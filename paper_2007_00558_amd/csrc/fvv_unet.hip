// fvv_unet.hip -- learned blend/inpaint network on gfx950 matrix cores.
//
// Every convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16: rows are
// output channels (A = bf16 weights, [rows][taps][K]), columns are pixels
// (B = bf16 NHWC activations gathered per tap), so each lane's accumulator
// holds four consecutive output channels of one pixel and stores them with
// one 8- or 16-byte write.  Weight gradients contract over pixels: tiles of
// the gradient and of the layer input are transposed through LDS and every
// workgroup writes an fp32 partial for its pixel chunk; a second kernel sums
// the partials in chunk order, so gradients are deterministic (no float
// atomics anywhere).  bfloat16 values are rounded to nearest even.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "fvv_unet.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

enum { TAP_CONV3 = 0, TAP_ONE = 1, TAP_FINE4 = 2 };
enum { EPI_RELU_BF16 = 0, EPI_F32 = 1, EPI_CONVT_BF16 = 2 };

// bfloat16 rounding to nearest even, written out on the bit pattern (the
// definition the hardware conversion below is checked against)
__device__ __forceinline__ uint16_t f2bf_ref(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two float32 values to packed bfloat16 (lo in the low half) with
// v_cvt_pk_bf16_f32, round to nearest even: the bits of f2bf_ref for every
// input but NaNs (fvv_check_bf16 compares the two over all 2^32 patterns).
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ uint16_t f2bf(float f) { return (uint16_t)pack_bf16(f, 0.f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) { return __builtin_bit_cast(bf16x8, *(const uint4 *)p); }

struct GemmArgs {
    const uint16_t *A;       // [M][taps][K] bf16
    const uint16_t *Bsrc;    // NHWC bf16 activations
    int b_cs, b_off;         // channel stride / offset of Bsrc
    const float *bias;       // per output channel (EPI_RELU_BF16, EPI_CONVT_BF16)
    void *out;
    int o_cs, o_off;
    int NB, H, W;            // column pixels: NB images of H x W
    int K;                   // channels per tap (multiple of 32)
    int k_src;               // channels Bsrc holds at b_off (0 = K); staged channels beyond are zero
    int M;                   // rows (multiple of 16)
    int cout;                // EPI_CONVT_BF16: output channels (M = 4 cout)
    uint16_t *pool;          // k_conv3w, EPI_RELU_BF16: also the 2x2 max-pooled output [NB][H/2][W/2][32] (or null)
    // k_conv3w<.., 2, .., UPC>: input chunk 0 is the 2x2 transposed
    // convolution (32 output channels, 64 input channels) of up_in
    // [NB][H/2][W/2][64] with weights up_w [4 x 32][64] and bias up_b,
    // computed per patch instead of read from Bsrc
    const uint16_t *up_in;
    const uint16_t *up_w;
    const float *up_b;
};

struct HeadArgs {
    const uint16_t *a;       // [P][32] bf16
    const uint16_t *w;       // [3][32] bf16
    const float *bias;       // [3]
    float *s_out;            // [P][3] or null
    uint8_t *rgb;            // image b at rgb + b * img_stride, or null
    int64_t pitch, img_stride;
    const unet_out *outs;    // or image b at outs[b] (device table), or null
    int NB, H, W, valid_h, valid_w;
    const float *target;     // [P][3] training
    float inv_n;             // 1 / (NB * valid_h * W * 3)
    float *g_a;              // [P][32] fp32 gradient at the head input
    float *part;             // per workgroup: 3*32 weight + 3 bias partials + 1 loss partial
};

// The head's 1x1 convolution (32 -> 3) of 32 pixels on one MFMA pair: A =
// the head weights as rows 0..2 of a 32-row tile (the other rows zero),
// B = the pixels' bfloat16 inputs, lane (lc, lh) holding channels 8 lh ..
// 8 lh + 7 (b0) and 16 + 8 lh .. 23 + 8 lh (b1) of pixel lc.  Lane lc (< 32)
// receives z_0..z_2 of pixel lc in d[0..2]; the result of a pixel depends
// only on its own inputs.
__device__ __forceinline__ f32x16 head_mfma(const uint16_t *w, bf16x8 b0, bf16x8 b1)
{
    const int lane = threadIdx.x & 63, lc = lane & 31, lh = lane >> 5;
    const bf16x8 zero8 = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
    const bf16x8 a0 = lc < 3 ? ld8(w + lc * 32 + 8 * lh) : zero8;
    const bf16x8 a1 = lc < 3 ? ld8(w + lc * 32 + 16 + 8 * lh) : zero8;
    f32x16 d;
#pragma unroll
    for (int r = 0; r < 16; ++r) d[r] = 0.f;
    d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, d, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, d, 0, 0, 0);
}

// Sigmoid outputs of the head for pixel p (image b, row y, column x): the
// float32 outputs (if h.s_out) and the RGB8 pixel where the three are finite.
__device__ __forceinline__ void head_store(const HeadArgs &h, const float z[3], int64_t p, int b, int y, int x)
{
    float s[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] = 1.0f / (1.0f + expf(-z[c]));
    if (h.s_out)
#pragma unroll
        for (int c = 0; c < 3; ++c) h.s_out[p * 3 + c] = s[c];
    const bool fin = isfinite(s[0]) && isfinite(s[1]) && isfinite(s[2]);
    uint8_t *o = nullptr;
    if (h.outs) {
        const unet_out d = h.outs[b];
        if (y < d.h && x < d.w) o = d.rgb + (int64_t)y * d.pitch + (int64_t)x * 3;
    } else if (h.rgb && y < h.valid_h && x < h.valid_w) {
        o = h.rgb + b * h.img_stride + (int64_t)y * h.pitch + (int64_t)x * 3;
    }
    if (o && fin)
#pragma unroll
        for (int c = 0; c < 3; ++c) o[c] = (uint8_t)fminf(floorf(s[c] * 255.f + 0.5f), 255.f);
}

// Source pixel of tap t for column pixel (b, y, x); -1 outside.
template <int TAP>
__device__ __forceinline__ int64_t tap_src(int b, int y, int x, int t, int H, int W)
{
    if (TAP == TAP_CONV3) {
        const int sy = y + t / 3 - 1, sx = x + t % 3 - 1;
        if (sy < 0 || sx < 0 || sy >= H || sx >= W) return -1;
        return ((int64_t)b * H + sy) * W + sx;
    } else if (TAP == TAP_FINE4) {
        return ((int64_t)b * 2 * H + 2 * y + (t >> 1)) * (2 * W) + 2 * x + (t & 1);
    } else {
        return ((int64_t)b * H + y) * W + x;
    }
}

template <int MC, int NP, int TAP, int EPI>
__global__ void __launch_bounds__(256) k_gemm(const GemmArgs g)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int HW = g.H * g.W;
    const int P = g.NB * HW;
    const int taps = TAP == TAP_CONV3 ? 9 : (TAP == TAP_FINE4 ? 4 : 1);
    int pb[NP], py[NP], px[NP];
    bool pv[NP];
    const int pbase = blockIdx.x * (64 * NP) + wave * (16 * NP);
#pragma unroll
    for (int n = 0; n < NP; ++n) {
        const int p = pbase + n * 16 + lr;
        pv[n] = p < P;
        const int pp = pv[n] ? p : 0;
        pb[n] = pp / HW;
        const int r = pp - pb[n] * HW;
        py[n] = r / g.W;
        px[n] = r - py[n] * g.W;
    }
    const int mbase = blockIdx.y * (16 * MC);
    f32x4 acc[MC][NP];
#pragma unroll
    for (int i = 0; i < MC; ++i)
#pragma unroll
        for (int n = 0; n < NP; ++n) acc[i][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero8 = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
    for (int t = 0; t < taps; ++t) {
        int64_t src[NP];
#pragma unroll
        for (int n = 0; n < NP; ++n) {
            const int64_t q = pv[n] ? tap_src<TAP>(pb[n], py[n], px[n], t, g.H, g.W) : -1;
            src[n] = q < 0 ? -1 : q * g.b_cs + g.b_off;
        }
        for (int c0 = 0; c0 < g.K; c0 += 32) {
            const int kk = c0 + 8 * lg;
            bf16x8 bfr[NP], afr[MC];
#pragma unroll
            for (int n = 0; n < NP; ++n) bfr[n] = src[n] >= 0 ? ld8(g.Bsrc + src[n] + kk) : zero8;
#pragma unroll
            for (int i = 0; i < MC; ++i) {
                const int m = mbase + i * 16 + lr;
                afr[i] = m < g.M ? ld8(g.A + ((int64_t)m * taps + t) * g.K + kk) : zero8;
            }
#pragma unroll
            for (int i = 0; i < MC; ++i)
#pragma unroll
                for (int n = 0; n < NP; ++n)
                    acc[i][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[i], bfr[n], acc[i][n], 0, 0, 0);
        }
    }
    // epilogue: lane holds rows m0..m0+3 of column pixel (pb, py, px)
#pragma unroll
    for (int i = 0; i < MC; ++i) {
        const int m0 = mbase + i * 16 + 4 * lg;
        if (m0 >= g.M) continue;
#pragma unroll
        for (int n = 0; n < NP; ++n) {
            if (!pv[n]) continue;
            const int64_t pix = ((int64_t)pb[n] * g.H + py[n]) * g.W + px[n];
            float v0 = acc[i][n][0], v1 = acc[i][n][1], v2 = acc[i][n][2], v3 = acc[i][n][3];
            if (EPI == EPI_F32) {
                float *o = (float *)g.out + pix * g.o_cs + g.o_off + m0;
                *(float4 *)o = make_float4(v0, v1, v2, v3);
            } else if (EPI == EPI_RELU_BF16) {
                v0 = fmaxf(v0 + g.bias[m0 + 0], 0.f);
                v1 = fmaxf(v1 + g.bias[m0 + 1], 0.f);
                v2 = fmaxf(v2 + g.bias[m0 + 2], 0.f);
                v3 = fmaxf(v3 + g.bias[m0 + 3], 0.f);
                uint16_t *o = (uint16_t *)g.out + pix * g.o_cs + g.o_off + m0;
                *(uint2 *)o = make_uint2(pack_bf16(v0, v1),
                                         pack_bf16(v2, v3));
            } else {
                const int d = m0 / g.cout, co = m0 - d * g.cout;
                const int64_t fp = ((int64_t)pb[n] * 2 * g.H + 2 * py[n] + (d >> 1)) * (2 * g.W) + 2 * px[n] + (d & 1);
                v0 += g.bias[co + 0];
                v1 += g.bias[co + 1];
                v2 += g.bias[co + 2];
                v3 += g.bias[co + 3];
                uint16_t *o = (uint16_t *)g.out + fp * g.o_cs + g.o_off + co;
                *(uint2 *)o = make_uint2(pack_bf16(v0, v1),
                                         pack_bf16(v2, v3));
            }
        }
    }
}

// ---------------------------------------------------------------- 3x3 convolution, LDS-staged
// 3x3 convolution (forward, or the data gradient with the mirrored weights)
// as an implicit GEMM on v_mfma_f32_32x32x16_bf16.  A block computes 32*MT
// output channels of a TH x 16 pixel patch of one image (a work item); for
// each 32-channel chunk of the input it stages the (TH+2) x 18 input patch
// and the weight slice (32*MT rows x 9 taps x 32 channels) in LDS once, and
// all nine taps read them from there.  Four waves split the patch's rows;
// each wave holds MT x NT tiles of 32 channels x 32 pixels (2 rows x 16
// columns).  The grid is the resident blocks; a block walks work items in
// steps of the grid and fetches the next chunk into registers while the
// current one's MFMAs run, across items too (the last chunk of an item
// fetches the first of the next), so no item starts on an exposed fetch.
// Per-pixel and per-row LDS strides are padded by 16 bytes so the 16-byte
// fragment reads of 8 consecutive lanes fall in distinct banks.
constexpr int C3_PXS = 80;             // bytes per staged pixel (32 bf16 + pad)
constexpr int C3_RS = 9 * 64 + 16;     // bytes per staged weight row

template <int MT, int TH>
constexpr int c3_lds_bytes() { return (TH + 2) * 18 * C3_PXS + 32 * MT * C3_RS; }

// 2x2 max-pool in a convolution epilogue: the window of a pooled pixel is
// lanes lc, lc^1 (columns) and lc^16 (rows) of the wave (patch origins, rows
// and widths even); returns the window's maximum of v (float32 before the
// bfloat16 rounding, whose maximum is the rounded maximum).
__device__ __forceinline__ float pool_max4(float v)
{
    const float m = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF,
                                                                         false)));   // quad_perm 1,0,3,2
    const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(m), __float_as_uint(m), false, false);
    return fmaxf(__uint_as_float(sw[0]), __uint_as_float(sw[1]));
}

template <int MT, int TH, int EPI, bool POOL = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_conv3(const GemmArgs g)
{
    static_assert(TH % 8 == 0, "each wave takes TH/4 rows, two per 32-pixel tile");
    constexpr int NT = TH / 8;         // 32-pixel tiles per wave (TH/4 rows of 16)
    constexpr int PW = 18;             // staged patch width
    constexpr int PH = TH + 2;
    extern __shared__ __attribute__((aligned(16))) uint8_t c3_smem[];
    uint8_t *patch = c3_smem;
    uint8_t *wts = c3_smem + PH * PW * C3_PXS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (g.W + 15) / 16, tiles_y = (g.H + TH - 1) / TH;
    const int mgroups = (g.M + 32 * MT - 1) / (32 * MT);
    const int items = tiles_x * tiles_y * g.NB * mgroups;
    const int k_src = g.k_src ? g.k_src : g.K;
    const int lc = lane & 31, lh = lane >> 5;
    // item of this block in step k (the grid is a multiple of 8): blocks on
    // one XCD (b mod 8) take consecutive items, the output-channel groups of
    // a patch and neighbouring patches, whose halos share that XCD's L2
    const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8, per_xcd = gridDim.x / 8;
    auto item_of = [&](int k) { return k * gridDim.x + xcd * per_xcd + slot; };
    struct Item {
        int b, x0, y0, mbase;
    };
    auto decode = [&](int it) {
        Item r;
        const int mg = it % mgroups;
        int t = it / mgroups;
        const int txi = t % tiles_x;
        t /= tiles_x;
        const int tyi = t % tiles_y;
        r.b = t / tiles_y;
        r.x0 = txi * 16;
        r.y0 = tyi * TH;
        r.mbase = mg * 32 * MT;
        return r;
    };
    // Chunks are fetched into registers (the input patch: PH x PW pixels x 4
    // quarters of 8 channels; the weight slice: 32*MT rows x 9 taps x 4
    // quarters) and stored to LDS once every wave is done with the previous.
    constexpr int NPF = (PH * PW * 4 + 255) / 256, NWF = (32 * MT * 36 + 255) / 256;
    uint4 fp[NPF], fw[NWF];
    // this thread's patch elements of an item: 32-bit element offsets of
    // their chunk-0 channels (-1 outside the image); every element of a
    // thread has the same quarter q = tid & 3
    auto offsets = [&](const Item &it, int32_t *po) {
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            const int e = tid + k * 256;
            const int px = e >> 2, pr = px / PW, pc = px - pr * PW;
            const int gy = it.y0 - 1 + pr, gx = it.x0 - 1 + pc;
            po[k] = (e < PH * PW * 4 && gy >= 0 && gy < g.H && gx >= 0 && gx < g.W)
                        ? ((it.b * g.H + gy) * g.W + gx) * g.b_cs + g.b_off + (tid & 3) * 8
                        : -1;
        }
    };
    // weights are stored chunk-major ([K/32][M][9][32]): a chunk's slice for
    // an item's rows is one contiguous run, element e of it at 8 e
    auto fetch = [&](const int32_t *po, int mbase, int c0) {
        const bool qin = c0 + (tid & 3) * 8 < k_src;
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            fp[k] = make_uint4(0, 0, 0, 0);
            if (po[k] >= 0 && qin) fp[k] = *(const uint4 *)(g.Bsrc + (uint32_t)(po[k] + c0));
        }
        const uint16_t *wc = g.A + (int64_t)mbase * 288 + (int64_t)(c0 >> 5) * g.M * 288;
#pragma unroll
        for (int k = 0; k < NWF; ++k) {
            const int e = tid + k * 256;
            fw[k] = make_uint4(0, 0, 0, 0);
            if (e < 32 * MT * 36 && mbase + e / 36 < g.M) fw[k] = *(const uint4 *)(wc + (uint32_t)e * 8);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            const int e = tid + k * 256;
            if (e < PH * PW * 4) *(uint4 *)(patch + (e >> 2) * C3_PXS + (e & 3) * 16) = fp[k];
        }
#pragma unroll
        for (int k = 0; k < NWF; ++k) {
            const int e = tid + k * 256;
            const int r = e / 36, rem = e - r * 36, tap = rem >> 2, q = rem & 3;
            if (e < 32 * MT * 36) *(uint4 *)(wts + r * C3_RS + tap * 64 + q * 16) = fw[k];
        }
    };
    // poff holds the offsets of the item whose chunks are being fetched: the
    // current one's, then (from its last chunk on) the next one's
    int cur = item_of(0);
    if (cur >= items) return;
    int32_t poff[NPF];
    {
        const Item it = decode(cur);
        offsets(it, poff);
        fetch(poff, it.mbase, 0);
    }
    stash();
    __syncthreads();
    // one loop over (item, chunk) steps, so the accumulators are carried
    // through a single loop
    int step = 1, nxt = item_of(1);
    int mbase = (cur % mgroups) * 32 * MT;
    f32x16 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int n = 0; n < NT; ++n)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][n][r] = 0.f;
    for (int c0 = 0;;) {
        // the next chunk: this item's, else the next item's first
        const bool last = c0 + 32 >= g.K;
        bool more = true;
        if (!last) {
            fetch(poff, mbase, c0 + 32);
        } else if (nxt < items) {
            const Item n = decode(nxt);
            offsets(n, poff);
            fetch(poff, n.mbase, 0);
        } else {
            more = false;
        }
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap - dy * 3;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int koff = (kk * 16 + 8 * lh) * 2;
                bf16x8 af[MT], bfr[NT];
#pragma unroll
                for (int i = 0; i < MT; ++i)
                    af[i] = __builtin_bit_cast(bf16x8, *(const uint4 *)(wts + (i * 32 + lc) * C3_RS + tap * 64 + koff));
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    const int pr = wave * (TH / 4) + 2 * n + (lc >> 4) + dy;
                    const int pc = (lc & 15) + dx;
                    bfr[n] = __builtin_bit_cast(bf16x8, *(const uint4 *)(patch + (pr * PW + pc) * C3_PXS + koff));
                }
#pragma unroll
                for (int i = 0; i < MT; ++i)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        acc[i][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[n], acc[i][n], 0, 0, 0);
            }
        }
        if (more) {
            __syncthreads();   // every wave is done with this chunk
            stash();
            __syncthreads();
        }
        if (!last) {
            c0 += 32;
            continue;
        }
        const Item it = decode(cur);
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int py = it.y0 + wave * (TH / 4) + 2 * n + (lc >> 4), px = it.x0 + (lc & 15);
            if (py >= g.H || px >= g.W) continue;
            const int64_t pix = ((int64_t)it.b * g.H + py) * g.W + px;
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int m0 = it.mbase + i * 32 + 8 * j + 4 * lh;
                    if (m0 >= g.M) continue;
                    float v0 = acc[i][n][4 * j + 0], v1 = acc[i][n][4 * j + 1];
                    float v2 = acc[i][n][4 * j + 2], v3 = acc[i][n][4 * j + 3];
                    if (EPI == EPI_F32) {
                        *(float4 *)((float *)g.out + pix * g.o_cs + g.o_off + m0) = make_float4(v0, v1, v2, v3);
                    } else {
                        v0 = fmaxf(v0 + g.bias[m0 + 0], 0.f);
                        v1 = fmaxf(v1 + g.bias[m0 + 1], 0.f);
                        v2 = fmaxf(v2 + g.bias[m0 + 2], 0.f);
                        v3 = fmaxf(v3 + g.bias[m0 + 3], 0.f);
                        *(uint2 *)((uint16_t *)g.out + pix * g.o_cs + g.o_off + m0) =
                            make_uint2(pack_bf16(v0, v1),
                                       pack_bf16(v2, v3));
                        if (POOL) {
                            // the window's four lanes share its maxima; lane
                            // (column bit a, row bit c) writes group j = 2 c + a
                            v0 = pool_max4(v0);
                            v1 = pool_max4(v1);
                            v2 = pool_max4(v2);
                            v3 = pool_max4(v3);
                            if (j == 2 * ((lc >> 4) & 1) + (lc & 1)) {
                                const int64_t pp = ((int64_t)it.b * (g.H / 2) + (py >> 1)) * (g.W / 2) + (px >> 1);
                                *(uint2 *)(g.pool + pp * g.M + m0) = make_uint2(pack_bf16(v0, v1), pack_bf16(v2, v3));
                            }
                        }
                    }
                }
        }
        if (!more) break;
        cur = nxt;
        nxt = item_of(++step);
        mbase = (cur % mgroups) * 32 * MT;
        c0 = 0;
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int n = 0; n < NT; ++n)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][n][r] = 0.f;
    }
}

// ---------------------------------------------------------------- 3x3 convolution, weights resident
// The 32-output-channel layers with one or two input chunks (the full-
// resolution level; 16-row patches with one chunk, 8-row ones with two, or
// with the head): the same implicit GEMM as k_conv3<1, TH>, but a block
// stages the whole weight slice (KC chunks x 32 rows x 9 taps x 32 channels)
// in LDS once and then walks over patches (TH x 16 pixels), so the weights
// are not fetched again for every patch; the next patch (all KC chunks) is
// fetched into registers while the current one's MFMAs and stores run.
// Blocks take patches in steps of the grid; block b's patches in one step
// are contiguous with those of the blocks on its XCD (b mod 8), so patches
// whose halos overlap are read through the same L2.
// A staged pixel holds its KC chunks side by side (KC x 64 bytes + 16 bytes
// of padding: 80 or 144 bytes, both keep the 16-byte fragment reads of 8
// consecutive lanes in distinct banks).
template <int KC>
constexpr int c3w_pxs() { return KC * 64 + 16; }
template <int TH, int KC>
constexpr int c3w_lds_bytes() { return (TH + 2) * 18 * c3w_pxs<KC>() + KC * 32 * C3_RS; }


template <int TH, int KC, int EPI, bool POOL, bool UPC = false, bool HEAD = false, bool K16 = false>
__global__ void __launch_bounds__(256) k_conv3w(const GemmArgs g, const HeadArgs hd)
{
    static_assert(!HEAD || EPI == EPI_RELU_BF16, "the head follows a ReLU output");
    static_assert(TH % 8 == 0, "each wave takes TH/4 rows, two per 32-pixel tile");
    static_assert(!UPC || (KC == 2 && TH == 8), "the transposed convolution feeds chunk 0 of 8-row patches");
    static_assert(!K16 || KC == 1, "K16: one chunk whose channels 16..31 are zero (not staged, not multiplied)");
    constexpr int NT = TH / 8;
    constexpr int PW = 18;
    constexpr int PH = TH + 2;
    constexpr int PXS = c3w_pxs<KC>();
    extern __shared__ __attribute__((aligned(16))) uint8_t c3w_smem[];
    uint8_t *patch = c3w_smem;                    // PH x PW pixels, KC chunks each
    uint8_t *wts = c3w_smem + PH * PW * PXS;      // KC weight slices
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (g.W + 15) / 16, tiles_y = (g.H + TH - 1) / TH;
    const int tiles = tiles_x * tiles_y * g.NB;
    const int k_src = g.k_src ? g.k_src : g.K;
    const int lc = lane & 31, lh = lane >> 5;
    // the weight slices, once: chunk-major [K/32][32][9][32]
    for (int e = tid; e < KC * 32 * 36; e += 256) {
        const int c = e / (32 * 36), r = (e / 36) % 32, rem = e % 36, tap = rem >> 2, q = rem & 3;
        *(uint4 *)(wts + (c * 32 + r) * C3_RS + tap * 64 + q * 16) = *(const uint4 *)(g.A + (int64_t)e * 8);
    }
    // patch index of this block in step k (the grid is a multiple of 8)
    const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8, per_xcd = gridDim.x / 8;
    auto tile_of = [&](int k) { return k * gridDim.x + xcd * per_xcd + slot; };
    // Transposed convolution feeding chunk 0 (UPC): the patch's fine rows
    // y0 - 1 .. y0 + 8 and columns x0 - 1 .. x0 + 16 come from the coarse
    // rows y0/2 - 1 .. y0/2 + 4 and columns x0/2 - 1 .. x0/2 + 8, 60 coarse
    // pixels in two 32-column tiles.  Wave w computes tap w (rows 32 w ..
    // 32 w + 31 of the weights, kept in registers) for all of them, in the
    // k-step order of the LDS-staged GEMM, so every value is the bytes that
    // GEMM would have stored; a fine pixel outside the image is 0 (the
    // convolution's zero padding).
    bf16x8 up_a[4], up_b[2][4];
    float up_bias[16];
    if constexpr (UPC) {
#pragma unroll
        for (int k = 0; k < 4; ++k) up_a[k] = ld8(g.up_w + (int64_t)(wave * 32 + lc) * 64 + 16 * k + 8 * lh);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) up_bias[4 * j + r] = g.up_b[8 * j + 4 * lh + r];
    }
    auto fetch_up = [&](int tl) {
        int t = tl;
        const int txi = t % tiles_x;
        t /= tiles_x;
        const int tyi = t % tiles_y;
        const int b = t / tiles_y;
        const int Hc = g.H / 2, Wc = g.W / 2;
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            const int sl = 32 * n + lc, cr = sl / 10, cc = sl - cr * 10;
            const int cy = tyi * 4 - 1 + cr, cx = txi * 8 - 1 + cc;
            const bool in = sl < 60 && cy >= 0 && cy < Hc && cx >= 0 && cx < Wc;
            const uint16_t *row = g.up_in + ((int64_t)(b * Hc + (in ? cy : 0)) * Wc + (in ? cx : 0)) * 64 + 8 * lh;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                up_b[n][k] = in ? ld8(row + 16 * k) : __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
        }
    };
    // the MFMAs run after the previous patch's (their inputs have landed by
    // then); their results wait in registers until the patch is staged
    f32x16 up_u[2];
    auto up_mfma = [&]() {
#pragma unroll
        for (int n = 0; n < 2; ++n) {
#pragma unroll
            for (int r = 0; r < 16; ++r) up_u[n][r] = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) up_u[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(up_a[k], up_b[n][k], up_u[n], 0, 0, 0);
        }
    };
    auto up_store = [&](int tl) {
        int t = tl;
        const int txi = t % tiles_x;
        t /= tiles_x;
        const int tyi = t % tiles_y;
        const int dy = wave >> 1, dx = wave & 1;
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            const int sl = 32 * n + lc, cr = sl / 10, cc = sl - cr * 10;
            const int pr = 2 * cr + dy - 1, pc = 2 * cc + dx - 1;       // patch row / column of this fine pixel
            const int fy = tyi * TH - 1 + pr, fx = txi * 16 - 1 + pc;
            if (sl < 60 && pr >= 0 && pr < PH && pc >= 0 && pc < PW) {
                const bool in = fy >= 0 && fy < g.H && fx >= 0 && fx < g.W;
                uint8_t *dst = patch + (pr * PW + pc) * PXS + 8 * lh;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    uint2 w2 = make_uint2(0, 0);
                    if (in)
                        w2 = make_uint2(pack_bf16(up_u[n][4 * j + 0] + up_bias[4 * j + 0], up_u[n][4 * j + 1] + up_bias[4 * j + 1]),
                                        pack_bf16(up_u[n][4 * j + 2] + up_bias[4 * j + 2], up_u[n][4 * j + 3] + up_bias[4 * j + 3]));
                    *(uint2 *)(dst + 16 * j) = w2;
                }
            }
        }
    };
    constexpr int NPF = (PH * PW * 4 + 255) / 256;
    uint4 fp[KC][NPF];
    auto fetch = [&](int tl) {
        int t = tl;
        const int txi = t % tiles_x;
        t /= tiles_x;
        const int tyi = t % tiles_y;
        const int b = t / tiles_y;
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            const int e = tid + k * 256;
            const int px = e >> 2, pr = px / PW, pc = px - pr * PW;
            const int gy = tyi * TH - 1 + pr, gx = txi * 16 - 1 + pc;
            const bool in = e < PH * PW * 4 && gy >= 0 && gy < g.H && gx >= 0 && gx < g.W;
            const int32_t off = ((b * g.H + gy) * g.W + gx) * g.b_cs + g.b_off + (tid & 3) * 8;
#pragma unroll
            for (int c = UPC ? 1 : 0; c < KC; ++c) {
                fp[c][k] = make_uint4(0, 0, 0, 0);
                if (in && c * 32 + (tid & 3) * 8 < k_src) fp[c][k] = *(const uint4 *)(g.Bsrc + (uint32_t)(off + c * 32));
            }
        }
        if constexpr (UPC) fetch_up(tl);
    };
    auto stash = [&]() {
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            const int e = tid + k * 256;
            if (e < PH * PW * 4 && !(K16 && (e & 3) >= 2))
#pragma unroll
                for (int c = UPC ? 1 : 0; c < KC; ++c) *(uint4 *)(patch + (e >> 2) * PXS + c * 64 + (e & 3) * 16) = fp[c][k];
        }
    };
    int cur = tile_of(0);
    if (cur < tiles) {
        fetch(cur);
        if constexpr (UPC) up_mfma();
    }
    for (int k = 0; cur < tiles; ++k) {
        __syncthreads();   // every wave is done with the previous patch (and the weights are staged)
        stash();
        if constexpr (UPC) up_store(cur);
        __syncthreads();
        const int nxt = tile_of(k + 1);
        if (nxt < tiles) fetch(nxt);
        f32x16 acc[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[n][r] = 0.f;
#pragma unroll
        for (int c = 0; c < KC; ++c)
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3, dx = tap - dy * 3;
#pragma unroll
                for (int kk = 0; kk < (K16 ? 1 : 2); ++kk) {
                    const int koff = (kk * 16 + 8 * lh) * 2;
                    const bf16x8 af = __builtin_bit_cast(bf16x8, *(const uint4 *)(wts + (c * 32 + lc) * C3_RS + tap * 64 + koff));
#pragma unroll
                    for (int n = 0; n < NT; ++n) {
                        const int pr = wave * (TH / 4) + 2 * n + (lc >> 4) + dy;
                        const int pc = (lc & 15) + dx;
                        const bf16x8 bfr = __builtin_bit_cast(bf16x8, *(const uint4 *)(patch + (pr * PW + pc) * PXS + c * 64 + koff));
                        acc[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bfr, acc[n], 0, 0, 0);
                    }
                }
            }
        if constexpr (UPC)
            if (nxt < tiles) up_mfma();
        // epilogue: lane holds, for pixel lc of each 32-pixel tile, channels
        // 8 j + 4 lh + {0..3} (j = 0..3)
        int t = cur;
        const int txi = t % tiles_x;
        t /= tiles_x;
        const int tyi = t % tiles_y;
        const int b = t / tiles_y;
        if constexpr (HEAD) {
            // the output as in the loop below (stored unless g.out is null:
            // only the head reads it), then the head on the matrix cores: the
            // packed bfloat16 halves of lanes l and l + 32 swapped
            // (v_permlane32_swap) into the B fragments of head_mfma
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int py = tyi * TH + wave * (TH / 4) + 2 * n + (lc >> 4), px = txi * 16 + (lc & 15);
                const bool ok = py < g.H && px < g.W;
                const int64_t pix = ((int64_t)b * g.H + py) * g.W + px;
                uint32_t w[4][2];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int m0 = 8 * j + 4 * lh;
                    w[j][0] = pack_bf16(fmaxf(acc[n][4 * j + 0] + g.bias[m0 + 0], 0.f),
                                        fmaxf(acc[n][4 * j + 1] + g.bias[m0 + 1], 0.f));
                    w[j][1] = pack_bf16(fmaxf(acc[n][4 * j + 2] + g.bias[m0 + 2], 0.f),
                                        fmaxf(acc[n][4 * j + 3] + g.bias[m0 + 3], 0.f));
                    if (ok && g.out)
                        *(uint2 *)((uint16_t *)g.out + pix * g.o_cs + g.o_off + m0) = make_uint2(w[j][0], w[j][1]);
                }
                uint4 o[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const auto s0 = __builtin_amdgcn_permlane32_swap(w[2 * q][0], w[2 * q + 1][0], false, false);
                    const auto s1 = __builtin_amdgcn_permlane32_swap(w[2 * q][1], w[2 * q + 1][1], false, false);
                    o[q] = make_uint4(s0[0], s1[0], s0[1], s1[1]);
                }
                const f32x16 dz = head_mfma(hd.w, __builtin_bit_cast(bf16x8, o[0]), __builtin_bit_cast(bf16x8, o[1]));
                if (ok && !lh) {
                    const float z[3] = {dz[0] + hd.bias[0], dz[1] + hd.bias[1], dz[2] + hd.bias[2]};
                    head_store(hd, z, pix, b, py, px);
                }
            }
            cur = nxt;
            continue;
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int py = tyi * TH + wave * (TH / 4) + 2 * n + (lc >> 4), px = txi * 16 + (lc & 15);
            if (py >= g.H || px >= g.W) continue;
            const int64_t pix = ((int64_t)b * g.H + py) * g.W + px;
            float v[16];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m0 = 8 * j + 4 * lh;
                float v0 = acc[n][4 * j + 0], v1 = acc[n][4 * j + 1];
                float v2 = acc[n][4 * j + 2], v3 = acc[n][4 * j + 3];
                if (EPI == EPI_F32) {
                    *(float4 *)((float *)g.out + pix * g.o_cs + g.o_off + m0) = make_float4(v0, v1, v2, v3);
                } else {
                    v0 = fmaxf(v0 + g.bias[m0 + 0], 0.f);
                    v1 = fmaxf(v1 + g.bias[m0 + 1], 0.f);
                    v2 = fmaxf(v2 + g.bias[m0 + 2], 0.f);
                    v3 = fmaxf(v3 + g.bias[m0 + 3], 0.f);
                    *(uint2 *)((uint16_t *)g.out + pix * g.o_cs + g.o_off + m0) =
                        make_uint2(pack_bf16(v0, v1),
                                   pack_bf16(v2, v3));
                    v[4 * j + 0] = v0;
                    v[4 * j + 1] = v1;
                    v[4 * j + 2] = v2;
                    v[4 * j + 3] = v3;
                }
            }
            if (EPI == EPI_RELU_BF16 && POOL) {
                // 2x2 max-pool: the window of pooled pixel (py/2, px/2) is
                // lanes lc, lc^1 (columns) and lc^16 (rows) of this wave
                // (patch origins, rows and widths are even).  The max of the
                // float32 values rounds to the max of their bfloat16 values.
#pragma unroll
                for (int r = 0; r < 16; ++r) v[r] = pool_max4(v[r]);
                // the four lanes of a window share its 32 channels' maxima;
                // lane (column bit a, row bit c) writes group j = 2 c + a
                const int jsel = 2 * ((lc >> 4) & 1) + (lc & 1);
                float q0 = v[0], q1 = v[1], q2 = v[2], q3 = v[3];
#pragma unroll
                for (int j = 1; j < 4; ++j)
                    if (jsel == j) {
                        q0 = v[4 * j + 0];
                        q1 = v[4 * j + 1];
                        q2 = v[4 * j + 2];
                        q3 = v[4 * j + 3];
                    }
                const int64_t pp = ((int64_t)b * (g.H / 2) + (py >> 1)) * (g.W / 2) + (px >> 1);
                *(uint2 *)(g.pool + pp * 32 + 8 * jsel + 4 * lh) =
                    make_uint2(pack_bf16(q0, q1),
                               pack_bf16(q2, q3));
            }
        }
        cur = nxt;
    }
}

// ---------------------------------------------------------------- 1x1 GEMM, LDS-staged
// out[p][m] = sum_k A[m][k] B[p][k] for the transposed convolutions (rows
// m = tap * C_out + co, scattered to the four fine pixels by the epilogue):
// TM rows x TN pixels per block (128 x 128, or 64 x 64 on small grids),
// 32-channel chunks of A and B staged in LDS, four waves of TM/2 x TN/2 on
// v_mfma_f32_32x32x16_bf16.
template <int EPI, int TM, int TN>
__global__ void __launch_bounds__(256) k_gemm1(const GemmArgs g)
{
    constexpr int MI = TM / 64, NI = TN / 64;   // 32x32 tiles per wave in each direction
    __shared__ __attribute__((aligned(16))) uint8_t As[TM * C3_PXS];
    __shared__ __attribute__((aligned(16))) uint8_t Bs[TN * C3_PXS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lc = lane & 31, lh = lane >> 5;
    const int wm = wave >> 1, wn = wave & 1;
    const int P = g.NB * g.H * g.W;
    const int pbase = blockIdx.x * TN, mbase = blockIdx.y * TM;
    f32x16 acc[MI][NI];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int n = 0; n < NI; ++n)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][n][r] = 0.f;
    for (int c0 = 0; c0 < g.K; c0 += 32) {
        for (int e = tid; e < TM * 4; e += 256) {
            const int r = e >> 2, q = e & 3;
            const int m = mbase + r;
            uint4 va = make_uint4(0, 0, 0, 0);
            if (m < g.M) va = *(const uint4 *)(g.A + (int64_t)m * g.K + c0 + q * 8);
            *(uint4 *)(As + r * C3_PXS + q * 16) = va;
        }
        for (int e = tid; e < TN * 4; e += 256) {
            const int r = e >> 2, q = e & 3;
            const int p = pbase + r;
            uint4 vb = make_uint4(0, 0, 0, 0);
            if (p < P) vb = *(const uint4 *)(g.Bsrc + (int64_t)p * g.b_cs + g.b_off + c0 + q * 8);
            *(uint4 *)(Bs + r * C3_PXS + q * 16) = vb;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int koff = (kk * 16 + 8 * lh) * 2;
            bf16x8 af[MI], bfr[NI];
#pragma unroll
            for (int i = 0; i < MI; ++i)
                af[i] = __builtin_bit_cast(bf16x8, *(const uint4 *)(As + (wm * 32 * MI + i * 32 + lc) * C3_PXS + koff));
#pragma unroll
            for (int n = 0; n < NI; ++n)
                bfr[n] = __builtin_bit_cast(bf16x8, *(const uint4 *)(Bs + (wn * 32 * NI + n * 32 + lc) * C3_PXS + koff));
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int n = 0; n < NI; ++n)
                    acc[i][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[n], acc[i][n], 0, 0, 0);
        }
        __syncthreads();
    }
    const int HW = g.H * g.W;
#pragma unroll
    for (int n = 0; n < NI; ++n) {
        const int p = pbase + wn * 32 * NI + n * 32 + lc;
        if (p >= P) continue;
        const int b = p / HW, rr = p - b * HW, y = rr / g.W, x = rr - y * g.W;
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m0 = mbase + wm * 32 * MI + i * 32 + 8 * j + 4 * lh;
                if (m0 >= g.M) continue;
                float v0 = acc[i][n][4 * j + 0], v1 = acc[i][n][4 * j + 1];
                float v2 = acc[i][n][4 * j + 2], v3 = acc[i][n][4 * j + 3];
                if (EPI == EPI_CONVT_BF16) {
                    const int d = m0 / g.cout, co = m0 - d * g.cout;
                    const int64_t fp = ((int64_t)b * 2 * g.H + 2 * y + (d >> 1)) * (2 * g.W) + 2 * x + (d & 1);
                    v0 += g.bias[co + 0];
                    v1 += g.bias[co + 1];
                    v2 += g.bias[co + 2];
                    v3 += g.bias[co + 3];
                    *(uint2 *)((uint16_t *)g.out + fp * g.o_cs + g.o_off + co) =
                        make_uint2(pack_bf16(v0, v1),
                                   pack_bf16(v2, v3));
                } else {
                    *(float4 *)((float *)g.out + (int64_t)p * g.o_cs + g.o_off + m0) = make_float4(v0, v1, v2, v3);
                }
            }
    }
}

// ---------------------------------------------------------------- 2x2 transposed convolution, registers only
// The transposed convolution into the half-resolution level (M = 4 C_out =
// 256 rows, K = C_in = 128; the kernel takes any M = 128 MTW): out[fine pixel of tap d][co] = sum_k A[d C_out + co][k] x[k]
// + bias.  Wave w of a block owns rows [32 MTW w, 32 MTW (w + 1)) and keeps
// their A fragments in registers for the whole launch; the block walks
// 32-pixel column tiles (in steps of the grid), every wave reading the same
// pixels' fragments straight from global memory (one 16-byte load per lane
// and 16 channels, the next tile's in flight while the current one's MFMAs
// and stores run).  Stores: the accumulator halves of lanes l and l + 32
// (channels 8 j + 4 lh + {0..3}) are exchanged with v_permlane32_swap so that
// each lane writes 8 consecutive channels, 16 bytes, and lanes l, l + 32
// together 32 contiguous bytes of a fine pixel.
template <int MTW, int KS>
__global__ void __launch_bounds__(256) k_convT(const GemmArgs g)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lc = lane & 31, lh = lane >> 5;
    const int P = g.NB * g.H * g.W;
    const int HW = g.H * g.W;
    bf16x8 af[MTW][KS];
#pragma unroll
    for (int i = 0; i < MTW; ++i)
#pragma unroll
        for (int k = 0; k < KS; ++k)
            af[i][k] = ld8(g.A + (int64_t)((wave * MTW + i) * 32 + lc) * g.K + 16 * k + 8 * lh);
    const bf16x8 zero8 = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
    auto fetch = [&](int p0, bf16x8 (&bf)[KS]) {
        const int p = p0 + lc;
        const uint16_t *row = g.Bsrc + (int64_t)(p < P ? p : 0) * g.b_cs + g.b_off + 8 * lh;
#pragma unroll
        for (int k = 0; k < KS; ++k) bf[k] = p < P ? ld8(row + 16 * k) : zero8;
    };
    bf16x8 bcur[KS], bnxt[KS];
    int p0 = blockIdx.x * 32;
    if (p0 < P) fetch(p0, bcur);
    for (; p0 < P; p0 += gridDim.x * 32) {
        const int pn = p0 + gridDim.x * 32;
        if (pn < P) fetch(pn, bnxt);
        f32x16 acc[MTW];
#pragma unroll
        for (int i = 0; i < MTW; ++i) {
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;
#pragma unroll
            for (int k = 0; k < KS; ++k) acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i][k], bcur[k], acc[i], 0, 0, 0);
        }
        const int p = p0 + lc;
        const int b = p / HW, rr = p - b * HW, y = rr / g.W, x = rr - y * g.W;
#pragma unroll
        for (int i = 0; i < MTW; ++i) {
            const int m0 = (wave * MTW + i) * 32;
            const int d = m0 / g.cout, co0 = m0 - d * g.cout;
            // packed bf16 pairs: w[j][h] = channels 8 j + 4 lh + 2 h, + 1
            uint32_t w[4][2];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 bj = *(const float4 *)(g.bias + co0 + 8 * j + 4 * lh);
                w[j][0] = pack_bf16(acc[i][4 * j + 0] + bj.x, acc[i][4 * j + 1] + bj.y);
                w[j][1] = pack_bf16(acc[i][4 * j + 2] + bj.z, acc[i][4 * j + 3] + bj.w);
            }
            // lanes < 32 end up with channels 16 q + 0..7, lanes >= 32 with
            // 16 q + 8..15 (q = 0, 1)
            uint4 o[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const auto s0 = __builtin_amdgcn_permlane32_swap(w[2 * q][0], w[2 * q + 1][0], false, false);
                const auto s1 = __builtin_amdgcn_permlane32_swap(w[2 * q][1], w[2 * q + 1][1], false, false);
                o[q] = make_uint4(s0[0], s1[0], s0[1], s1[1]);
            }
            if (p < P) {
                const int64_t fp = ((int64_t)b * 2 * g.H + 2 * y + (d >> 1)) * (2 * g.W) + 2 * x + (d & 1);
                uint16_t *dst = (uint16_t *)g.out + fp * g.o_cs + g.o_off + co0 + 8 * lh;
                *(uint4 *)dst = o[0];
                *(uint4 *)(dst + 16) = o[1];
            }
        }
#pragma unroll
        for (int k = 0; k < KS; ++k) bcur[k] = bnxt[k];
    }
}

// ---------------------------------------------------------------- weight gradient
struct WgradArgs {
    const uint16_t *G;       // bf16 gradient of the layer output (rows)
    int g_cs, g_off;
    const uint16_t *X;       // bf16 layer input (columns)
    int x_cs, x_off;
    float *part;             // [chunks][M][taps*K] fp32 partial sums
    int NB, H, W;            // pixel grid of the contraction (the coarse grid for convT)
    int M, K;                // rows; input channels per tap (multiple of 32)
    int x_src;               // channels X holds at x_off (0 = K); staged channels beyond are zero
    int chunk;               // pixels per workgroup (multiple of 32)
};

constexpr int WG_LD = 40;    // LDS row length in bf16 (32 pixels + pad, 16-byte aligned rows)

// grid: x = tap * (K/32) + column block of 32 channels, y = 64-row block,
// z = pixel chunk.  LDS holds the chunk's 32-pixel steps transposed to
// [channel][pixel] so each lane reads 8 consecutive pixels of one channel.
template <int TAP>
__global__ void __launch_bounds__(256) k_wgrad(const WgradArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t Gt[64 * WG_LD];
    __shared__ __attribute__((aligned(16))) uint16_t Xt[32 * WG_LD];
    const int taps = TAP == TAP_CONV3 ? 9 : (TAP == TAP_FINE4 ? 4 : 1);
    const int ncb = a.K / 32;
    const int t = blockIdx.x / ncb, cb = blockIdx.x - t * ncb;
    const int mb = blockIdx.y * 64;
    const int HW = a.H * a.W, P = a.NB * HW;
    const int p_begin = blockIdx.z * a.chunk, p_end = min(P, p_begin + a.chunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
    for (int p0 = p_begin; p0 < p_end; p0 += 32) {
        // gradient tile: 32 pixels x 64 rows (8 rows per thread)
        {
            const int pl = tid >> 3, rg = tid & 7;
            const int p = p0 + pl;
            uint4 v = make_uint4(0, 0, 0, 0);
            const int m = mb + rg * 8;
            if (p < p_end && m < a.M) {
                const int b = p / HW, r = p - b * HW, y = r / a.W, x = r - y * a.W;
                int64_t gp;
                if (TAP == TAP_FINE4)
                    gp = ((int64_t)b * 2 * a.H + 2 * y + (t >> 1)) * (2 * a.W) + 2 * x + (t & 1);
                else
                    gp = p;
                v = *(const uint4 *)(a.G + gp * a.g_cs + a.g_off + m);
            }
            const uint16_t *h = (const uint16_t *)&v;
#pragma unroll
            for (int j = 0; j < 8; ++j) Gt[(rg * 8 + j) * WG_LD + pl] = h[j];
        }
        // input tile: 32 pixels x 32 channels (threads 0..127)
        if (tid < 128) {
            const int pl = tid >> 2, cg = tid & 3;
            const int p = p0 + pl;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (p < p_end) {
                const int b = p / HW, r = p - b * HW, y = r / a.W, x = r - y * a.W;
                int64_t xp = -1;
                if (TAP == TAP_CONV3) {
                    const int sy = y + t / 3 - 1, sx = x + t % 3 - 1;
                    if (sy >= 0 && sx >= 0 && sy < a.H && sx < a.W) xp = ((int64_t)b * a.H + sy) * a.W + sx;
                } else {
                    xp = p;
                }
                if (xp >= 0 && cb * 32 + cg * 8 < (a.x_src ? a.x_src : a.K))
                    v = *(const uint4 *)(a.X + xp * a.x_cs + a.x_off + cb * 32 + cg * 8);
            }
            const uint16_t *h = (const uint16_t *)&v;
#pragma unroll
            for (int j = 0; j < 8; ++j) Xt[(cg * 8 + j) * WG_LD + pl] = h[j];
        }
        __syncthreads();
        const bf16x8 af = __builtin_bit_cast(bf16x8, *(const uint4 *)&Gt[(wave * 16 + lr) * WG_LD + 8 * lg]);
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            const bf16x8 bf = __builtin_bit_cast(bf16x8, *(const uint4 *)&Xt[(n * 16 + lr) * WG_LD + 8 * lg]);
            acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[n], 0, 0, 0);
        }
        __syncthreads();
    }
    const int cols = taps * a.K;
    float *out = a.part + (int64_t)blockIdx.z * a.M * cols;
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = mb + wave * 16 + 4 * lg + r;
            if (m < a.M) out[(int64_t)m * cols + t * a.K + cb * 32 + n * 16 + lr] = acc[n][r];
        }
}

// Weight gradient of a 3x3 convolution with all nine taps in one workgroup:
// the 32-pixel gradient tile is staged once per step and reused by the
// nine shifted input tiles (9 x 2 MFMAs per wave per step).  grid: x = input
// channel block of 32, y = 64-row block, z = pixel chunk.
__global__ void __launch_bounds__(256) k_wgrad3(const WgradArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t Gt[64 * WG_LD];
    __shared__ __attribute__((aligned(16))) uint16_t Xt[9 * 32 * WG_LD];
    const int cb = blockIdx.x;
    const int mb = blockIdx.y * 64;
    const int HW = a.H * a.W, P = a.NB * HW;
    const int p_begin = blockIdx.z * a.chunk, p_end = min(P, p_begin + a.chunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    f32x4 acc[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t][0] = acc[t][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int p0 = p_begin; p0 < p_end; p0 += 32) {
        {   // gradient tile: 32 pixels x 64 rows
            const int pl = tid >> 3, rg = tid & 7;
            const int p = p0 + pl, m = mb + rg * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (p < p_end && m < a.M) v = *(const uint4 *)(a.G + (int64_t)p * a.g_cs + a.g_off + m);
            const uint16_t *h = (const uint16_t *)&v;
#pragma unroll
            for (int j = 0; j < 8; ++j) Gt[(rg * 8 + j) * WG_LD + pl] = h[j];
        }
        // nine input tiles: 32 pixels x 32 channels each, shifted by the tap
        for (int e = tid; e < 9 * 128; e += 256) {
            const int t = e >> 7, rem = e & 127, pl = rem >> 2, cg = rem & 3;
            const int p = p0 + pl;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (p < p_end) {
                const int b = p / HW, r = p - b * HW, y = r / a.W, x = r - y * a.W;
                const int sy = y + t / 3 - 1, sx = x + t % 3 - 1;
                if (sy >= 0 && sx >= 0 && sy < a.H && sx < a.W && cb * 32 + cg * 8 < (a.x_src ? a.x_src : a.K))
                    v = *(const uint4 *)(a.X + (((int64_t)b * a.H + sy) * a.W + sx) * a.x_cs + a.x_off + cb * 32 +
                                         cg * 8);
            }
            const uint16_t *h = (const uint16_t *)&v;
#pragma unroll
            for (int j = 0; j < 8; ++j) Xt[(t * 32 + cg * 8 + j) * WG_LD + pl] = h[j];
        }
        __syncthreads();
        const bf16x8 af = __builtin_bit_cast(bf16x8, *(const uint4 *)&Gt[(wave * 16 + lr) * WG_LD + 8 * lg]);
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                const bf16x8 bf =
                    __builtin_bit_cast(bf16x8, *(const uint4 *)&Xt[(t * 32 + n * 16 + lr) * WG_LD + 8 * lg]);
                acc[t][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[t][n], 0, 0, 0);
            }
        __syncthreads();
    }
    const int cols = 9 * a.K;
    float *out = a.part + (int64_t)blockIdx.z * a.M * cols;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = mb + wave * 16 + 4 * lg + r;
                if (m < a.M) out[(int64_t)m * cols + t * a.K + cb * 32 + n * 16 + lr] = acc[t][n][r];
            }
}

// Sum the partials in chunk order into the canonical gradient (rows x taps x
// cin, dropping padded input channels).
__global__ void __launch_bounds__(256) k_wgrad_reduce(const float *__restrict__ part, int chunks, int M, int taps,
                                                      int K, int cin, float *__restrict__ gw)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = M * taps * cin;
    if (e >= n) return;
    const int ci = e % cin, mt = e / cin, t = mt % taps, m = mt / taps;
    const int64_t cols = (int64_t)taps * K;
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * M * cols + (int64_t)m * cols + t * K + ci];
    gw[e] = s;
}

// ---------------------------------------------------------------- elementwise layers
// 2x2 max-pool, bf16 NHWC; thread per (output pixel, 8 channels).
__global__ void __launch_bounds__(256) k_pool(const uint16_t *in, int i_cs, int i_off, uint16_t *out, int NB, int H,
                                              int W, int C)
{
    const int groups = C / 8;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int Ho = H / 2, Wo = W / 2;
    if (e >= (int64_t)NB * Ho * Wo * groups) return;
    const int gi = (int)(e % groups);
    const int64_t op = e / groups;
    const int b = (int)(op / (Ho * Wo)), r = (int)(op % (Ho * Wo)), y = r / Wo, x = r - y * Wo;
    uint16_t best[8];
    for (int d = 0; d < 4; ++d) {
        const int64_t ip = ((int64_t)b * H + 2 * y + (d >> 1)) * W + 2 * x + (d & 1);
        const uint4 v = *(const uint4 *)(in + ip * i_cs + i_off + gi * 8);
        const uint16_t *h = (const uint16_t *)&v;
        for (int j = 0; j < 8; ++j)
            if (d == 0 || bf2f(h[j]) > bf2f(best[j])) best[j] = h[j];
    }
    *(uint4 *)(out + op * C + gi * 8) = *(const uint4 *)best;
}

// Pool backward fused with the skip-connection gradient: g_fine[p] =
// (p is the first maximum of its window ? g_coarse : 0) + skip[p].
__global__ void __launch_bounds__(256) k_pool_back(const uint16_t *a, int a_cs, int a_off, const float *g_coarse,
                                                   const float *skip, int s_cs, int s_off, float *g_fine, int NB,
                                                   int H, int W, int C)
{
    const int groups = C / 8;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int Ho = H / 2, Wo = W / 2;
    if (e >= (int64_t)NB * Ho * Wo * groups) return;
    const int gi = (int)(e % groups);
    const int64_t op = e / groups;
    const int b = (int)(op / (Ho * Wo)), r = (int)(op % (Ho * Wo)), y = r / Wo, x = r - y * Wo;
    float best[8];
    int arg[8];
    for (int d = 0; d < 4; ++d) {
        const int64_t ip = ((int64_t)b * H + 2 * y + (d >> 1)) * W + 2 * x + (d & 1);
        const uint4 v = *(const uint4 *)(a + ip * a_cs + a_off + gi * 8);
        const uint16_t *h = (const uint16_t *)&v;
        for (int j = 0; j < 8; ++j) {
            const float f = bf2f(h[j]);
            if (d == 0 || f > best[j]) {
                best[j] = f;
                arg[j] = d;
            }
        }
    }
    for (int d = 0; d < 4; ++d) {
        const int64_t ip = ((int64_t)b * H + 2 * y + (d >> 1)) * W + 2 * x + (d & 1);
        for (int j = 0; j < 8; ++j) {
            const int c = gi * 8 + j;
            const float gv = arg[j] == d ? g_coarse[op * C + c] : 0.f;
            g_fine[ip * C + c] = gv + skip[ip * s_cs + s_off + c];
        }
    }
}

// Gradient at a layer output -> bf16 matrix-core operand (masked by the ReLU
// when relu != 0) and per-workgroup bias partial sums of the fp32 masked
// gradient.  Workgroup: 64 pixels; thread: 8 channels.
__global__ void __launch_bounds__(256) k_mask_round(const float *g, int g_cs, int g_off, const uint16_t *act, int a_cs,
                                                    int a_off, int relu, uint16_t *G, int C, int P, float *bpart)
{
    const int groups = C / 8;
    const int tid = threadIdx.x;
    const int gi = tid % groups;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int p0 = blockIdx.x * 64;
    for (int e = tid; e < 64 * groups; e += 256) {
        const int p = p0 + e / groups;
        if (p >= P) break;
        const float4 ga = *(const float4 *)(g + (int64_t)p * g_cs + g_off + gi * 8);
        const float4 gb = *(const float4 *)(g + (int64_t)p * g_cs + g_off + gi * 8 + 4);
        float v[8] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w};
        if (relu) {
            const uint4 av = *(const uint4 *)(act + (int64_t)p * a_cs + a_off + gi * 8);
            const uint16_t *h = (const uint16_t *)&av;
            for (int j = 0; j < 8; ++j)
                if (!(bf2f(h[j]) > 0.f)) v[j] = 0.f;
        }
        uint16_t o[8];
        for (int j = 0; j < 8; ++j) {
            s[j] += v[j];
            o[j] = f2bf(v[j]);
        }
        *(uint4 *)(G + (int64_t)p * C + gi * 8) = *(const uint4 *)o;
    }
    __shared__ float red[256 * 8];
    for (int j = 0; j < 8; ++j) red[tid * 8 + j] = s[j];
    __syncthreads();
    if (tid < groups) {
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int u = tid; u < 256; u += groups)
            for (int j = 0; j < 8; ++j) acc[j] += red[u * 8 + j];
        for (int j = 0; j < 8; ++j) bpart[(int64_t)blockIdx.x * C + tid * 8 + j] = acc[j];
    }
}

// Column sums of a rows x n matrix of partials: one workgroup per column,
// thread t adds rows t, t+256, ... in order, then a fixed tree combines the
// 256 sums -- the same result on every run.
__global__ void __launch_bounds__(256) k_reduce_rows(const float *part, int rows, int n, float *out)
{
    __shared__ float red[256];
    const int col = blockIdx.x;
    float acc = 0.f;
    for (int r = threadIdx.x; r < rows; r += 256) acc += part[(int64_t)r * n + col];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[col] = red[0];
}

// Head: 1x1 conv 32->3 + bias, sigmoid.  mode 0: inference (s and/or RGB8
// of finite pixels); mode 1: training (loss partials, d loss / d z, the
// gradient at the head input and the head's weight/bias partials).

__global__ void __launch_bounds__(256) k_head(const HeadArgs h, int mode)
{
    __shared__ float red[256 * 4];
    __shared__ float wred[32 * 4];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int P = h.NB * h.H * h.W;
    const bool in = p < P;
    // z on the matrix cores: the wave's 64 pixels as two 32-pixel columns
    // (head_mfma), pixel 32 t + lc of the wave in lane lc of column t; the
    // second column's results move to lanes 32..63 (v_permlane32_swap)
    const int lane = threadIdx.x & 63, lc = lane & 31, lh = lane >> 5;
    const int64_t wbase = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    f32x16 d[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int64_t q = wbase + 32 * t + lc;
        const bf16x8 zero8 = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
        const bf16x8 b0 = q < P ? ld8(h.a + q * 32 + 8 * lh) : zero8;
        const bf16x8 b1 = q < P ? ld8(h.a + q * 32 + 16 + 8 * lh) : zero8;
        d[t] = head_mfma(h.w, b0, b1);
    }
    float z[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(d[1][c]), __float_as_uint(d[1][c]), false,
                                                         false);
        const float zc = lh ? __uint_as_float(sw[0]) : d[0][c];
        if (in) z[c] = zc + h.bias[c];
    }
    float a[32];
    if (in && mode != 0)
        for (int q = 0; q < 4; ++q) {
            const uint4 v = *(const uint4 *)(h.a + p * 32 + q * 8);
            const uint16_t *hv = (const uint16_t *)&v;
            for (int j = 0; j < 8; ++j) a[q * 8 + j] = bf2f(hv[j]);
        }
    const int b = in ? (int)(p / (h.H * h.W)) : 0;
    const int r = in ? (int)(p % (h.H * h.W)) : 0;
    const int y = r / h.W, x = r - y * h.W;
    if (mode == 0) {
        if (in) head_store(h, z, p, b, y, x);
        return;
    }
    float s[3];
    for (int c = 0; c < 3; ++c) s[c] = 1.0f / (1.0f + expf(-z[c]));
    // training
    float gz[3] = {0.f, 0.f, 0.f}, loss = 0.f;
    if (in && y < h.valid_h) {
        for (int c = 0; c < 3; ++c) {
            const float d = s[c] - h.target[p * 3 + c];
            loss += fabsf(d);
            const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
            gz[c] = sg * h.inv_n * s[c] * (1.f - s[c]);
        }
    }
    float gzr[3];
    for (int c = 0; c < 3; ++c) gzr[c] = bf2f(f2bf(gz[c]));
    if (in)
        for (int ci = 0; ci < 32; ++ci) {
            float acc = 0.f;
            for (int c = 0; c < 3; ++c) acc += gzr[c] * bf2f(h.w[c * 32 + ci]);
            h.g_a[p * 32 + ci] = acc;
        }
    // per-workgroup partials: weights (3 x 32), bias (3), loss (1), fixed order
    const int tid = threadIdx.x;
    float *outp = h.part + (int64_t)blockIdx.x * (96 + 4);
    for (int c = 0; c < 3; ++c) {
        for (int q = 0; q < 8; ++q) {   // 32 input channels in 8 rounds of 4
            for (int j = 0; j < 4; ++j) red[tid * 4 + j] = in ? gzr[c] * a[q * 4 + j] : 0.f;
            __syncthreads();
            if (tid < 4) {
                float acc = 0.f;
                for (int u = 0; u < 256; ++u) acc += red[u * 4 + tid];
                wred[(q * 4 + tid)] = acc;
            }
            __syncthreads();
        }
        if (tid < 32) outp[c * 32 + tid] = wred[tid];
        __syncthreads();
    }
    red[tid * 4 + 0] = gz[0];
    red[tid * 4 + 1] = gz[1];
    red[tid * 4 + 2] = gz[2];
    red[tid * 4 + 3] = loss;
    __syncthreads();
    if (tid < 4) {
        float acc = 0.f;
        for (int u = 0; u < 256; ++u) acc += red[u * 4 + tid];
        outp[96 + tid] = acc;
    }
}

// Adam on the fp32 master parameters of one layer, and the bf16 copies in
// the forward layout and the data-gradient layout (taps mirrored for 3x3):
// 3x3 convolutions chunk-major, [cin_pad/32][cout][9][32] and
// [cout/32][cin][9][32], so one 32-channel chunk of a block's rows is one
// contiguous run; transposed convolutions [tap][cout][cin] and
// [cin][tap][cout]; the head [cout][cin].
struct AdamArgs {
    float *w, *m, *v;
    const float *g;
    int n;                   // floats of this parameter block
    int is_weight;
    int kind, cin, cin_pad, cout, taps;
    uint16_t *wf, *wd;
    float lr, b1, b2, eps, c1, c2;   // c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
    int apply;
};

__global__ void __launch_bounds__(256) k_adam(const AdamArgs a)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n) return;
    float w = a.w[e];
    if (a.apply) {
        const float g = a.g[e];
        const float m = a.b1 * a.m[e] + (1.f - a.b1) * g;
        const float v = a.b2 * a.v[e] + (1.f - a.b2) * g * g;
        a.m[e] = m;
        a.v[e] = v;
        w = w - a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
        a.w[e] = w;
    }
    if (!a.is_weight) return;
    const int ci = e % a.cin, rest = e / a.cin, t = rest % a.taps, co = rest / a.taps;
    const uint16_t wb = f2bf(w);
    if (a.kind == 1) {   // convT: forward rows are (tap, cout)
        a.wf[((int64_t)(t * a.cout + co)) * a.cin_pad + ci] = wb;
    } else if (a.kind == 0) {   // 3x3: chunk-major [cin_pad/32][cout][9][32]
        a.wf[(((int64_t)(ci >> 5) * a.cout + co) * 9 + t) * 32 + (ci & 31)] = wb;
    } else {
        a.wf[((int64_t)co * a.taps + t) * a.cin_pad + ci] = wb;
    }
    if (a.wd) {
        const int td = a.kind == 0 ? a.taps - 1 - t : t;
        if (a.kind == 0)   // data gradient, chunk-major over the output channels: [cout/32][cin][9][32]
            a.wd[(((int64_t)(co >> 5) * a.cin + ci) * 9 + td) * 32 + (co & 31)] = wb;
        else
            a.wd[((int64_t)ci * a.taps + td) * a.cout + co] = wb;
    }
}

// Every float32 bit pattern but the NaNs: the hardware conversion against
// the written-out rounding.
__global__ void __launch_bounds__(256) k_check_bf16(unsigned long long *bad)
{
    uint32_t miss = 0;
    const uint32_t stride = gridDim.x * 256u;
    for (uint32_t u = blockIdx.x * 256u + threadIdx.x;; u += stride) {
        const float f = __uint_as_float(u);
        if (!((u & 0x7fffffffu) > 0x7f800000u)) miss += (uint16_t)pack_bf16(f, 0.f) != f2bf_ref(f);
        if (u > 0xFFFFFFFFu - stride) break;
    }
    if (miss) atomicAdd(bad, (unsigned long long)miss);
}

// ---------------------------------------------------------------- host side
const struct {
    const char *name;
    int kind, cin, cout;
} kLayers[] = {
    {"enc0a", 0, UNET_IN, 32}, {"enc0b", 0, 32, 32},  {"enc1a", 0, 32, 64},   {"enc1b", 0, 64, 64},
    {"enc2a", 0, 64, 128},              {"enc2b", 0, 128, 128}, {"mid_a", 0, 128, 256}, {"mid_b", 0, 256, 256},
    {"up2", 1, 256, 128},               {"dec2a", 0, 256, 128}, {"dec2b", 0, 128, 128}, {"up1", 1, 128, 64},
    {"dec1a", 0, 128, 64},              {"dec1b", 0, 64, 64},   {"up0", 1, 64, 32},     {"dec0a", 0, 64, 32},
    {"dec0b", 0, 32, 32},               {"head", 2, 32, 3},
};
constexpr int kNL = sizeof(kLayers) / sizeof(kLayers[0]);
enum { L_E0A, L_E0B, L_E1A, L_E1B, L_E2A, L_E2B, L_MA, L_MB, L_UP2, L_D2A, L_D2B, L_UP1, L_D1A, L_D1B, L_UP0,
       L_D0A, L_D0B, L_HEAD };
// resolution level (0 = full) of each layer's output, and of its weight-gradient contraction
constexpr int kOutLevel[kNL] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 2, 1, 1, 1, 0, 0, 0, 0};
constexpr int kSumLevel[kNL] = {0, 0, 1, 1, 2, 2, 3, 3, 3, 2, 2, 2, 1, 1, 1, 0, 0, 0};

struct Layers {
    unet_layer L[kNL];
    size_t n_params = 0, n_wf = 0, n_wd = 0;
    Layers()
    {
        for (int i = 0; i < kNL; ++i) {
            unet_layer &l = L[i];
            l.name = kLayers[i].name;
            l.kind = kLayers[i].kind;
            l.cin = kLayers[i].cin;
            l.cout = kLayers[i].cout;
            l.cin_pad = l.kind == 2 ? l.cin : std::max(32, l.cin);
            l.taps = l.kind == 0 ? 9 : (l.kind == 1 ? 4 : 1);
            l.w_off = n_params;
            n_params += (size_t)l.cout * l.taps * l.cin;
            l.b_off = n_params;
            n_params += (size_t)l.cout;
            l.wf_off = n_wf;
            n_wf += (size_t)l.cout * l.taps * l.cin_pad;
            l.wd_off = n_wd;
            if (l.kind != 2 && i != L_E0A) n_wd += (size_t)l.cout * l.taps * l.cin;
        }
    }
};
const Layers &layers()
{
    static const Layers t;
    return t;
}

// chunking of a weight-gradient contraction over P pixels
// Pixel chunking of a weight-gradient contraction over P pixels for a
// layer whose grid has `wgs` workgroups per chunk: about 1024 workgroups in
// all, chunks of at least 256 pixels (multiples of 32).
int wgrad_chunks(size_t P, int wgs)
{
    const size_t want = std::max<size_t>(1, 1024 / (size_t)std::max(1, wgs));
    return (int)std::max<size_t>(1, std::min<size_t>((P + 255) / 256, want));
}
int wgrad_chunk(size_t P, int wgs)
{
    const size_t c = (P + wgrad_chunks(P, wgs) - 1) / wgrad_chunks(P, wgs);
    return (int)((c + 31) / 32 * 32);
}
int wgrad_wgs(const unet_layer &l)
{
    const int mblk = (l.cout + 63) / 64, kblk = l.cin_pad / 32;
    return l.kind == 0 ? mblk * kblk : mblk * kblk * l.taps;
}

size_t partial_floats(size_t P0)
{
    const Layers &T = layers();
    size_t m = ((P0 + 63) / 64) * 256;   // bias partials (<= 256 channels per 64-pixel group)
    for (int i = 0; i < kNL; ++i) {
        const unet_layer &l = T.L[i];
        if (l.kind == 2) continue;
        // a contraction over P <= Pk pixels has ceil(P / chunk) <= wgrad_chunks(P)
        // <= wgrad_chunks(Pk) chunks (chunk >= P / wgrad_chunks(P), monotone in P)
        const size_t Pk = P0 >> (2 * kSumLevel[i]);
        const size_t chunks = (size_t)wgrad_chunks(Pk, wgrad_wgs(l));
        m = std::max(m, chunks * l.cout * l.taps * l.cin_pad);
    }
    return m;
}

#define NCHK(expr)                                  \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return e_;            \
    } while (0)

}  // namespace

struct unet_state {
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    uint16_t *wf = nullptr, *wd = nullptr;
    int step = 0;
    bool loaded = false;
};

// Forward activations (bf16; concat buffers hold [up | skip]) and, for
// training, the fp32 gradient ping-pong, the concat gradients, the bf16
// matrix-core operand and the partial sums.
struct unet_act {
    size_t cap = 0;          // pixels at full resolution
    bool train = false;
    bool up0_stored = true;  // the last forward stored the finest transposed convolution's output
    bool d0b_stored = true;  // ... and dec0b's output
    size_t bytes = 0;
    int NB = 0, H = 0, W = 0;
    uint16_t *e0a = nullptr, *cat0 = nullptr, *p1 = nullptr, *e1a = nullptr, *cat1 = nullptr, *p2 = nullptr,
             *e2a = nullptr, *cat2 = nullptr, *p3 = nullptr, *ma = nullptr, *mb = nullptr, *d2a = nullptr,
             *d2b = nullptr, *d1a = nullptr, *d1b = nullptr, *d0a = nullptr, *d0b = nullptr;
    float *g0 = nullptr, *g1 = nullptr;                  // [P0][32] each
    float *gs0 = nullptr, *gs1 = nullptr, *gs2 = nullptr;   // [P0][64], [P1][128], [P2][256]
    uint16_t *G = nullptr;                                // [P0][32]
    float *part = nullptr;
    float *head_part = nullptr;
    float *loss_dev = nullptr;
    void *blocks[40] = {};
    int n_blocks = 0;
};

namespace {

struct Plan {
    size_t off[40];
    int n = 0;
    size_t total = 0;
    size_t add(size_t bytes)
    {
        off[n++] = total;
        const size_t o = total;
        total += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

// One allocation per set; the plan gives every buffer its offset.
template <typename F>
void act_plan(size_t P0, bool train, F &&put)
{
    const size_t P1 = P0 / 4, P2 = P1 / 4, P3 = P2 / 4;
    put(0, P0 * 32 * 2);     // e0a
    put(1, P0 * 64 * 2);     // cat0
    put(2, P1 * 32 * 2);     // p1
    put(3, P1 * 64 * 2);     // e1a
    put(4, P1 * 128 * 2);    // cat1
    put(5, P2 * 64 * 2);     // p2
    put(6, P2 * 128 * 2);    // e2a
    put(7, P2 * 256 * 2);    // cat2
    put(8, P3 * 128 * 2);    // p3
    put(9, P3 * 256 * 2);    // ma
    put(10, P3 * 256 * 2);   // mb
    put(11, P2 * 128 * 2);   // d2a
    put(12, P2 * 128 * 2);   // d2b
    put(13, P1 * 64 * 2);    // d1a
    put(14, P1 * 64 * 2);    // d1b
    put(15, P0 * 32 * 2);    // d0a
    put(16, P0 * 32 * 2);    // d0b
    if (!train) return;
    put(17, P0 * 32 * 4);    // g0
    put(18, P0 * 32 * 4);    // g1
    put(19, P0 * 64 * 4);    // gs0
    put(20, P1 * 128 * 4);   // gs1
    put(21, P2 * 256 * 4);   // gs2
    put(22, P0 * 32 * 2);    // G
    put(23, partial_floats(P0) * 4);
    put(24, ((P0 + 255) / 256) * 100 * 4);
    put(25, 256);            // loss
}

}  // namespace

unet_state *unet_new() { return new (std::nothrow) unet_state(); }

void unet_free(unet_state *n)
{
    if (!n) return;
    for (void *p : {(void *)n->w, (void *)n->m, (void *)n->v, (void *)n->g, (void *)n->wf, (void *)n->wd})
        if (p) (void)hipFree(p);
    delete n;
}

unet_act *unet_act_new() { return new (std::nothrow) unet_act(); }

void unet_act_free(unet_act *a)
{
    if (!a) return;
    if (a->blocks[0]) (void)hipFree(a->blocks[0]);
    delete a;
}

size_t unet_param_floats() { return layers().n_params; }
int unet_layer_count() { return kNL; }
const unet_layer *unet_layer_info(int i) { return (i >= 0 && i < kNL) ? &layers().L[i] : nullptr; }
size_t unet_weight_bytes()
{
    const Layers &T = layers();
    return T.n_params * 4 * 4 + (T.n_wf + T.n_wd) * 2;
}
size_t unet_act_need(size_t pixels, bool train)
{
    size_t total = 0;
    act_plan(pixels, train, [&](int, size_t b) { total += (b + 255) & ~(size_t)255; });
    return total;
}
size_t unet_act_bytes(const unet_act *a) { return a ? a->bytes : 0; }
size_t unet_act_cap(const unet_act *a) { return a ? a->cap : 0; }
bool unet_act_trainable(const unet_act *a) { return a && a->train; }
bool unet_loaded(const unet_state *n) { return n && n->loaded; }

hipError_t unet_act_reserve(unet_act *a, size_t pixels, bool train)
{
    if (a->cap >= pixels && (a->train || !train)) return hipSuccess;
    const size_t cap = std::max(pixels, a->cap);
    train = train || a->train;
    NCHK(hipDeviceSynchronize());
    if (a->blocks[0]) (void)hipFree(a->blocks[0]);
    *a = unet_act();
    size_t off[32] = {}, total = 0;
    act_plan(cap, train, [&](int i, size_t b) {
        off[i] = total;
        total += (b + 255) & ~(size_t)255;
    });
    uint8_t *base = nullptr;
    NCHK(hipMalloc((void **)&base, total));
    a->blocks[0] = base;
    a->bytes = total;
    a->cap = cap;
    a->train = train;
    uint16_t **bf[17] = {&a->e0a, &a->cat0, &a->p1, &a->e1a, &a->cat1, &a->p2, &a->e2a, &a->cat2, &a->p3,
                         &a->ma,  &a->mb,   &a->d2a, &a->d2b, &a->d1a, &a->d1b, &a->d0a, &a->d0b};
    for (int i = 0; i < 17; ++i) *bf[i] = (uint16_t *)(base + off[i]);
    if (train) {
        a->g0 = (float *)(base + off[17]);
        a->g1 = (float *)(base + off[18]);
        a->gs0 = (float *)(base + off[19]);
        a->gs1 = (float *)(base + off[20]);
        a->gs2 = (float *)(base + off[21]);
        a->G = (uint16_t *)(base + off[22]);
        a->part = (float *)(base + off[23]);
        a->head_part = (float *)(base + off[24]);
        a->loss_dev = (float *)(base + off[25]);
    }
    return hipSuccess;
}

namespace {

// Blocks of a kernel that the device holds at once (its occupancy times the
// compute units), for the kernels that walk their work in steps of the grid;
// computed once per kernel.
template <typename F>
int resident_blocks(F kernel, size_t lds)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, lds) != hipSuccess)
        return 256;
    return std::max(1, per) * std::max(1, cus);
}

template <int MC, int NP, int TAP, int EPI>
hipError_t gemm(const GemmArgs &g, hipStream_t s)
{
    const int P = g.NB * g.H * g.W;
    dim3 grid((P + 64 * NP - 1) / (64 * NP), (g.M + 16 * MC - 1) / (16 * MC));
    hipLaunchKernelGGL((k_gemm<MC, NP, TAP, EPI>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

template <int MT, int TH, int EPI, bool POOL = false>
hipError_t conv3_launch(const GemmArgs &g, hipStream_t s)
{
    constexpr int lds = c3_lds_bytes<MT, TH>();
    static_assert(lds <= 65536, "staged patch and weights must fit 64 KB");
    const int64_t items = (int64_t)((g.W + 15) / 16) * ((g.H + TH - 1) / TH) * g.NB * ((g.M + 32 * MT - 1) / (32 * MT));
    static const int rb = std::max(8, resident_blocks(k_conv3<MT, TH, EPI, POOL>, lds) / 8 * 8);
    const int grid = (int)std::min<int64_t>(rb, (items + 7) / 8 * 8);
    hipLaunchKernelGGL((k_conv3<MT, TH, EPI, POOL>), dim3(grid), dim3(256), lds, s, g);
    return hipGetLastError();
}

// 3x3 convolution shapes (measured on the 960x544 network): the
// 32-output-channel layers of large grids with their weights resident
// (16-row patches with one input chunk, 8-row ones with two); otherwise 32
// output channels x 8-row patches for grids under 64 K pixels (more blocks
// where there are few pixels), else 64 channels x 16-row patches
template <int TH, int KC, int EPI, bool POOL, bool UPC = false, bool HEAD = false, bool K16 = false>
hipError_t conv3w_launch(const GemmArgs &g, hipStream_t s, const HeadArgs &h = HeadArgs{})
{
    constexpr int lds = c3w_lds_bytes<TH, KC>();
    static_assert(lds <= 65536, "staged patches and weights must fit 64 KB");
    static const int grid = std::max(8, resident_blocks(k_conv3w<TH, KC, EPI, POOL, UPC, HEAD, K16>, lds) / 8 * 8);
    hipLaunchKernelGGL((k_conv3w<TH, KC, EPI, POOL, UPC, HEAD, K16>), dim3(grid), dim3(256), lds, s, g, h);
    return hipGetLastError();
}

// *pooled (if given) tells whether the launch also wrote the 2x2 max-pool
// of the output to g.pool; *headed (if given) whether it also ran the head
// (only the weights-resident kernel with one input chunk runs it), and then
// head_only leaves the output itself unstored.
template <int EPI>
hipError_t conv3(GemmArgs g, hipStream_t s, bool *pooled = nullptr, const HeadArgs *head = nullptr,
                 bool *headed = nullptr, bool head_only = false)
{
    if (g.K % 32 != 0) return hipErrorInvalidValue;
    if (pooled) *pooled = false;
    if (headed) *headed = false;
    // 32 output channels from one or two input chunks, with patches for
    // every block several times over: weights resident, blocks walk patches
    const int64_t tiles8 = (int64_t)((g.W + 15) / 16) * ((g.H + 7) / 8) * g.NB;
    if (g.M == 32 && g.K == 32 && tiles8 >= 2048 && g.H % 2 == 0 && g.W % 2 == 0) {
        if constexpr (EPI == EPI_RELU_BF16) {
            if (pooled && g.pool) {
                *pooled = true;
                return conv3w_launch<16, 1, EPI, true>(g, s);
            }
            if (headed && head) {
                *headed = true;
                if (head_only) g.out = nullptr;
                return conv3w_launch<16, 1, EPI, false, false, true>(g, s, *head);
            }
        }
        // an input of 16 channels or fewer (the stack): the zero half of the
        // chunk is neither staged nor multiplied
        if (g.k_src > 0 && g.k_src <= 16) return conv3w_launch<16, 1, EPI, false, false, false, true>(g, s);
        return conv3w_launch<16, 1, EPI, false>(g, s);
    }
    if (g.M == 32 && g.K == 64 && tiles8 >= 2048) return conv3w_launch<8, 2, EPI, false>(g, s);
    const bool big = g.M > 32 && (int64_t)g.NB * g.H * g.W >= 65536;
    if constexpr (EPI == EPI_RELU_BF16) {
        if (pooled && g.pool && g.H % 2 == 0 && g.W % 2 == 0) {
            *pooled = true;
            return big ? conv3_launch<2, 16, EPI, true>(g, s) : conv3_launch<1, 8, EPI, true>(g, s);
        }
    }
    return big ? conv3_launch<2, 16, EPI>(g, s) : conv3_launch<1, 8, EPI>(g, s);
}

// 3x3 conv + bias + ReLU into (out, o_cs, o_off); with pool_out, *pooled
// tells whether the 2x2 max-pool of the output was written there as well,
// with head, *headed whether the head ran on the output as well (and
// head_only then leaves out unwritten)
hipError_t conv_fwd(unet_state *n, int li, const uint16_t *in, int i_cs, int i_off, uint16_t *out, int o_cs, int o_off,
                    int NB, int H, int W, hipStream_t s, uint16_t *pool_out = nullptr, bool *pooled = nullptr,
                    const HeadArgs *head = nullptr, bool *headed = nullptr, bool head_only = false)
{
    const unet_layer &l = layers().L[li];
    GemmArgs g{};
    g.A = n->wf + l.wf_off;
    g.Bsrc = in;
    g.b_cs = i_cs;
    g.b_off = i_off;
    g.bias = n->w + l.b_off;
    g.out = out;
    g.o_cs = o_cs;
    g.o_off = o_off;
    g.NB = NB;
    g.H = H;
    g.W = W;
    g.K = l.cin_pad;
    g.k_src = std::min(i_cs - i_off, l.cin_pad);
    g.M = l.cout;
    g.pool = pool_out;
    return conv3<EPI_RELU_BF16>(g, s, pooled, head, headed, head_only);
}

hipError_t convT_fwd(unet_state *n, int li, const uint16_t *in, int i_cs, int NB, int H, int W, uint16_t *out,
                     int o_cs, hipStream_t s)
{
    const unet_layer &l = layers().L[li];
    GemmArgs g{};
    g.A = n->wf + l.wf_off;
    g.Bsrc = in;
    g.b_cs = i_cs;
    g.bias = n->w + l.b_off;
    g.out = out;
    g.o_cs = o_cs;
    g.NB = NB;
    g.H = H;
    g.W = W;
    g.K = l.cin_pad;
    g.M = 4 * l.cout;
    g.cout = l.cout;
    const int P = NB * H * W;
    // the half-resolution level with a thousand pixel tiles or more: A in
    // registers, no LDS (at the finest level, with one 32-row tile per
    // wave, the LDS-staged GEMM below is faster)
    if (P >= 32768) {
        if (g.M == 256 && g.K == 128) {
            static const int rb = resident_blocks(k_convT<2, 8>, 0);
            hipLaunchKernelGGL((k_convT<2, 8>), dim3(std::min(rb, (P + 31) / 32)), dim3(256), 0, s, g);
            return hipGetLastError();
        }
    }
    // 128 x 128 blocks where they number a thousand or more, else 64 x 64
    // (small grids are latency-bound: more, shorter blocks)
    const int64_t big = (int64_t)((P + 127) / 128) * ((g.M + 127) / 128);
    if (big >= 1024) {
        dim3 grid((P + 127) / 128, (g.M + 127) / 128);
        hipLaunchKernelGGL((k_gemm1<EPI_CONVT_BF16, 128, 128>), grid, dim3(256), 0, s, g);
    } else {
        dim3 grid((P + 63) / 64, (g.M + 63) / 64);
        hipLaunchKernelGGL((k_gemm1<EPI_CONVT_BF16, 64, 64>), grid, dim3(256), 0, s, g);
    }
    return hipGetLastError();
}

hipError_t pool(const uint16_t *in, int i_cs, int i_off, uint16_t *out, int NB, int H, int W, int C, hipStream_t s)
{
    const int64_t n = (int64_t)NB * (H / 2) * (W / 2) * (C / 8);
    hipLaunchKernelGGL(k_pool, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, i_cs, i_off, out, NB, H, W, C);
    return hipGetLastError();
}

// Whether the finest transposed convolution can run inside the next
// convolution (weights-resident kernel with two input chunks).
bool up0_fusable(int NB, int H, int W)
{
    return (int64_t)((W + 15) / 16) * ((H + 7) / 8) * NB >= 2048;
}

// dec0a with its input chunk 0 (the finest transposed convolution of d1b)
// computed per patch: cat0's first 32 channels are neither written nor read
hipError_t dec0a_fused(unet_state *n, unet_act *a, int NB, int H, int W, hipStream_t s)
{
    const unet_layer &l = layers().L[L_D0A], &u = layers().L[L_UP0];
    GemmArgs g{};
    g.A = n->wf + l.wf_off;
    g.Bsrc = a->cat0;
    g.b_cs = 64;
    g.bias = n->w + l.b_off;
    g.out = a->d0a;
    g.o_cs = 32;
    g.NB = NB;
    g.H = H;
    g.W = W;
    g.K = l.cin_pad;
    g.M = l.cout;
    g.up_in = a->d1b;
    g.up_w = n->wf + u.wf_off;
    g.up_b = n->w + u.b_off;
    if (g.K != 64 || g.M != 32 || u.cout != 32 || u.cin_pad != 64) return hipErrorInvalidValue;
    return conv3w_launch<8, 2, EPI_RELU_BF16, false, true>(g, s);
}

// The forward pass up to the last 3x3 convolution.  lean (inference) stores
// only what a later launch reads: the finest transposed convolution may run
// inside dec0a, and dec0b's output, when the head runs in its epilogue, is
// not stored.  With head, *head_done tells whether the head ran there.
hipError_t forward_all(unet_state *n, unet_act *a, const uint16_t *stack, int NB, int H, int W, hipStream_t s,
                       bool lean = false, const HeadArgs *head = nullptr, bool *head_done = nullptr)
{
    a->NB = NB;
    a->H = H;
    a->W = W;
    const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
    NCHK(conv_fwd(n, L_E0A, stack, UNET_IN, 0, a->e0a, 32, 0, NB, H, W, s));
    bool pooled = false;
    NCHK(conv_fwd(n, L_E0B, a->e0a, 32, 0, a->cat0, 64, 32, NB, H, W, s, a->p1, &pooled));
    if (!pooled) NCHK(pool(a->cat0, 64, 32, a->p1, NB, H, W, 32, s));
    NCHK(conv_fwd(n, L_E1A, a->p1, 32, 0, a->e1a, 64, 0, NB, H1, W1, s));
    NCHK(conv_fwd(n, L_E1B, a->e1a, 64, 0, a->cat1, 128, 64, NB, H1, W1, s, a->p2, &pooled));
    if (!pooled) NCHK(pool(a->cat1, 128, 64, a->p2, NB, H1, W1, 64, s));
    NCHK(conv_fwd(n, L_E2A, a->p2, 64, 0, a->e2a, 128, 0, NB, H2, W2, s));
    NCHK(conv_fwd(n, L_E2B, a->e2a, 128, 0, a->cat2, 256, 128, NB, H2, W2, s, a->p3, &pooled));
    if (!pooled) NCHK(pool(a->cat2, 256, 128, a->p3, NB, H2, W2, 128, s));
    NCHK(conv_fwd(n, L_MA, a->p3, 128, 0, a->ma, 256, 0, NB, H3, W3, s));
    NCHK(conv_fwd(n, L_MB, a->ma, 256, 0, a->mb, 256, 0, NB, H3, W3, s));
    NCHK(convT_fwd(n, L_UP2, a->mb, 256, NB, H3, W3, a->cat2, 256, s));
    NCHK(conv_fwd(n, L_D2A, a->cat2, 256, 0, a->d2a, 128, 0, NB, H2, W2, s));
    NCHK(conv_fwd(n, L_D2B, a->d2a, 128, 0, a->d2b, 128, 0, NB, H2, W2, s));
    NCHK(convT_fwd(n, L_UP1, a->d2b, 128, NB, H2, W2, a->cat1, 128, s));
    NCHK(conv_fwd(n, L_D1A, a->cat1, 128, 0, a->d1a, 64, 0, NB, H1, W1, s));
    NCHK(conv_fwd(n, L_D1B, a->d1a, 64, 0, a->d1b, 64, 0, NB, H1, W1, s));
    a->up0_stored = !(lean && up0_fusable(NB, H, W));
    if (a->up0_stored) {
        NCHK(convT_fwd(n, L_UP0, a->d1b, 64, NB, H1, W1, a->cat0, 64, s));
        NCHK(conv_fwd(n, L_D0A, a->cat0, 64, 0, a->d0a, 32, 0, NB, H, W, s));
    } else {
        NCHK(dec0a_fused(n, a, NB, H, W, s));
    }
    bool headed = false;
    NCHK(conv_fwd(n, L_D0B, a->d0a, 32, 0, a->d0b, 32, 0, NB, H, W, s, nullptr, nullptr, head, &headed, lean));
    a->d0b_stored = !(lean && headed);
    if (head_done) *head_done = headed;
    return hipSuccess;
}

// gradient g (fp32, C channels at g_off of a g_cs-channel buffer) of layer
// li's output -> bf16 operand a->G [P][C] (ReLU-masked by the stored output
// when relu) and the layer's bias gradient
hipError_t mask_round(unet_state *n, unet_act *a, const float *g, int g_cs, int g_off, const uint16_t *act,
                      int a_cs, int a_off, bool relu, int C, int P, int li, hipStream_t s)
{
    const int wgs = (P + 63) / 64;
    hipLaunchKernelGGL(k_mask_round, dim3(wgs), dim3(256), 0, s, g, g_cs, g_off, act, a_cs, a_off, relu ? 1 : 0, a->G,
                       C, P, a->part);
    NCHK(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_rows, dim3(C), dim3(256), 0, s, (const float *)a->part, wgs, C,
                       n->g + layers().L[li].b_off);
    return hipGetLastError();
}

// weight gradient of layer li from a->G (its masked output gradient) and
// its input X; (NB, H, W) is the contraction grid (the coarse grid for convT)
template <int TAP>
hipError_t wgrad(unet_state *n, unet_act *a, int li, const uint16_t *X, int x_cs, int NB, int H, int W, hipStream_t s)
{
    const unet_layer &l = layers().L[li];
    const int P = NB * H * W;
    const int chunk = wgrad_chunk((size_t)P, wgrad_wgs(l));
    const int chunks = (P + chunk - 1) / chunk;
    WgradArgs w{};
    w.G = a->G;
    w.g_cs = l.cout;
    w.X = X;
    w.x_cs = x_cs;
    w.part = a->part;
    w.NB = NB;
    w.H = H;
    w.W = W;
    w.M = l.cout;
    w.K = l.cin_pad;
    w.x_src = l.cin;
    w.chunk = chunk;
    constexpr int taps = TAP == TAP_CONV3 ? 9 : (TAP == TAP_FINE4 ? 4 : 1);
    if (TAP == TAP_CONV3) {
        dim3 grid(l.cin_pad / 32, (l.cout + 63) / 64, chunks);
        hipLaunchKernelGGL(k_wgrad3, grid, dim3(256), 0, s, w);
    } else {
        dim3 grid(taps * (l.cin_pad / 32), (l.cout + 63) / 64, chunks);
        hipLaunchKernelGGL(k_wgrad<TAP>, grid, dim3(256), 0, s, w);
    }
    NCHK(hipGetLastError());
    const int nel = l.cout * taps * l.cin;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((nel + 255) / 256), dim3(256), 0, s, (const float *)a->part, chunks,
                       l.cout, taps, l.cin_pad, l.cin, n->g + l.w_off);
    return hipGetLastError();
}

// data gradient of a 3x3 conv from a->G: fp32 [P][cin]
hipError_t conv_dgrad(unet_state *n, unet_act *a, int li, float *out, int NB, int H, int W, hipStream_t s)
{
    const unet_layer &l = layers().L[li];
    GemmArgs g{};
    g.A = n->wd + l.wd_off;
    g.Bsrc = a->G;
    g.b_cs = l.cout;
    g.out = out;
    g.o_cs = l.cin;
    g.NB = NB;
    g.H = H;
    g.W = W;
    g.K = l.cout;
    g.M = l.cin;
    return conv3<EPI_F32>(g, s);
}

// data gradient of a 2x2 transposed conv: a->G on the fine grid -> fp32 [P_coarse][cin]
hipError_t convT_dgrad(unet_state *n, unet_act *a, int li, float *out, int NB, int Hc, int Wc, hipStream_t s)
{
    const unet_layer &l = layers().L[li];
    GemmArgs g{};
    g.A = n->wd + l.wd_off;
    g.Bsrc = a->G;
    g.b_cs = l.cout;
    g.out = out;
    g.o_cs = l.cin;
    g.NB = NB;
    g.H = Hc;
    g.W = Wc;
    g.K = l.cout;
    g.M = l.cin;
    return gemm<4, 1, TAP_FINE4, EPI_F32>(g, s);
}

hipError_t pool_back(const uint16_t *act, int a_cs, int a_off, const float *g_coarse, const float *skip, int s_cs,
                     int s_off, float *g_fine, int NB, int H, int W, int C, hipStream_t s)
{
    const int64_t n = (int64_t)NB * (H / 2) * (W / 2) * (C / 8);
    hipLaunchKernelGGL(k_pool_back, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, act, a_cs, a_off, g_coarse,
                       skip, s_cs, s_off, g_fine, NB, H, W, C);
    return hipGetLastError();
}

// Adam (apply) and the bf16 copies of every layer
hipError_t prep_weights(unet_state *n, float lr, int apply, hipStream_t s)
{
    float c1 = 1.f, c2 = 1.f;
    if (apply) {
        c1 = (float)(1.0 / (1.0 - std::pow(0.9, n->step)));
        c2 = (float)(1.0 / (1.0 - std::pow(0.999, n->step)));
    }
    const Layers &T = layers();
    for (int i = 0; i < kNL; ++i) {
        const unet_layer &l = T.L[i];
        for (int part = 0; part < 2; ++part) {
            AdamArgs a{};
            const size_t off = part == 0 ? l.w_off : l.b_off;
            a.w = n->w + off;
            a.m = n->m + off;
            a.v = n->v + off;
            a.g = n->g + off;
            a.n = part == 0 ? l.cout * l.taps * l.cin : l.cout;
            a.is_weight = part == 0;
            a.kind = l.kind;
            a.cin = l.cin;
            a.cin_pad = l.cin_pad;
            a.cout = l.cout;
            a.taps = l.taps;
            a.wf = n->wf + l.wf_off;
            a.wd = (l.kind != 2 && i != L_E0A) ? n->wd + l.wd_off : nullptr;
            a.lr = lr;
            a.b1 = 0.9f;
            a.b2 = 0.999f;
            a.eps = 1e-8f;
            a.c1 = c1;
            a.c2 = c2;
            a.apply = apply;
            hipLaunchKernelGGL(k_adam, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
            NCHK(hipGetLastError());
        }
    }
    return hipSuccess;
}

// The convolutions address activations with 32-bit element offsets: the
// widest buffer holds 64 channels per full-resolution pixel.
bool geometry_ok(unet_act *a, int NB, int H, int W)
{
    return NB >= 1 && H >= UNET_ALIGN && W >= UNET_ALIGN && H % UNET_ALIGN == 0 && W % UNET_ALIGN == 0 &&
           (size_t)NB * H * W <= a->cap && (size_t)NB * H * W * 64 < ((size_t)1 << 31);
}

}  // namespace

hipError_t unet_set_params(unet_state *n, const float *host, hipStream_t s)
{
    const Layers &T = layers();
    if (!n->w) {
        NCHK(hipMalloc((void **)&n->w, T.n_params * 4));
        NCHK(hipMalloc((void **)&n->m, T.n_params * 4));
        NCHK(hipMalloc((void **)&n->v, T.n_params * 4));
        NCHK(hipMalloc((void **)&n->g, T.n_params * 4));
        NCHK(hipMalloc((void **)&n->wf, T.n_wf * 2));
        NCHK(hipMalloc((void **)&n->wd, T.n_wd * 2));
    }
    // host buffers are the caller's pageable memory: blocking copies with the
    // stream idle
    NCHK(hipStreamSynchronize(s));
    NCHK(hipMemcpy(n->w, host, T.n_params * 4, hipMemcpyHostToDevice));
    NCHK(hipMemsetAsync(n->m, 0, T.n_params * 4, s));
    NCHK(hipMemsetAsync(n->v, 0, T.n_params * 4, s));
    NCHK(hipMemsetAsync(n->g, 0, T.n_params * 4, s));
    NCHK(hipMemsetAsync(n->wf, 0, T.n_wf * 2, s));   // padded input channels stay zero
    n->step = 0;
    NCHK(prep_weights(n, 0.f, 0, s));
    NCHK(hipStreamSynchronize(s));
    n->loaded = true;
    return hipSuccess;
}

hipError_t unet_get_params(unet_state *n, float *host, hipStream_t s)
{
    NCHK(hipStreamSynchronize(s));
    return hipMemcpy(host, n->w, layers().n_params * 4, hipMemcpyDeviceToHost);
}

hipError_t unet_get_grads(unet_state *n, float *host, hipStream_t s)
{
    NCHK(hipStreamSynchronize(s));
    return hipMemcpy(host, n->g, layers().n_params * 4, hipMemcpyDeviceToHost);
}

hipError_t unet_forward(unet_state *n, unet_act *a, const uint16_t *stack, int NB, int H, int W, float *s_out,
                           uint8_t *rgb, int64_t pitch, int64_t img_stride, int valid_h, int valid_w,
                           hipStream_t s, std::string &err, bool keep)
{
    if (!n->loaded) {
        err = "no network parameters loaded";
        return hipErrorInvalidValue;
    }
    if (!geometry_ok(a, NB, H, W)) {
        err = "network input must be a multiple of 8 in both dimensions and fit the activation set";
        return hipErrorInvalidValue;
    }
    const unet_layer &hl = layers().L[L_HEAD];
    HeadArgs h{};
    h.a = a->d0b;
    h.w = n->wf + hl.wf_off;
    h.bias = n->w + hl.b_off;
    h.s_out = s_out;
    h.rgb = rgb;
    h.pitch = pitch;
    h.img_stride = img_stride;
    h.NB = NB;
    h.H = H;
    h.W = W;
    h.valid_h = valid_h;
    h.valid_w = valid_w;
    bool done = false;
    NCHK(forward_all(n, a, stack, NB, H, W, s, !keep, &h, &done));
    if (done) return hipSuccess;
    const int P = NB * H * W;
    hipLaunchKernelGGL(k_head, dim3((P + 255) / 256), dim3(256), 0, s, h, 0);
    return hipGetLastError();
}

hipError_t unet_forward_batch(unet_state *n, unet_act *a, const uint16_t *stack, int NB, int H, int W,
                              const unet_out *outs, hipStream_t s, std::string &err, bool keep)
{
    if (!n->loaded) {
        err = "no network parameters loaded";
        return hipErrorInvalidValue;
    }
    if (!outs || !geometry_ok(a, NB, H, W)) {
        err = "network input must be a multiple of 8 in both dimensions and fit the activation set";
        return hipErrorInvalidValue;
    }
    const unet_layer &hl = layers().L[L_HEAD];
    HeadArgs h{};
    h.a = a->d0b;
    h.w = n->wf + hl.wf_off;
    h.bias = n->w + hl.b_off;
    h.outs = outs;
    h.NB = NB;
    h.H = H;
    h.W = W;
    bool done = false;
    NCHK(forward_all(n, a, stack, NB, H, W, s, !keep, &h, &done));
    if (done) return hipSuccess;
    const int P = NB * H * W;
    hipLaunchKernelGGL(k_head, dim3((P + 255) / 256), dim3(256), 0, s, h, 0);
    return hipGetLastError();
}

hipError_t unet_train(unet_state *n, unet_act *a, const uint16_t *stack, const float *target, int NB, int H,
                         int W, int valid_h, float lr, int apply, float *loss_host, hipStream_t s, std::string &err)
{
    if (!n->loaded) {
        err = "no network parameters loaded";
        return hipErrorInvalidValue;
    }
    if (!a->train || !geometry_ok(a, NB, H, W) || valid_h < 1 || valid_h > H) {
        err = "bad training geometry";
        return hipErrorInvalidValue;
    }
    NCHK(forward_all(n, a, stack, NB, H, W, s));
    const int P0 = NB * H * W, P1 = P0 / 4, P2 = P1 / 4, P3 = P2 / 4;
    const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
    const Layers &T = layers();
    // head: loss, gradient at dec0b, head weight/bias gradients
    HeadArgs h{};
    h.a = a->d0b;
    h.w = n->wf + T.L[L_HEAD].wf_off;
    h.bias = n->w + T.L[L_HEAD].b_off;
    h.NB = NB;
    h.H = H;
    h.W = W;
    h.valid_h = valid_h;
    h.valid_w = W;
    h.target = target;
    h.inv_n = (float)(1.0 / ((double)NB * valid_h * W * 3));
    h.g_a = a->g0;
    h.part = a->head_part;
    const int hwg = (P0 + 255) / 256;
    hipLaunchKernelGGL(k_head, dim3(hwg), dim3(256), 0, s, h, 1);
    NCHK(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_rows, dim3(100), dim3(256), 0, s, (const float *)a->head_part, hwg, 100, a->part);
    NCHK(hipGetLastError());
    NCHK(hipMemcpyAsync(n->g + T.L[L_HEAD].w_off, a->part, 96 * 4, hipMemcpyDeviceToDevice, s));
    NCHK(hipMemcpyAsync(n->g + T.L[L_HEAD].b_off, a->part + 96, 3 * 4, hipMemcpyDeviceToDevice, s));
    NCHK(hipMemcpyAsync(a->loss_dev, a->part + 99, 4, hipMemcpyDeviceToDevice, s));
    // decoder, level 0
    NCHK(mask_round(n, a, a->g0, 32, 0, a->d0b, 32, 0, true, 32, P0, L_D0B, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_D0B, a->d0a, 32, NB, H, W, s));
    NCHK(conv_dgrad(n, a, L_D0B, a->g1, NB, H, W, s));
    NCHK(mask_round(n, a, a->g1, 32, 0, a->d0a, 32, 0, true, 32, P0, L_D0A, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_D0A, a->cat0, 64, NB, H, W, s));
    NCHK(conv_dgrad(n, a, L_D0A, a->gs0, NB, H, W, s));              // [g_up0 | g_skip0]
    NCHK(mask_round(n, a, a->gs0, 64, 0, nullptr, 0, 0, false, 32, P0, L_UP0, s));
    NCHK(wgrad<TAP_FINE4>(n, a, L_UP0, a->d1b, 64, NB, H1, W1, s));
    NCHK(convT_dgrad(n, a, L_UP0, a->g0, NB, H1, W1, s));            // g(d1b) [P1][64]
    // level 1
    NCHK(mask_round(n, a, a->g0, 64, 0, a->d1b, 64, 0, true, 64, P1, L_D1B, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_D1B, a->d1a, 64, NB, H1, W1, s));
    NCHK(conv_dgrad(n, a, L_D1B, a->g1, NB, H1, W1, s));
    NCHK(mask_round(n, a, a->g1, 64, 0, a->d1a, 64, 0, true, 64, P1, L_D1A, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_D1A, a->cat1, 128, NB, H1, W1, s));
    NCHK(conv_dgrad(n, a, L_D1A, a->gs1, NB, H1, W1, s));            // [g_up1 | g_skip1]
    NCHK(mask_round(n, a, a->gs1, 128, 0, nullptr, 0, 0, false, 64, P1, L_UP1, s));
    NCHK(wgrad<TAP_FINE4>(n, a, L_UP1, a->d2b, 128, NB, H2, W2, s));
    NCHK(convT_dgrad(n, a, L_UP1, a->g0, NB, H2, W2, s));            // g(d2b) [P2][128]
    // level 2
    NCHK(mask_round(n, a, a->g0, 128, 0, a->d2b, 128, 0, true, 128, P2, L_D2B, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_D2B, a->d2a, 128, NB, H2, W2, s));
    NCHK(conv_dgrad(n, a, L_D2B, a->g1, NB, H2, W2, s));
    NCHK(mask_round(n, a, a->g1, 128, 0, a->d2a, 128, 0, true, 128, P2, L_D2A, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_D2A, a->cat2, 256, NB, H2, W2, s));
    NCHK(conv_dgrad(n, a, L_D2A, a->gs2, NB, H2, W2, s));            // [g_up2 | g_skip2]
    NCHK(mask_round(n, a, a->gs2, 256, 0, nullptr, 0, 0, false, 128, P2, L_UP2, s));
    NCHK(wgrad<TAP_FINE4>(n, a, L_UP2, a->mb, 256, NB, H3, W3, s));
    NCHK(convT_dgrad(n, a, L_UP2, a->g0, NB, H3, W3, s));            // g(mb) [P3][256]
    // bottleneck
    NCHK(mask_round(n, a, a->g0, 256, 0, a->mb, 256, 0, true, 256, P3, L_MB, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_MB, a->ma, 256, NB, H3, W3, s));
    NCHK(conv_dgrad(n, a, L_MB, a->g1, NB, H3, W3, s));
    NCHK(mask_round(n, a, a->g1, 256, 0, a->ma, 256, 0, true, 256, P3, L_MA, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_MA, a->p3, 128, NB, H3, W3, s));
    NCHK(conv_dgrad(n, a, L_MA, a->g0, NB, H3, W3, s));              // g(p3) [P3][128]
    // encoder, level 2: g(enc2b) = pool routing of g(p3) + skip
    NCHK(pool_back(a->cat2, 256, 128, a->g0, a->gs2, 256, 128, a->g1, NB, H2, W2, 128, s));
    NCHK(mask_round(n, a, a->g1, 128, 0, a->cat2, 256, 128, true, 128, P2, L_E2B, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_E2B, a->e2a, 128, NB, H2, W2, s));
    NCHK(conv_dgrad(n, a, L_E2B, a->g0, NB, H2, W2, s));
    NCHK(mask_round(n, a, a->g0, 128, 0, a->e2a, 128, 0, true, 128, P2, L_E2A, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_E2A, a->p2, 64, NB, H2, W2, s));
    NCHK(conv_dgrad(n, a, L_E2A, a->g1, NB, H2, W2, s));             // g(p2) [P2][64]
    // level 1
    NCHK(pool_back(a->cat1, 128, 64, a->g1, a->gs1, 128, 64, a->g0, NB, H1, W1, 64, s));
    NCHK(mask_round(n, a, a->g0, 64, 0, a->cat1, 128, 64, true, 64, P1, L_E1B, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_E1B, a->e1a, 64, NB, H1, W1, s));
    NCHK(conv_dgrad(n, a, L_E1B, a->g1, NB, H1, W1, s));
    NCHK(mask_round(n, a, a->g1, 64, 0, a->e1a, 64, 0, true, 64, P1, L_E1A, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_E1A, a->p1, 32, NB, H1, W1, s));
    NCHK(conv_dgrad(n, a, L_E1A, a->g0, NB, H1, W1, s));             // g(p1) [P1][32]
    // level 0
    NCHK(pool_back(a->cat0, 64, 32, a->g0, a->gs0, 64, 32, a->g1, NB, H, W, 32, s));
    NCHK(mask_round(n, a, a->g1, 32, 0, a->cat0, 64, 32, true, 32, P0, L_E0B, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_E0B, a->e0a, 32, NB, H, W, s));
    NCHK(conv_dgrad(n, a, L_E0B, a->g0, NB, H, W, s));
    NCHK(mask_round(n, a, a->g0, 32, 0, a->e0a, 32, 0, true, 32, P0, L_E0A, s));
    NCHK(wgrad<TAP_CONV3>(n, a, L_E0A, stack, UNET_IN, NB, H, W, s));
    if (apply) {
        n->step += 1;
        NCHK(prep_weights(n, lr, 1, s));
    }
    if (loss_host) {
        float sum = 0.f;
        NCHK(hipStreamSynchronize(s));
        NCHK(hipMemcpy(&sum, a->loss_dev, 4, hipMemcpyDeviceToHost));
        *loss_host = (float)(sum / ((double)NB * valid_h * W * 3));
    }
    return hipSuccess;
}

hipError_t unet_read_act(unet_act *a, int layer, void *host, size_t bytes, hipStream_t s)
{
    const uint16_t *src = nullptr;
    int cs = 0, off = 0, C = 0;
    switch (layer) {
    case L_E0A: src = a->e0a; cs = 32; C = 32; break;
    case L_E0B: src = a->cat0; cs = 64; off = 32; C = 32; break;
    case L_E1A: src = a->e1a; cs = 64; C = 64; break;
    case L_E1B: src = a->cat1; cs = 128; off = 64; C = 64; break;
    case L_E2A: src = a->e2a; cs = 128; C = 128; break;
    case L_E2B: src = a->cat2; cs = 256; off = 128; C = 128; break;
    case L_MA: src = a->ma; cs = 256; C = 256; break;
    case L_MB: src = a->mb; cs = 256; C = 256; break;
    case L_UP2: src = a->cat2; cs = 256; C = 128; break;
    case L_D2A: src = a->d2a; cs = 128; C = 128; break;
    case L_D2B: src = a->d2b; cs = 128; C = 128; break;
    case L_UP1: src = a->cat1; cs = 128; C = 64; break;
    case L_D1A: src = a->d1a; cs = 64; C = 64; break;
    case L_D1B: src = a->d1b; cs = 64; C = 64; break;
    case L_UP0:
        if (!a->up0_stored) return hipErrorInvalidValue;
        src = a->cat0;
        cs = 64;
        C = 32;
        break;
    case L_D0A: src = a->d0a; cs = 32; C = 32; break;
    case L_D0B:
        if (!a->d0b_stored) return hipErrorInvalidValue;
        src = a->d0b;
        cs = 32;
        C = 32;
        break;
    default: return hipErrorInvalidValue;
    }
    if (!src || a->NB == 0) return hipErrorInvalidValue;
    const size_t P = ((size_t)a->NB * a->H * a->W) >> (2 * kOutLevel[layer]);
    if (bytes != P * C * 2) return hipErrorInvalidValue;
    NCHK(hipStreamSynchronize(s));
    return hipMemcpy2D(host, (size_t)C * 2, src + off, (size_t)cs * 2, (size_t)C * 2, P, hipMemcpyDeviceToHost);
}

hipError_t unet_check_bf16(unsigned long long *bad_dev, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_bf16, dim3(4096), dim3(256), 0, s, bad_dev);
    return hipGetLastError();
}
