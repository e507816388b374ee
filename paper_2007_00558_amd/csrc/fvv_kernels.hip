// fvv_kernels.hip -- gfx950 kernels of the DIBR view-synthesis path.
//
// Stages (FVV Live, arXiv 2007.00558, Section VI):
//   repack     MVD ingest, once per frame set: RGB8 -> 8-byte texels {RGBA8,
//              depth}, millimetres (or 12-bit coded depth, Section V-A,
//              decoded to millimetres) -> metres with the Eq. (1) correction
//              (Section IV-A)
//   desc       copy of the view descriptors from coherent pinned host memory
//   bin        every pixel of each selected source camera is warped into
//              the virtual image once: its splat record (projected depth and
//              packed footprint) is stored, and each 8x8 source block,
//              bounded by the exact union of its pixels' footprints, is
//              appended to the lists of the output tiles it touches
//   tile       one workgroup per 32x32 output tile: splats its binned blocks
//              (from their pixels' splat records) into an LDS z-buffer of packed
//              (depth, camera, pixel) keys with 64-bit LDS atomicMin, 3x3
//              crack/speckle filter in LDS, backward depth-consistent
//              bilinear fetch from each selected camera mixed by camera
//              distance, hole fill for holes whose neighbours lie inside the
//              tile, writes the RGB8 output
//   fill_open  the remaining holes: nearest covered pixel left/right/up/down
//              through per-tile row and column summaries, larger depth wins
//
// The z-buffer never leaves LDS; the only per-pixel HBM traffic besides the
// source gathers is the RGB8 output and a 4-byte slot per pixel.
//
// Arithmetic contract shared with the definition of the method: every
// decision (pixel coverage, key order, tap validity, hole) is computed in
// float32 op by op -- built with -ffp-contract=off and correctly rounded
// division -- so the key map and the hole map are bit-exact.
#include <algorithm>
#include <climits>

#include "fvv_internal.h"
#include "fvv_y12.h"

namespace {

// Pointers the kernels read from global memory, as global-address-space
// pointers: loads then compile to global_load (not flat_load, which also
// waits on the LDS counter).
template <typename V> using gmem = __attribute__((address_space(1))) const V;
template <typename V> __device__ __forceinline__ gmem<V> *gptr(const V *p) { return (gmem<V> *)p; }

constexpr int T = FVV_TILE;
constexpr int WN = FVV_TILE + 2;   // tile window edge with a 1-pixel halo
constexpr int TNT = T * T / 4;     // threads of a tile workgroup: four pixels each
constexpr int TNW = TNT / 64;      // its waves
constexpr int TPR = T / 4;         // threads per tile row
static_assert(T % 4 == 0 && TNT % 64 == 0 && TNT >= 2 * T && TNT <= 1024, "tile workgroup shape");

__device__ __forceinline__ uint32_t f2u(float f) { return __float_as_uint(f); }
__device__ __forceinline__ float u2f(uint32_t u) { return __uint_as_float(u); }
// two float32 values to packed bfloat16 bits (lo in the low half), round
// to nearest even, by v_cvt_pk_bf16_f32 (fvv_check_bf16 compares it with
// the rounding written out on the bits over every non-NaN float32)
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pack(float lo, float hi)
{
    const f32x2_t v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// p_r = ((M_r0 i + M_r1 j) + M_r2) z + m_r, each op rounded to float32
__device__ __forceinline__ void project(const float *M, const float *m, float i, float j, float z,
                                        float &p0, float &p1, float &p2)
{
    p0 = __fadd_rn(__fmul_rn(__fadd_rn(__fadd_rn(__fmul_rn(M[0], i), __fmul_rn(M[1], j)), M[2]), z), m[0]);
    p1 = __fadd_rn(__fmul_rn(__fadd_rn(__fadd_rn(__fmul_rn(M[3], i), __fmul_rn(M[4], j)), M[5]), z), m[1]);
    p2 = __fadd_rn(__fmul_rn(__fadd_rn(__fadd_rn(__fmul_rn(M[6], i), __fmul_rn(M[7], j)), M[8]), z), m[2]);
}

// a / b rounded to nearest from y = RN(1/b), bit for bit what a correctly
// rounded division gives (Markstein's theorem: q = RN(a y) is within one ulp
// of a/b, the remainder a - b q is exact in one fused multiply-add, and
// RN(q + rem y) = RN(a/b); no overflow or underflow for the magnitudes of
// image coordinates and depths).  Lets one division serve every quotient by
// the same projected depth at three instructions per extra quotient.
__device__ __forceinline__ float div_by(float a, float b, float y)
{
    const float q = __fmul_rn(a, y);
    const float rem = __fmaf_rn(-b, q, a);
    return __fmaf_rn(rem, y, q);
}

// RN(1/b) for a normal b with a normal reciprocal (every projected depth,
// 0.01 < b < 2^126): the hardware reciprocal (within one ulp of 1/b) refined
// by one Newton step in fused multiply-adds, y0 + y0 (1 - b y0), is the
// correctly rounded reciprocal for every significand of b except all ones.
// There the step can stay on the even neighbour one ulp below RN(1/b), whose
// significand is odd (1/b lies just above the midpoint of the two), so that
// significand gets its low bit set.  Three instructions fewer than the
// correctly rounded division; fvv_check_reciprocal compares the two over
// every significand of a range of binades on the device.
__device__ __forceinline__ float rcp_rn(float b)
{
    const float y0 = __builtin_amdgcn_rcpf(b);
    const float y1 = __fmaf_rn(__fmaf_rn(-b, y0, 1.0f), y0, y0);
    const uint32_t ones = ((f2u(b) & 0x7FFFFFu) + 1u) >> 23;   // 1 iff the significand is all ones
    return u2f(f2u(y1) | ones);
}

// Row of source block blk (< 2^24; nbx <= 8192): with m = ceil(2^40 / nbx),
// blk m / 2^40 exceeds blk / nbx by less than blk / 2^40 < 2^-16 <= 1 / nbx,
// too little to reach the next integer, so its floor is the quotient: a
// 64-bit multiply on the scalar unit instead of an integer division.
__device__ __forceinline__ int block_row(int blk, const fvv_src_desc &s)
{
    return (int)(((uint64_t)(uint32_t)blk * s.nbx_magic) >> 40);
}

struct Footprint {
    int x0, x1, y0, y1;
    unsigned long long key;
};

// Forward warp of source pixel (i, j) at depth z: the output pixel centres
// x with u - mx/2 <= x < u + mx/2 (rows likewise), mx = clamp(sx z / p2, 1,
// max_fp), clipped to the output image; key = depth bits | camera | pixel.
// In float32 with correctly rounded quotients u = p0/p2, v = p1/p2,
// mx = (sx z)/p2, my = (sy z)/p2 (one division, see div_by).
__device__ __forceinline__ bool splat_point(const fvv_src_desc &s, int W, int H, float max_fp, int i, int j,
                                            float z, Footprint &f)
{
    float q0, q1, q2;
    project(s.A, s.a, (float)i, (float)j, z, q0, q1, q2);
    if (!(q2 > FVV_ZCLIP)) return false;
    const float r = rcp_rn(q2);   // one correctly rounded reciprocal per point
    const float u = div_by(q0, q2, r), v = div_by(q1, q2, r);
    if (!isfinite(u) || !isfinite(v)) return false;
    float mx = div_by(__fmul_rn(s.sx, z), q2, r);
    float my = div_by(__fmul_rn(s.sy, z), q2, r);
    mx = fminf(fmaxf(mx, 1.0f), max_fp);
    my = fminf(fmaxf(my, 1.0f), max_fp);
    const float hx = __fmul_rn(0.5f, mx), hy = __fmul_rn(0.5f, my);
    float x0f = ceilf(__fsub_rn(u, hx)), x1f = __fsub_rn(ceilf(__fadd_rn(u, hx)), 1.0f);
    float y0f = ceilf(__fsub_rn(v, hy)), y1f = __fsub_rn(ceilf(__fadd_rn(v, hy)), 1.0f);
    x0f = fmaxf(x0f, 0.0f);
    y0f = fmaxf(y0f, 0.0f);
    x1f = fminf(x1f, (float)(W - 1));
    y1f = fminf(y1f, (float)(H - 1));
    if (x0f > x1f || y0f > y1f) return false;
    f.x0 = (int)x0f;
    f.x1 = (int)x1f;
    f.y0 = (int)y0f;
    f.y1 = (int)y1f;
    f.key = ((unsigned long long)f2u(q2) << 32) | ((unsigned long long)(uint32_t)s.cam << 27) |
            (unsigned long long)(uint32_t)(j * s.W + i);   // < 2^27 pixels
    return true;
}

// Wave-wide min / max of a u32 with DPP lane moves: pairs, quads, half rows
// and rows inside each 16-lane row, then the row broadcasts carry rows
// 0 -> 1, 2 -> 3 and 1 -> 2, 3; lane 63 then holds the result for the whole
// wave.  Each step folds into one v_min_u32_dpp / v_max_u32_dpp: lanes a
// move does not write keep their own value, the identity of min and max.
template <bool MIN>
__device__ __forceinline__ uint32_t wave_reduce_u32(uint32_t v)
{
    constexpr int id = MIN ? (int)0xFFFFFFFF : 0;
    auto op = [](uint32_t a, int b) { return MIN ? min(a, (uint32_t)b) : max(a, (uint32_t)b); };
    v = op(v, __builtin_amdgcn_update_dpp(id, (int)v, 0xB1, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(id, (int)v, 0x4E, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(id, (int)v, 0x141, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(id, (int)v, 0x140, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(id, (int)v, 0x142, 0xA, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(id, (int)v, 0x143, 0xC, 0xF, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ float wave_minf(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_maxf(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// ---------------------------------------------------------------- repack
// One thread per source pixel (grid.z = camera): 8-byte texel {RGBA8,
// decoded depth bits} for the backward gathers and the decoded depth plane
// for the splat.  Millimetres 0 and 0xFFFF (the background signal) carry no
// live depth; holes (0) may first be closed by the pre-filter.  With a background model the background layer's texel and
// depth planes are written too (layered synthesis, Section VI).
// live millimetres of source pixel (x, y): uint16, or decoded from the I420
// 12-bit coding (Y, then U with the even rows' MSBs, then V with the odd rows')
__device__ __forceinline__ uint32_t live_mm(const fvv_repack_batch &b, const fvv_repack_cam &c, int x, int y)
{
    if (b.y12) {
        const int64_t uvp = c.depth_pitch >> 1;
        const uint8_t *pl = c.depth + (int64_t)c.H * c.depth_pitch + ((y & 1) ? (int64_t)(c.H >> 1) * uvp : 0);
        const uint32_t uv = pl[(int64_t)(y >> 1) * uvp + (x >> 1)];
        return y12_dequantise(y12_unfold(c.depth[(int64_t)y * c.depth_pitch + x], y12_msb(uv, x & 1)), b.planes);
    }
    return *(const uint16_t *)(c.depth + (int64_t)y * c.depth_pitch + (int64_t)x * 2);
}

// Hole-filling joint bilateral pre-filter (Section VI pre-processing of the
// live depth): the integer bilateral mean of the valid depths around a hole,
// spatial weight times the weight of the L1 colour distance, when at least
// jbf_min neighbours carry weight; 0 (still a hole) otherwise.  Inlined: the
// batch lives in the kernel arguments, and a call would copy it to scratch.
__device__ __forceinline__ uint32_t jbf_fill(const fvv_repack_batch &b, const fvv_repack_cam &c, int x, int y,
                                             const uint8_t *p)
{
    const int r = b.jbf_radius, n = 2 * r + 1;
    const uint32_t *ws = b.jbf, *wc = b.jbf + FVV_JBF_WS;
    uint64_t sw = 0, swd = 0;
    int cnt = 0;
    for (int dy = -r; dy <= r; ++dy) {
        const int yy = y + dy;
        if (yy < 0 || yy >= c.H) continue;
        for (int dx = -r; dx <= r; ++dx) {
            const int xx = x + dx;
            if ((dx | dy) == 0 || xx < 0 || xx >= c.W) continue;
            const uint32_t q = live_mm(b, c, xx, yy);
            if (q == 0 || q == FVV_BG_MM) continue;
            const uint8_t *pq = c.rgb + (int64_t)yy * c.rgb_pitch + (int64_t)xx * 3;
            const int dist = abs((int)p[0] - (int)pq[0]) + abs((int)p[1] - (int)pq[1]) + abs((int)p[2] - (int)pq[2]);
            const uint64_t w = (uint64_t)(ws[(dy + r) * n + dx + r] * wc[dist]);
            if (w == 0) continue;
            sw += w;
            swd += w * q;
            ++cnt;
        }
    }
    return (cnt >= b.jbf_min && sw > 0) ? (uint32_t)((swd + sw / 2) / sw) : 0u;
}

__global__ void __launch_bounds__(256) k_repack(const fvv_repack_batch b)
{
    const fvv_repack_cam &c = b.cam[blockIdx.z];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= c.W || y >= c.H) return;
    const uint8_t *p = c.rgb + (int64_t)y * c.rgb_pitch + (int64_t)x * 3;
    const uint32_t col = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | 0xFF000000u;
    uint32_t d = live_mm(b, c, x, y);
    if (d == 0 && b.jbf) d = jbf_fill(b, c, x, y, p);
    uint32_t zb = FVV_NO_DEPTH;
    if (d != 0 && d != FVV_BG_MM) {
        const float z = __fdiv_rn((float)d, 1000.0f);
        const float s = __fadd_rn(__fmul_rn(c.alpha, z), c.beta);   // Eq. (1): (alpha z + beta) z
        zb = f2u(__fmul_rn(s, z));
    }
    const int64_t o = (int64_t)y * c.W + x;
    c.texel_out[o] = make_uint2(col, zb);
    c.depth_out[o] = u2f(zb);
    if (c.bg_texel_out) {
        // background layer: the model's depth (calibrated geometry, no Eq. 1)
        // under the live colour of pixels that carry the background signal
        uint32_t bz = FVV_NO_DEPTH;
        const uint32_t m = c.bg_model ? c.bg_model[o] : 0u;
        if (d == FVV_BG_MM && m != 0 && m != FVV_BG_MM) bz = f2u(__fdiv_rn((float)m, 1000.0f));
        c.bg_texel_out[o] = make_uint2(col, bz);
        c.bg_depth_out[o] = u2f(bz);
    }
}

// ---------------------------------------------------------------- descriptors
__global__ void __launch_bounds__(256) k_desc(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int n)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = src[e];
}

// One view's descriptor passed by value (calls that allocate nothing have
// no pinned host copy to read): thread 0 stores it, and every thread clears
// the view's tile counters, which the binning expects at zero.
__global__ void __launch_bounds__(256) k_desc_one(const fvv_view_desc d, fvv_view_desc *__restrict__ dst,
                                                  int32_t *__restrict__ counts, int n_counts)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = d;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_counts; e += gridDim.x * blockDim.x) counts[e] = 0;
}

// ---------------------------------------------------------------- binning
// One wave per (view, camera slot, 8x8 source block), one lane per pixel:
// the exact output bounds of the block's footprints (each pixel projected as
// the splat projects it), turned into the range of tiles whose window -- the
// tile plus a 1-pixel halo -- they touch, and appended to those tiles' lists.
// Entries past a tile's capacity are dropped and that tile then scans every
// block's range instead.  (Bounds from the corners of the block's depth range
// would save the per-pixel projections, but depth noise widens them along
// the epipolar lines by several pixels and roughly doubles the tile work.)
__global__ void __launch_bounds__(256) k_bin(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.z];
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) *vd.open_count = 0;
    const int k = blockIdx.y;
    const int lane = threadIdx.x & 63;
    if (k >= fvv_nsrc(vd)) return;
    const fvv_src_desc &s = vd.src[k];
    // FVV_BIN_BPW consecutive blocks per wave (wave-uniform indices: the
    // block arithmetic stays on the scalar unit).  A wave is bound by the
    // latency of its depth loads and list atomics, so each wave carries
    // independent blocks whose loads, reductions and atomics overlap.
    const int blk0 = __builtin_amdgcn_readfirstlane((blockIdx.x * 4 + (threadIdx.x >> 6)) * FVV_BIN_BPW);
    if (blk0 >= s.nblk) return;
    uint32_t zb[FVV_BIN_BPW];
    int pi[FVV_BIN_BPW], pj[FVV_BIN_BPW];
#pragma unroll
    for (int q = 0; q < FVV_BIN_BPW; ++q) {
        const int by = block_row(blk0 + q, s), bx = blk0 + q - by * s.nbx;
        pi[q] = bx * FVV_SBLK + (lane & (FVV_SBLK - 1));
        pj[q] = by * FVV_SBLK + lane / FVV_SBLK;
        zb[q] = FVV_NO_DEPTH;
        if (blk0 + q < s.nblk && pi[q] < s.W && pj[q] < s.H) zb[q] = f2u(gptr(s.depth)[(uint32_t)(pj[q] * s.W + pi[q])]);
    }
    // footprint bounds, clipped to the output (< 8192); 0x7FFF as the
    // smallest x0 marks "none"
    int4 t[FVV_BIN_BPW];
#pragma unroll
    for (int q = 0; q < FVV_BIN_BPW; ++q) {
        uint32_t x0 = 0x7FFFu, y0 = 0x7FFFu, x1 = 0u, y1 = 0u;
        Footprint f;
        uint32_t rz = FVV_NO_DEPTH, rf = 0u;   // this pixel's splat record
        if (zb[q] != FVV_NO_DEPTH && splat_point(s, vd.W, vd.H, vd.max_fp, pi[q], pj[q], u2f(zb[q]), f)) {
            x0 = (uint32_t)f.x0;
            y0 = (uint32_t)f.y0;
            x1 = (uint32_t)f.x1;
            y1 = (uint32_t)f.y1;
            rz = (uint32_t)(f.key >> 32);
            rf = (x1 - x0 <= 7u && y1 - y0 <= 7u) ? (x0 | y0 << 13 | (x1 - x0) << 26 | (y1 - y0) << 29)
                                                  : FVV_SPL_RECOMPUTE;
        }
        if (blk0 + q < s.nblk)
            ((__attribute__((address_space(1))) unsigned long long *)
                 vd.spl)[((uint32_t)(k * vd.blk_stride + blk0 + q) << 6) + (uint32_t)lane] =
                (unsigned long long)rf << 32 | rz;
        const int fx0 = (int)wave_reduce_u32<true>(x0), fy0 = (int)wave_reduce_u32<true>(y0);
        const int fx1 = (int)wave_reduce_u32<false>(x1), fy1 = (int)wave_reduce_u32<false>(y1);
        t[q] = make_int4(1, 0, 1, 0);   // empty
        if (fx0 != 0x7FFF) {
            t[q].x = max(0, (fx0 + T - 1) / T - 1);
            t[q].y = min(vd.ntx - 1, (fx1 + 1) / T);
            t[q].z = max(0, (fy0 + T - 1) / T - 1);
            t[q].w = min(vd.nty - 1, (fy1 + 1) / T);
        }
        if (lane == 0 && blk0 + q < s.nblk) vd.bbox[(int64_t)k * vd.blk_stride + blk0 + q] = t[q];
    }
    auto append = [&](int tile, int blk) {
        const int pos = __hip_atomic_fetch_add((__attribute__((address_space(1))) int32_t *)(vd.counts + tile), 1,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (pos < vd.tile_cap)
            ((__attribute__((address_space(1))) int32_t *)vd.list)[(uint64_t)(uint32_t)tile * (uint32_t)vd.tile_cap +
                                                                   (uint32_t)pos] = (k << 24) | blk;
    };
    // the usual case, every range within 8 x (64 / 8 / FVV_BIN_BPW) tiles:
    // one atomic instruction appends all blocks of the wave, lane group q
    // (64 / FVV_BIN_BPW lanes) taking block q's tiles
    constexpr int GL = 64 / FVV_BIN_BPW, GY = GL / 8;
    bool small = true;
#pragma unroll
    for (int q = 0; q < FVV_BIN_BPW; ++q)
        small = small && (t[q].x > t[q].y || (t[q].y - t[q].x < 8 && t[q].w - t[q].z < GY));
    if (small) {
        const int g = lane / GL, ex = lane & 7, ey = (lane % GL) >> 3;
        int4 r = t[0];
#pragma unroll
        for (int q = 1; q < FVV_BIN_BPW; ++q)
            if (g == q) r = t[q];
        if (r.x + ex <= r.y && r.z + ey <= r.w) append((r.z + ey) * vd.ntx + r.x + ex, blk0 + g);
    } else {
#pragma unroll
        for (int q = 0; q < FVV_BIN_BPW; ++q) {
            if (t[q].x > t[q].y) continue;
            const int nx = t[q].y - t[q].x + 1, n = nx * (t[q].w - t[q].z + 1);
            for (int e = lane; e < n; e += 64) append((t[q].z + e / nx) * vd.ntx + t[q].x + e % nx, blk0 + q);
        }
    }
}

// ---------------------------------------------------------------- filter
#define CSWAP(a, b)                                     \
    {                                                   \
        const unsigned long long lo_ = min(v[a], v[b]); \
        const unsigned long long hi_ = max(v[a], v[b]); \
        v[a] = lo_;                                     \
        v[b] = hi_;                                     \
    }

// Lower median (element (n-1)/2 in key order) of the valid keys among the 8
// neighbours.  Empty keys (all ones) order last, so sorting all eight with a
// 19-comparator network and taking that element is exact.
__device__ __forceinline__ unsigned long long lower_median8(unsigned long long v[8], int n)
{
    CSWAP(0, 2) CSWAP(1, 3) CSWAP(4, 6) CSWAP(5, 7)
    CSWAP(0, 4) CSWAP(1, 5) CSWAP(2, 6) CSWAP(3, 7)
    CSWAP(0, 1) CSWAP(2, 3) CSWAP(4, 5) CSWAP(6, 7)
    CSWAP(2, 4) CSWAP(3, 5)
    CSWAP(1, 4) CSWAP(3, 6)
    CSWAP(1, 2) CSWAP(3, 4) CSWAP(5, 6)
    const int m = (n - 1) >> 1;
    unsigned long long res = v[0];
#pragma unroll
    for (int e = 1; e < 8; ++e)
        if (m == e) res = v[e];
    return res;
}
#undef CSWAP

__device__ __forceinline__ int valid_count(const unsigned long long v[8])
{
    int n = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) n += v[e] != FVV_KEY_EMPTY;
    return n;
}

// Crack fill (empty key, >= 5 valid neighbours) and speckle removal (valid
// key, >= 5 valid neighbours, none within tau z0) take the lower median of
// the valid neighbours; every other pixel keeps its key.
__device__ __forceinline__ bool filter_needs_median(unsigned long long c, const unsigned long long v[8], float tau)
{
    // an empty key's depth word is all ones, a valid key's is the bit
    // pattern of a positive float (sign bit clear): the sign bits count the
    // empty neighbours
    uint32_t empty = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) empty += (uint32_t)(v[e] >> 63);
    if (empty > 3) return false;   // fewer than five valid neighbours
    if (c == FVV_KEY_EMPTY) return true;
    const float z0 = u2f((uint32_t)(c >> 32));
    const float lim = __fmul_rn(tau, z0);
    // a neighbour within tau: the smallest |z_k - z0| is <= lim (an empty
    // neighbour's depth is a NaN, which the minimum passes over; all NaN
    // compares false)
    float d = fabsf(__fsub_rn(u2f((uint32_t)(v[0] >> 32)), z0));
#pragma unroll
    for (int e = 1; e < 8; ++e) d = fminf(d, fabsf(__fsub_rn(u2f((uint32_t)(v[e] >> 32)), z0)));
    return !(d <= lim);
}

__device__ __forceinline__ unsigned long long filter_key(unsigned long long c, unsigned long long v[8], float tau)
{
    return filter_needs_median(c, v, tau) ? lower_median8(v, valid_count(v)) : c;
}

// ---------------------------------------------------------------- blend
// Backward warp of output pixel (x, y) at depth zf into the K source slots
// from k0 (one layer's selected cameras); taps whose source depth agrees with
// the warped depth within tau are mixed bilinearly, cameras by their
// distance weights.  Returns true and the RGBA8 colour if any camera
// contributes.
//
// ST (learned path): also the pixel's stack channels ch[0..14] from the
// same per-camera samples: for each of the first three slots that
// contributes, its bilinear colour (R, G, B / 255), the inverse source depth
// 0.5 / q_z capped at 1 and a validity flag 1 (the caller zeroes ch first:
// slots without a consistent tap stay zero).
template <bool ST>
__device__ __forceinline__ bool blend_pixel(const fvv_view_desc &vd, int k0, int x, int y, float zf, uint32_t &rgba,
                                            float *ch = nullptr)
{
    // Decisions (sample in range, tap valid and depth-consistent, camera
    // survives) in float32 op by op; the colour mix is value arithmetic and
    // uses fused multiply-adds and hardware reciprocals.
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, wsum = 0.f;
    auto camera = [&](int k, float *chk) {
        const fvv_src_desc &s = vd.src[k];
        float q0, q1, q2;
        project(s.B, s.b, (float)x, (float)y, zf, q0, q1, q2);
        if (!(q2 > FVV_ZCLIP)) return;
        const float r = rcp_rn(q2);
        const float u = div_by(q0, q2, r), v = div_by(q1, q2, r);
        if (!(u >= -0.5f && u <= s.umax)) return;
        if (!(v >= -0.5f && v <= s.vmax)) return;
        const float fi0 = floorf(u), fj0 = floorf(v);
        const float fu = __fsub_rn(u, fi0), fv = __fsub_rn(v, fj0);
        const int i0 = (int)fi0, j0 = (int)fj0;
        const float lim = __fmul_rn(vd.tau, q2);
        // i0 >= -1 and i0 <= W - 1 (likewise j0): only the outer taps can fall
        // off.  The four taps are read together from clamped coordinates; a
        // tap off the image or not depth-consistent gets weight 0 (adding
        // 0 * colour and 0 to the sums leaves them unchanged, as skipping it
        // would).
        const float gu = 1.0f - fu, gv = 1.0f - fv;
        const float wx0 = i0 >= 0 ? gu : 0.0f, wx1 = i0 + 1 < s.W ? fu : 0.0f;
        const float wy0 = j0 >= 0 ? gv : 0.0f, wy1 = j0 + 1 < s.H ? fv : 0.0f;
        const float wt[4] = {wx0 * wy0, wx1 * wy0, wx0 * wy1, wx1 * wy1};
        const int ic[2] = {max(i0, 0), min(i0 + 1, s.W - 1)};
        // 32-bit texel indices (a source has < 2^27 pixels): a uniform base
        // plus a 32-bit offset needs no 64-bit address arithmetic
        const uint32_t jr[2] = {(uint32_t)__umul24((uint32_t)max(j0, 0), (uint32_t)s.W),
                                (uint32_t)__umul24((uint32_t)min(j0 + 1, s.H - 1), (uint32_t)s.W)};
        const gmem<unsigned long long> *tex = gptr((const unsigned long long *)s.texel);
        uint2 tx[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const unsigned long long t = tex[jr[n >> 1] + (uint32_t)ic[n & 1]];
            tx[n] = make_uint2((uint32_t)t, (uint32_t)(t >> 32));
        }
        float c0 = 0.f, c1 = 0.f, c2 = 0.f, csum = 0.f;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            // a texel without depth holds FVV_NO_DEPTH, a NaN as float32,
            // so the consistency test alone rejects it (NaN <= lim is false)
            const float w = fabsf(__fsub_rn(u2f(tx[n].y), q2)) <= lim ? wt[n] : 0.0f;
            c0 = fmaf(w, (float)(tx[n].x & 0xFF), c0);
            c1 = fmaf(w, (float)((tx[n].x >> 8) & 0xFF), c1);
            c2 = fmaf(w, (float)((tx[n].x >> 16) & 0xFF), c2);
            csum += w;
        }
        // a camera without a consistent tap adds nothing (no branch, so the
        // colour words are read with the depths)
        const bool any = csum > 0.f;
        const float inv = any ? s.wgt * __builtin_amdgcn_rcpf(csum) : 0.0f;
        acc0 = fmaf(c0, inv, acc0);
        acc1 = fmaf(c1, inv, acc1);
        acc2 = fmaf(c2, inv, acc2);
        wsum += any ? s.wgt : 0.0f;
        if (ST && chk && any) {
            // colour / csum / 255: value arithmetic (within a bfloat16 step
            // of the exact quotient); the inverse depth 0.5 / q2 is exact:
            // half of the correctly rounded reciprocal
            const float icol = __builtin_amdgcn_rcpf(csum) * (1.0f / 255.0f);
            chk[0] = c0 * icol;
            chk[1] = c1 * icol;
            chk[2] = c2 * icol;
            chk[3] = fminf(0.5f * r, 1.0f);
            chk[4] = 1.0f;
        }
    };
    if (ST) {
        // the stack's three slots unrolled, so their channels stay in registers
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k < vd.K) camera(k0 + k, ch + 5 * k);
        for (int k = 3; k < vd.K; ++k) camera(k0 + k, nullptr);
    } else {
        for (int k = 0; k < vd.K; ++k) camera(k0 + k, nullptr);
    }
    if (!(wsum > 0.f)) return false;
    const float iw = __builtin_amdgcn_rcpf(wsum);
    const float r = fminf(floorf(fmaf(acc0, iw, 0.5f)), 255.f);
    const float g = fminf(floorf(fmaf(acc1, iw, 0.5f)), 255.f);
    const float b = fminf(floorf(fmaf(acc2, iw, 0.5f)), 255.f);
    rgba = (uint32_t)r | ((uint32_t)g << 8) | ((uint32_t)b << 16) | 0xFF000000u;
    return true;
}

// Learned-path input of output pixel (x, y): channels ch[0..14] from
// blend_pixel (zeros for pixels without a filtered point and for the
// padding beyond the image), the last of 16 bf16 channels zero, 32 bytes
// per pixel.
__device__ __forceinline__ void store_stack(const fvv_view_desc &vd, int x, int y, const float ch[16])
{
    uint4 *o = (uint4 *)(vd.stack + ((int64_t)y * vd.stack_w + x) * 16);
    o[0] = make_uint4(bf16_pack(ch[0], ch[1]), bf16_pack(ch[2], ch[3]), bf16_pack(ch[4], ch[5]), bf16_pack(ch[6], ch[7]));
    o[1] = make_uint4(bf16_pack(ch[8], ch[9]), bf16_pack(ch[10], ch[11]), bf16_pack(ch[12], ch[13]),
                      bf16_pack(ch[14], 0.f));
}

__device__ __forceinline__ void put_rgb(uint8_t *out, int64_t pitch, int x, int y, uint32_t c)
{
    uint8_t *p = out + (int64_t)y * pitch + (int64_t)x * 3;
    p[0] = (uint8_t)c;
    p[1] = (uint8_t)(c >> 8);
    p[2] = (uint8_t)(c >> 16);
}

__device__ __forceinline__ uint32_t get_rgb(const uint8_t *out, int64_t pitch, int x, int y)
{
    const uint8_t *p = out + (int64_t)y * pitch + (int64_t)x * 3;
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
}

// Hole-fill preference: larger depth, then nearer, then the earlier
// direction (callers offer candidates in the order left, right, up, down).
struct Cand {
    float z;
    int dist;
    int idx;    // tile-local or image index of the chosen pixel, -1 none
};

__device__ __forceinline__ void offer(Cand &b, float z, int dist, int idx)
{
    if (b.idx < 0 || z > b.z || (z == b.z && dist < b.dist)) {
        b.z = z;
        b.dist = dist;
        b.idx = idx;
    }
}

// ---------------------------------------------------------------- fused tile
// STACK: views may carry a learned-path stack (a separate instantiation, so
// the plain kernel keeps its register budget and occupancy).
template <bool STACK, bool LAYERED>
__device__ __forceinline__ void tile_body(const fvv_view_desc *__restrict__ views, int mtx, int mty, int n_views)
{
    // XCD-aware order: workgroups are dealt to the 8 XCDs round-robin, so
    // dispatch index b runs on XCD b % 8.  Each XCD takes a contiguous
    // eighth of the (view, tile) sequence in raster order; neighbouring
    // tiles, which splat many of the same source blocks, then share one L2.
    const int per_view = mtx * mty;
    const int total = per_view * n_views;
    const int per_xcd = (total + FVV_XCDS - 1) / FVV_XCDS;
    const int b = blockIdx.x;
    const int w = (b % FVV_XCDS) * per_xcd + b / FVV_XCDS;
    if (w >= total) return;
    const int view = w / per_view, rem = w - view * per_view;
    const int ty = rem / mtx, tx = rem - ty * mtx;
    const fvv_view_desc &vd = views[view];
    if (tx >= vd.ntx || ty >= vd.nty) return;
    const int W = vd.W, H = vd.H;
    const int tile = ty * vd.ntx + tx;
    const int X0 = tx * T, Y0 = ty * T;
    const int WX0 = X0 - 1, WY0 = Y0 - 1;
    const int tw = min(T, W - X0), th = min(T, H - Y0);
    // z-buffer window(s): layered views keep the foreground layer in the
    // first and the background layer in the second
    constexpr int NZ = LAYERED ? 2 * WN * WN : WN * WN;
    __shared__ unsigned long long zk[NZ];
    // the tile's filtered keys during the filter, then its slots and colours
    __shared__ unsigned long long s_buf[T * T];
    uint32_t *const s_slot = (uint32_t *)s_buf;
    uint32_t *const s_rgb = s_slot + T * T;
    unsigned long long *const s_kf = s_buf;
    // pixels whose filtered key is a median (the two-window variant filters
    // in place: its LDS budget has no room for the list)
    __shared__ uint16_t s_med[LAYERED ? 2 : T * T];
    __shared__ int s_open, s_hole, s_nmed;
    const int t = threadIdx.x;
    const int n_entries = vd.counts[tile];
    for (int e = t; e < NZ; e += TNT) zk[e] = FVV_KEY_EMPTY;
    if (t == 0) {
        s_open = 0;
        s_hole = 0;
        s_nmed = 0;
    }
    __syncthreads();

    // ---- S1: splat every binned source block into the window; each wave
    // takes its own list entries (one 8x8 source block = one wave)
    const bool scan_all = n_entries > vd.tile_cap;
    // the wave index and every list entry are wave-uniform: kept in scalar
    // registers, the source descriptor of an entry is read with scalar loads
    // and its block arithmetic runs on the scalar unit
    const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int si = lane & (FVV_SBLK - 1), sj = lane / FVV_SBLK;
    // this lane's splat record of block `ent`, written by the binning
    // (the same projection and footprint as splat_point, computed once per
    // block instead of once per tile that lists it)
    auto block_rec = [&](int ent) -> unsigned long long {
        ent = __builtin_amdgcn_readfirstlane(ent);   // uniform (see above)
        return gptr(vd.spl)[((uint32_t)((ent >> 24) * vd.blk_stride + (ent & 0xFFFFFF)) << 6) + (uint32_t)lane];
    };
    auto splat_entry = [&](int ent, unsigned long long rec) {
        ent = __builtin_amdgcn_readfirstlane(ent);   // uniform; the pipeline's copies lose that
        const uint32_t rz = (uint32_t)rec, rf = (uint32_t)(rec >> 32);
        // a point without depth (its record's footprint is 0) is dropped
        // with the empty footprints below: one lane branch per entry, not two
        const bool live = rz != FVV_NO_DEPTH;
        const fvv_src_desc &s = vd.src[(uint32_t)ent >> 24];
        const int blk = ent & 0xFFFFFF;
        const int by = block_row(blk, s), bx = blk - by * s.nbx;
        const int i = bx * FVV_SBLK + si, j = by * FVV_SBLK + sj;
        Footprint f;
        if (rf != FVV_SPL_RECOMPUTE) {
            f.x0 = (int)(rf & 0x1FFFu);
            f.y0 = (int)((rf >> 13) & 0x1FFFu);
            f.x1 = f.x0 + (int)((rf >> 26) & 7u);
            f.y1 = f.y0 + (int)(rf >> 29);
            f.key = ((unsigned long long)rz << 32) | ((unsigned long long)(uint32_t)s.cam << 27) |
                    (unsigned long long)(uint32_t)(j * s.W + i);
        } else if (!splat_point(s, W, H, vd.max_fp, i, j, gptr(s.depth)[(uint32_t)(j * s.W + i)], f)) {
            return;
        }
        const int xa = max(f.x0, WX0), xb = live ? min(f.x1, WX0 + WN - 1) : xa - 1;
        const int ya = max(f.y0, WY0), yb = min(f.y1, WY0 + WN - 1);
        unsigned long long *zl = (LAYERED && (ent >> 24) >= vd.K) ? zk + WN * WN : zk;
        if (xa > xb || ya > yb) return;
        // the first 2 x 2 pixels of the footprint (all of it at the usual
        // magnifications) as predicated atomics, the rest in a loop
        unsigned long long *z0 = zl + (ya - WY0) * WN + (xa - WX0);
        const bool wx = xa < xb, wy = ya < yb;
        atomicMin(z0, f.key);
        if (wx) atomicMin(z0 + 1, f.key);
        if (wy) atomicMin(z0 + WN, f.key);
        if (wx && wy) atomicMin(z0 + WN + 1, f.key);
        if (xb - xa > 1 || yb - ya > 1) {
            for (int y = ya; y <= yb; ++y)
                for (int x = xa; x <= xb; ++x)
                    if (x - xa > 1 || y - ya > 1) atomicMin(&zl[(y - WY0) * WN + (x - WX0)], f.key);
        }
    };
    if (!scan_all) {
        // The wave's entries are e = wave + TNW q; the splat records of the
        // next two entries are in flight while the current one is splatted,
        // so the dependent loads of consecutive entries overlap instead of
        // queueing.
        // the list was written by the binning and is only read here: wave-
        // uniform entries come through the scalar cache (constant address
        // space), straight into scalar registers
        const __attribute__((address_space(4))) int32_t *lst =
            (const __attribute__((address_space(4))) int32_t *)(vd.list + (int64_t)tile * vd.tile_cap + wave);
        const int nq = __builtin_amdgcn_readfirstlane(n_entries > wave ? (n_entries - wave + TNW - 1) / TNW : 0);
        auto entry = [&](int q) -> int { return lst[(uint32_t)(TNW * q)]; };
        // Two records in flight, in two registers that alternate (the loop
        // takes two entries per trip): a register is reloaded only after its
        // record has been taken, so taking one waits for that load alone.
        // Past the last entry the last record is loaded again (unused), so
        // the loads need no branches.
        if (nq > 0) {
            int e0 = entry(0), e1 = entry(min(1, nq - 1));
            unsigned long long z0 = block_rec(e0), z1 = block_rec(e1);
            for (int q = 0; q < nq; q += 2) {
                const int ec0 = e0;
                const unsigned long long zc0 = z0;
                e0 = entry(min(q + 2, nq - 1));
                z0 = block_rec(e0);
                splat_entry(ec0, zc0);
                if (q + 1 >= nq) break;
                const int ec1 = e1;
                const unsigned long long zc1 = z1;
                e1 = entry(min(q + 3, nq - 1));
                z1 = block_rec(e1);
                splat_entry(ec1, zc1);
            }
        }
    } else {
        // more entries than the list holds: test every block's tile range
        for (int e = wave; e < fvv_nsrc(vd) * vd.blk_stride; e += TNW) {
            const int k = e / vd.blk_stride, blk = e - k * vd.blk_stride;
            if (blk >= vd.src[k].nblk) continue;
            const int4 r = vd.bbox[e];
            if (!(r.x <= tx && tx <= r.y && r.z <= ty && ty <= r.w)) continue;
            const int ent = (k << 24) | blk;
            splat_entry(ent, block_rec(ent));
        }
    }
    __syncthreads();

    // ---- S2: 3x3 filter of four horizontally adjacent pixels per thread.
    // Most pixels keep their key (fewer than five valid neighbours, or a
    // neighbour within tau); only the rest need the lower median, whose
    // sorting network a wave would otherwise run whenever one of its lanes
    // needs it.  Those pixels are listed and the list is spread over every
    // thread of the tile.
    const int ly = t / TPR, lx0 = (t % TPR) * 4;
    const int y = Y0 + ly;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x = X0 + lx0 + q;
        unsigned long long kf = FVV_KEY_EMPTY;
        bool need = false;
        if (x < W && y < H) {
            const unsigned long long *w3 = zk + ly * WN + lx0 + q;
            const unsigned long long c = w3[WN + 1];
            unsigned long long nb[8] = {w3[0], w3[1], w3[2], w3[WN], w3[WN + 2], w3[2 * WN], w3[2 * WN + 1],
                                        w3[2 * WN + 2]};
            if (LAYERED) {
                kf = filter_key(c, nb, vd.tau);
            } else {
                kf = c;
                need = filter_needs_median(c, nb, vd.tau);
            }
        }
        s_kf[ly * T + lx0 + q] = kf;
        const unsigned long long m = __ballot(need);
        if (m) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&s_nmed, __popcll(m));
            base = __builtin_amdgcn_readfirstlane(base);   // every lane is active here: lane 0's value
            const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
            if (need) s_med[base + rank] = (uint16_t)(ly * T + lx0 + q);
        }
    }
    __syncthreads();
    for (int e = t; e < s_nmed; e += TNT) {
        const int pix = s_med[e];
        const unsigned long long *w3 = zk + (pix / T) * WN + (pix % T);
        unsigned long long nb[8] = {w3[0], w3[1], w3[2], w3[WN], w3[WN + 2], w3[2 * WN], w3[2 * WN + 1],
                                    w3[2 * WN + 2]};
        s_kf[pix] = lower_median8(nb, valid_count(nb));
    }
    __syncthreads();
    unsigned long long kfs[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) kfs[q] = s_kf[ly * T + lx0 + q];
    __syncthreads();   // the key buffer becomes the slot and colour buffers

    // ---- S3: backward fetch and blend
    uint32_t pslot[4], prgb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x = X0 + lx0 + q;
        pslot[q] = FVV_HOLE;
        prgb[q] = 0;
        const unsigned long long kf = kfs[q];
        float ch[STACK ? 16 : 1];   // the learned-path stack channels of the pixel
#pragma unroll
        for (int c = 0; c < (STACK ? 16 : 1); ++c) ch[c] = 0.f;
        if (x < W && y < H) {
            if (kf != FVV_KEY_EMPTY) {
                const float zf = u2f((uint32_t)(kf >> 32));
                uint32_t col;
                if (blend_pixel<STACK>(vd, 0, x, y, zf, col, ch)) {
                    pslot[q] = f2u(zf);
                    prgb[q] = col;
                }
            }
            const int64_t o = (int64_t)y * W + x;
            if (LAYERED) {
                // the background layer shows wherever the foreground layer
                // has no colour (the foreground is stacked over it)
                const bool tap = vd.dbg_bz != nullptr;
                if ((pslot[q] & FVV_HOLE) || tap) {
                    const unsigned long long *zb = zk + WN * WN + ly * WN + lx0 + q;
                    const unsigned long long cb = zb[WN + 1];
                    unsigned long long nbb[8] = {zb[0], zb[1], zb[2], zb[WN], zb[WN + 2], zb[2 * WN], zb[2 * WN + 1],
                                                 zb[2 * WN + 2]};
                    const unsigned long long kb = filter_key(cb, nbb, vd.tau);
                    if ((pslot[q] & FVV_HOLE) && kb != FVV_KEY_EMPTY) {
                        const float zf = u2f((uint32_t)(kb >> 32));
                        uint32_t col;
                        if (blend_pixel<false>(vd, vd.K, x, y, zf, col)) {
                            pslot[q] = f2u(zf);
                            prgb[q] = col;
                        }
                    }
                    if (tap) {
                        vd.dbg_bz[o] = cb;
                        vd.dbg_bzf[o] = kb;
                    }
                }
            }
            if (vd.dbg_z) vd.dbg_z[o] = zk[(ly + 1) * WN + lx0 + q + 1];
            if (vd.dbg_zf) vd.dbg_zf[o] = kf;
            if (vd.dbg_rgba) vd.dbg_rgba[o] = prgb[q];
            if (vd.dbg_depth) vd.dbg_depth[o] = (pslot[q] & FVV_HOLE) ? 0.0f : u2f(pslot[q]);
        }
        if (STACK && vd.stack && x < vd.stack_w && y < vd.stack_h) store_stack(vd, x, y, ch);
    }
    bool any_hole = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        s_slot[ly * T + lx0 + q] = pslot[q];
        s_rgb[ly * T + lx0 + q] = prgb[q];
        any_hole |= (pslot[q] & FVV_HOLE) && lx0 + q < tw && ly < th;
    }
    if (any_hole) s_hole = 1;
    __syncthreads();

    // ---- S4 (local): holes whose nearest covered pixel in every direction
    // lies inside the tile (or beyond the image edge) are filled here; the
    // others are marked open for the second pass.
    const bool fill = vd.fill_mode == 0;
    // nearest covered pixel inside the tile in each direction for every
    // pixel (tile-local column for left / right, row for up / down; -1 =
    // none): one scan per row and column, in the z-buffer's LDS, which is
    // dead by now; only tiles with holes
    int8_t *s_in = (int8_t *)zk;
    static_assert(4 * T * T <= WN * WN * 8, "the scan arrays fit the key window");
    if (fill && s_hole) {
        if (t < 4 * T) {
            const int d = t / T, q = t - d * T;
            int last = -1;
            if (d == 0 && q < th) {
                for (int lx = 0; lx < tw; ++lx) {
                    s_in[q * T + lx] = (int8_t)last;
                    if (!(s_slot[q * T + lx] & FVV_HOLE)) last = lx;
                }
            } else if (d == 1 && q < th) {
                for (int lx = tw - 1; lx >= 0; --lx) {
                    s_in[T * T + q * T + lx] = (int8_t)last;
                    if (!(s_slot[q * T + lx] & FVV_HOLE)) last = lx;
                }
            } else if (d == 2 && q < tw) {
                for (int ly2 = 0; ly2 < th; ++ly2) {
                    s_in[2 * T * T + ly2 * T + q] = (int8_t)last;
                    if (!(s_slot[ly2 * T + q] & FVV_HOLE)) last = ly2;
                }
            } else if (d == 3 && q < tw) {
                for (int ly2 = th - 1; ly2 >= 0; --ly2) {
                    s_in[3 * T * T + ly2 * T + q] = (int8_t)last;
                    if (!(s_slot[ly2 * T + q] & FVV_HOLE)) last = ly2;
                }
            }
        }
        __syncthreads();
    }
    uint32_t osl[4], ocol[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int lx = lx0 + q;
        osl[q] = FVV_HOLE;
        ocol[q] = 0;
        if (lx >= tw || ly >= th) continue;
        uint32_t sl = pslot[q], col = prgb[q];
        if (sl & FVV_HOLE) {
            col = 0;
            sl = FVV_HOLE;
            if (fill) {
                Cand b{0.f, 0, -1};
                const int e = ly * T + lx;
                const int xl = s_in[e], xr = s_in[T * T + e], yu = s_in[2 * T * T + e], yd = s_in[3 * T * T + e];
                // open: some direction has no covered pixel inside the tile
                // and the tile does not end at the image edge there
                const bool open = (xl < 0 && X0 > 0) || (xr < 0 && X0 + tw < W) || (yu < 0 && Y0 > 0) ||
                                  (yd < 0 && Y0 + th < H);
                if (!open) {
                    if (xl >= 0) offer(b, u2f(s_slot[ly * T + xl]), lx - xl, ly * T + xl);
                    if (xr >= 0) offer(b, u2f(s_slot[ly * T + xr]), xr - lx, ly * T + xr);
                    if (yu >= 0) offer(b, u2f(s_slot[yu * T + lx]), ly - yu, yu * T + lx);
                    if (yd >= 0) offer(b, u2f(s_slot[yd * T + lx]), yd - ly, yd * T + lx);
                }
                if (open) {
                    sl = FVV_HOLE_OPEN;
                    s_open = 1;
                } else if (b.idx >= 0) {
                    col = s_rgb[b.idx];
                }
            }
        }
        osl[q] = sl;
        ocol[q] = col;
    }
    // the thread's four pixels are adjacent: one 16-byte slot store and
    // three 4-byte colour stores where alignment allows, else per pixel
    if (ly < th) {
        const int x = X0 + lx0;
        const int64_t so = (int64_t)y * W + x;
        uint8_t *po = vd.out + (int64_t)y * vd.out_pitch + (int64_t)x * 3;
        if (lx0 + 3 < tw && (so & 3) == 0 && ((uintptr_t)po & 3) == 0) {
            *(uint4 *)(vd.slot + so) = make_uint4(osl[0], osl[1], osl[2], osl[3]);
            uint32_t *pw = (uint32_t *)po;
            pw[0] = (ocol[0] & 0xFFFFFFu) | (ocol[1] << 24);
            pw[1] = ((ocol[1] >> 8) & 0xFFFFu) | (ocol[2] << 16);
            pw[2] = ((ocol[2] >> 16) & 0xFFu) | ((ocol[3] & 0xFFFFFFu) << 8);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (lx0 + q >= tw) continue;
                vd.slot[so + q] = osl[q];
                put_rgb(vd.out, vd.out_pitch, x + q, y, ocol[q]);
            }
        }
    }

    // ---- per-tile row / column summaries of covered pixels for the open pass
    // (a tile without holes is covered edge to edge)
    const bool holes = s_hole != 0;
    if (t < T) {
        int first = -1, last = -1;
        if (t < th && !holes) {
            first = X0;
            last = X0 + tw - 1;
        } else if (t < th)
            for (int c = 0; c < tw; ++c)
                if (!(s_slot[t * T + c] & FVV_HOLE)) {
                    if (first < 0) first = X0 + c;
                    last = X0 + c;
                }
        vd.rowsum[(int64_t)tile * T + t] = make_int2(first, last);
    } else if (t < 2 * T) {
        const int c = t - T;
        int first = -1, last = -1;
        if (c < tw && !holes) {
            first = Y0;
            last = Y0 + th - 1;
        } else if (c < tw)
            for (int r = 0; r < th; ++r)
                if (!(s_slot[r * T + c] & FVV_HOLE)) {
                    if (first < 0) first = Y0 + r;
                    last = Y0 + r;
                }
        vd.colsum[(int64_t)tile * T + c] = make_int2(first, last);
    }
    __syncthreads();
    if (t == 0) {
        if (vd.dbg_tiles) vd.dbg_tiles[tile] = make_int2(n_entries, vd.tile_cap);
        vd.counts[tile] = 0;   // ready for the next call
        if (s_open > 0) vd.open_list[atomicAdd(vd.open_count, 1)] = make_int2(vd.view, tile);
    }
}

// The plain kernel is held to 64 VGPRs (8 waves per SIMD; it uses 52), so
// the waves of eight workgroups share each SIMD; the stack variant keeps
// its registers.
__global__ void __launch_bounds__(TNT) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_tile_plain(const fvv_view_desc *__restrict__ views, int mtx, int mty, int n_views)
{
    tile_body<false, false>(views, mtx, mty, n_views);
}

__global__ void __launch_bounds__(TNT) k_tile_stack(const fvv_view_desc *__restrict__ views, int mtx, int mty,
                                                    int n_views)
{
    tile_body<true, false>(views, mtx, mty, n_views);
}

// Layered synthesis (Section VI): foreground and background layers splatted
// into their own LDS z-buffers, each filtered and mixed over its own source
// slots, the foreground stacked over the background.  Plain views of a batch
// that also holds layered views run here too (their second window stays
// empty), and a batch that also holds learned views takes the variant that
// writes their stacks.  The two windows bound occupancy to 5 workgroups per
// CU through LDS, so registers are not capped.
__global__ void __launch_bounds__(TNT) k_tile_layered(const fvv_view_desc *__restrict__ views, int mtx, int mty, int n_views)
{
    tile_body<false, true>(views, mtx, mty, n_views);
}

__global__ void __launch_bounds__(TNT) k_tile_stack_layered(const fvv_view_desc *__restrict__ views, int mtx,
                                                            int mty, int n_views)
{
    tile_body<true, true>(views, mtx, mty, n_views);
}

// ---------------------------------------------------------------- open holes
// Holes whose nearest covered neighbour in some direction lies outside their
// tile: scan the tile, then walk the per-tile summaries of the row or column.
// A fixed grid walks the batch's list of tiles with open holes.
// threads per open tile: one per row and direction of the walks and scans
// (4 x 32), every thread busy in those serial phases; twice the tiles in
// flight of a 256-thread block
constexpr int FILL_NT = 4 * T;
__global__ void __launch_bounds__(FILL_NT) k_fill_open(const fvv_view_desc *__restrict__ views)
{
    // The tile's slots are staged in LDS (the scans inside the tile then
    // cost no dependent global loads), and the walks beyond the tile, which
    // every hole of a tile row (or column) would repeat, are done once per
    // row and direction: s_ox[d][q] = the nearest covered image coordinate
    // outside the tile (x for left / right of row q, y for up / down of
    // column q; -1 = none) and s_oz[d][q] its depth bits.
    __shared__ uint32_t s_slot[T * T];
    __shared__ int s_ox[4][T];
    __shared__ uint32_t s_oz[4][T];
    // nearest covered pixel inside the tile in each direction (tile-local
    // column for left / right, row for up / down; -1 = none), one scan per
    // row or column instead of one per hole
    __shared__ int8_t s_in[4][T * T];
    const int n_open = *views[0].open_count;
    for (int item = blockIdx.x; item < n_open; item += gridDim.x) {
        const int2 vt = views[0].open_list[item];
        const fvv_view_desc &vd = views[vt.x];
        const int tile = vt.y;
        const int ty = tile / vd.ntx, tx = tile - ty * vd.ntx;
        const int W = vd.W;
        const int X0 = tx * T, Y0 = ty * T;
        const int tw = min(T, W - X0), th = min(T, vd.H - Y0);
        const uint32_t *slot = vd.slot;
        __syncthreads();   // the previous item's readers are done
        for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
            const int ly = e / T, lx = e - ly * T;
            s_slot[e] = (lx < tw && ly < th) ? slot[(int64_t)(Y0 + ly) * W + X0 + lx] : FVV_HOLE;
        }
        if (threadIdx.x < 4 * T) {
            const int d = threadIdx.x / T, q = threadIdx.x - d * T;
            int pos = -1;
            if (d < 2 && q < th) {
                const int y = Y0 + q;
                if (d == 0) {
                    for (int t2 = tx - 1; t2 >= 0 && pos < 0; --t2) pos = vd.rowsum[(int64_t)(ty * vd.ntx + t2) * T + q].y;
                } else {
                    for (int t2 = tx + 1; t2 < vd.ntx && pos < 0; ++t2)
                        pos = vd.rowsum[(int64_t)(ty * vd.ntx + t2) * T + q].x;
                }
                s_oz[d][q] = pos >= 0 ? slot[(int64_t)y * W + pos] : 0u;
            } else if (d >= 2 && q < tw) {
                const int x = X0 + q;
                if (d == 2) {
                    for (int t2 = ty - 1; t2 >= 0 && pos < 0; --t2) pos = vd.colsum[(int64_t)(t2 * vd.ntx + tx) * T + q].y;
                } else {
                    for (int t2 = ty + 1; t2 < vd.nty && pos < 0; ++t2)
                        pos = vd.colsum[(int64_t)(t2 * vd.ntx + tx) * T + q].x;
                }
                s_oz[d][q] = pos >= 0 ? slot[(int64_t)pos * W + x] : 0u;
            }
            s_ox[d][q] = pos;
        }
        __syncthreads();
        if (threadIdx.x < 4 * T) {
            const int d = threadIdx.x / T, q = threadIdx.x - d * T;
            int last = -1;
            if (d == 0 && q < th) {
                for (int lx = 0; lx < tw; ++lx) {
                    s_in[0][q * T + lx] = (int8_t)last;
                    if (!(s_slot[q * T + lx] & FVV_HOLE)) last = lx;
                }
            } else if (d == 1 && q < th) {
                for (int lx = tw - 1; lx >= 0; --lx) {
                    s_in[1][q * T + lx] = (int8_t)last;
                    if (!(s_slot[q * T + lx] & FVV_HOLE)) last = lx;
                }
            } else if (d == 2 && q < tw) {
                for (int ly = 0; ly < th; ++ly) {
                    s_in[2][ly * T + q] = (int8_t)last;
                    if (!(s_slot[ly * T + q] & FVV_HOLE)) last = ly;
                }
            } else if (d == 3 && q < tw) {
                for (int ly = th - 1; ly >= 0; --ly) {
                    s_in[3][ly * T + q] = (int8_t)last;
                    if (!(s_slot[ly * T + q] & FVV_HOLE)) last = ly;
                }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
            const int ly = e / T, lx = e - ly * T;
            if (lx >= tw || ly >= th || s_slot[e] != FVV_HOLE_OPEN) continue;
            const int x = X0 + lx, y = Y0 + ly;
            // candidates carry image indices y*W + x; depths from the slots
            Cand c{0.f, 0, -1};
            // left
            const int l = s_in[0][e];
            if (l >= 0) offer(c, u2f(s_slot[ly * T + l]), lx - l, y * W + X0 + l);
            else if (s_ox[0][ly] >= 0) offer(c, u2f(s_oz[0][ly]), x - s_ox[0][ly], y * W + s_ox[0][ly]);
            // right
            const int r = s_in[1][e];
            if (r >= 0) offer(c, u2f(s_slot[ly * T + r]), r - lx, y * W + X0 + r);
            else if (s_ox[1][ly] >= 0) offer(c, u2f(s_oz[1][ly]), s_ox[1][ly] - x, y * W + s_ox[1][ly]);
            // up
            const int u = s_in[2][e];
            if (u >= 0) offer(c, u2f(s_slot[u * T + lx]), ly - u, (Y0 + u) * W + x);
            else if (s_ox[2][lx] >= 0) offer(c, u2f(s_oz[2][lx]), y - s_ox[2][lx], s_ox[2][lx] * W + x);
            // down
            const int d = s_in[3][e];
            if (d >= 0) offer(c, u2f(s_slot[d * T + lx]), d - ly, (Y0 + d) * W + x);
            else if (s_ox[3][lx] >= 0) offer(c, u2f(s_oz[3][lx]), s_ox[3][lx] - y, s_ox[3][lx] * W + x);
            uint32_t col = 0;
            if (c.idx >= 0) {
                const int cy = c.idx / W, cx = c.idx - cy * W;
                col = get_rgb(vd.out, vd.out_pitch, cx, cy);
            }
            put_rgb(vd.out, vd.out_pitch, x, y, col);
        }
    }
}

}  // namespace

hipError_t fvv_launch_repack(const fvv_repack_batch &b, int max_w, int max_h, hipStream_t s, fvv_prof *prof)
{
    if (b.n <= 0) return hipSuccess;
    dim3 grid((max_w + 255) / 256, max_h, b.n);
    hipEvent_t e0;
    fvv_prof_begin(prof, s, e0);
    hipLaunchKernelGGL(k_repack, grid, dim3(256), 0, s, b);
    fvv_prof_end(prof, s, FVV_ST_REPACK, e0);
    return hipGetLastError();
}

namespace {

// binning, tile kernel and open-hole pass over the descriptors at d_views
hipError_t launch_stages(fvv_view_desc *d_views, const fvv_batch_dims &b, hipStream_t s, fvv_prof *prof)
{
    hipEvent_t e0;
    fvv_prof_begin(prof, s, e0);
    const int bin_waves = (b.max_blocks + FVV_BIN_BPW - 1) / FVV_BIN_BPW;
    hipLaunchKernelGGL(k_bin, dim3((bin_waves + 3) / 4, b.max_k, b.n_views), dim3(256), 0, s, d_views);
    fvv_prof_end(prof, s, FVV_ST_BIN, e0);
    fvv_prof_begin(prof, s, e0);
    {
        // 1-D dispatch of every (view, tile), rounded up to whole XCD rounds
        const int total = b.max_tiles_x * b.max_tiles_y * b.n_views;
        const dim3 grid((total + FVV_XCDS - 1) / FVV_XCDS * FVV_XCDS);
        if (b.any_layered && b.any_stack)
            hipLaunchKernelGGL(k_tile_stack_layered, grid, dim3(TNT), 0, s, d_views, b.max_tiles_x, b.max_tiles_y,
                               b.n_views);
        else if (b.any_layered)
            hipLaunchKernelGGL(k_tile_layered, grid, dim3(TNT), 0, s, d_views, b.max_tiles_x, b.max_tiles_y,
                               b.n_views);
        else if (b.any_stack)
            hipLaunchKernelGGL(k_tile_stack, grid, dim3(TNT), 0, s, d_views, b.max_tiles_x, b.max_tiles_y, b.n_views);
        else
            hipLaunchKernelGGL(k_tile_plain, grid, dim3(TNT), 0, s, d_views, b.max_tiles_x, b.max_tiles_y, b.n_views);
    }
    fvv_prof_end(prof, s, FVV_ST_TILE, e0);
    if (b.fill_bg) {
        fvv_prof_begin(prof, s, e0);
        const int grid = std::max(1, std::min(b.total_tiles, 2048 * 256 / FILL_NT));
        hipLaunchKernelGGL(k_fill_open, dim3(grid), dim3(FILL_NT), 0, s, d_views);
        fvv_prof_end(prof, s, FVV_ST_FILL_OPEN, e0);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t fvv_launch_synthesis(const fvv_view_desc *h_views, fvv_view_desc *d_views, const fvv_batch_dims &b,
                                size_t extra_bytes, hipStream_t s, fvv_prof *prof)
{
    if (b.n_views <= 0) return hipSuccess;
    static_assert(sizeof(fvv_view_desc) % 16 == 0, "descriptors are copied in 16-byte words");
    if (extra_bytes % 16) return hipErrorInvalidValue;
    const int words = (int)((b.n_views * sizeof(fvv_view_desc) + extra_bytes) / 16);
    hipEvent_t e0;
    fvv_prof_begin(prof, s, e0);
    hipLaunchKernelGGL(k_desc, dim3((words + 255) / 256), dim3(256), 0, s, (const uint4 *)h_views, (uint4 *)d_views,
                       words);
    fvv_prof_end(prof, s, FVV_ST_DESC, e0);
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_stages(d_views, b, s, prof);
}

namespace {

// Every significand m of b = 2^e (1 + m 2^-23), e_lo <= e <= e_hi: rcp_rn(b)
// against the correctly rounded 1/b, and the quotients div_by(a, b, rcp_rn(b))
// of two dividends per b against the correctly rounded a / b.
__global__ void __launch_bounds__(256) k_check_rcp(int e_lo, int n_exp, unsigned long long *bad)
{
    const uint32_t n = (uint32_t)n_exp << 23;
    uint32_t miss = 0;
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        const uint32_t m = i & 0x7FFFFFu;
        const int e = e_lo + (int)(i >> 23);
        const float b = u2f(((uint32_t)(127 + e) << 23) | m);
        const float y = rcp_rn(b);
        miss += f2u(y) != f2u(__fdiv_rn(1.0f, b));
        // dividends of both signs, image-coordinate-like magnitudes
        const float a0 = u2f(((uint32_t)(118 + (m * 2654435761u >> 27) % 24u) << 23) | ((m * 40503u) & 0x7FFFFFu));
        const float a1 = -u2f(((uint32_t)(118 + (m * 2246822519u >> 27) % 24u) << 23) | ((m * 69069u) & 0x7FFFFFu));
        miss += f2u(div_by(a0, b, y)) != f2u(__fdiv_rn(a0, b));
        miss += f2u(div_by(a1, b, y)) != f2u(__fdiv_rn(a1, b));
    }
    if (miss) atomicAdd(bad, (unsigned long long)miss);
}

}  // namespace

hipError_t fvv_check_reciprocal_impl(int e_lo, int e_hi, unsigned long long *bad_dev, hipStream_t s)
{
    if (e_lo < -125 || e_hi > 125 || e_lo > e_hi) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_check_rcp, dim3(4096), dim3(256), 0, s, e_lo, e_hi - e_lo + 1, bad_dev);
    return hipGetLastError();
}

hipError_t fvv_launch_synthesis_one(const fvv_view_desc &view, fvv_view_desc *d_view, int32_t *counts,
                                    const fvv_batch_dims &b, hipStream_t s, fvv_prof *prof)
{
    if (b.n_views != 1) return hipErrorInvalidValue;
    hipEvent_t e0;
    fvv_prof_begin(prof, s, e0);
    const int grid = std::max(1, std::min(64, (b.total_tiles + 255) / 256));
    hipLaunchKernelGGL(k_desc_one, dim3(grid), dim3(256), 0, s, view, d_view, counts, b.total_tiles);
    fvv_prof_end(prof, s, FVV_ST_DESC, e0);
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_stages(d_view, b, s, prof);
}
