// fvv_kernels.hip -- gfx950 kernels of the DIBR view-synthesis path.
//
// Stages (FVV Live, arXiv 2007.00558, Section VI):
//   repack     MVD ingest: RGB8 -> 8-byte texels {RGBA8, depth}, millimetres ->
//              metres with the Eq. (1) correction (Section IV-A); per frame set
//   bin_count  every 16x16 block of each selected source camera is projected
//              (3D warping of its valid pixels) and the output tiles its
//              footprints touch are counted
//   bin_scan   per-tile list offsets
//   bin_fill   per-tile lists of source blocks
//   tile       one workgroup per 32x32 output tile: splats its binned blocks
//              into an LDS z-buffer of packed (depth, camera, pixel) keys with
//              64-bit LDS atomicMin, 3x3 crack/speckle filter in LDS, backward
//              depth-consistent bilinear fetch from each selected camera mixed
//              by camera distance, hole fill for holes whose neighbours lie
//              inside the tile, writes the RGB8 output
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

namespace {

constexpr int T = FVV_TILE;
constexpr int WN = FVV_TILE + 2;   // tile window edge with a 1-pixel halo

__device__ __forceinline__ uint32_t f2u(float f) { return __float_as_uint(f); }
__device__ __forceinline__ float u2f(uint32_t u) { return __uint_as_float(u); }

// p_r = ((M_r0 i + M_r1 j) + M_r2) z + m_r, each op rounded to float32
__device__ __forceinline__ void project(const float *M, const float *m, float i, float j, float z,
                                        float &p0, float &p1, float &p2)
{
    p0 = __fadd_rn(__fmul_rn(__fadd_rn(__fadd_rn(__fmul_rn(M[0], i), __fmul_rn(M[1], j)), M[2]), z), m[0]);
    p1 = __fadd_rn(__fmul_rn(__fadd_rn(__fadd_rn(__fmul_rn(M[3], i), __fmul_rn(M[4], j)), M[5]), z), m[1]);
    p2 = __fadd_rn(__fmul_rn(__fadd_rn(__fadd_rn(__fmul_rn(M[6], i), __fmul_rn(M[7], j)), M[8]), z), m[2]);
}

struct Footprint {
    int x0, x1, y0, y1;
    unsigned long long key;
};

// Forward warp of source pixel (i, j) at depth z: the output pixel centres
// x with u - mx/2 <= x < u + mx/2 (rows likewise), mx = clamp(sx z / p2, 1,
// max_fp), clipped to the output image; key = depth bits | camera | pixel.
__device__ __forceinline__ bool splat_point(const fvv_src_desc &s, int W, int H, float max_fp, int i, int j,
                                            float z, Footprint &f)
{
    float q0, q1, q2;
    project(s.A, s.a, (float)i, (float)j, z, q0, q1, q2);
    if (!(q2 > FVV_ZCLIP)) return false;
    const float u = __fdiv_rn(q0, q2), v = __fdiv_rn(q1, q2);
    if (!isfinite(u) || !isfinite(v)) return false;
    float mx = __fdiv_rn(__fmul_rn(s.sx, z), q2);
    float my = __fdiv_rn(__fmul_rn(s.sy, z), q2);
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
            (unsigned long long)((int64_t)j * s.W + i);
    return true;
}

// ---------------------------------------------------------------- repack
// One launch per frame set: grid.z = camera.
__global__ void __launch_bounds__(256) k_repack(const fvv_repack_batch b)
{
    const fvv_repack_cam &c = b.cam[blockIdx.z];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= c.W || y >= c.H) return;
    const uint8_t *p = c.rgb + (int64_t)y * c.rgb_pitch + (int64_t)x * 3;
    const uint32_t col = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | 0xFF000000u;
    const uint16_t d = *(const uint16_t *)(c.depth + (int64_t)y * c.depth_pitch + (int64_t)x * 2);
    uint32_t zb = FVV_NO_DEPTH;
    if (d != 0) {
        const float z = __fdiv_rn((float)d, 1000.0f);
        const float s = __fadd_rn(__fmul_rn(c.alpha, z), c.beta);   // Eq. (1): (alpha z + beta) z
        zb = f2u(__fmul_rn(s, z));
    }
    c.texel_out[(int64_t)y * c.W + x] = make_uint2(col, zb);
    c.depth_out[(int64_t)y * c.W + x] = u2f(zb);
}

// ---------------------------------------------------------------- binning
__device__ __forceinline__ int wave_min(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// One wave per (view, camera slot, 8x8 source block), four blocks per
// workgroup: exact bounding box of the block's footprints, turned into the
// range of output tiles whose window (tile plus 1-pixel halo) it touches;
// each such tile is counted.
__global__ void __launch_bounds__(256) k_bin_count(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.z];
    const int k = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int blk = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= vd.K) return;
    const fvv_src_desc &s = vd.src[k];
    if (blk >= s.nblk) return;
    const int by = blk / s.nbx, bx = blk - by * s.nbx;
    const int i = bx * FVV_SBLK + (lane & (FVV_SBLK - 1));
    const int j = by * FVV_SBLK + (lane / FVV_SBLK);
    int x0 = INT_MAX, x1 = -1, y0 = INT_MAX, y1 = -1;
    if (i < s.W && j < s.H) {
        const uint32_t zb = f2u(s.depth[(int64_t)j * s.W + i]);
        Footprint f;
        if (zb != FVV_NO_DEPTH && splat_point(s, vd.W, vd.H, vd.max_fp, i, j, u2f(zb), f)) {
            x0 = f.x0;
            x1 = f.x1;
            y0 = f.y0;
            y1 = f.y1;
        }
    }
    // every lane ends with the block's bounds
    x0 = wave_min(x0);
    y0 = wave_min(y0);
    x1 = wave_max(x1);
    y1 = wave_max(y1);
    int4 t = make_int4(1, 0, 1, 0);   // empty
    if (x1 >= 0) {
        t.x = max(0, (x0 + T - 1) / T - 1);
        t.y = min(vd.ntx - 1, (x1 + 1) / T);
        t.z = max(0, (y0 + T - 1) / T - 1);
        t.w = min(vd.nty - 1, (y1 + 1) / T);
    }
    if (lane == 0) vd.bbox[(int64_t)k * vd.blk_stride + blk] = t;
    if (t.x > t.y) return;
    const int nx = t.y - t.x + 1, n = nx * (t.w - t.z + 1);
    for (int e = lane; e < n; e += 64) {
        const int ty = t.z + e / nx, tx = t.x + e % nx;
        atomicAdd(&vd.counts[ty * vd.ntx + tx], 1);
    }
}

// One workgroup per view: exclusive scan of the tile counts into list
// offsets (and fill cursors); counters are cleared for the next call.
__global__ void __launch_bounds__(256) k_bin_scan(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.x];
    const int n = vd.ntx * vd.nty;
    const int t = threadIdx.x;
    const int C = (n + 255) / 256;
    const int e0 = min(t * C, n), e1 = min(e0 + C, n);
    int sum = 0;
    for (int e = e0; e < e1; ++e) sum += vd.counts[e];
    __shared__ int sc[256];
    sc[t] = sum;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int a = t >= d ? sc[t - d] : 0;
        __syncthreads();
        sc[t] += a;
        __syncthreads();
    }
    int run = sc[t] - sum;
    for (int e = e0; e < e1; ++e) {
        const int c = vd.counts[e];
        vd.offs[e] = run;
        vd.cursor[e] = run;
        vd.counts[e] = 0;
        run += c;
    }
    if (t == 255) *vd.overflow = sc[255] > vd.list_cap ? 1 : 0;
}

// One thread per (view, camera slot, source block): append the block to the
// list of every tile in its range.
__global__ void __launch_bounds__(256) k_bin_fill(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.z];
    const int k = blockIdx.y;
    const int blk = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= vd.K || blk >= vd.src[k].nblk) return;
    if (*vd.overflow) return;
    const int4 t = vd.bbox[(int64_t)k * vd.blk_stride + blk];
    for (int ty = t.z; ty <= t.w; ++ty)
        for (int tx = t.x; tx <= t.y; ++tx) {
            const int pos = atomicAdd(&vd.cursor[ty * vd.ntx + tx], 1);
            vd.list[pos] = (k << 24) | blk;
        }
}

// ---------------------------------------------------------------- filter
// Lower median (element (n-1)/2 in key order) of the valid keys among the 8
// neighbours; empty keys (all ones) order last, so a rank selection over all
// eight picks it directly.
__device__ __forceinline__ unsigned long long lower_median8(const unsigned long long v[8], int n)
{
    const int m = (n - 1) >> 1;
    unsigned long long res = FVV_KEY_EMPTY;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        int r = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) r += (v[b] < v[a]) || (v[b] == v[a] && b < a);
        if (r == m) res = v[a];
    }
    return res;
}

// Crack fill (empty key, >= 5 valid neighbours) and speckle removal (valid
// key, >= 5 valid neighbours, none within tau z0) take the lower median.
__device__ __forceinline__ unsigned long long filter_key(unsigned long long c, const unsigned long long v[8],
                                                         float tau)
{
    int n = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) n += v[e] != FVV_KEY_EMPTY;
    if (n < 5) return c;
    if (c != FVV_KEY_EMPTY) {
        const float z0 = u2f((uint32_t)(c >> 32));
        const float lim = __fmul_rn(tau, z0);
        bool near = false;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (v[e] != FVV_KEY_EMPTY && fabsf(__fsub_rn(u2f((uint32_t)(v[e] >> 32)), z0)) <= lim) near = true;
        if (near) return c;
    }
    return lower_median8(v, n);
}

// ---------------------------------------------------------------- blend
// Backward warp of output pixel (x, y) at depth zf into every selected
// camera; taps whose source depth agrees with the warped depth within tau
// are mixed bilinearly, cameras by their distance weights.  Returns true and
// the RGBA8 colour if any camera contributes.
__device__ __forceinline__ bool blend_pixel(const fvv_view_desc &vd, int x, int y, float zf, uint32_t &rgba)
{
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, wsum = 0.f;
    for (int k = 0; k < vd.K; ++k) {
        const fvv_src_desc &s = vd.src[k];
        float q0, q1, q2;
        project(s.B, s.b, (float)x, (float)y, zf, q0, q1, q2);
        if (!(q2 > FVV_ZCLIP)) continue;
        const float u = __fdiv_rn(q0, q2), v = __fdiv_rn(q1, q2);
        if (!(u >= -0.5f && u <= __fsub_rn((float)s.W, 0.5f))) continue;
        if (!(v >= -0.5f && v <= __fsub_rn((float)s.H, 0.5f))) continue;
        const float fi0 = floorf(u), fj0 = floorf(v);
        const float fu = __fsub_rn(u, fi0), fv = __fsub_rn(v, fj0);
        const int i0 = (int)fi0, j0 = (int)fj0;
        const float lim = __fmul_rn(vd.tau, q2);
        const float gu = 1.0f - fu, gv = 1.0f - fv;
        const float wt[4] = {gu * gv, fu * gv, gu * fv, fu * fv};
        float c0 = 0.f, c1 = 0.f, c2 = 0.f, csum = 0.f;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const int ti = i0 + (n & 1), tj = j0 + (n >> 1);
            if (ti < 0 || tj < 0 || ti >= s.W || tj >= s.H) continue;
            const uint2 tx = s.texel[(int64_t)tj * s.W + ti];
            if (tx.y == FVV_NO_DEPTH) continue;
            if (!(fabsf(__fsub_rn(u2f(tx.y), q2)) <= lim)) continue;
            c0 += wt[n] * (float)(tx.x & 0xFF);
            c1 += wt[n] * (float)((tx.x >> 8) & 0xFF);
            c2 += wt[n] * (float)((tx.x >> 16) & 0xFF);
            csum += wt[n];
        }
        if (!(csum > 0.f)) continue;
        const float inv = s.wgt / csum;
        acc0 += c0 * inv;
        acc1 += c1 * inv;
        acc2 += c2 * inv;
        wsum += s.wgt;
    }
    if (!(wsum > 0.f)) return false;
    const float r = fminf(floorf(acc0 / wsum + 0.5f), 255.f);
    const float g = fminf(floorf(acc1 / wsum + 0.5f), 255.f);
    const float b = fminf(floorf(acc2 / wsum + 0.5f), 255.f);
    rgba = (uint32_t)r | ((uint32_t)g << 8) | ((uint32_t)b << 16) | 0xFF000000u;
    return true;
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
__global__ void __launch_bounds__(256) k_tile(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.z];
    const int tx = blockIdx.x, ty = blockIdx.y;
    if (tx >= vd.ntx || ty >= vd.nty) return;
    const int W = vd.W, H = vd.H;
    const int tile = ty * vd.ntx + tx;
    const int X0 = tx * T, Y0 = ty * T;
    const int WX0 = X0 - 1, WY0 = Y0 - 1;
    const int tw = min(T, W - X0), th = min(T, H - Y0);
    __shared__ unsigned long long zk[WN * WN];
    __shared__ uint32_t s_slot[T * T];
    __shared__ uint32_t s_rgb[T * T];
    __shared__ int s_open;
    const int t = threadIdx.x;
    for (int e = t; e < WN * WN; e += 256) zk[e] = FVV_KEY_EMPTY;
    if (t == 0) s_open = 0;
    __syncthreads();

    // ---- S1: splat every binned source block into the window
    const bool scan_all = *vd.overflow != 0;
    const int beg = scan_all ? 0 : vd.offs[tile];
    const int end = scan_all ? vd.K * vd.blk_stride : vd.cursor[tile];
    // each wave splats its own list entries (one 8x8 source block per entry)
    const int lane = t & 63, wave = t >> 6;
    const int si = lane & (FVV_SBLK - 1), sj = lane / FVV_SBLK;
    for (int e = beg + wave; e < end; e += 4) {
        int k, blk;
        if (!scan_all) {
            const int ent = vd.list[e];
            k = ent >> 24;
            blk = ent & 0xFFFFFF;
        } else {
            k = e / vd.blk_stride;
            blk = e - k * vd.blk_stride;
            if (blk >= vd.src[k].nblk) continue;
            const int4 r = vd.bbox[e];
            if (!(r.x <= tx && tx <= r.y && r.z <= ty && ty <= r.w)) continue;
        }
        const fvv_src_desc &s = vd.src[k];
        const int by = blk / s.nbx, bx = blk - by * s.nbx;
        const int i = bx * FVV_SBLK + si, j = by * FVV_SBLK + sj;
        if (i >= s.W || j >= s.H) continue;
        const uint32_t zb = f2u(s.depth[(int64_t)j * s.W + i]);
        if (zb == FVV_NO_DEPTH) continue;
        Footprint f;
        if (!splat_point(s, W, H, vd.max_fp, i, j, u2f(zb), f)) continue;
        const int xa = max(f.x0, WX0), xb = min(f.x1, WX0 + WN - 1);
        const int ya = max(f.y0, WY0), yb = min(f.y1, WY0 + WN - 1);
        for (int y = ya; y <= yb; ++y)
            for (int x = xa; x <= xb; ++x) atomicMin(&zk[(y - WY0) * WN + (x - WX0)], f.key);
    }
    __syncthreads();

    // ---- S2 + S3: filter and blend four horizontally adjacent pixels
    const int ly = t >> 3, lx0 = (t & 7) * 4;
    const int y = Y0 + ly;
    unsigned long long w3[3][6];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) w3[r][c] = zk[(ly + r) * WN + lx0 + c];
    uint32_t pslot[4], prgb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x = X0 + lx0 + q;
        pslot[q] = FVV_HOLE;
        prgb[q] = 0;
        if (x >= W || y >= H) continue;
        const unsigned long long c = w3[1][q + 1];
        const unsigned long long nb[8] = {w3[0][q], w3[0][q + 1], w3[0][q + 2], w3[1][q],
                                          w3[1][q + 2], w3[2][q], w3[2][q + 1], w3[2][q + 2]};
        const unsigned long long kf = filter_key(c, nb, vd.tau);
        if (kf != FVV_KEY_EMPTY) {
            const float zf = u2f((uint32_t)(kf >> 32));
            uint32_t col;
            if (blend_pixel(vd, x, y, zf, col)) {
                pslot[q] = f2u(zf);
                prgb[q] = col;
            }
        }
        const int64_t o = (int64_t)y * W + x;
        if (vd.dbg_z) vd.dbg_z[o] = c;
        if (vd.dbg_zf) vd.dbg_zf[o] = kf;
        if (vd.dbg_rgba) vd.dbg_rgba[o] = prgb[q];
        if (vd.dbg_depth) vd.dbg_depth[o] = (pslot[q] & FVV_HOLE) ? 0.0f : u2f(pslot[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        s_slot[ly * T + lx0 + q] = pslot[q];
        s_rgb[ly * T + lx0 + q] = prgb[q];
    }
    __syncthreads();

    // ---- S4 (local): holes whose nearest covered pixel in every direction
    // lies inside the tile (or beyond the image edge) are filled here; the
    // others are marked open for the second pass.
    const bool fill = vd.fill_mode == 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int lx = lx0 + q;
        if (lx >= tw || ly >= th) continue;
        const int x = X0 + lx;
        uint32_t sl = pslot[q], col = prgb[q];
        if (sl & FVV_HOLE) {
            col = 0;
            if (fill) {
                Cand b{0.f, 0, -1};
                bool open = false;
                int xl = lx - 1;
                while (xl >= 0 && (s_slot[ly * T + xl] & FVV_HOLE)) --xl;
                if (xl >= 0) offer(b, u2f(s_slot[ly * T + xl]), lx - xl, ly * T + xl);
                else open = X0 > 0;
                if (!open) {
                    int xr = lx + 1;
                    while (xr < tw && (s_slot[ly * T + xr] & FVV_HOLE)) ++xr;
                    if (xr < tw) offer(b, u2f(s_slot[ly * T + xr]), xr - lx, ly * T + xr);
                    else open = X0 + tw < W;
                }
                if (!open) {
                    int yu = ly - 1;
                    while (yu >= 0 && (s_slot[yu * T + lx] & FVV_HOLE)) --yu;
                    if (yu >= 0) offer(b, u2f(s_slot[yu * T + lx]), ly - yu, yu * T + lx);
                    else open = Y0 > 0;
                }
                if (!open) {
                    int yd = ly + 1;
                    while (yd < th && (s_slot[yd * T + lx] & FVV_HOLE)) ++yd;
                    if (yd < th) offer(b, u2f(s_slot[yd * T + lx]), yd - ly, yd * T + lx);
                    else open = Y0 + th < H;
                }
                if (open) {
                    sl = FVV_HOLE_OPEN;
                    atomicAdd(&s_open, 1);
                } else {
                    sl = FVV_HOLE;
                    if (b.idx >= 0) col = s_rgb[b.idx];
                }
            } else {
                sl = FVV_HOLE;
            }
        }
        vd.slot[(int64_t)y * W + x] = sl;
        put_rgb(vd.out, vd.out_pitch, x, y, col);
    }

    // ---- per-tile row / column summaries of covered pixels for the open pass
    if (t < T) {
        int first = -1, last = -1;
        if (t < th)
            for (int c = 0; c < tw; ++c)
                if (!(s_slot[t * T + c] & FVV_HOLE)) {
                    if (first < 0) first = X0 + c;
                    last = X0 + c;
                }
        vd.rowsum[(int64_t)tile * T + t] = make_int2(first, last);
    } else if (t < 2 * T) {
        const int c = t - T;
        int first = -1, last = -1;
        if (c < tw)
            for (int r = 0; r < th; ++r)
                if (!(s_slot[r * T + c] & FVV_HOLE)) {
                    if (first < 0) first = Y0 + r;
                    last = Y0 + r;
                }
        vd.colsum[(int64_t)tile * T + c] = make_int2(first, last);
    }
    __syncthreads();
    if (t == 0) vd.open[tile] = s_open;
}

// ---------------------------------------------------------------- open holes
// Holes whose nearest covered neighbour in some direction lies outside their
// tile: scan the tile, then walk the per-tile summaries of the row or column.
__global__ void __launch_bounds__(256) k_fill_open(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.z];
    const int tx = blockIdx.x, ty = blockIdx.y;
    if (tx >= vd.ntx || ty >= vd.nty) return;
    const int tile = ty * vd.ntx + tx;
    if (vd.open[tile] == 0) return;
    const int W = vd.W, H = vd.H;
    const int X0 = tx * T, Y0 = ty * T;
    const int tw = min(T, W - X0), th = min(T, H - Y0);
    const uint32_t *slot = vd.slot;
    for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
        const int ly = e / T, lx = e - ly * T;
        if (lx >= tw || ly >= th) continue;
        const int x = X0 + lx, y = Y0 + ly;
        if (slot[(int64_t)y * W + x] != FVV_HOLE_OPEN) continue;
        const int64_t row = (int64_t)y * W;
        // left
        int xl = x - 1;
        while (xl >= X0 && (slot[row + xl] & FVV_HOLE)) --xl;
        if (xl < X0) {
            xl = -1;
            for (int t2 = tx - 1; t2 >= 0; --t2) {
                const int l = vd.rowsum[(int64_t)(ty * vd.ntx + t2) * T + ly].y;
                if (l >= 0) {
                    xl = l;
                    break;
                }
            }
        }
        // right
        int xr = x + 1;
        while (xr < X0 + tw && (slot[row + xr] & FVV_HOLE)) ++xr;
        if (xr >= X0 + tw) {
            xr = -1;
            for (int t2 = tx + 1; t2 < vd.ntx; ++t2) {
                const int f = vd.rowsum[(int64_t)(ty * vd.ntx + t2) * T + ly].x;
                if (f >= 0) {
                    xr = f;
                    break;
                }
            }
        }
        // candidates carry image indices y*W + x
        Cand c{0.f, 0, -1};
        if (xl >= 0) offer(c, u2f(slot[row + xl]), x - xl, y * W + xl);
        if (xr >= 0) offer(c, u2f(slot[row + xr]), xr - x, y * W + xr);
        // up
        int yu = y - 1;
        while (yu >= Y0 && (slot[(int64_t)yu * W + x] & FVV_HOLE)) --yu;
        if (yu < Y0) {
            yu = -1;
            for (int t2 = ty - 1; t2 >= 0; --t2) {
                const int l = vd.colsum[(int64_t)(t2 * vd.ntx + tx) * T + lx].y;
                if (l >= 0) {
                    yu = l;
                    break;
                }
            }
        }
        if (yu >= 0) offer(c, u2f(slot[(int64_t)yu * W + x]), y - yu, yu * W + x);
        // down
        int yd = y + 1;
        while (yd < Y0 + th && (slot[(int64_t)yd * W + x] & FVV_HOLE)) ++yd;
        if (yd >= Y0 + th) {
            yd = -1;
            for (int t2 = ty + 1; t2 < vd.nty; ++t2) {
                const int f = vd.colsum[(int64_t)(t2 * vd.ntx + tx) * T + lx].x;
                if (f >= 0) {
                    yd = f;
                    break;
                }
            }
        }
        if (yd >= 0) offer(c, u2f(slot[(int64_t)yd * W + x]), yd - y, yd * W + x);
        uint32_t col = 0;
        if (c.idx >= 0) {
            const int cy = c.idx / W, cx = c.idx - cy * W;
            col = get_rgb(vd.out, vd.out_pitch, cx, cy);
        }
        put_rgb(vd.out, vd.out_pitch, x, y, col);
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

hipError_t fvv_launch_synthesis(const fvv_view_desc *d_views, const fvv_batch_dims &b, hipStream_t s,
                                fvv_prof *prof)
{
    if (b.n_views <= 0) return hipSuccess;
    hipEvent_t e0;
    fvv_prof_begin(prof, s, e0);
    hipLaunchKernelGGL(k_bin_count, dim3((b.max_blocks + 3) / 4, b.max_k, b.n_views), dim3(256), 0, s, d_views);
    fvv_prof_end(prof, s, FVV_ST_BIN_COUNT, e0);
    fvv_prof_begin(prof, s, e0);
    hipLaunchKernelGGL(k_bin_scan, dim3(b.n_views), dim3(256), 0, s, d_views);
    fvv_prof_end(prof, s, FVV_ST_BIN_SCAN, e0);
    fvv_prof_begin(prof, s, e0);
    hipLaunchKernelGGL(k_bin_fill, dim3((b.max_blocks + 255) / 256, b.max_k, b.n_views), dim3(256), 0, s,
                       d_views);
    fvv_prof_end(prof, s, FVV_ST_BIN_FILL, e0);
    fvv_prof_begin(prof, s, e0);
    hipLaunchKernelGGL(k_tile, dim3(b.max_tiles_x, b.max_tiles_y, b.n_views), dim3(256), 0, s, d_views);
    fvv_prof_end(prof, s, FVV_ST_TILE, e0);
    if (b.fill_bg) {
        fvv_prof_begin(prof, s, e0);
        hipLaunchKernelGGL(k_fill_open, dim3(b.max_tiles_x, b.max_tiles_y, b.n_views), dim3(256), 0, s,
                           d_views);
        fvv_prof_end(prof, s, FVV_ST_FILL_OPEN, e0);
    }
    return hipGetLastError();
}
