// fvv_kernels.hip -- gfx950 kernels of the DIBR view-synthesis path.
//
// Stages (FVV Live, arXiv 2007.00558, Section VI):
//   repack   MVD upload: RGB8 -> RGBA8 texels, millimetres -> metres with the
//            Eq. (1) correction (Section IV-A), once per frame set
//   splat    3D warping of every valid source pixel into the virtual view,
//            z-buffered by 64-bit packed (depth, camera, pixel) keys
//   filter   3x3 crack fill / speckle removal on the key map ("image
//            filtering" that accompanies backward warping against cracks)
//   blend    backward warping into each selected camera, depth-consistent
//            bilinear fetch, mix by camera distance
//   fill     disocclusion holes take the nearest uncovered-free neighbour
//            with the largest depth (background)
//
// Arithmetic contract shared with the definition of the method: every
// decision (pixel coverage, key order, tap validity, hole) is computed in
// float32 op by op -- built with -ffp-contract=off and correctly rounded
// division -- so the key map and the hole map are bit-exact.
#include <algorithm>

#include "fvv_internal.h"

namespace {

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

// ---------------------------------------------------------------- repack
__global__ void __launch_bounds__(256) k_repack(const uint8_t *__restrict__ rgb, int64_t rgb_pitch,
                                                const uint16_t *__restrict__ depth, int64_t depth_pitch,
                                                int W, int H, float alpha, float beta,
                                                uint32_t *__restrict__ rgba_out,
                                                float *__restrict__ depth_out)
{
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    int y = blockIdx.y;
    if (x >= W || y >= H) return;
    const uint8_t *p = rgb + (int64_t)y * rgb_pitch + (int64_t)x * 3;
    uint32_t c = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | 0xFF000000u;
    uint16_t d = *(const uint16_t *)((const uint8_t *)depth + (int64_t)y * depth_pitch + (int64_t)x * 2);
    uint32_t zb = FVV_NO_DEPTH;
    if (d != 0) {
        float z = __fdiv_rn((float)d, 1000.0f);
        float s = __fadd_rn(__fmul_rn(alpha, z), beta);   // Eq. (1): (alpha z + beta) z
        zb = f2u(__fmul_rn(s, z));
    }
    rgba_out[(int64_t)y * W + x] = c;
    depth_out[(int64_t)y * W + x] = u2f(zb);
}

// ---------------------------------------------------------------- z clear
__global__ void __launch_bounds__(256) k_zclear(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.y];
    int64_t n = (int64_t)vd.W * vd.H;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        vd.Z[e] = FVV_KEY_EMPTY;
}

// ---------------------------------------------------------------- splat
// One thread per source pixel of one selected camera of one view.
__global__ void __launch_bounds__(256) k_splat(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.z];
    const int k = blockIdx.y;
    if (k >= vd.K) return;
    const fvv_src_desc &s = vd.src[k];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= s.W * s.H) return;
    const uint32_t zb = f2u(s.depth[p]);
    if (zb == FVV_NO_DEPTH) return;
    const float z = u2f(zb);
    const int j = p / s.W, i = p - j * s.W;
    float q0, q1, q2;
    project(s.A, s.a, (float)i, (float)j, z, q0, q1, q2);
    if (!(q2 > FVV_ZCLIP)) return;
    const float u = __fdiv_rn(q0, q2), v = __fdiv_rn(q1, q2);
    if (!isfinite(u) || !isfinite(v)) return;
    float mx = __fdiv_rn(__fmul_rn(s.sx, z), q2);
    float my = __fdiv_rn(__fmul_rn(s.sy, z), q2);
    mx = fminf(fmaxf(mx, 1.0f), vd.max_fp);
    my = fminf(fmaxf(my, 1.0f), vd.max_fp);
    const float hx = __fmul_rn(0.5f, mx), hy = __fmul_rn(0.5f, my);
    float x0f = ceilf(__fsub_rn(u, hx)), x1f = __fsub_rn(ceilf(__fadd_rn(u, hx)), 1.0f);
    float y0f = ceilf(__fsub_rn(v, hy)), y1f = __fsub_rn(ceilf(__fadd_rn(v, hy)), 1.0f);
    x0f = fmaxf(x0f, 0.0f);
    y0f = fmaxf(y0f, 0.0f);
    x1f = fminf(x1f, (float)(vd.W - 1));
    y1f = fminf(y1f, (float)(vd.H - 1));
    if (x0f > x1f || y0f > y1f) return;
    const unsigned long long key = ((unsigned long long)f2u(q2) << 32) |
                                   ((unsigned long long)(uint32_t)s.cam << 27) | (unsigned long long)p;
    const int x0 = (int)x0f, x1 = (int)x1f, y0 = (int)y0f, y1 = (int)y1f;
    for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x)
            atomicMin(&vd.Z[(int64_t)y * vd.W + x], key);
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
        for (int b = 0; b < 8; ++b)
            r += (v[b] < v[a]) || (v[b] == v[a] && b < a);
        if (r == m) res = v[a];
    }
    return res;
}

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
// Returns true and the RGBA8 colour if any camera contributes.
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
            const int64_t o = (int64_t)tj * s.W + ti;
            const uint32_t zs = f2u(s.depth[o]);
            if (zs == FVV_NO_DEPTH) continue;
            if (!(fabsf(__fsub_rn(u2f(zs), q2)) <= lim)) continue;
            const uint32_t t = s.rgba[o];
            c0 += wt[n] * (float)(t & 0xFF);
            c1 += wt[n] * (float)((t >> 8) & 0xFF);
            c2 += wt[n] * (float)((t >> 16) & 0xFF);
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

// 16x16 output tile per workgroup; the raw key map with a 1-pixel halo is
// staged in LDS, filtered, then each pixel is blended.
#define TB 16
__global__ void __launch_bounds__(256) k_filter_blend(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.z];
    const int W = vd.W, H = vd.H;
    const int tx0 = blockIdx.x * TB, ty0 = blockIdx.y * TB;
    if (tx0 >= W || ty0 >= H) return;
    __shared__ unsigned long long tile[TB + 2][TB + 2];
    const int tid = threadIdx.y * TB + threadIdx.x;
    for (int e = tid; e < (TB + 2) * (TB + 2); e += TB * TB) {
        const int ly = e / (TB + 2), lx = e - ly * (TB + 2);
        const int gx = tx0 + lx - 1, gy = ty0 + ly - 1;
        tile[ly][lx] = (gx >= 0 && gy >= 0 && gx < W && gy < H) ? vd.Z[(int64_t)gy * W + gx] : FVV_KEY_EMPTY;
    }
    __syncthreads();
    const int x = tx0 + threadIdx.x, y = ty0 + threadIdx.y;
    if (x >= W || y >= H) return;
    const int lx = threadIdx.x + 1, ly = threadIdx.y + 1;
    const unsigned long long nb[8] = {tile[ly - 1][lx - 1], tile[ly - 1][lx], tile[ly - 1][lx + 1],
                                      tile[ly][lx - 1],                       tile[ly][lx + 1],
                                      tile[ly + 1][lx - 1], tile[ly + 1][lx], tile[ly + 1][lx + 1]};
    const unsigned long long kf = filter_key(tile[ly][lx], nb, vd.tau);
    const int64_t o = (int64_t)y * W + x;
    if (vd.Zf) vd.Zf[o] = kf;
    uint32_t col = 0, slot = FVV_HOLE_BIT;
    if (kf != FVV_KEY_EMPTY) {
        const float zf = u2f((uint32_t)(kf >> 32));
        if (blend_pixel(vd, x, y, zf, col)) slot = f2u(zf);
    }
    vd.rgba[o] = col;
    vd.slot[o] = slot;
    if (vd.dbg_depth) vd.dbg_depth[o] = (slot & FVV_HOLE_BIT) ? 0.0f : u2f(slot);
}

// ---------------------------------------------------------------- hole fill
// Row pass: for every hole, the better of its nearest non-hole neighbours to
// the left and right (larger depth, then nearer, then left) is stored in the
// hole's slot as FVV_HOLE_BIT | (x + 1); FVV_HOLE_BIT alone = none.
__global__ void __launch_bounds__(256) k_fill_rows(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.y];
    const int y = blockIdx.x;
    const int W = vd.W;
    if (y >= vd.H) return;
    uint32_t *row = vd.slot + (int64_t)y * W;
    const int t = threadIdx.x;
    const int C = (W + 255) >> 8;
    const int x0 = min(t * C, W), x1 = min(x0 + C, W);
    int last = -1, first = W;
    for (int x = x0; x < x1; ++x)
        if (!(row[x] & FVV_HOLE_BIT)) {
            if (first == W) first = x;
            last = x;
        }
    __shared__ int sl[256], sf[256];
    sl[t] = last;
    sf[t] = first;
    __syncthreads();
    // inclusive prefix max of `last` and suffix min of `first` (Hillis-Steele)
    for (int d = 1; d < 256; d <<= 1) {
        const int a = t >= d ? sl[t - d] : -1;
        const int b = t + d < 256 ? sf[t + d] : W;
        __syncthreads();
        sl[t] = max(sl[t], a);
        sf[t] = min(sf[t], b);
        __syncthreads();
    }
    int L = t > 0 ? sl[t - 1] : -1;
    const int carryR = t < 255 ? sf[t + 1] : W;
    for (int x = x0; x < x1; ++x) {
        const uint32_t s = row[x];
        if (!(s & FVV_HOLE_BIT)) {
            L = x;
            continue;
        }
        int R = carryR;
        for (int xr = x + 1; xr < x1; ++xr)
            if (!(row[xr] & FVV_HOLE_BIT)) {
                R = xr;
                break;
            }
        int win = -1;
        if (L >= 0 && R < W) {
            const float zl = u2f(row[L]), zr = u2f(row[R]);
            win = (zl > zr || (zl == zr && x - L <= R - x)) ? L : R;
        } else if (L >= 0) {
            win = L;
        } else if (R < W) {
            win = R;
        }
        row[x] = FVV_HOLE_BIT | (uint32_t)(win + 1);
    }
}

// Column summaries: first and last non-hole row of each FVV_FILL_SEG-row
// segment of each column (-1 if none).
__global__ void __launch_bounds__(64) k_fill_colsum(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.z];
    const int x = blockIdx.x * 64 + threadIdx.x, seg = blockIdx.y;
    if (x >= vd.W || seg >= vd.n_seg) return;
    const int r0 = seg * FVV_FILL_SEG, r1 = min(r0 + FVV_FILL_SEG, vd.H);
    int first = -1, last = -1;
    for (int r = r0; r < r1; ++r)
        if (!(vd.slot[(int64_t)r * vd.W + x] & FVV_HOLE_BIT)) {
            if (first < 0) first = r;
            last = r;
        }
    vd.colsum[(int64_t)seg * vd.W + x] = make_int2(first, last);
}

__device__ __forceinline__ void put_rgb(uint8_t *out, int64_t pitch, int x, int y, uint32_t c)
{
    uint8_t *p = out + (int64_t)y * pitch + (int64_t)x * 3;
    p[0] = (uint8_t)c;
    p[1] = (uint8_t)(c >> 8);
    p[2] = (uint8_t)(c >> 16);
}

// Column pass: combine the row winner with the nearest non-holes above and
// below (larger depth, then nearer; row candidates before up before down),
// copy the winner's colour; non-holes copy their own.  Writes the output.
__global__ void __launch_bounds__(64) k_fill_resolve(const fvv_view_desc *__restrict__ views)
{
    const fvv_view_desc &vd = views[blockIdx.z];
    const int x = blockIdx.x * 64 + threadIdx.x, seg = blockIdx.y;
    const int W = vd.W, H = vd.H;
    if (x >= W || seg >= vd.n_seg) return;
    const int r0 = seg * FVV_FILL_SEG, r1 = min(r0 + FVV_FILL_SEG, H);
    const bool fill = vd.fill_mode == 0;
    __shared__ short below[FVV_FILL_SEG][64];
    int up = -1;
    if (fill) {
        for (int s2 = seg - 1; s2 >= 0; --s2) {
            const int l = vd.colsum[(int64_t)s2 * W + x].y;
            if (l >= 0) {
                up = l;
                break;
            }
        }
        int nd = H;
        for (int s2 = seg + 1; s2 < vd.n_seg; ++s2) {
            const int f = vd.colsum[(int64_t)s2 * W + x].x;
            if (f >= 0) {
                nd = f;
                break;
            }
        }
        for (int r = r1 - 1; r >= r0; --r) {
            below[r - r0][threadIdx.x] = (short)min(nd, 32767);
            if (!(vd.slot[(int64_t)r * W + x] & FVV_HOLE_BIT)) nd = r;
        }
    }
    for (int r = r0; r < r1; ++r) {
        const uint32_t s = vd.slot[(int64_t)r * W + x];
        if (!(s & FVV_HOLE_BIT)) {
            put_rgb(vd.out, vd.out_pitch, x, r, vd.rgba[(int64_t)r * W + x]);
            up = r;
            continue;
        }
        uint32_t col = 0;
        if (fill) {
            int64_t src = -1;
            float zb = 0.f;
            int db = 0;
            const int rw = (int)(s & ~FVV_HOLE_BIT);
            if (rw > 0) {
                const int xw = rw - 1;
                src = (int64_t)r * W + xw;
                zb = u2f(vd.slot[src]);
                db = abs(xw - x);
            }
            if (up >= 0) {
                const int64_t o = (int64_t)up * W + x;
                const float zu = u2f(vd.slot[o]);
                const int du = r - up;
                if (src < 0 || zu > zb || (zu == zb && du < db)) {
                    src = o;
                    zb = zu;
                    db = du;
                }
            }
            const int dn = below[r - r0][threadIdx.x];
            if (dn < H) {
                const int64_t o = (int64_t)dn * W + x;
                const float zd = u2f(vd.slot[o]);
                const int dd = dn - r;
                if (src < 0 || zd > zb || (zd == zb && dd < db)) src = o;
            }
            if (src >= 0) col = vd.rgba[src];
        }
        put_rgb(vd.out, vd.out_pitch, x, r, col);
    }
}

}  // namespace

hipError_t fvv_launch_repack(const uint8_t *rgb, int64_t rgb_pitch, const uint16_t *depth,
                             int64_t depth_pitch, int W, int H, float alpha, float beta,
                             uint32_t *rgba_out, float *depth_out, hipStream_t s, fvv_prof *prof)
{
    dim3 grid((W + 255) / 256, H);
    hipEvent_t e0;
    fvv_prof_begin(prof, s, e0);
    hipLaunchKernelGGL(k_repack, grid, dim3(256), 0, s, rgb, rgb_pitch, depth, depth_pitch, W, H, alpha,
                       beta, rgba_out, depth_out);
    fvv_prof_end(prof, s, FVV_ST_REPACK, e0);
    return hipGetLastError();
}

hipError_t fvv_launch_synthesis(const fvv_view_desc *d_views, int n_views, int max_w, int max_h,
                                int max_src_px, int max_k, bool fill_bg, hipStream_t s, fvv_prof *prof)
{
    if (n_views <= 0) return hipSuccess;
    const int64_t max_px = (int64_t)max_w * max_h;
    const int zblocks = (int)std::min<int64_t>((max_px + 255) / 256, 4096);
    const int n_seg = (max_h + FVV_FILL_SEG - 1) / FVV_FILL_SEG;
    hipEvent_t e0;
    fvv_prof_begin(prof, s, e0);
    hipLaunchKernelGGL(k_zclear, dim3(zblocks, n_views), dim3(256), 0, s, d_views);
    fvv_prof_end(prof, s, FVV_ST_ZCLEAR, e0);
    fvv_prof_begin(prof, s, e0);
    hipLaunchKernelGGL(k_splat, dim3((max_src_px + 255) / 256, max_k, n_views), dim3(256), 0, s, d_views);
    fvv_prof_end(prof, s, FVV_ST_SPLAT, e0);
    fvv_prof_begin(prof, s, e0);
    hipLaunchKernelGGL(k_filter_blend, dim3((max_w + TB - 1) / TB, (max_h + TB - 1) / TB, n_views),
                       dim3(TB, TB), 0, s, d_views);
    fvv_prof_end(prof, s, FVV_ST_FILTER_BLEND, e0);
    if (fill_bg) {
        fvv_prof_begin(prof, s, e0);
        hipLaunchKernelGGL(k_fill_rows, dim3(max_h, n_views), dim3(256), 0, s, d_views);
        fvv_prof_end(prof, s, FVV_ST_FILL_ROWS, e0);
        fvv_prof_begin(prof, s, e0);
        hipLaunchKernelGGL(k_fill_colsum, dim3((max_w + 63) / 64, n_seg, n_views), dim3(64), 0, s, d_views);
        fvv_prof_end(prof, s, FVV_ST_FILL_COLSUM, e0);
    }
    fvv_prof_begin(prof, s, e0);
    hipLaunchKernelGGL(k_fill_resolve, dim3((max_w + 63) / 64, n_seg, n_views), dim3(64), 0, s, d_views);
    fvv_prof_end(prof, s, FVV_ST_FILL_RESOLVE, e0);
    return hipGetLastError();
}
