// fvv_codec.hip -- 12-bit depth coding onto 8-bit I420 images (Section V-A):
// the capture-side encoder (Eq. 2 quantisation, Eq. 3 folding, MSB
// interleave) and the standalone decoder.  The frame-store ingest decodes
// the same format inside its repack kernel.
//
// One thread per 2x2 block, numbered row-major over the image (grid.y =
// image of a batch of equal-sized images), so no lane idles at a row end
// and every plane is read and written in contiguous runs.  The double
// divisions of Eq. 2 dominate (three per pixel to encode, two to decode;
// the plane terms come precomputed): fp64-issue bound, not HBM bound.
#include "fvv_internal.h"
#include "fvv_y12.h"

namespace {

// block (r, c) of image blockIdx.y handled by this thread, false past the end
__device__ __forceinline__ bool y12_block(const fvv_y12_batch &b, int &r, int &c)
{
    const int bw = b.W >> 1;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= bw * (b.H >> 1)) return false;
    r = e / bw;
    c = e - r * bw;
    return true;
}

__global__ void __launch_bounds__(256) k_y12_encode(const fvv_y12_batch b)
{
    int r, c;
    if (!y12_block(b, r, c)) return;
    const int n = blockIdx.y;
    const uint8_t *dep = b.mm[n];
    const int64_t dpitch = b.mm_pitch[n], ypitch = b.yuv_pitch[n], uvpitch = ypitch / 2;
    uint8_t *Y = b.yuv[n];
    uint8_t *U = Y + (int64_t)b.H * ypitch;
    uint8_t *V = U + (int64_t)(b.H / 2) * uvpitch;
    const uint16_t *d0 = (const uint16_t *)(dep + (int64_t)(2 * r) * dpitch) + 2 * c;
    const uint16_t *d1 = (const uint16_t *)(dep + (int64_t)(2 * r + 1) * dpitch) + 2 * c;
    const uint32_t p11 = y12_quantise(d0[0], b.planes), p12 = y12_quantise(d0[1], b.planes);
    const uint32_t p21 = y12_quantise(d1[0], b.planes), p22 = y12_quantise(d1[1], b.planes);
    uint8_t *y0 = Y + (int64_t)(2 * r) * ypitch + 2 * c;
    uint8_t *y1 = y0 + ypitch;
    y0[0] = (uint8_t)y12_fold(p11);
    y0[1] = (uint8_t)y12_fold(p12);
    y1[0] = (uint8_t)y12_fold(p21);
    y1[1] = (uint8_t)y12_fold(p22);
    U[(int64_t)r * uvpitch + c] = (uint8_t)(y12_spread4(p11 >> 8) | y12_spread4(p12 >> 8) << 1);
    V[(int64_t)r * uvpitch + c] = (uint8_t)(y12_spread4(p21 >> 8) | y12_spread4(p22 >> 8) << 1);
}

__global__ void __launch_bounds__(256) k_y12_decode(const fvv_y12_batch b)
{
    int r, c;
    if (!y12_block(b, r, c)) return;
    const int n = blockIdx.y;
    const int64_t ypitch = b.yuv_pitch[n], uvpitch = ypitch / 2, dpitch = b.mm_pitch[n];
    const uint8_t *Y = b.yuv[n];
    const uint8_t *U = Y + (int64_t)b.H * ypitch;
    const uint8_t *V = U + (int64_t)(b.H / 2) * uvpitch;
    uint8_t *dep = (uint8_t *)b.mm[n];
    const uint8_t *y0 = Y + (int64_t)(2 * r) * ypitch + 2 * c;
    const uint8_t *y1 = y0 + ypitch;
    const uint32_t u = U[(int64_t)r * uvpitch + c], v = V[(int64_t)r * uvpitch + c];
    uint16_t *d0 = (uint16_t *)(dep + (int64_t)(2 * r) * dpitch) + 2 * c;
    uint16_t *d1 = (uint16_t *)(dep + (int64_t)(2 * r + 1) * dpitch) + 2 * c;
    d0[0] = (uint16_t)y12_dequantise(y12_unfold(y0[0], y12_msb(u, 0)), b.planes);
    d0[1] = (uint16_t)y12_dequantise(y12_unfold(y0[1], y12_msb(u, 1)), b.planes);
    d1[0] = (uint16_t)y12_dequantise(y12_unfold(y1[0], y12_msb(v, 0)), b.planes);
    d1[1] = (uint16_t)y12_dequantise(y12_unfold(y1[1], y12_msb(v, 1)), b.planes);
}

}  // namespace

hipError_t fvv_launch_y12(const fvv_y12_batch &b, bool encode, hipStream_t s)
{
    if (b.n <= 0) return hipSuccess;
    const int64_t blocks = (int64_t)(b.W / 2) * (b.H / 2);
    const dim3 grid((unsigned)((blocks + 255) / 256), b.n);
    if (encode)
        hipLaunchKernelGGL(k_y12_encode, grid, dim3(256), 0, s, b);
    else
        hipLaunchKernelGGL(k_y12_decode, grid, dim3(256), 0, s, b);
    return hipGetLastError();
}
