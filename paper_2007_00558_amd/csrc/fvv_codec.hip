// fvv_codec.hip -- 12-bit depth coding onto 8-bit I420 images (Section V-A):
// the capture-side encoder (Eq. 2 quantisation, Eq. 3 folding, MSB
// interleave) and the standalone decoder.  The frame-store ingest decodes
// the same format inside its repack kernel.
//
// One thread per 2x2 block: a wave covers 128 columns of two rows, so every
// plane is read and written in contiguous runs.  Memory bound (HBM): the
// encoder moves 2 + 1.5 bytes per pixel, the decoder 1.5 + 2.
#include "fvv_internal.h"
#include "fvv_y12.h"

namespace {

__global__ void __launch_bounds__(256) k_y12_encode(const uint8_t *__restrict__ dep, int64_t dpitch, int bw,
                                                      float z_near, float z_far, uint8_t *__restrict__ Y,
                                                      int64_t ypitch, uint8_t *__restrict__ U,
                                                      uint8_t *__restrict__ V, int64_t uvpitch)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= bw) return;
    const double zn = z_near, zf = z_far;
    const uint16_t *d0 = (const uint16_t *)(dep + (int64_t)(2 * r) * dpitch) + 2 * c;
    const uint16_t *d1 = (const uint16_t *)(dep + (int64_t)(2 * r + 1) * dpitch) + 2 * c;
    const uint32_t p11 = y12_quantise(d0[0], zn, zf), p12 = y12_quantise(d0[1], zn, zf);
    const uint32_t p21 = y12_quantise(d1[0], zn, zf), p22 = y12_quantise(d1[1], zn, zf);
    uint8_t *y0 = Y + (int64_t)(2 * r) * ypitch + 2 * c;
    uint8_t *y1 = y0 + ypitch;
    y0[0] = (uint8_t)y12_fold(p11);
    y0[1] = (uint8_t)y12_fold(p12);
    y1[0] = (uint8_t)y12_fold(p21);
    y1[1] = (uint8_t)y12_fold(p22);
    U[(int64_t)r * uvpitch + c] = (uint8_t)(y12_spread4(p11 >> 8) | y12_spread4(p12 >> 8) << 1);
    V[(int64_t)r * uvpitch + c] = (uint8_t)(y12_spread4(p21 >> 8) | y12_spread4(p22 >> 8) << 1);
}

__global__ void __launch_bounds__(256) k_y12_decode(const uint8_t *__restrict__ Y, int64_t ypitch,
                                                      const uint8_t *__restrict__ U, const uint8_t *__restrict__ V,
                                                      int64_t uvpitch, int bw, float z_near, float z_far,
                                                      uint8_t *__restrict__ dep, int64_t dpitch)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= bw) return;
    const double zn = z_near, zf = z_far;
    const uint8_t *y0 = Y + (int64_t)(2 * r) * ypitch + 2 * c;
    const uint8_t *y1 = y0 + ypitch;
    const uint32_t u = U[(int64_t)r * uvpitch + c], v = V[(int64_t)r * uvpitch + c];
    uint16_t *d0 = (uint16_t *)(dep + (int64_t)(2 * r) * dpitch) + 2 * c;
    uint16_t *d1 = (uint16_t *)(dep + (int64_t)(2 * r + 1) * dpitch) + 2 * c;
    d0[0] = (uint16_t)y12_dequantise(y12_unfold(y0[0], y12_msb(u, 0)), zn, zf);
    d0[1] = (uint16_t)y12_dequantise(y12_unfold(y0[1], y12_msb(u, 1)), zn, zf);
    d1[0] = (uint16_t)y12_dequantise(y12_unfold(y1[0], y12_msb(v, 0)), zn, zf);
    d1[1] = (uint16_t)y12_dequantise(y12_unfold(y1[1], y12_msb(v, 1)), zn, zf);
}

}  // namespace

hipError_t fvv_launch_y12_encode(const uint8_t *dep, int64_t dpitch, int W, int H, float zn, float zf, uint8_t *yuv,
                                 int64_t ypitch, hipStream_t s)
{
    const int bw = W / 2, bh = H / 2;
    uint8_t *U = yuv + (int64_t)H * ypitch;
    uint8_t *V = U + (int64_t)bh * (ypitch / 2);
    hipLaunchKernelGGL(k_y12_encode, dim3((bw + 255) / 256, bh), dim3(256), 0, s, dep, dpitch, bw, zn, zf, yuv,
                       ypitch, U, V, ypitch / 2);
    return hipGetLastError();
}

hipError_t fvv_launch_y12_decode(const uint8_t *yuv, int64_t ypitch, int W, int H, float zn, float zf, uint8_t *dep,
                                 int64_t dpitch, hipStream_t s)
{
    const int bw = W / 2, bh = H / 2;
    const uint8_t *U = yuv + (int64_t)H * ypitch;
    const uint8_t *V = U + (int64_t)bh * (ypitch / 2);
    hipLaunchKernelGGL(k_y12_decode, dim3((bw + 255) / 256, bh), dim3(256), 0, s, yuv, ypitch, U, V, ypitch / 2, bw,
                       zn, zf, dep, dpitch);
    return hipGetLastError();
}
