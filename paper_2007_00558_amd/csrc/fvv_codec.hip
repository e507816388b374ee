// fvv_codec.hip -- 12-bit depth coding onto 8-bit I420 images (Section V-A):
// the capture-side encoder (Eq. 2 quantisation, Eq. 3 folding, MSB
// interleave) and the standalone decoder.  The frame-store ingest decodes
// the same format inside its repack kernel.
//
// One thread per 2x2 block (grid.z = image of a batch of equal-sized
// images): a wave covers 128 columns of two rows, so every plane is read and
// written in contiguous runs.  Memory bound (HBM): the encoder moves 2 + 1.5
// bytes per pixel, the decoder 1.5 + 2.
#include "fvv_internal.h"
#include "fvv_y12.h"

namespace {

__global__ void __launch_bounds__(256) k_y12_encode(const fvv_y12_batch b)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    const int bw = b.W / 2;
    if (c >= bw) return;
    const uint8_t *dep = b.mm[blockIdx.z];
    const int64_t dpitch = b.mm_pitch[blockIdx.z], ypitch = b.yuv_pitch[blockIdx.z], uvpitch = ypitch / 2;
    uint8_t *Y = b.yuv[blockIdx.z];
    uint8_t *U = Y + (int64_t)b.H * ypitch;
    uint8_t *V = U + (int64_t)(b.H / 2) * uvpitch;
    const double zn = b.z_near, zf = b.z_far;
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

__global__ void __launch_bounds__(256) k_y12_decode(const fvv_y12_batch b)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    const int bw = b.W / 2;
    if (c >= bw) return;
    const int64_t ypitch = b.yuv_pitch[blockIdx.z], uvpitch = ypitch / 2, dpitch = b.mm_pitch[blockIdx.z];
    const uint8_t *Y = b.yuv[blockIdx.z];
    const uint8_t *U = Y + (int64_t)b.H * ypitch;
    const uint8_t *V = U + (int64_t)(b.H / 2) * uvpitch;
    uint8_t *dep = (uint8_t *)b.mm[blockIdx.z];
    const double zn = b.z_near, zf = b.z_far;
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

hipError_t fvv_launch_y12(const fvv_y12_batch &b, bool encode, hipStream_t s)
{
    if (b.n <= 0) return hipSuccess;
    const dim3 grid((b.W / 2 + 255) / 256, b.H / 2, b.n);
    if (encode)
        hipLaunchKernelGGL(k_y12_encode, grid, dim3(256), 0, s, b);
    else
        hipLaunchKernelGGL(k_y12_decode, grid, dim3(256), 0, s, b);
    return hipGetLastError();
}
