// fvv_y12.h -- device helpers of the 12-bit depth coding for 8-bit YUV420
// video codecs (Section V-A), shared by the codec kernels and the frame-store
// ingest.  Internal to the library.
//
// Codes: 0 = background (0xFFFF in millimetre maps, the background signal of
// the layered transmission), 1 = no depth (0 mm) or out of range,
// 2..4095 = Eq. 2 of the depth, which is linear in
// 1/z between the clipping planes.  Eq. 2 and its inverse run in double
// precision op by op (the library is built without contraction), rounded
// half up; "out of range" means the rounded code leaves 2..4095.
//
// I420 placement of each 2x2 block p11 p12 / p21 p22: every pixel's Y is its
// 8 LSBs, mirrored to 255 - LSBs when its 4 MSBs are odd (Eq. 3), so that
// consecutive codes never jump in Y; U carries the MSBs of p11 on its even
// bits and those of p12 on its odd bits (bit 2k = bit k of p11, bit 2k+1 =
// bit k of p12), V the same for p21 and p22.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// The two plane terms of Eq. 2, 1/z_far and 1/z_near - 1/z_far, each one
// correctly rounded double operation; the host evaluates them once per call
// (the same IEEE operations give the same bits there).
struct y12_planes {
    double inv_zf, span;
};
__host__ __device__ inline y12_planes y12_make_planes(float z_near, float z_far)
{
    const double zn = z_near, zf = z_far;
    return {1.0 / zf, 1.0 / zn - 1.0 / zf};
}

// Eq. 2: millimetres -> code
__device__ __forceinline__ uint32_t y12_quantise(uint32_t mm, y12_planes p)
{
    if (mm == 0xFFFFu) return 0u;
    if (mm == 0) return 1u;
    const double z = (double)mm / 1000.0;
    const double a = 1.0 / z - p.inv_zf;
    const double r = floor(4093.0 * a / p.span + 2.0 + 0.5);
    return (r >= 2.0 && r <= 4095.0) ? (uint32_t)r : 1u;
}

// inverse of Eq. 2 -> whole millimetres in 1..65535 (0xFFFF for code 0, 0 for
// code 1)
__device__ __forceinline__ uint32_t y12_dequantise(uint32_t code, y12_planes p)
{
    if (code == 0u) return 0xFFFFu;
    if (code == 1u) return 0u;
    const double t = (double)(code - 2u) / 4093.0;
    const double inv = t * p.span + p.inv_zf;
    const double mm = floor(1.0 / inv * 1000.0 + 0.5);
    return mm < 1.0 ? 1u : mm > 65535.0 ? 65535u : (uint32_t)mm;
}

// Eq. 3 and its inverse
__device__ __forceinline__ uint32_t y12_fold(uint32_t code)
{
    return ((code >> 8) & 1u) ? 255u - (code & 0xFFu) : (code & 0xFFu);
}
__device__ __forceinline__ uint32_t y12_unfold(uint32_t yv, uint32_t msb)
{
    return msb << 8 | ((msb & 1u) ? 255u - yv : yv);
}

// 4 bits b3..b0 -> the even bits of a byte, and back
__device__ __forceinline__ uint32_t y12_spread4(uint32_t m)
{
    m = (m | m << 2) & 0x33u;
    return (m | m << 1) & 0x55u;
}
__device__ __forceinline__ uint32_t y12_gather4(uint32_t v)
{
    v &= 0x55u;
    v = (v | v >> 1) & 0x33u;
    return (v | v >> 2) & 0x0Fu;
}

// MSBs of pixel column `odd` (0 = left, 1 = right) of a U or V byte
__device__ __forceinline__ uint32_t y12_msb(uint32_t uv, uint32_t odd) { return y12_gather4(uv >> odd); }
