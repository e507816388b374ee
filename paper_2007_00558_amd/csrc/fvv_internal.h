// fvv_internal.h -- descriptors shared by the host runtime and the gfx950
// kernels of libfvv.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fvv_y12.h"

#include <string>
#include <utility>
#include <vector>

#define FVV_KMAX 8
#define FVV_KEY_EMPTY 0xFFFFFFFFFFFFFFFFull
#define FVV_NO_DEPTH 0xFFFFFFFFu    // depth-plane marker of a pixel without depth
#ifndef FVV_BG_MM
#define FVV_BG_MM 0xFFFF            // background signal of live millimetre maps (no live depth), as in fvv.h
#endif
#define FVV_HOLE 0x80000000u        // slot of a hole filled inside its tile (or left black)
#define FVV_HOLE_OPEN 0x80000001u   // slot of a hole whose neighbours lie beyond its tile
#define FVV_ZCLIP 0.01f             // points and samples nearer than this are dropped
#define FVV_SPL_RECOMPUTE 0xFFFFFFFFu   // splat record whose footprint does not pack (x0 = 8191 with x1 > x0)
#define FVV_TILE 32                 // output tile edge (pixels) of the fused kernel
#define FVV_SBLK 8                  // source block edge (pixels) of the binning
#define FVV_BIN_BPW 4               // source blocks per wave of the binning
#define FVV_TILE_CAP_MIN 128        // minimum bin-list entries per output tile
#define FVV_MAX_RIG 32              // cameras in a rig
#define FVV_XCDS 8                  // XCDs of an MI355X: workgroup i runs on XCD i mod 8

// One selected source camera of one view.  The float32 pair matrices are
// computed on the host in double and rounded once (Section VI pinhole warp):
//   forward  p = ((A_r0 i + A_r1 j) + A_r2) z + a_r   (source pixel -> virtual)
//   backward q = ((B_r0 x + B_r1 y) + B_r2) z + b_r   (virtual pixel -> source)
struct fvv_src_desc {
    const uint2 *texel;     // H*W: x = RGBA8 (R in the low byte), y = depth bits (FVV_NO_DEPTH = none)
    const float *depth;     // H*W decoded depth (Eq. 1 applied); FVV_NO_DEPTH bits = none
    int32_t W, H;
    int32_t cam;            // rig index (key bits 27..31)
    int32_t nbx;            // source blocks per row: ceil(W / FVV_SBLK)
    int32_t nblk;           // source blocks: nbx * ceil(H / FVV_SBLK)
    uint64_t nbx_magic;     // ceil(2^40 / nbx): blk / nbx = (blk nbx_magic) >> 40 (blk < 2^24)
    float wgt;              // view weight, 1 / centre distance
    float A[9], a[3], B[9], b[3];
    float sx, sy;           // focal ratios virtual / source (footprint scale)
    float umax, vmax;       // W - 0.5, H - 0.5: last sample coordinates on the image (exact in float32)
};

// One virtual view of a batched synthesis call.
struct fvv_view_desc {
    int32_t W, H, K, fill_mode;     // K selected cameras
    float tau, max_fp;
    int32_t ntx, nty;       // output tiles per row / column
    int32_t blk_stride;     // bbox entries reserved per camera slot (>= max nblk)
    int32_t tile_cap;       // bin-list entries per tile
    int32_t view;           // index of this view in the batch
    int32_t layered;        // layered synthesis: src[0..K) foreground layers,
                            // src[K..2K) background layers of the same cameras
    // binning
    int32_t *counts;        // ntx*nty tile counters (zero between calls; cleared by the tile kernel)
    int32_t *list;          // ntx*nty*tile_cap entries: source slot << 24 | source block
    int4 *bbox;             // nsrc*blk_stride tile ranges (x0, x1, y0, y1; x0 > x1 = empty)
    // per-pixel splat records written by the binning, nsrc*blk_stride*64
    // (slot, block, lane): x = depth bits of the projected point
    // (FVV_NO_DEPTH = no splat), y = footprint x0 | y0 << 13 | (x1 - x0) << 26
    // | (y1 - y0) << 29, or FVV_SPL_RECOMPUTE when an extent exceeds 7
    unsigned long long *spl;
    int2 *dbg_tiles;        // debug tap (null unless enabled): per tile, the entries the
                            // binning appended and the list capacity
    // per-tile results
    uint32_t *slot;         // W*H depth bits of covered pixels / FVV_HOLE / FVV_HOLE_OPEN
    int2 *rowsum;           // ntx*nty*FVV_TILE (first, last) covered x of each tile row
    int2 *colsum;           // ntx*nty*FVV_TILE (first, last) covered y of each tile column
    int2 *open_list;        // batch-wide list of (view, tile) with open holes
    int32_t *open_count;    // its length (cleared by the binning kernel)
    uint8_t *out;           // final RGB8, out_pitch bytes per row
    int64_t out_pitch;
    // learned path: network input [stack_h][stack_w][16] bf16 (null = plain view)
    uint16_t *stack;
    int32_t stack_w, stack_h;   // W, H rounded up to multiples of 8
    // debug taps (null unless enabled); dbg_bz / dbg_bzf: background layer
    unsigned long long *dbg_z;
    unsigned long long *dbg_zf;
    unsigned long long *dbg_bz;
    unsigned long long *dbg_bzf;
    uint32_t *dbg_rgba;
    float *dbg_depth;
    fvv_src_desc src[FVV_KMAX];
};

// source slots of a view: one per selected camera, two when layered
__host__ __device__ inline int fvv_nsrc(const fvv_view_desc &d) { return d.layered ? 2 * d.K : d.K; }

// Stage timing: when a context has profiling on, every kernel launch is
// bracketed by a pair of HIP events on its stream; durations are summed per
// stage when the profile is read.
enum fvv_stage {
    FVV_ST_REPACK = 0,
    FVV_ST_DESC,
    FVV_ST_BIN,
    FVV_ST_TILE,
    FVV_ST_FILL_OPEN,
    FVV_ST_NET,         // learned path: network forward of one view
    FVV_ST_TRAIN,       // learned path: one training step
    FVV_NSTAGES
};

struct fvv_prof {
    std::vector<hipEvent_t> pool;
    size_t next = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
    double total_ms[FVV_NSTAGES] = {};
    int64_t launches[FVV_NSTAGES] = {};
    hipEvent_t take()
    {
        if (next == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[next++];
    }
};

inline void fvv_prof_begin(fvv_prof *p, hipStream_t s, hipEvent_t &e0)
{
    e0 = nullptr;
    if (p && (e0 = p->take())) (void)hipEventRecord(e0, s);
}

inline void fvv_prof_end(fvv_prof *p, hipStream_t s, int stage, hipEvent_t e0)
{
    if (!p || !e0) return;
    hipEvent_t e1 = p->take();
    if (!e1) return;
    (void)hipEventRecord(e1, s);
    p->marks.push_back({stage, {e0, e1}});
}

// Launch geometry of one batched synthesis call.
struct fvv_batch_dims {
    int n_views;
    int max_k;            // largest source-slot count of the batch
    int max_blocks;       // largest source-block count of a selected camera
    int max_tiles_x;      // largest ntx
    int max_tiles_y;      // largest nty
    int total_tiles;      // tiles of all views
    bool fill_bg;         // any view fills holes
    bool any_stack;       // any view writes a learned-path stack
    bool any_layered;     // any view is layered (no view is both)
};

// Ingest of one frame set: every present camera's caller buffers (device
// memory, or the runtime's staging copy of host memory) in one launch.
struct fvv_repack_cam {
    const uint8_t *rgb;
    int64_t rgb_pitch;      // bytes
    const uint8_t *depth;   // uint16 millimetres, or (12-bit coding) an I420 image:
                            // Y rows of depth_pitch bytes, then the U and V
                            // planes, H/2 rows of depth_pitch/2 bytes each
    int64_t depth_pitch;    // bytes
    uint2 *texel_out;
    float *depth_out;
    int32_t W, H;
    float alpha, beta;      // Eq. (1)
    // layered frame sets: the camera's background model (uint16 mm, W per
    // row; null = none) and the background-layer planes it fills
    const uint16_t *bg_model;
    uint2 *bg_texel_out;
    float *bg_depth_out;
};
// Joint bilateral pre-filter tables: FVV_JBF_WS spatial weights (a
// (2r+1)^2 window, row-major, padded to 7x7) then FVV_JBF_WC range weights
// by L1 colour distance, 12-bit integers.
#define FVV_JBF_WS 49
#define FVV_JBF_WC 766
struct fvv_repack_batch {
    int32_t n;
    int32_t y12;            // depth arrives 12-bit coded (Section V-A)
    y12_planes planes;      // plane terms of that coding (clipping planes in metres)
    const uint32_t *jbf;    // pre-filter weight tables (null = filter off)
    int32_t jbf_radius, jbf_min;
    fvv_repack_cam cam[FVV_MAX_RIG];
};

// 12-bit depth coding (fvv_codec.hip) of n equal-sized images in one
// launch: millimetres (mm[i], rows of mm_pitch[i] bytes) <-> an I420 image
// (yuv[i]: Y rows of yuv_pitch[i] bytes, then U and V of H/2 rows of
// yuv_pitch[i]/2 bytes).  W and H even.
struct fvv_y12_batch {
    int32_t n, W, H;
    y12_planes planes;      // of the clipping planes z_near, z_far
    const uint8_t *mm[FVV_MAX_RIG];
    int64_t mm_pitch[FVV_MAX_RIG];
    uint8_t *yuv[FVV_MAX_RIG];
    int64_t yuv_pitch[FVV_MAX_RIG];
};
hipError_t fvv_launch_y12(const fvv_y12_batch &b, bool encode, hipStream_t s);

// Host-side launchers (fvv_kernels.hip).  All return hipError_t of the launch.
hipError_t fvv_launch_repack(const fvv_repack_batch &b, int max_w, int max_h, hipStream_t s, fvv_prof *prof);
// h_views: device-visible pointer to the coherent pinned host copy of the
// descriptors and extra_bytes (a multiple of 16) that follow them, copied
// into d_views by the first kernel of the sequence.
hipError_t fvv_launch_synthesis(const fvv_view_desc *h_views, fvv_view_desc *d_views,
                                const fvv_batch_dims &dims, size_t extra_bytes, hipStream_t s, fvv_prof *prof);
// One view whose descriptor travels in the kernel arguments: stored to
// d_view, and the view's dims.total_tiles counters at `counts` cleared, by
// the first kernel of the sequence (no host staging, nothing allocated).
hipError_t fvv_launch_synthesis_one(const fvv_view_desc &view, fvv_view_desc *d_view, int32_t *counts,
                                    const fvv_batch_dims &dims, hipStream_t s, fvv_prof *prof);

// Measured machine peaks (fvv_peaks.hip) on the current device; see
// fvv_measure_peaks in fvv.h for the five figures written to out.
hipError_t fvv_measure_peaks_impl(double *out, std::string &err);
// fvv_check_reciprocal's kernel: adds the mismatch count to *bad_dev
hipError_t fvv_check_reciprocal_impl(int e_lo, int e_hi, unsigned long long *bad_dev, hipStream_t s);
