// fvv_internal.h -- descriptors shared by the host runtime and the gfx950
// kernels of libfvv.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

#define FVV_KMAX 8
#define FVV_KEY_EMPTY 0xFFFFFFFFFFFFFFFFull
#define FVV_NO_DEPTH 0xFFFFFFFFu    // depth-plane marker of a pixel without depth
#define FVV_HOLE_BIT 0x80000000u    // slot marker of a hole (valid depths are positive floats)
#define FVV_ZCLIP 0.01f             // points and samples nearer than this are dropped
#define FVV_FILL_SEG 64             // rows per column segment in the hole fill

// One selected source camera of one view.  The float32 pair matrices are
// computed on the host in double and rounded once (Section VI pinhole warp):
//   forward  p = ((A_r0 i + A_r1 j) + A_r2) z + a_r   (source pixel -> virtual)
//   backward q = ((B_r0 x + B_r1 y) + B_r2) z + b_r   (virtual pixel -> source)
struct fvv_src_desc {
    const uint32_t *rgba;   // H*W texels, RGBA8 with R in the low byte
    const float *depth;     // H*W decoded depth (Eq. 1 applied); FVV_NO_DEPTH bits = none
    int32_t W, H;
    int32_t cam;            // rig index (key bits 27..31)
    float wgt;              // view weight, 1 / centre distance
    float A[9], a[3], B[9], b[3];
    float sx, sy;           // focal ratios virtual / source (footprint scale)
};

// One virtual view of a batched synthesis call.
struct fvv_view_desc {
    int32_t W, H, K, fill_mode;
    float tau, max_fp;
    int32_t n_seg;          // ceil(H / FVV_FILL_SEG)
    int32_t pad0;
    unsigned long long *Z;  // W*H raw keys (splat target)
    unsigned long long *Zf; // W*H filtered keys (debug tap; may be null)
    float *dbg_depth;       // W*H blend depth (debug tap; may be null)
    uint32_t *rgba;         // W*H blend result, A = 255 covered, 0 hole
    uint32_t *slot;         // W*H depth bits of covered pixels / hole codes
    int2 *colsum;           // n_seg*W column-segment summaries
    uint8_t *out;           // final RGB8, out_pitch bytes per row
    int64_t out_pitch;
    fvv_src_desc src[FVV_KMAX];
};

// Stage timing: when a context has profiling on, every kernel launch is
// bracketed by a pair of HIP events on its stream; durations are summed per
// stage when the profile is read.
enum fvv_stage {
    FVV_ST_REPACK = 0,
    FVV_ST_ZCLEAR,
    FVV_ST_SPLAT,
    FVV_ST_FILTER_BLEND,
    FVV_ST_FILL_ROWS,
    FVV_ST_FILL_COLSUM,
    FVV_ST_FILL_RESOLVE,
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

// Host-side launchers (fvv_kernels.hip).  All return hipError_t of the launch.
hipError_t fvv_launch_repack(const uint8_t *rgb, int64_t rgb_pitch, const uint16_t *depth,
                             int64_t depth_pitch, int W, int H, float alpha, float beta,
                             uint32_t *rgba_out, float *depth_out, hipStream_t s, fvv_prof *prof);
hipError_t fvv_launch_synthesis(const fvv_view_desc *d_views, int n_views, int max_w,
                                int max_h, int max_src_px, int max_k, bool fill_bg,
                                hipStream_t s, fvv_prof *prof);
