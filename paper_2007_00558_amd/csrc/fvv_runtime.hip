// fvv_runtime.hip -- host runtime behind the C ABI of libfvv.so (include/fvv.h).
//
// Owns the device state of one context: the rig, a double-buffered frame
// store of repacked MVD frames, workspaces for batched synthesis, debug taps,
// stage timing, and the continuous-batching server.  Camera selection and
// the pair matrices are computed here in double and handed to the kernels as
// float32 (Section VI: the pinhole warp and the mix by camera distance).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/fvv.h"
#include "fvv_internal.h"
#include "fvv_unet.h"

namespace {

using Clock = std::chrono::steady_clock;

thread_local std::string g_create_error;

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// One resident frame set.  Every stream that reads it records an event;
// an upload into the slot waits for all of them.
struct FrameSlot {
    uint64_t version = 0;                 // 0 = empty
    std::vector<uint2 *> texel;           // per camera {RGBA8, depth bits}
    std::vector<float *> depth;
    std::vector<uint2 *> bg_texel;        // layered sets: background layer of each camera
    std::vector<float *> bg_depth;
    bool layered = false;                 // holds background layers
    std::vector<int32_t> present;
    hipEvent_t ready = nullptr;           // recorded after the repack
    hipStream_t ready_stream = nullptr;   // the stream it was recorded on
    std::vector<std::pair<hipStream_t, hipEvent_t>> readers;
};

// Device buffers of one batched launch sequence.
struct Workspace {
    uint8_t *ws = nullptr;
    size_t ws_bytes = 0;
    int32_t *counts = nullptr;            // tile counters, zero between calls
    size_t counts_cap = 0;
    fvv_view_desc *d_desc = nullptr;
    size_t desc_cap = 0;
    int2 *open_list = nullptr;            // batch list of tiles with open holes
    int32_t *open_count = nullptr;
    bool dirty = false;                   // a launch failed: clear the counters first
    static constexpr int kRing = 4;       // coherent pinned host descriptor buffers
    fvv_view_desc *h_desc[kRing] = {};
    fvv_view_desc *h_desc_dev[kRing] = {};   // their device-visible addresses
    hipEvent_t h_ev[kRing] = {};
    bool h_live[kRing] = {};
    size_t h_cap = 0;
    int ring = 0;
};

struct ViewLayout {
    int ntx, nty, n_tiles, blk_stride, tile_cap, K;
    int nsrc;             // source slots: K, or 2K when layered
    int32_t idx[FVV_MAX_K];
    double w[FVV_MAX_K];
};

struct Request {
    uint64_t ticket;
    fvv_camera cam;
    fvv_synth_params P;
    void *out;
    int64_t pitch;
    Clock::time_point arrive;
    size_t bytes;     // workspace bound
    size_t tiles;
};

struct Result {
    bool done = false;
    int32_t status = FVV_OK;
    double latency = 0.0;
};

struct Server {
    int max_slots = 0;
    size_t step_bytes = 0;
    size_t step_tiles = 0;
    Workspace ws[2];
    hipStream_t stream[2] = {nullptr, nullptr};
    hipEvent_t done_ev[2] = {nullptr, nullptr};
    bool busy[2] = {false, false};
    std::vector<Request> inflight[2];
    std::thread sched, compl_[2];
    std::mutex qmu;                       // pending, busy, stop
    std::condition_variable qcv;
    std::deque<Request> pending;
    // viewpoints of recent requests (arrival time, camera) for the
    // transmission set; bounded
    std::deque<std::pair<Clock::time_point, fvv_camera>> recent;
    bool stop = false;
    bool paused = false;
    std::mutex cmu[2];
    std::condition_variable ccv[2];
    bool launched[2] = {false, false};
    Clock::time_point launch_t[2];
    std::mutex dmu;                       // results, stats
    std::unordered_map<uint64_t, Result> results;
    std::atomic<uint64_t> next_ticket{1};
    unet_act *act[2] = {nullptr, nullptr};   // network activations of each stream's steps
    // statistics
    uint64_t n_steps = 0, n_done = 0, n_failed = 0, pixels = 0, batch_sum = 0;
    double busy_s = 0.0;
};

}  // namespace

struct fvv_ctx {
    int device = 0;
    uint64_t budget = 0;     // 0 = unlimited
    uint64_t allocated = 0;
    std::mutex mu;           // guards everything below against the server thread
    std::string err;
    std::vector<fvv_camera> rig;
    FrameSlot slots[2];
    int latest = -1;
    uint64_t next_version = 1;
    std::vector<hipEvent_t> event_pool;
    // background models of the layered synthesis: uint16 mm per camera
    // (width per row; null = none), set while has_bg
    std::vector<uint16_t *> bg_model;
    bool has_bg = false;
    // joint bilateral pre-filter of live depth at ingest (null tables = off)
    uint32_t *jbf = nullptr;
    int32_t jbf_radius = 0, jbf_min = 0;
    bool jbf_on = false;
    // depth format of uploads (FVV_DEPTH_*) and the clipping planes of the
    // 12-bit coding
    int32_t depth_format = FVV_DEPTH_MM16;
    float z_near = 0.f, z_far = 0.f;
    // upload staging: raw RGB8 + depth planes of all cameras
    uint8_t *staging = nullptr;
    size_t staging_bytes = 0;
    hipEvent_t staging_free = nullptr;
    // pinned bounce buffer (two halves) for copies into the caller's
    // pageable host memory, and an event per half
    uint8_t *bounce = nullptr;
    hipEvent_t bounce_ev[2] = {nullptr, nullptr};
    Workspace user;          // workspace of direct synthesis calls
    uint8_t *scratch = nullptr;   // device address of this device's no-allocation scratch
    // Direct calls (synthesis, stacks, network forward and training) share
    // the user workspace, the activation set, the network's gradient and
    // the debug taps: the last such call's stream and an event recorded
    // after its work; a call on another stream waits for that event first.
    hipEvent_t last_ev = nullptr;
    hipStream_t last_stream = nullptr;
    bool last_live = false;
    // debug taps of view 0 of the last direct synthesis
    bool debug = false;
    unsigned long long *dbg_z = nullptr;
    unsigned long long *dbg_zf = nullptr;
    unsigned long long *dbg_bz = nullptr;     // background layer (layered views)
    unsigned long long *dbg_bzf = nullptr;
    bool last_layered = false;
    uint32_t *dbg_rgba = nullptr;
    float *dbg_depth = nullptr;
    size_t dbg_px = 0;
    int2 *dbg_tiles = nullptr;     // per tile: bin-list entries appended, list capacity
    size_t dbg_tiles_n = 0;
    int32_t debug_view = 0;        // view of a batched call whose stages are tapped
    int64_t last_tiles = 0;
    int64_t last_px = 0;
    bool have_taps = false;
    // stage timing
    bool profiling = false;
    fvv_prof prof;
    Server *server = nullptr;
    // learned path: network weights and the activation set of direct calls
    unet_state *net = nullptr;
    unet_act *act = nullptr;
    uint64_t net_bytes = 0;     // device bytes held by the network and every activation set
};

namespace {

int32_t fail(fvv_ctx *c, int32_t code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_create_error = buf;
    return code;
}

#define HIPCHECK(ctx, expr)                                                                       \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail((ctx), FVV_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

int32_t dalloc(fvv_ctx *c, void **p, size_t bytes)
{
    if (c->budget && c->allocated + bytes > c->budget)
        return fail(c, FVV_E_NOMEM, "device memory budget exceeded (%llu + %zu > %llu bytes)",
                    (unsigned long long)c->allocated, bytes, (unsigned long long)c->budget);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, FVV_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    c->allocated += bytes;
    return FVV_OK;
}

void dfree(fvv_ctx *c, void *p, size_t bytes)
{
    if (p) {
        (void)hipFree(p);
        c->allocated -= std::min<uint64_t>(bytes, c->allocated);
    }
}

bool finite_all(const float *v, int n)
{
    for (int e = 0; e < n; ++e)
        if (!std::isfinite(v[e])) return false;
    return true;
}

int32_t check_camera(fvv_ctx *c, const fvv_camera &cam, bool source, const char *what)
{
    if (cam.width < 1 || cam.height < 1 || cam.width > 65535 || cam.height > 65535)
        return fail(c, FVV_E_ARG, "%s: bad size %dx%d", what, cam.width, cam.height);
    if (source && (int64_t)cam.width * cam.height > FVV_MAX_SRC_PIXELS)
        return fail(c, FVV_E_ARG, "%s: %dx%d exceeds %d pixels", what, cam.width, cam.height,
                    FVV_MAX_SRC_PIXELS);
    if (!source && (cam.width > FVV_MAX_OUT_DIM || cam.height > FVV_MAX_OUT_DIM))
        return fail(c, FVV_E_ARG, "%s: output %dx%d exceeds %d", what, cam.width, cam.height, FVV_MAX_OUT_DIM);
    const float sc[6] = {cam.fx, cam.fy, cam.cx, cam.cy, cam.depth_alpha, cam.depth_beta};
    if (!finite_all(sc, 6) || !finite_all(cam.R, 9) || !finite_all(cam.t, 3))
        return fail(c, FVV_E_ARG, "%s: non-finite parameter", what);
    if (!(cam.fx > 0.f) || !(cam.fy > 0.f)) return fail(c, FVV_E_ARG, "%s: fx/fy must be > 0", what);
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += (double)cam.R[r * 3 + k] * (double)cam.R[q * 3 + k];
            if (std::fabs(s - (r == q ? 1.0 : 0.0)) > 1e-4)
                return fail(c, FVV_E_ARG, "%s: R is not orthonormal", what);
        }
    return FVV_OK;
}

// camera centre C = -R^T t in double
void centre(const fvv_camera &c, double C[3])
{
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += (double)c.R[k * 3 + r] * (double)c.t[k];
        C[r] = -s;
    }
}

// Adaptive view transmission (Section V-C): OR into m the n_tx rig cameras
// nearest to viewpoint v (centre distance, ties to the lower index).
void tx_union(const fvv_camera *rig, int n, const fvv_camera &v, int n_tx, uint32_t &m)
{
    double Cv[3];
    centre(v, Cv);
    std::vector<std::pair<double, int>> d;
    for (int c = 0; c < n; ++c) {
        double Cc[3];
        centre(rig[c], Cc);
        const double dx = Cc[0] - Cv[0], dy = Cc[1] - Cv[1], dz = Cc[2] - Cv[2];
        d.emplace_back(std::sqrt(dx * dx + dy * dy + dz * dz), c);
    }
    std::stable_sort(d.begin(), d.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    for (int e = 0; e < n_tx && e < n; ++e) m |= 1u << d[e].second;
}

int popcount32(uint32_t m)
{
    int c = 0;
    for (; m; m &= m - 1) ++c;
    return c;
}

// Rank present cameras by centre distance (stable: ties keep the lower index);
// weights 1/d; a coincident camera (d < 1e-6 m) is used alone with weight 1.
int select_k(const fvv_camera *rig, const int32_t *present, int n, const fvv_camera &v, int k, int32_t *idx,
             double *w)
{
    double Cv[3];
    centre(v, Cv);
    // insertion by distance into a fixed array (stable: a camera goes after
    // every earlier one at the same distance; no heap use)
    std::pair<double, int> d[FVV_MAX_CAMERAS];
    int nd = 0;
    for (int c = 0; c < n && c < FVV_MAX_CAMERAS; ++c) {
        if (present && !present[c]) continue;
        double Cc[3];
        centre(rig[c], Cc);
        const double dx = Cc[0] - Cv[0], dy = Cc[1] - Cv[1], dz = Cc[2] - Cv[2];
        const double dist = std::sqrt(dx * dx + dy * dy + dz * dz);
        int e = nd++;
        for (; e > 0 && dist < d[e - 1].first; --e) d[e] = d[e - 1];
        d[e] = {dist, c};
    }
    int K = std::min<int>({nd, k, FVV_MAX_K});
    if (K > 0 && d[0].first < 1e-6) {
        idx[0] = d[0].second;
        w[0] = 1.0;
        return 1;
    }
    for (int e = 0; e < K; ++e) {
        idx[e] = d[e].second;
        w[e] = 1.0 / d[e].first;
    }
    return K;
}

// Pair matrices of the pinhole warp from camera s (points) to camera d
// (image): M = K_d (R_d R_s^T) K_s^-1, m = K_d (t_d - R_d R_s^T t_s); double,
// fixed association order, rounded once to float32.
void pair_dir(const fvv_camera &s, const fvv_camera &d, float M[9], float m[3])
{
    double Rrel[9], T1[9], T2[9], tr[3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += (double)d.R[r * 3 + k] * (double)s.R[c * 3 + k];
            Rrel[r * 3 + c] = acc;
        }
    const double fx = s.fx, fy = s.fy;
    const double Ksi[9] = {1.0 / fx, 0.0, -(double)s.cx / fx, 0.0, 1.0 / fy, -(double)s.cy / fy, 0.0, 0.0, 1.0};
    const double Kd[9] = {(double)d.fx, 0.0, (double)d.cx, 0.0, (double)d.fy, (double)d.cy, 0.0, 0.0, 1.0};
    auto mm = [](const double *X, const double *Y, double *Z) {
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += X[r * 3 + k] * Y[k * 3 + c];
                Z[r * 3 + c] = acc;
            }
    };
    mm(Rrel, Ksi, T1);
    mm(Kd, T1, T2);
    for (int r = 0; r < 3; ++r) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += Rrel[r * 3 + k] * (double)s.t[k];
        tr[r] = (double)d.t[r] - acc;
    }
    for (int r = 0; r < 3; ++r) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += Kd[r * 3 + k] * tr[k];
        m[r] = (float)acc;
    }
    for (int e = 0; e < 9; ++e) M[e] = (float)T2[e];
}

int nblocks(const fvv_camera &c)
{
    return ((c.width + FVV_SBLK - 1) / FVV_SBLK) * ((c.height + FVV_SBLK - 1) / FVV_SBLK);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// bytes of workspace one view needs: slot plane, tile arrays, bin list,
// block ranges, and (host-memory output) an RGB8 staging image
size_t stack_w(int W) { return (size_t)(W + UNET_ALIGN - 1) / UNET_ALIGN * UNET_ALIGN; }
size_t stack_bytes(int W, int H) { return stack_w(W) * stack_w(H) * UNET_IN * 2; }

size_t view_ws_bytes(int W, int H, const ViewLayout &L, bool host_out, bool learned = false)
{
    const size_t px = (size_t)W * H;
    const size_t nt = (size_t)L.n_tiles;
    size_t b = align256(px * 4);                                   // slot
    b += align256(nt * FVV_TILE * sizeof(int2)) * 2;               // rowsum, colsum
    b += align256(nt * (size_t)L.tile_cap * 4);                    // bin lists
    b += align256((size_t)L.nsrc * L.blk_stride * sizeof(int4));   // block tile ranges
    b += align256((size_t)L.nsrc * L.blk_stride * 64 * 8);         // splat records
    if (host_out) b += align256(px * 3);
    if (learned) b += align256(stack_bytes(W, H));
    return b;
}

// Tile grid and list sizes of a view drawing on K cameras of the rig whose
// block counts are given (each twice when layered); used both for exact
// layouts and for upper bounds.
void layout_sizes(ViewLayout &L, int W, int H, const int *nblk, int K, bool layered)
{
    L.K = K;
    L.nsrc = layered ? 2 * K : K;
    L.ntx = (W + FVV_TILE - 1) / FVV_TILE;
    L.nty = (H + FVV_TILE - 1) / FVV_TILE;
    L.n_tiles = L.ntx * L.nty;
    int sum = 0, mx = 0;
    for (int k = 0; k < L.nsrc; ++k) {
        sum += nblk[k % K];
        mx = std::max(mx, nblk[k % K]);
    }
    L.blk_stride = mx;
    // a block touches about two tiles; room for four times the average
    const int cap = (int)std::min<int64_t>(65536, (8LL * sum + L.n_tiles - 1) / L.n_tiles);
    L.tile_cap = std::max(FVV_TILE_CAP_MIN, (cap + 31) / 32 * 32);
}

hipEvent_t take_event(fvv_ctx *c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// record that `s` reads frame slot fs (an upload into the slot waits for it)
constexpr size_t kBounceHalf = (size_t)8 << 20;   // bytes per half; holds a row of any output width

// Copy `rows` rows of `row` bytes from device memory (src_pitch apart) into
// the caller's host memory (dst_pitch apart) after the work already on
// stream s: device -> pinned bounce half (asynchronous, on s) -> host
// memcpy, two halves in flight.  Returns with the copy complete.
int32_t to_host(fvv_ctx *c, uint8_t *dst, int64_t dst_pitch, const uint8_t *src, int64_t src_pitch, size_t row,
                size_t rows, hipStream_t s)
{
    if (rows == 0 || row == 0) return FVV_OK;
    if (row > kBounceHalf) return fail(c, FVV_E_ARG, "rows of %zu bytes exceed the %zu-byte host bounce buffer", row,
                                       kBounceHalf);
    if (!c->bounce) {
        HIPCHECK(c, hipHostMalloc((void **)&c->bounce, 2 * kBounceHalf, hipHostMallocDefault));
        for (auto &e : c->bounce_ev) HIPCHECK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    const size_t per = kBounceHalf / row;          // rows per piece
    const size_t n = (rows + per - 1) / per;
    auto issue = [&](size_t i) -> int32_t {
        const size_t r0 = i * per, nr = std::min(per, rows - r0);
        uint8_t *b = c->bounce + (i & 1) * kBounceHalf;
        HIPCHECK(c, hipMemcpy2DAsync(b, row, src + (int64_t)r0 * src_pitch, (size_t)src_pitch, row, nr,
                                     hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipEventRecord(c->bounce_ev[i & 1], s));
        return FVV_OK;
    };
    int32_t rc = issue(0);
    for (size_t i = 0; i < n && rc == FVV_OK; ++i) {
        if (i + 1 < n && (rc = issue(i + 1))) break;   // the other half was consumed in the last iteration
        HIPCHECK(c, hipEventSynchronize(c->bounce_ev[i & 1]));
        const size_t r0 = i * per, nr = std::min(per, rows - r0);
        const uint8_t *b = c->bounce + (i & 1) * kBounceHalf;
        if (dst_pitch == (int64_t)row) {
            std::memcpy(dst + r0 * row, b, nr * row);
        } else {
            for (size_t r = 0; r < nr; ++r) std::memcpy(dst + (int64_t)(r0 + r) * dst_pitch, b + r * row, row);
        }
    }
    return rc;
}

int32_t note_reader(fvv_ctx *c, FrameSlot &fs, hipStream_t s)
{
    for (auto &r : fs.readers)
        if (r.first == s) {
            HIPCHECK(c, hipEventRecord(r.second, s));
            return FVV_OK;
        }
    hipEvent_t e = take_event(c);
    if (!e) return fail(c, FVV_E_DEVICE, "hipEventCreate failed");
    HIPCHECK(c, hipEventRecord(e, s));
    fs.readers.emplace_back(s, e);
    return FVV_OK;
}

int32_t ensure_frame_slot(fvv_ctx *c, FrameSlot &s)
{
    const int n = (int)c->rig.size();
    if ((int)s.texel.size() == n && s.layered == c->has_bg && s.ready) return FVV_OK;
    if (!s.texel.empty()) return fail(c, FVV_E_STATE, "frame slot layout out of date");
    s.texel.assign(n, nullptr);
    s.depth.assign(n, nullptr);
    s.bg_texel.assign(n, nullptr);
    s.bg_depth.assign(n, nullptr);
    s.layered = c->has_bg;
    s.present.assign(n, 0);
    for (int k = 0; k < n; ++k) {
        const size_t px = (size_t)c->rig[k].width * c->rig[k].height;
        int32_t rc = dalloc(c, (void **)&s.texel[k], px * 8);
        if (rc) return rc;
        rc = dalloc(c, (void **)&s.depth[k], px * 4);
        if (rc) return rc;
        if (s.layered) {
            if ((rc = dalloc(c, (void **)&s.bg_texel[k], px * 8))) return rc;
            if ((rc = dalloc(c, (void **)&s.bg_depth[k], px * 4))) return rc;
        }
    }
    if (!s.ready) HIPCHECK(c, hipEventCreateWithFlags(&s.ready, hipEventDisableTiming));
    return FVV_OK;
}

void release_bg(fvv_ctx *c)
{
    for (size_t k = 0; k < c->bg_model.size(); ++k)
        if (c->bg_model[k]) dfree(c, c->bg_model[k], (size_t)c->rig[k].width * c->rig[k].height * 2);
    c->bg_model.clear();
    c->has_bg = false;
}

void release_frames(fvv_ctx *c)
{
    for (auto &s : c->slots) {
        for (size_t k = 0; k < s.texel.size(); ++k) {
            const size_t px = (size_t)c->rig[k].width * c->rig[k].height;
            dfree(c, s.texel[k], px * 8);
            dfree(c, s.depth[k], px * 4);
            if (s.layered) {
                dfree(c, s.bg_texel[k], px * 8);
                dfree(c, s.bg_depth[k], px * 4);
            }
        }
        s.texel.clear();
        s.depth.clear();
        s.bg_texel.clear();
        s.bg_depth.clear();
        s.layered = false;
        s.present.clear();
        for (auto &r : s.readers) c->event_pool.push_back(r.second);
        s.readers.clear();
        s.version = 0;
    }
    c->latest = -1;
}

// Per view of a launch: its descriptor and one entry of the network's output
// table (learned views), both copied to the device by the first kernel.
constexpr size_t kDescBytes = sizeof(fvv_view_desc) + sizeof(unet_out);
static_assert(sizeof(unet_out) % 16 == 0, "output tables copy in 16-byte words");

// Learned views of a launch batched through the network: views with one
// stack size, at most this many pixels per forward (bounds the activation
// set: about 420 bytes per pixel).
constexpr size_t kNetBatchPixels = (size_t)8 << 20;

// Grow a workspace (synchronising the device first) so it holds `bytes` of
// per-view buffers, `tiles` tile counters and `n` view descriptors.
int32_t ws_reserve(fvv_ctx *c, Workspace &W, size_t bytes, size_t tiles, size_t n)
{
    int32_t rc;
    if (W.ws_bytes < bytes) {
        HIPCHECK(c, hipDeviceSynchronize());
        dfree(c, W.ws, W.ws_bytes);
        W.ws = nullptr;
        W.ws_bytes = 0;
        if ((rc = dalloc(c, (void **)&W.ws, bytes))) return rc;
        W.ws_bytes = bytes;
    }
    if (W.counts_cap < tiles) {
        HIPCHECK(c, hipDeviceSynchronize());
        dfree(c, W.counts, W.counts_cap * 4);
        dfree(c, W.open_list, W.counts_cap * sizeof(int2));
        dfree(c, W.open_count, 256);
        W.counts = nullptr;
        W.open_list = nullptr;
        W.open_count = nullptr;
        W.counts_cap = 0;
        if ((rc = dalloc(c, (void **)&W.counts, tiles * 4))) return rc;
        if ((rc = dalloc(c, (void **)&W.open_list, tiles * sizeof(int2)))) return rc;
        if ((rc = dalloc(c, (void **)&W.open_count, 256))) return rc;
        HIPCHECK(c, hipMemset(W.counts, 0, tiles * 4));
        W.counts_cap = tiles;
        W.dirty = false;
    }
    if (W.desc_cap < n) {
        HIPCHECK(c, hipDeviceSynchronize());
        dfree(c, W.d_desc, W.desc_cap * kDescBytes);
        W.d_desc = nullptr;
        W.desc_cap = 0;
        if ((rc = dalloc(c, (void **)&W.d_desc, n * kDescBytes))) return rc;
        W.desc_cap = n;
    }
    if (W.h_cap < n) {
        for (int r = 0; r < Workspace::kRing; ++r) {
            if (W.h_live[r]) HIPCHECK(c, hipEventSynchronize(W.h_ev[r]));
            W.h_live[r] = false;
            if (W.h_desc[r]) (void)hipHostFree(W.h_desc[r]);
            W.h_desc[r] = nullptr;
            // fine-grained (coherent) so the copy kernel always sees this call's data
            HIPCHECK(c, hipHostMalloc((void **)&W.h_desc[r], n * kDescBytes,
                                      hipHostMallocMapped | hipHostMallocCoherent));
            HIPCHECK(c, hipHostGetDevicePointer((void **)&W.h_desc_dev[r], W.h_desc[r], 0));
            if (!W.h_ev[r]) HIPCHECK(c, hipEventCreateWithFlags(&W.h_ev[r], hipEventDisableTiming));
        }
        W.h_cap = n;
    }
    return FVV_OK;
}

void ws_release(fvv_ctx *c, Workspace &W)
{
    dfree(c, W.ws, W.ws_bytes);
    dfree(c, W.counts, W.counts_cap * 4);
    dfree(c, W.open_list, W.counts_cap * sizeof(int2));
    dfree(c, W.open_count, 256);
    dfree(c, W.d_desc, W.desc_cap * kDescBytes);
    for (int r = 0; r < Workspace::kRing; ++r) {
        if (W.h_desc[r]) (void)hipHostFree(W.h_desc[r]);
        if (W.h_ev[r]) (void)hipEventDestroy(W.h_ev[r]);
    }
    W = Workspace();
}

int32_t resolve_params(fvv_ctx *c, const fvv_synth_params *p, fvv_synth_params &o)
{
    o = fvv_synth_params{3, 0.05f, 4.0f, FVV_FILL_BG, FVV_PATH_PLAIN, 0u, 0};
    if (!p) return FVV_OK;
    o = *p;
    if (o.k_nearest == 0) o.k_nearest = 3;
    if (o.tau_rel == 0.f) o.tau_rel = 0.05f;
    if (o.max_footprint == 0.f) o.max_footprint = 4.0f;
    if (o.k_nearest < 1 || o.k_nearest > FVV_MAX_K)
        return fail(c, FVV_E_ARG, "k_nearest %d outside 1..%d", o.k_nearest, FVV_MAX_K);
    if (!std::isfinite(o.tau_rel) || !(o.tau_rel > 0.f))
        return fail(c, FVV_E_ARG, "tau_rel must be finite and > 0");
    if (!std::isfinite(o.max_footprint) || !(o.max_footprint >= 1.f) || o.max_footprint > 64.f)
        return fail(c, FVV_E_ARG, "max_footprint must lie in [1, 64]");
    if (o.fill_mode != FVV_FILL_BG && o.fill_mode != FVV_FILL_NONE)
        return fail(c, FVV_E_ARG, "unknown fill_mode %d", o.fill_mode);
    if (o.path != FVV_PATH_PLAIN && o.path != FVV_PATH_LEARNED && o.path != FVV_PATH_LAYERED)
        return fail(c, FVV_E_ARG, "unknown path %d", o.path);
    if (o.path == FVV_PATH_LAYERED && o.k_nearest > FVV_MAX_K / 2)
        return fail(c, FVV_E_ARG, "layered synthesis blends at most %d cameras", FVV_MAX_K / 2);
    return FVV_OK;
}

int32_t find_slot(fvv_ctx *c, uint64_t version, int &si)
{
    si = c->latest;
    if (version) {
        si = -1;
        for (int q = 0; q < 2; ++q)
            if (c->slots[q].version == version) si = q;
        if (si < 0) return fail(c, FVV_E_STATE, "frame version %llu is not resident", (unsigned long long)version);
    }
    if (si < 0 || c->slots[si].version == 0) return fail(c, FVV_E_STATE, "no frame set uploaded");
    return FVV_OK;
}

// Grow an activation set to hold `px` network pixels (and the training
// buffers if train), within the context's memory budget.
int32_t reserve_act(fvv_ctx *c, unet_act *a, size_t px, bool train)
{
    const bool tr = train || unet_act_trainable(a);
    const size_t cap = std::max(px, unet_act_cap(a));
    if (cap == unet_act_cap(a) && tr == unet_act_trainable(a)) return FVV_OK;
    const size_t before = unet_act_bytes(a), after = unet_act_need(cap, tr);
    if (c->budget && c->allocated - before + after > c->budget)
        return fail(c, FVV_E_NOMEM, "device memory budget exceeded by the network activations (%zu bytes)", after);
    const hipError_t e = unet_act_reserve(a, cap, tr);
    c->allocated = c->allocated - before + unet_act_bytes(a);
    c->net_bytes = c->net_bytes - before + unet_act_bytes(a);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, FVV_E_NOMEM, "network activations (%zu bytes): %s", after, hipGetErrorString(e));
    }
    return FVV_OK;
}

int32_t net_status(fvv_ctx *c, hipError_t e, const std::string &err, const char *what)
{
    if (e == hipSuccess) return FVV_OK;
    if (!err.empty()) return fail(c, FVV_E_ARG, "%s: %s", what, err.c_str());
    return fail(c, FVV_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Learned-path inputs and outputs of one launch sequence.
struct LearnedIO {
    unet_act *act = nullptr;           // activation set of the stream (null: the network does not run)
    uint16_t *stack_out = nullptr;     // caller's stacks [n][stack_h][stack_w][16] (every view learned)
    bool scratch_out = false;          // RGB goes to workspace scratch (stack-only calls)
};

// Order a direct call on stream s after the previous direct call's device
// work when that ran on another stream (they share buffers).
int32_t order_direct(fvv_ctx *c, hipStream_t s)
{
    if (c->last_live && c->last_stream != s) HIPCHECK(c, hipStreamWaitEvent(s, c->last_ev, 0));
    return FVV_OK;
}

// Mark the end of a direct call's device work on stream s.
int32_t mark_direct(fvv_ctx *c, hipStream_t s)
{
    if (!c->last_ev) HIPCHECK(c, hipEventCreateWithFlags(&c->last_ev, hipEventDisableTiming));
    HIPCHECK(c, hipEventRecord(c->last_ev, s));
    c->last_stream = s;
    c->last_live = true;
    return FVV_OK;
}

// Camera selection and tile layout of one view: the frame slot it reads
// (si), its selected cameras and weights, tile grid and list sizes (L).
int32_t plan_view(fvv_ctx *c, const fvv_camera &vc, const fvv_synth_params &P, int &si, ViewLayout &L)
{
    int32_t rc;
    if ((rc = find_slot(c, P.frame_version, si))) return rc;
    const FrameSlot &fs = c->slots[si];
    const bool layered = P.path == FVV_PATH_LAYERED;
    if (layered && !fs.layered)
        return fail(c, FVV_E_STATE, "layered synthesis needs a frame set uploaded with background models");
    const int n = (int)c->rig.size();
    int32_t pres[FVV_MAX_CAMERAS];
    for (int q = 0; q < n; ++q) pres[q] = ((P.exclude_mask >> q) & 1u) ? 0 : fs.present[q];
    const int K = select_k(c->rig.data(), pres, n, vc, P.k_nearest, L.idx, L.w);
    if (K < 1) return fail(c, FVV_E_STATE, "no camera present in the frame set");
    int nb[FVV_MAX_K];
    for (int k = 0; k < K; ++k) nb[k] = nblocks(c->rig[L.idx[k]]);
    layout_sizes(L, vc.width, vc.height, nb, K, layered);
    return FVV_OK;
}

// Descriptor of view `view` of a launch: geometry, parameters, the selected
// cameras with their weights and float32 pair matrices, and the view's
// buffers (slot plane, tile summaries, bin lists, block ranges, splat
// records) carved from `cur`, tile counters from `cnt` (both advanced).
// Output, stack, taps and the batch's open-tile list are the caller's.
void fill_desc(fvv_ctx *c, fvv_view_desc &d, const fvv_camera &vc, const ViewLayout &L, const FrameSlot &fs,
               const fvv_synth_params &P, int view, uint8_t *&cur, int32_t *&cnt)
{
    std::memset(&d, 0, sizeof d);
    d.W = vc.width;
    d.H = vc.height;
    d.K = L.K;
    d.fill_mode = P.fill_mode;
    d.tau = P.tau_rel;
    d.max_fp = P.max_footprint;
    d.ntx = L.ntx;
    d.nty = L.nty;
    d.blk_stride = L.blk_stride;
    d.tile_cap = L.tile_cap;
    d.view = view;
    d.layered = L.nsrc > L.K;
    const size_t px = (size_t)vc.width * vc.height;
    const size_t nt = (size_t)L.n_tiles;
    auto carve = [&](size_t bytes) {
        uint8_t *p = cur;
        cur += align256(bytes);
        return p;
    };
    d.slot = (uint32_t *)carve(px * 4);
    d.rowsum = (int2 *)carve(nt * FVV_TILE * sizeof(int2));
    d.colsum = (int2 *)carve(nt * FVV_TILE * sizeof(int2));
    d.list = (int32_t *)carve(nt * (size_t)L.tile_cap * 4);
    d.bbox = (int4 *)carve((size_t)L.nsrc * L.blk_stride * sizeof(int4));
    d.spl = (unsigned long long *)carve((size_t)L.nsrc * L.blk_stride * 64 * 8);
    d.counts = cnt;
    cnt += nt;
    for (int k = 0; k < L.K; ++k) {
        const fvv_camera &sc = c->rig[L.idx[k]];
        fvv_src_desc &sd = d.src[k];
        sd.texel = fs.texel[L.idx[k]];
        sd.depth = fs.depth[L.idx[k]];
        sd.W = sc.width;
        sd.H = sc.height;
        sd.cam = L.idx[k];
        sd.nbx = (sc.width + FVV_SBLK - 1) / FVV_SBLK;
        sd.nbx_magic = ((1ULL << 40) + (uint64_t)sd.nbx - 1) / (uint64_t)sd.nbx;
        sd.nblk = nblocks(sc);
        sd.wgt = (float)L.w[k];
        pair_dir(sc, vc, sd.A, sd.a);
        pair_dir(vc, sc, sd.B, sd.b);
        sd.sx = (float)((double)vc.fx / (double)sc.fx);
        sd.sy = (float)((double)vc.fy / (double)sc.fy);
        sd.umax = (float)sc.width - 0.5f;
        sd.vmax = (float)sc.height - 0.5f;
        if (d.layered) {
            // the camera's background layer: same geometry and weight
            fvv_src_desc &bd = d.src[L.K + k];
            bd = sd;
            bd.texel = fs.bg_texel[L.idx[k]];
            bd.depth = fs.bg_depth[L.idx[k]];
        }
    }
}

// One batched launch sequence over n views (caller holds c->mu, has checked
// the arguments and resolved each view's parameters).  grow: the workspace
// may be enlarged; otherwise the caller guarantees it fits.  Views on the
// learned path also write the network input stack in the tile kernel, and
// the network then overwrites their plain result with its own wherever its
// output is finite; without a loaded network they stay plain.
int32_t launch_views(fvv_ctx *c, Workspace &Wk, const fvv_camera *virts, const fvv_synth_params *Ps, int n_views,
                     void *const *outs, const int64_t *pitches, bool host_out, hipStream_t s, bool grow,
                     bool taps, const LearnedIO &lio = LearnedIO())
{
    const bool have_net = lio.act && c->net && unet_loaded(c->net);
    std::vector<char> learned(n_views, 0);
    for (int v = 0; v < n_views; ++v) learned[v] = lio.stack_out || (have_net && Ps[v].path == FVV_PATH_LEARNED);
    // network batches: learned views grouped by stack size (first appearance
    // order, views in call order), split at kNetBatchPixels; each batch's
    // stacks are contiguous and its output-table entries consecutive
    struct NetBatch {
        int H, W;
        std::vector<int> views;
    };
    std::vector<NetBatch> batches;
    size_t net_px = 0;
    if (!lio.stack_out) {
        for (int v = 0; v < n_views; ++v) {
            if (!learned[v]) continue;
            const int sh = (int)stack_w(virts[v].height), sw = (int)stack_w(virts[v].width);
            const size_t px = (size_t)sh * sw;
            NetBatch *b = nullptr;
            for (auto it = batches.rbegin(); it != batches.rend(); ++it)
                if (it->H == sh && it->W == sw) {
                    b = &*it;
                    break;
                }
            if (!b || (b->views.size() + 1) * px > std::max(kNetBatchPixels, px)) {
                batches.push_back(NetBatch{sh, sw, {}});
                b = &batches.back();
            }
            b->views.push_back(v);
            net_px = std::max(net_px, b->views.size() * px);
        }
    }
    std::vector<ViewLayout> lay(n_views);
    std::vector<int> slot_of(n_views);
    size_t total = 0, total_tiles = 0;
    fvv_batch_dims dims{n_views, 0, 0, 0, 0, 0, false, false, false};
    int32_t rc;
    for (int v = 0; v < n_views; ++v) {
        if ((rc = plan_view(c, virts[v], Ps[v], slot_of[v], lay[v]))) return rc;
        const ViewLayout &L = lay[v];
        const fvv_camera &vc = virts[v];
        const bool layered = Ps[v].path == FVV_PATH_LAYERED;
        total += view_ws_bytes(vc.width, vc.height, L, host_out || lio.scratch_out, learned[v] && !lio.stack_out);
        total_tiles += (size_t)L.n_tiles;
        dims.total_tiles += L.n_tiles;
        dims.max_k = std::max(dims.max_k, L.nsrc);
        dims.any_layered = dims.any_layered || layered;
        dims.max_blocks = std::max(dims.max_blocks, L.blk_stride);
        dims.max_tiles_x = std::max(dims.max_tiles_x, L.ntx);
        dims.max_tiles_y = std::max(dims.max_tiles_y, L.nty);
        dims.fill_bg = dims.fill_bg || Ps[v].fill_mode == FVV_FILL_BG;
        dims.any_stack = dims.any_stack || learned[v];
    }
    if (grow) {
        if ((rc = ws_reserve(c, Wk, total, total_tiles, n_views))) return rc;
    } else if (Wk.ws_bytes < total || Wk.counts_cap < total_tiles || Wk.desc_cap < (size_t)n_views) {
        return fail(c, FVV_E_NOMEM, "step does not fit its workspace");
    }
    if (net_px && (rc = reserve_act(c, lio.act, net_px, false))) return rc;
    const int tv = taps && c->debug_view < n_views ? c->debug_view : -1;   // tapped view
    if (tv >= 0) {
        const size_t nt = (size_t)lay[tv].n_tiles;
        if (c->dbg_tiles_n < nt) {
            HIPCHECK(c, hipDeviceSynchronize());
            dfree(c, c->dbg_tiles, c->dbg_tiles_n * sizeof(int2));
            c->dbg_tiles = nullptr;
            c->dbg_tiles_n = 0;
            if ((rc = dalloc(c, (void **)&c->dbg_tiles, nt * sizeof(int2)))) return rc;
            c->dbg_tiles_n = nt;
        }
        const size_t px = (size_t)virts[tv].width * virts[tv].height;
        if (c->dbg_px < px) {
            HIPCHECK(c, hipDeviceSynchronize());
            dfree(c, c->dbg_z, c->dbg_px * 8);
            dfree(c, c->dbg_zf, c->dbg_px * 8);
            dfree(c, c->dbg_bz, c->dbg_px * 8);
            dfree(c, c->dbg_bzf, c->dbg_px * 8);
            dfree(c, c->dbg_rgba, c->dbg_px * 4);
            dfree(c, c->dbg_depth, c->dbg_px * 4);
            c->dbg_z = c->dbg_zf = c->dbg_bz = c->dbg_bzf = nullptr;
            c->dbg_rgba = nullptr;
            c->dbg_depth = nullptr;
            c->dbg_px = 0;
            if ((rc = dalloc(c, (void **)&c->dbg_z, px * 8))) return rc;
            if ((rc = dalloc(c, (void **)&c->dbg_zf, px * 8))) return rc;
            if ((rc = dalloc(c, (void **)&c->dbg_bz, px * 8))) return rc;
            if ((rc = dalloc(c, (void **)&c->dbg_bzf, px * 8))) return rc;
            if ((rc = dalloc(c, (void **)&c->dbg_rgba, px * 4))) return rc;
            if ((rc = dalloc(c, (void **)&c->dbg_depth, px * 4))) return rc;
            c->dbg_px = px;
        }
    }
    const int r = Wk.ring;
    Wk.ring = (Wk.ring + 1) % Workspace::kRing;
    if (Wk.h_live[r]) HIPCHECK(c, hipEventSynchronize(Wk.h_ev[r]));
    fvv_view_desc *hd = Wk.h_desc[r];
    uint8_t *cur = Wk.ws;
    int32_t *cnt = Wk.counts;
    std::vector<uint8_t *> host_stage(n_views, nullptr);
    for (int v = 0; v < n_views; ++v) {
        const fvv_camera &vc = virts[v];
        fvv_view_desc &d = hd[v];
        fill_desc(c, d, vc, lay[v], c->slots[slot_of[v]], Ps[v], v, cur, cnt);
        d.open_list = Wk.open_list;
        d.open_count = Wk.open_count;
        const size_t px = (size_t)vc.width * vc.height;
        auto carve = [&](size_t bytes) {
            uint8_t *p = cur;
            cur += align256(bytes);
            return p;
        };
        if (host_out || lio.scratch_out) {
            host_stage[v] = carve(px * 3);
            d.out = host_stage[v];
            d.out_pitch = (int64_t)vc.width * 3;
        } else {
            d.out = (uint8_t *)outs[v];
            d.out_pitch = pitches[v];
        }
        if (learned[v]) {
            d.stack_w = (int32_t)stack_w(vc.width);
            d.stack_h = (int32_t)stack_w(vc.height);
            if (lio.stack_out) d.stack = lio.stack_out + (size_t)v * stack_bytes(vc.width, vc.height) / 2;
        }
        if (v == tv) {
            d.dbg_tiles = c->dbg_tiles;
            d.dbg_z = c->dbg_z;
            d.dbg_zf = c->dbg_zf;
            if (d.layered) {
                d.dbg_bz = c->dbg_bz;
                d.dbg_bzf = c->dbg_bzf;
            }
            d.dbg_rgba = c->dbg_rgba;
            d.dbg_depth = c->dbg_depth;
        }
    }
    // network batches: contiguous stacks, output table after the descriptors
    unet_out *ht = (unet_out *)(hd + n_views);
    std::vector<int> batch_first;
    int n_tab = 0;
    for (const NetBatch &b : batches) {
        batch_first.push_back(n_tab);
        const size_t sb = stack_bytes(b.W, b.H);
        uint8_t *base = cur;
        cur += align256(sb * b.views.size());
        for (size_t q = 0; q < b.views.size(); ++q) {
            fvv_view_desc &d = hd[b.views[q]];
            d.stack = (uint16_t *)(base + q * sb);
            ht[n_tab++] = unet_out{d.out, d.out_pitch, d.H, d.W, 0};
        }
    }
    bool waited[2] = {false, false};
    for (int v = 0; v < n_views; ++v)
        if (!waited[slot_of[v]]) {
            // a stream's own earlier work is ordered already
            if (c->slots[slot_of[v]].ready_stream != s)
                HIPCHECK(c, hipStreamWaitEvent(s, c->slots[slot_of[v]].ready, 0));
            waited[slot_of[v]] = true;
        }
    if (Wk.dirty) {
        HIPCHECK(c, hipMemsetAsync(Wk.counts, 0, Wk.counts_cap * 4, s));
        Wk.dirty = false;
    }
    const hipError_t le = fvv_launch_synthesis(Wk.h_desc_dev[r], Wk.d_desc, dims, n_tab * sizeof(unet_out), s,
                                               c->profiling ? &c->prof : nullptr);
    if (le != hipSuccess) {
        Wk.dirty = true;
        return fail(c, FVV_E_DEVICE, "synthesis launch failed: %s", hipGetErrorString(le));
    }
    if (!batches.empty()) {
        fvv_prof *prof = c->profiling ? &c->prof : nullptr;
        const unet_out *dt = (const unet_out *)(Wk.d_desc + n_views);
        for (size_t bi = 0; bi < batches.size(); ++bi) {
            const NetBatch &b = batches[bi];
            std::string err;
            hipEvent_t e0;
            fvv_prof_begin(prof, s, e0);
            const hipError_t e = unet_forward_batch(c->net, lio.act, hd[b.views[0]].stack, (int)b.views.size(), b.H,
                                                    b.W, dt + batch_first[bi], s, err, taps);
            fvv_prof_end(prof, s, FVV_ST_NET, e0);
            if ((rc = net_status(c, e, err, "network forward"))) return rc;
        }
    }
    HIPCHECK(c, hipEventRecord(Wk.h_ev[r], s));
    Wk.h_live[r] = true;
    for (int q = 0; q < 2; ++q)
        if (waited[q] && (rc = note_reader(c, c->slots[q], s))) return rc;
    if (host_out && !lio.scratch_out) {
        // caller's (pageable) host memory: through the pinned bounce buffer
        for (int v = 0; v < n_views; ++v) {
            const size_t row = (size_t)virts[v].width * 3;
            if ((rc = to_host(c, (uint8_t *)outs[v], pitches[v], host_stage[v], (int64_t)row, row,
                              (size_t)virts[v].height, s)))
                return rc;
        }
    }
    return FVV_OK;
}

int32_t synthesize_impl(fvv_ctx *c, const fvv_camera *virts, int n_views, const fvv_synth_params *params,
                        void *const *outs, const int64_t *pitches, int32_t mem_kind, void *stream)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!virts || n_views < 1 || !outs || !pitches) return fail(c, FVV_E_ARG, "null argument or n_views < 1");
    if (mem_kind != FVV_MEM_HOST && mem_kind != FVV_MEM_DEVICE) return fail(c, FVV_E_ARG, "bad mem_kind");
    if (c->rig.empty()) return fail(c, FVV_E_STATE, "no rig set");
    fvv_synth_params P;
    int32_t rc = resolve_params(c, params, P);
    if (rc) return rc;
    int si;
    if ((rc = find_slot(c, P.frame_version, si))) return rc;
    for (int v = 0; v < n_views; ++v) {
        if ((rc = check_camera(c, virts[v], false, "virtual camera"))) return rc;
        if (!outs[v]) return fail(c, FVV_E_ARG, "outs[%d] is null", v);
        if (pitches[v] < (int64_t)virts[v].width * 3) return fail(c, FVV_E_ARG, "pitches[%d] too small", v);
    }
    DeviceGuard g(c->device);
    std::vector<fvv_synth_params> Ps(n_views, P);
    LearnedIO lio;
    lio.act = c->act;
    const hipStream_t s = (hipStream_t)stream;
    if ((rc = order_direct(c, s))) return rc;
    rc = launch_views(c, c->user, virts, Ps.data(), n_views, outs, pitches, mem_kind == FVV_MEM_HOST, s, true,
                      c->debug, lio);
    const int32_t rm = mark_direct(c, s);
    if (rc) return rc;
    if (rm) return rm;
    c->have_taps = c->debug && c->debug_view < n_views;
    if (c->have_taps) {
        const fvv_camera &tvc = virts[c->debug_view];
        c->last_px = (int64_t)tvc.width * tvc.height;
        c->last_tiles = (int64_t)((tvc.width + FVV_TILE - 1) / FVV_TILE) * ((tvc.height + FVV_TILE - 1) / FVV_TILE);
    }
    c->last_layered = P.path == FVV_PATH_LAYERED;
    return FVV_OK;
}

// ---------------------------------------------------------------- server
// Upper bound of the workspace one request can need (any K cameras of the rig).
void request_bounds(const fvv_ctx *c, const fvv_camera &v, int k, bool learned, bool layered, size_t &bytes,
                    size_t &tiles)
{
    std::vector<int> nb;
    for (const auto &cam : c->rig) nb.push_back(nblocks(cam));
    std::sort(nb.rbegin(), nb.rend());
    const int K = std::min<int>({k, (int)nb.size(), FVV_MAX_K});
    ViewLayout L;
    layout_sizes(L, v.width, v.height, nb.data(), K, layered);
    bytes = view_ws_bytes(v.width, v.height, L, false, learned);
    tiles = (size_t)L.n_tiles;
}

void finish(Server *S, const Request &r, int32_t status, double latency)
{
    std::lock_guard<std::mutex> lk(S->dmu);
    Result &res = S->results[r.ticket];
    res.done = true;
    res.status = status;
    res.latency = latency;
    if (status == FVV_OK) {
        ++S->n_done;
        S->pixels += (uint64_t)r.cam.width * r.cam.height;
    } else {
        ++S->n_failed;
    }
}

// Continuous batching: whenever one of the two step workspaces is free, the
// pending requests are admitted in arrival order while step slots and
// workspace memory last, and launched as one batch on that workspace's
// stream; the other workspace's step may still be running.
void scheduler(fvv_ctx *c)
{
    Server *S = c->server;
    for (;;) {
        std::vector<Request> batch;
        int w = -1;
        {
            std::unique_lock<std::mutex> lk(S->qmu);
            S->qcv.wait(lk, [&] { return (S->stop && S->pending.empty()) ||
                                         (!S->pending.empty() && (!S->paused || S->stop) &&
                                          (!S->busy[0] || !S->busy[1])); });
            if (S->pending.empty()) break;
            w = S->busy[0] ? 1 : 0;
            size_t bytes = 0, tiles = 0;
            while (!S->pending.empty() && (int)batch.size() < S->max_slots) {
                Request &r = S->pending.front();
                if (r.bytes > S->step_bytes || r.tiles > S->step_tiles) {
                    Request bad = r;
                    S->pending.pop_front();
                    lk.unlock();
                    finish(S, bad, FVV_E_NOMEM, 0.0);
                    lk.lock();
                    continue;
                }
                if (bytes + r.bytes > S->step_bytes || tiles + r.tiles > S->step_tiles) break;
                bytes += r.bytes;
                tiles += r.tiles;
                batch.push_back(r);
                S->pending.pop_front();
            }
            if (batch.empty()) continue;
            S->busy[w] = true;
        }
        int32_t rc;
        {
            std::lock_guard<std::mutex> lk(c->mu);
            DeviceGuard g(c->device);
            std::vector<fvv_camera> cams;
            std::vector<fvv_synth_params> Ps;
            std::vector<void *> outs;
            std::vector<int64_t> pitches;
            for (auto &r : batch) {
                cams.push_back(r.cam);
                Ps.push_back(r.P);
                outs.push_back(r.out);
                pitches.push_back(r.pitch);
            }
            LearnedIO lio;
            lio.act = S->act[w];
            rc = launch_views(c, S->ws[w], cams.data(), Ps.data(), (int)batch.size(), outs.data(), pitches.data(),
                              false, S->stream[w], false, false, lio);
            if (rc == FVV_OK && hipEventRecord(S->done_ev[w], S->stream[w]) != hipSuccess) rc = FVV_E_DEVICE;
        }
        if (rc != FVV_OK) {
            for (auto &r : batch) finish(S, r, rc, 0.0);
            std::lock_guard<std::mutex> lk(S->qmu);
            S->busy[w] = false;
            S->qcv.notify_all();
            continue;
        }
        {
            std::lock_guard<std::mutex> lk(S->cmu[w]);
            S->inflight[w] = std::move(batch);
            S->launched[w] = true;
            S->launch_t[w] = Clock::now();
        }
        S->ccv[w].notify_all();
    }
    for (int w = 0; w < 2; ++w) {
        std::lock_guard<std::mutex> lk(S->cmu[w]);
        S->ccv[w].notify_all();
    }
}

// Completion of workspace w's steps: wait for the step's event, stamp every
// request of the step (latency = completion - submission, host clock) and
// hand the workspace back to the scheduler.
void completer(fvv_ctx *c, int w)
{
    Server *S = c->server;
    for (;;) {
        std::vector<Request> batch;
        Clock::time_point t0;
        {
            std::unique_lock<std::mutex> lk(S->cmu[w]);
            S->ccv[w].wait(lk, [&] {
                if (S->launched[w]) return true;
                std::lock_guard<std::mutex> q(S->qmu);
                return S->stop && S->pending.empty() && !S->busy[w];
            });
            if (!S->launched[w]) break;
            batch = std::move(S->inflight[w]);
            S->launched[w] = false;
            t0 = S->launch_t[w];
        }
        int32_t status = FVV_OK;
        {
            DeviceGuard g(c->device);
            if (hipEventSynchronize(S->done_ev[w]) != hipSuccess) status = FVV_E_DEVICE;
        }
        const Clock::time_point t = Clock::now();
        for (auto &r : batch) finish(S, r, status, std::chrono::duration<double>(t - r.arrive).count());
        {
            std::lock_guard<std::mutex> lk(S->dmu);
            ++S->n_steps;
            S->batch_sum += batch.size();
            S->busy_s += std::chrono::duration<double>(t - t0).count();
        }
        {
            std::lock_guard<std::mutex> lk(S->qmu);
            S->busy[w] = false;
        }
        S->qcv.notify_all();
        for (int o = 0; o < 2; ++o) S->ccv[o].notify_all();
    }
}

void server_teardown(fvv_ctx *c)
{
    Server *S = c->server;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->qmu);
        S->stop = true;
    }
    S->qcv.notify_all();
    if (S->sched.joinable()) S->sched.join();
    for (int w = 0; w < 2; ++w) {
        {
            std::lock_guard<std::mutex> lk(S->cmu[w]);
        }
        S->ccv[w].notify_all();
        if (S->compl_[w].joinable()) S->compl_[w].join();
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    for (int w = 0; w < 2; ++w) {
        if (S->stream[w]) {
            (void)hipStreamSynchronize(S->stream[w]);
            for (auto &slot : c->slots) {
                auto &rd = slot.readers;
                for (size_t e = 0; e < rd.size();)
                    if (rd[e].first == S->stream[w]) {
                        c->event_pool.push_back(rd[e].second);
                        rd.erase(rd.begin() + e);
                    } else {
                        ++e;
                    }
            }
            (void)hipStreamDestroy(S->stream[w]);
        }
        if (S->done_ev[w]) (void)hipEventDestroy(S->done_ev[w]);
        ws_release(c, S->ws[w]);
        const size_t ab = unet_act_bytes(S->act[w]);
        c->allocated -= std::min<uint64_t>(ab, c->allocated);
        c->net_bytes -= std::min<uint64_t>(ab, c->net_bytes);
        unet_act_free(S->act[w]);
    }
    delete S;
    c->server = nullptr;
}

}  // namespace

// Device scratch of fvv_synthesize_noalloc, one instance per GPU (each device
// holds its own copy at its own address until the process ends).  In host
// code `scratch` names a host-side stand-in: host code uses only the device
// address hipGetSymbolAddress returns, kept per device below.
static __device__ __align__(256) uint8_t scratch[FVV_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device dev, looked up once per device with
// that device current (at context creation).
int32_t scratch_address(int dev, uint8_t **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        DeviceGuard g(dev);
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(nullptr, FVV_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        }
        g_scratch[dev] = (uint8_t *)p;
    }
    *out = g_scratch[dev];
    return FVV_OK;
}

}  // namespace

extern "C" {

int32_t fvv_abi_version(void) { return FVV_ABI_VERSION; }

int32_t fvv_create(int32_t hip_device, uint64_t mem_budget_bytes, fvv_ctx **out)
{
    if (!out) return fail(nullptr, FVV_E_ARG, "out is null");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return fail(nullptr, FVV_E_DEVICE, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (hip_device < 0 || hip_device >= n)
        return fail(nullptr, FVV_E_ARG, "device %d outside 0..%d", hip_device, n - 1);
    if (hip_device >= kMaxDevices) return fail(nullptr, FVV_E_UNSUPPORTED, "device %d beyond %d", hip_device, kMaxDevices);
    uint8_t *scr = nullptr;
    const int32_t rc = scratch_address(hip_device, &scr);
    if (rc) return rc;
    fvv_ctx *c = new (std::nothrow) fvv_ctx();
    if (!c) return fail(nullptr, FVV_E_NOMEM, "out of host memory");
    c->device = hip_device;
    c->scratch = scr;
    c->budget = mem_budget_bytes;
    *out = c;
    return FVV_OK;
}

void fvv_destroy(fvv_ctx *c)
{
    if (!c) return;
    server_teardown(c);
    {
        std::lock_guard<std::mutex> lk(c->mu);
        DeviceGuard g(c->device);
        (void)hipDeviceSynchronize();
        if (!c->rig.empty()) release_frames(c);
        for (auto &s : c->slots)
            if (s.ready) (void)hipEventDestroy(s.ready);
        dfree(c, c->staging, c->staging_bytes);
        if (c->staging_free) (void)hipEventDestroy(c->staging_free);
        if (c->bounce) (void)hipHostFree(c->bounce);
        for (hipEvent_t e : c->bounce_ev)
            if (e) (void)hipEventDestroy(e);
        ws_release(c, c->user);
        dfree(c, c->dbg_z, c->dbg_px * 8);
        dfree(c, c->dbg_zf, c->dbg_px * 8);
        dfree(c, c->dbg_bz, c->dbg_px * 8);
        dfree(c, c->dbg_bzf, c->dbg_px * 8);
        dfree(c, c->dbg_rgba, c->dbg_px * 4);
        dfree(c, c->dbg_depth, c->dbg_px * 4);
        dfree(c, c->dbg_tiles, c->dbg_tiles_n * sizeof(int2));
        release_bg(c);
        dfree(c, c->jbf, (FVV_JBF_WS + FVV_JBF_WC) * 4);
        for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
        for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
        if (c->last_ev) (void)hipEventDestroy(c->last_ev);
        unet_act_free(c->act);
        unet_free(c->net);
    }
    delete c;
}

const char *fvv_last_error(const fvv_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int32_t fvv_set_rig(fvv_ctx *c, const fvv_camera *cams, int32_t n)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->server) return fail(c, FVV_E_STATE, "stop the server before changing the rig");
    if (!cams || n < 1 || n > FVV_MAX_CAMERAS) return fail(c, FVV_E_ARG, "rig size %d outside 1..%d", n, FVV_MAX_CAMERAS);
    for (int k = 0; k < n; ++k) {
        int32_t rc = check_camera(c, cams[k], true, "rig camera");
        if (rc) return rc;
    }
    DeviceGuard g(c->device);
    HIPCHECK(c, hipDeviceSynchronize());
    if (!c->rig.empty()) release_frames(c);
    release_bg(c);
    c->rig.assign(cams, cams + n);
    return FVV_OK;
}

int32_t fvv_set_bg_model(fvv_ctx *c, const void *const *depth_mm, const int64_t *pitches, int32_t n,
                         int32_t mem_kind, void *stream)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->server) return fail(c, FVV_E_STATE, "stop the server before changing the background models");
    if (c->rig.empty()) return fail(c, FVV_E_STATE, "no rig set");
    if (mem_kind != FVV_MEM_HOST && mem_kind != FVV_MEM_DEVICE) return fail(c, FVV_E_ARG, "bad mem_kind");
    if (depth_mm && (n != (int)c->rig.size() || !pitches))
        return fail(c, FVV_E_ARG, "need one model (or NULL) per rig camera (%zu) and their pitches", c->rig.size());
    if (depth_mm)
        for (int k = 0; k < n; ++k) {
            if (!depth_mm[k]) continue;
            if (pitches[k] < 2 * (int64_t)c->rig[k].width || pitches[k] % 2 || ((uintptr_t)depth_mm[k] & 1))
                return fail(c, FVV_E_ARG, "model %d: rows must be 2-byte aligned and hold width values", k);
        }
    DeviceGuard g(c->device);
    HIPCHECK(c, hipDeviceSynchronize());
    // resident frame sets lose their layers: the next upload rebuilds them
    release_frames(c);
    release_bg(c);
    if (!depth_mm) return FVV_OK;
    c->bg_model.assign(n, nullptr);
    c->has_bg = true;
    hipStream_t s = (hipStream_t)stream;
    for (int k = 0; k < n; ++k) {
        if (!depth_mm[k]) continue;
        const int W = c->rig[k].width, H = c->rig[k].height;
        int32_t rc = dalloc(c, (void **)&c->bg_model[k], (size_t)W * H * 2);
        if (rc) return rc;
        if (mem_kind == FVV_MEM_HOST)
            HIPCHECK(c, hipMemcpy2D(c->bg_model[k], (size_t)W * 2, depth_mm[k], pitches[k], (size_t)W * 2, H,
                                    hipMemcpyHostToDevice));
        else
            HIPCHECK(c, hipMemcpy2DAsync(c->bg_model[k], (size_t)W * 2, depth_mm[k], pitches[k], (size_t)W * 2, H,
                                         hipMemcpyDeviceToDevice, s));
    }
    HIPCHECK(c, hipStreamSynchronize(s));
    // models are set rarely: finish every copy (a pageable host copy may
    // still be in flight on return) before any stream's ingest reads them
    HIPCHECK(c, hipDeviceSynchronize());
    return FVV_OK;
}

int32_t fvv_upload_mvd(fvv_ctx *c, const fvv_view *views, int32_t n, int32_t mem_kind, void *stream,
                       uint64_t *out_version)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->rig.empty()) return fail(c, FVV_E_STATE, "no rig set");
    if (!views || n != (int)c->rig.size()) return fail(c, FVV_E_ARG, "need one view per rig camera (%zu)", c->rig.size());
    if (mem_kind != FVV_MEM_HOST && mem_kind != FVV_MEM_DEVICE) return fail(c, FVV_E_ARG, "bad mem_kind");
    const bool y12 = c->depth_format == FVV_DEPTH_Y12;
    // staged depth plane: uint16 rows, or an I420 image (Y, then U and V)
    auto depth_bytes = [y12](int W, int H) { return y12 ? (size_t)W * H * 3 / 2 : (size_t)W * H * 2; };
    size_t need = 0;
    int n_present = 0;
    for (int k = 0; k < n; ++k) {
        const fvv_view &v = views[k];
        const fvv_camera &cam = c->rig[k];
        if (!v.rgb && !v.depth_mm) continue;
        if (!v.rgb || !v.depth_mm) return fail(c, FVV_E_ARG, "view %d: rgb and depth must both be given", k);
        if (y12) {
            if (cam.width % 2 || cam.height % 2)
                return fail(c, FVV_E_ARG, "view %d: 12-bit coded depth needs even width and height", k);
            if (v.rgb_pitch < (int64_t)cam.width * 3 || v.depth_pitch < (int64_t)cam.width || v.depth_pitch % 2)
                return fail(c, FVV_E_ARG, "view %d: pitch too small (or odd I420 luma pitch)", k);
        } else {
            if (v.rgb_pitch < (int64_t)cam.width * 3 || v.depth_pitch < (int64_t)cam.width * 2)
                return fail(c, FVV_E_ARG, "view %d: pitch too small", k);
            if (v.depth_pitch % 2 || ((uintptr_t)v.depth_mm & 1))
                return fail(c, FVV_E_ARG, "view %d: depth must be 2-byte aligned (pointer and pitch)", k);
        }
        need += align256((size_t)cam.width * cam.height * 3) + align256(depth_bytes(cam.width, cam.height));
        ++n_present;
    }
    if (n_present == 0) return fail(c, FVV_E_ARG, "no camera present in the upload");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const bool host = mem_kind == FVV_MEM_HOST;
    const int dst = c->latest < 0 ? 0 : 1 - c->latest;
    FrameSlot &fs = c->slots[dst];
    int32_t rc = ensure_frame_slot(c, fs);
    if (rc) return rc;
    if (host && c->staging_bytes < need) {
        HIPCHECK(c, hipDeviceSynchronize());
        dfree(c, c->staging, c->staging_bytes);
        c->staging = nullptr;
        c->staging_bytes = 0;
        if ((rc = dalloc(c, (void **)&c->staging, need))) return rc;
        c->staging_bytes = need;
    }
    if (!c->staging_free) HIPCHECK(c, hipEventCreateWithFlags(&c->staging_free, hipEventDisableTiming));
    else if (host) HIPCHECK(c, hipStreamWaitEvent(s, c->staging_free, 0));
    for (auto &r : fs.readers)
        if (r.first != s) HIPCHECK(c, hipStreamWaitEvent(s, r.second, 0));
    // device memory is read in place by the repack kernel; host memory is
    // first copied into the staging buffer, with blocking copies from the
    // caller's pageable memory once the stream is idle
    if (host) HIPCHECK(c, hipStreamSynchronize(s));
    fvv_repack_batch b{};
    int max_w = 0, max_h = 0;
    uint8_t *cur = c->staging;
    for (int k = 0; k < n; ++k) {
        const fvv_view &v = views[k];
        const fvv_camera &cam = c->rig[k];
        fs.present[k] = (v.rgb && v.depth_mm) ? 1 : 0;
        if (!fs.present[k]) continue;
        const int W = cam.width, H = cam.height;
        fvv_repack_cam &rc_ = b.cam[b.n++];
        if (host) {
            uint8_t *rgb = cur;
            cur += align256((size_t)W * H * 3);
            uint8_t *dep = cur;
            cur += align256(depth_bytes(W, H));
            HIPCHECK(c, hipMemcpy2D(rgb, (size_t)W * 3, v.rgb, v.rgb_pitch, (size_t)W * 3, H,
                                    hipMemcpyHostToDevice));
            if (y12) {
                // Y rows, then the U and V planes at half the pitch
                const uint8_t *src = (const uint8_t *)v.depth_mm;
                const int64_t sp = v.depth_pitch, up = sp / 2;
                HIPCHECK(c, hipMemcpy2D(dep, (size_t)W, src, sp, (size_t)W, H, hipMemcpyHostToDevice));
                HIPCHECK(c, hipMemcpy2D(dep + (size_t)W * H, (size_t)W / 2, src + (int64_t)H * sp, up, (size_t)W / 2,
                                        H, hipMemcpyHostToDevice));
                rc_.depth_pitch = W;
            } else {
                HIPCHECK(c, hipMemcpy2D(dep, (size_t)W * 2, v.depth_mm, v.depth_pitch, (size_t)W * 2, H,
                                        hipMemcpyHostToDevice));
                rc_.depth_pitch = (int64_t)W * 2;
            }
            rc_.rgb = rgb;
            rc_.rgb_pitch = (int64_t)W * 3;
            rc_.depth = dep;
        } else {
            rc_.rgb = (const uint8_t *)v.rgb;
            rc_.rgb_pitch = v.rgb_pitch;
            rc_.depth = (const uint8_t *)v.depth_mm;
            rc_.depth_pitch = v.depth_pitch;
        }
        rc_.texel_out = fs.texel[k];
        rc_.depth_out = fs.depth[k];
        if (fs.layered) {
            rc_.bg_model = c->bg_model[k];
            rc_.bg_texel_out = fs.bg_texel[k];
            rc_.bg_depth_out = fs.bg_depth[k];
        }
        rc_.W = W;
        rc_.H = H;
        rc_.alpha = cam.depth_alpha;
        rc_.beta = cam.depth_beta;
        max_w = std::max(max_w, W);
        max_h = std::max(max_h, H);
    }
    b.y12 = y12;
    if (y12) b.planes = y12_make_planes(c->z_near, c->z_far);
    if (c->jbf_on) {
        b.jbf = c->jbf;
        b.jbf_radius = c->jbf_radius;
        b.jbf_min = c->jbf_min;
    }
    HIPCHECK(c, fvv_launch_repack(b, max_w, max_h, s, c->profiling ? &c->prof : nullptr));
    if (host) HIPCHECK(c, hipEventRecord(c->staging_free, s));
    HIPCHECK(c, hipEventRecord(fs.ready, s));
    fs.ready_stream = s;
    if (mem_kind == FVV_MEM_HOST) HIPCHECK(c, hipStreamSynchronize(s));
    fs.version = c->next_version++;
    c->latest = dst;
    if (out_version) *out_version = fs.version;
    return FVV_OK;
}

int32_t fvv_set_prefilter(fvv_ctx *c, int32_t enable, int32_t radius, float sigma_s, float sigma_c,
                          int32_t min_valid)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!enable) {
        c->jbf_on = false;
        return FVV_OK;
    }
    if (radius < 1 || radius > 3) return fail(c, FVV_E_ARG, "pre-filter radius %d outside 1..3", radius);
    if (!(std::isfinite(sigma_s) && sigma_s > 0.f && std::isfinite(sigma_c) && sigma_c > 0.f))
        return fail(c, FVV_E_ARG, "pre-filter sigmas must be finite and > 0");
    const int n = 2 * radius + 1;
    if (min_valid < 1 || min_valid > n * n - 1)
        return fail(c, FVV_E_ARG, "pre-filter min_valid %d outside 1..%d", min_valid, n * n - 1);
    // weight tables: 12-bit integers of the spatial and range Gaussians
    uint32_t t[FVV_JBF_WS + FVV_JBF_WC] = {};
    for (int dy = -radius; dy <= radius; ++dy)
        for (int dx = -radius; dx <= radius; ++dx) {
            const double e = std::exp(-(double)(dx * dx + dy * dy) / (2.0 * (double)sigma_s * (double)sigma_s));
            t[(dy + radius) * n + dx + radius] = (uint32_t)std::floor(4096.0 * e + 0.5);
        }
    for (int d = 0; d < FVV_JBF_WC; ++d) {
        const double e = std::exp(-(double)d * (double)d / (2.0 * (double)sigma_c * (double)sigma_c));
        t[FVV_JBF_WS + d] = (uint32_t)std::floor(4096.0 * e + 0.5);
    }
    DeviceGuard g(c->device);
    int32_t rc;
    if (!c->jbf && (rc = dalloc(c, (void **)&c->jbf, sizeof t))) return rc;
    HIPCHECK(c, hipDeviceSynchronize());
    HIPCHECK(c, hipMemcpy(c->jbf, t, sizeof t, hipMemcpyHostToDevice));
    c->jbf_radius = radius;
    c->jbf_min = min_valid;
    c->jbf_on = true;
    return FVV_OK;
}

int32_t fvv_read_frame_depth(fvv_ctx *c, int32_t cam, int32_t layer, uint64_t version, void *host_out,
                             int64_t bytes)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!host_out) return fail(c, FVV_E_ARG, "host_out is null");
    if (cam < 0 || cam >= (int)c->rig.size()) return fail(c, FVV_E_ARG, "camera %d outside the rig", cam);
    if (layer != 0 && layer != 1) return fail(c, FVV_E_ARG, "layer must be 0 (live / foreground) or 1 (background)");
    int si;
    int32_t rc = find_slot(c, version, si);
    if (rc) return rc;
    const FrameSlot &fs = c->slots[si];
    if (!fs.present[cam]) return fail(c, FVV_E_STATE, "camera %d is absent from that frame set", cam);
    if (layer == 1 && !fs.layered) return fail(c, FVV_E_STATE, "that frame set has no background layers");
    const int64_t need = (int64_t)c->rig[cam].width * c->rig[cam].height * 4;
    if (bytes != need) return fail(c, FVV_E_ARG, "the plane holds %lld bytes, asked %lld", (long long)need,
                                   (long long)bytes);
    DeviceGuard g(c->device);
    HIPCHECK(c, hipDeviceSynchronize());
    const size_t row = (size_t)c->rig[cam].width * 4;
    return to_host(c, (uint8_t *)host_out, (int64_t)row, (const uint8_t *)(layer ? fs.bg_depth[cam] : fs.depth[cam]),
                   (int64_t)row, row, (size_t)c->rig[cam].height, nullptr);
}

int32_t fvv_set_depth_format(fvv_ctx *c, int32_t format, float z_near, float z_far)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (format == FVV_DEPTH_MM16) {
        c->depth_format = format;
        return FVV_OK;
    }
    if (format != FVV_DEPTH_Y12) return fail(c, FVV_E_ARG, "unknown depth format %d", format);
    if (!(std::isfinite(z_near) && std::isfinite(z_far) && z_near > 0.f && z_near < z_far))
        return fail(c, FVV_E_ARG, "clipping planes need 0 < z_near < z_far (finite)");
    c->depth_format = format;
    c->z_near = z_near;
    c->z_far = z_far;
    return FVV_OK;
}

namespace {

// arguments shared by the standalone encoder and decoder
int32_t check_y12_args(const void *a, const void *b, int32_t W, int32_t H, float zn, float zf, int64_t ypitch,
                       int64_t dpitch)
{
    if (!a || !b) return fail(nullptr, FVV_E_ARG, "null buffer");
    if (W < 2 || H < 2 || W % 2 || H % 2 || (int64_t)W * H > FVV_MAX_SRC_PIXELS || H > 65536)
        return fail(nullptr, FVV_E_ARG, "width and height must be even, >= 2, with width*height <= %d",
                    FVV_MAX_SRC_PIXELS);
    if (ypitch < W || ypitch % 2) return fail(nullptr, FVV_E_ARG, "I420 luma pitch must be even and >= width");
    if (dpitch < 2 * (int64_t)W || dpitch % 2 || ((uintptr_t)b & 1))
        return fail(nullptr, FVV_E_ARG, "depth rows must be 2-byte aligned and hold width values");
    if (!(std::isfinite(zn) && std::isfinite(zf) && zn > 0.f && zn < zf))
        return fail(nullptr, FVV_E_ARG, "clipping planes need 0 < z_near < z_far (finite)");
    return FVV_OK;
}

}  // namespace

namespace {

int32_t y12_batch(int32_t n, const void *const *depth_mm, const int64_t *depth_pitch, int32_t W, int32_t H,
                  float zn, float zf, void *const *yuv, const int64_t *y_pitch, bool encode, void *stream)
{
    if (n < 1 || n > FVV_MAX_RIG || !depth_mm || !depth_pitch || !yuv || !y_pitch)
        return fail(nullptr, FVV_E_ARG, "need 1..%d images and their pointer and pitch arrays", FVV_MAX_RIG);
    fvv_y12_batch b{};
    b.n = n;
    b.W = W;
    b.H = H;
    b.planes = y12_make_planes(zn, zf);
    for (int i = 0; i < n; ++i) {
        int32_t rc = check_y12_args(yuv[i], depth_mm[i], W, H, zn, zf, y_pitch[i], depth_pitch[i]);
        if (rc) return rc;
        b.mm[i] = (const uint8_t *)depth_mm[i];
        b.mm_pitch[i] = depth_pitch[i];
        b.yuv[i] = (uint8_t *)yuv[i];
        b.yuv_pitch[i] = y_pitch[i];
    }
    hipError_t e = fvv_launch_y12(b, encode, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, FVV_E_DEVICE, "coding launch: %s", hipGetErrorString(e));
    return FVV_OK;
}

}  // namespace

int32_t fvv_depth_encode_y12(const void *depth_mm, int64_t depth_pitch, int32_t width, int32_t height, float z_near,
                             float z_far, void *yuv, int64_t y_pitch, void *stream)
{
    return y12_batch(1, &depth_mm, &depth_pitch, width, height, z_near, z_far, &yuv, &y_pitch, true, stream);
}

int32_t fvv_depth_decode_y12(const void *yuv, int64_t y_pitch, int32_t width, int32_t height, float z_near,
                             float z_far, void *depth_mm, int64_t depth_pitch, void *stream)
{
    const void *mm = depth_mm;
    void *y = const_cast<void *>(yuv);
    return y12_batch(1, &mm, &depth_pitch, width, height, z_near, z_far, &y, &y_pitch, false, stream);
}

int32_t fvv_depth_encode_y12_batch(int32_t n, const void *const *depth_mm, const int64_t *depth_pitch, int32_t width,
                                   int32_t height, float z_near, float z_far, void *const *yuv, const int64_t *y_pitch,
                                   void *stream)
{
    return y12_batch(n, depth_mm, depth_pitch, width, height, z_near, z_far, yuv, y_pitch, true, stream);
}

int32_t fvv_depth_decode_y12_batch(int32_t n, const void *const *yuv, const int64_t *y_pitch, int32_t width,
                                   int32_t height, float z_near, float z_far, void *const *depth_mm,
                                   const int64_t *depth_pitch, void *stream)
{
    return y12_batch(n, (const void *const *)depth_mm, depth_pitch, width, height, z_near, z_far,
                     (void *const *)yuv, y_pitch, false, stream);
}

int32_t fvv_synthesize(fvv_ctx *c, const fvv_camera *virt, const fvv_synth_params *params, void *out_rgb8,
                       int64_t out_pitch, int32_t mem_kind, void *stream)
{
    void *outs[1] = {out_rgb8};
    int64_t pitches[1] = {out_pitch};
    return synthesize_impl(c, virt, 1, params, outs, pitches, mem_kind, stream);
}

int32_t fvv_synthesize_batch(fvv_ctx *c, const fvv_camera *virts, int32_t n_views, const fvv_synth_params *params,
                             void *const *outs, const int64_t *pitches, int32_t mem_kind, void *stream)
{
    return synthesize_impl(c, virts, n_views, params, outs, pitches, mem_kind, stream);
}

int32_t fvv_synthesize_noalloc(fvv_ctx *c, const fvv_camera *virt, const fvv_synth_params *params, void *out_dev,
                               int64_t out_pitch, void *stream)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!virt || !out_dev) return fail(c, FVV_E_ARG, "null argument");
    if (c->rig.empty()) return fail(c, FVV_E_STATE, "no rig set");
    fvv_synth_params P;
    int32_t rc = resolve_params(c, params, P);
    if (rc) return rc;
    if (P.path == FVV_PATH_LEARNED)
        return fail(c, FVV_E_UNSUPPORTED, "the learned path needs network activation memory: use fvv_synthesize");
    if ((rc = check_camera(c, *virt, false, "virtual camera"))) return rc;
    if (out_pitch < (int64_t)virt->width * 3) return fail(c, FVV_E_ARG, "out_pitch too small");
    int si;
    ViewLayout L;
    if ((rc = plan_view(c, *virt, P, si, L))) return rc;
    // scratch layout: open-tile count | descriptor | tile counters |
    // open-tile list | the view's buffers (as a workspace carves them)
    const size_t nt = (size_t)L.n_tiles;
    const size_t off_desc = 256;
    const size_t off_counts = off_desc + align256(sizeof(fvv_view_desc));
    const size_t off_open = off_counts + align256(nt * 4);
    const size_t off_view = off_open + align256(nt * sizeof(int2));
    const size_t need = off_view + view_ws_bytes(virt->width, virt->height, L, false);
    if (need > FVV_NOALLOC_SCRATCH_BYTES)
        return fail(c, FVV_E_NOMEM, "the view needs %zu bytes of scratch, more than the %llu bytes of the "
                    "no-allocation entry point", need, (unsigned long long)FVV_NOALLOC_SCRATCH_BYTES);
    DeviceGuard g(c->device);
    uint8_t *const base = c->scratch;
    fvv_view_desc d;
    uint8_t *cur = base + off_view;
    int32_t *cnt = (int32_t *)(base + off_counts);
    fill_desc(c, d, *virt, L, c->slots[si], P, 0, cur, cnt);
    d.open_count = (int32_t *)base;
    d.open_list = (int2 *)(base + off_open);
    d.out = (uint8_t *)out_dev;
    d.out_pitch = out_pitch;
    const fvv_batch_dims dims{1, L.nsrc, L.blk_stride, L.ntx, L.nty, L.n_tiles, P.fill_mode == FVV_FILL_BG, false,
                              P.path == FVV_PATH_LAYERED};
    const hipStream_t s = (hipStream_t)stream;
    if (c->slots[si].ready_stream != s) HIPCHECK(c, hipStreamWaitEvent(s, c->slots[si].ready, 0));
    const hipError_t le = fvv_launch_synthesis_one(d, (fvv_view_desc *)(base + off_desc),
                                                   (int32_t *)(base + off_counts), dims, s, nullptr);
    if (le != hipSuccess) return fail(c, FVV_E_DEVICE, "synthesis launch failed: %s", hipGetErrorString(le));
    return note_reader(c, c->slots[si], s);
}

int32_t fvv_measure_peaks(int32_t hip_device, double *out, int32_t n)
{
    if (!out || n < FVV_PEAKS) return fail(nullptr, FVV_E_ARG, "out needs %d entries", FVV_PEAKS);
    int nd = 0;
    hipError_t e = hipGetDeviceCount(&nd);
    if (e != hipSuccess) return fail(nullptr, FVV_E_DEVICE, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (hip_device < 0 || hip_device >= nd) return fail(nullptr, FVV_E_ARG, "device %d outside 0..%d", hip_device, nd - 1);
    DeviceGuard g(hip_device);
    for (int k = 0; k < FVV_PEAKS; ++k) out[k] = 0.0;
    std::string err;
    e = fvv_measure_peaks_impl(out, err);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(nullptr, e == hipErrorOutOfMemory ? FVV_E_NOMEM : FVV_E_DEVICE, "peak measurement%s%s: %s",
                    err.empty() ? "" : " ", err.c_str(), hipGetErrorString(e));
    }
    return FVV_PEAKS;
}

int32_t fvv_check_reciprocal(int32_t hip_device, int32_t e_lo, int32_t e_hi, uint64_t *mismatches)
{
    if (!mismatches) return fail(nullptr, FVV_E_ARG, "mismatches is null");
    if (e_lo < -125 || e_hi > 125 || e_lo > e_hi) return fail(nullptr, FVV_E_ARG, "binades %d..%d outside -125..125", e_lo, e_hi);
    int nd = 0;
    hipError_t e = hipGetDeviceCount(&nd);
    if (e != hipSuccess) return fail(nullptr, FVV_E_DEVICE, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (hip_device < 0 || hip_device >= nd) return fail(nullptr, FVV_E_ARG, "device %d outside 0..%d", hip_device, nd - 1);
    DeviceGuard g(hip_device);
    unsigned long long *bad = nullptr;
    if ((e = hipMalloc((void **)&bad, sizeof *bad)) != hipSuccess)
        return fail(nullptr, FVV_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
    unsigned long long h = 0;
    e = hipMemcpy(bad, &h, sizeof h, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = fvv_check_reciprocal_impl(e_lo, e_hi, bad, nullptr);
    if (e == hipSuccess) e = hipMemcpy(&h, bad, sizeof h, hipMemcpyDeviceToHost);
    (void)hipFree(bad);
    if (e != hipSuccess) return fail(nullptr, FVV_E_DEVICE, "reciprocal check: %s", hipGetErrorString(e));
    *mismatches = h;
    return FVV_OK;
}

int32_t fvv_check_bf16(int32_t hip_device, uint64_t *mismatches)
{
    if (!mismatches) return fail(nullptr, FVV_E_ARG, "mismatches is null");
    int nd = 0;
    hipError_t e = hipGetDeviceCount(&nd);
    if (e != hipSuccess) return fail(nullptr, FVV_E_DEVICE, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (hip_device < 0 || hip_device >= nd) return fail(nullptr, FVV_E_ARG, "device %d outside 0..%d", hip_device, nd - 1);
    DeviceGuard g(hip_device);
    unsigned long long *bad = nullptr;
    if ((e = hipMalloc((void **)&bad, sizeof *bad)) != hipSuccess)
        return fail(nullptr, FVV_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
    unsigned long long h = 0;
    e = hipMemcpy(bad, &h, sizeof h, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = unet_check_bf16(bad, nullptr);
    if (e == hipSuccess) e = hipMemcpy(&h, bad, sizeof h, hipMemcpyDeviceToHost);
    (void)hipFree(bad);
    if (e != hipSuccess) return fail(nullptr, FVV_E_DEVICE, "bfloat16 check: %s", hipGetErrorString(e));
    *mismatches = h;
    return FVV_OK;
}

int32_t fvv_select_cameras(const fvv_camera *rig, const int32_t *present, int32_t n, const fvv_camera *virt,
                           int32_t k, int32_t *idx, float *w)
{
    if (!rig || !virt || !idx || !w || n < 1 || n > FVV_MAX_CAMERAS || k < 1) return FVV_E_ARG;
    int32_t id[FVV_MAX_K];
    double wd[FVV_MAX_K];
    const int K = select_k(rig, present, n, *virt, k, id, wd);
    for (int e = 0; e < K; ++e) {
        idx[e] = id[e];
        w[e] = (float)wd[e];
    }
    return K;
}

int32_t fvv_tx_cameras(const fvv_camera *rig, int32_t n, const fvv_camera *views, int32_t n_views, int32_t n_tx,
                       uint32_t *mask)
{
    if (!rig || !mask || n < 1 || n > FVV_MAX_CAMERAS || n_tx < 1 || n_views < 0 || (n_views > 0 && !views))
        return FVV_E_ARG;
    uint32_t m = 0;
    for (int v = 0; v < n_views; ++v) tx_union(rig, n, views[v], n_tx, m);
    *mask = m;
    return popcount32(m);
}

int32_t fvv_pair_matrices(const fvv_camera *src, const fvv_camera *virt, float *out26)
{
    if (!src || !virt || !out26) return FVV_E_ARG;
    pair_dir(*src, *virt, out26, out26 + 9);
    pair_dir(*virt, *src, out26 + 12, out26 + 21);
    out26[24] = (float)((double)virt->fx / (double)src->fx);
    out26[25] = (float)((double)virt->fy / (double)src->fy);
    return FVV_OK;
}

static const char *k_stage_names[FVV_NSTAGES] = {"repack", "desc", "bin", "tile", "fill_open", "net", "net_train"};

int32_t fvv_set_profiling(fvv_ctx *c, int32_t enable)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    c->profiling = enable != 0;
    return FVV_OK;
}

int32_t fvv_stage_count(void) { return FVV_NSTAGES; }

const char *fvv_stage_name(int32_t stage)
{
    return (stage >= 0 && stage < FVV_NSTAGES) ? k_stage_names[stage] : nullptr;
}

int32_t fvv_profile_read(fvv_ctx *c, double *total_ms, int64_t *launches, int32_t n, int32_t reset)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!total_ms || !launches || n < FVV_NSTAGES) return fail(c, FVV_E_ARG, "need %d entries", FVV_NSTAGES);
    DeviceGuard g(c->device);
    for (auto &m : c->prof.marks) {
        HIPCHECK(c, hipEventSynchronize(m.second.second));
        float ms = 0.f;
        HIPCHECK(c, hipEventElapsedTime(&ms, m.second.first, m.second.second));
        c->prof.total_ms[m.first] += ms;
        c->prof.launches[m.first] += 1;
    }
    c->prof.marks.clear();
    c->prof.next = 0;
    for (int k = 0; k < FVV_NSTAGES; ++k) {
        total_ms[k] = c->prof.total_ms[k];
        launches[k] = c->prof.launches[k];
        if (reset) {
            c->prof.total_ms[k] = 0.0;
            c->prof.launches[k] = 0;
        }
    }
    return FVV_OK;
}

int32_t fvv_set_debug(fvv_ctx *c, int32_t enable)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    c->debug = enable != 0;
    return FVV_OK;
}

int32_t fvv_set_debug_view(fvv_ctx *c, int32_t view)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (view < 0) return fail(c, FVV_E_ARG, "view %d < 0", view);
    c->debug_view = view;
    return FVV_OK;
}

int32_t fvv_debug_read(fvv_ctx *c, int32_t tap, void *host_out, int64_t bytes)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!host_out) return fail(c, FVV_E_ARG, "host_out is null");
    if (!c->have_taps) return fail(c, FVV_E_STATE, "no debug taps: enable with fvv_set_debug before synthesis");
    DeviceGuard g(c->device);
    const void *src = nullptr;
    int64_t need = 0;
    switch (tap) {
    case FVV_TAP_Z_RAW: src = c->dbg_z; need = c->last_px * 8; break;
    case FVV_TAP_Z_FILT: src = c->dbg_zf; need = c->last_px * 8; break;
    case FVV_TAP_BLEND: src = c->dbg_rgba; need = c->last_px * 4; break;
    case FVV_TAP_DEPTH: src = c->dbg_depth; need = c->last_px * 4; break;
    case FVV_TAP_TILES: src = c->dbg_tiles; need = c->last_tiles * 8; break;
    case FVV_TAP_BG_Z_RAW:
    case FVV_TAP_BG_Z_FILT:
        if (!c->last_layered) return fail(c, FVV_E_STATE, "background-layer taps need a layered synthesis");
        src = tap == FVV_TAP_BG_Z_RAW ? c->dbg_bz : c->dbg_bzf;
        need = c->last_px * 8;
        break;
    default: return fail(c, FVV_E_ARG, "unknown tap %d", tap);
    }
    if (bytes != need) return fail(c, FVV_E_ARG, "tap %d holds %lld bytes, asked %lld", tap, (long long)need, (long long)bytes);
    HIPCHECK(c, hipDeviceSynchronize());
    // as rows of at most 8 KB so any tap fits the bounce buffer's halves
    const size_t row = std::min<size_t>((size_t)need, 8192);
    const size_t rows = row ? (size_t)need / row : 0, tail = (size_t)need - rows * row;
    int32_t rc = to_host(c, (uint8_t *)host_out, (int64_t)row, (const uint8_t *)src, (int64_t)row, row, rows, nullptr);
    if (rc == FVV_OK && tail)
        rc = to_host(c, (uint8_t *)host_out + rows * row, (int64_t)tail, (const uint8_t *)src + rows * row,
                     (int64_t)tail, tail, 1, nullptr);
    return rc;
}

int32_t fvv_server_start(fvv_ctx *c, int32_t max_slots, uint64_t step_bytes)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->server) return fail(c, FVV_E_STATE, "server already running");
    if (c->rig.empty()) return fail(c, FVV_E_STATE, "no rig set");
    if (max_slots < 1 || max_slots > 4096) return fail(c, FVV_E_ARG, "max_slots %d outside 1..4096", max_slots);
    DeviceGuard g(c->device);
    Server *S = new (std::nothrow) Server();
    if (!S) return fail(c, FVV_E_NOMEM, "out of host memory");
    S->max_slots = max_slots;
    if (step_bytes == 0) {
        // default: room for max_slots 1920x1080 views drawing on three cameras
        fvv_camera v1080{};
        v1080.width = 1920;
        v1080.height = 1080;
        size_t b, t;
        request_bounds(c, v1080, 3, false, false, b, t);
        step_bytes = (uint64_t)b * max_slots;
    }
    S->step_bytes = step_bytes;
    // tile counters: a 1920x1080 view has 2040 tiles in under 9 MB of workspace
    S->step_tiles = std::max<size_t>(4096, step_bytes / 2048);
    int32_t rc = FVV_OK;
    for (int w = 0; w < 2 && rc == FVV_OK; ++w) {
        rc = ws_reserve(c, S->ws[w], S->step_bytes, S->step_tiles, (size_t)max_slots);
        if (rc == FVV_OK && !(S->act[w] = unet_act_new())) rc = fail(c, FVV_E_NOMEM, "out of host memory");
        if (rc == FVV_OK && hipStreamCreateWithFlags(&S->stream[w], hipStreamNonBlocking) != hipSuccess)
            rc = fail(c, FVV_E_DEVICE, "hipStreamCreate failed");
        if (rc == FVV_OK &&
            hipEventCreateWithFlags(&S->done_ev[w], hipEventDisableTiming | hipEventBlockingSync) != hipSuccess)
            rc = fail(c, FVV_E_DEVICE, "hipEventCreate failed");
    }
    if (rc != FVV_OK) {
        for (int w = 0; w < 2; ++w) {
            if (S->stream[w]) (void)hipStreamDestroy(S->stream[w]);
            if (S->done_ev[w]) (void)hipEventDestroy(S->done_ev[w]);
            ws_release(c, S->ws[w]);
            unet_act_free(S->act[w]);
        }
        delete S;
        return rc;
    }
    c->server = S;
    S->sched = std::thread(scheduler, c);
    for (int w = 0; w < 2; ++w) S->compl_[w] = std::thread(completer, c, w);
    return FVV_OK;
}

int32_t fvv_server_pause(fvv_ctx *c, int32_t paused)
{
    if (!c) return FVV_E_ARG;
    Server *S = c->server;
    if (!S) return fail(c, FVV_E_STATE, "server not running");
    {
        std::lock_guard<std::mutex> lk(S->qmu);
        S->paused = paused != 0;
    }
    S->qcv.notify_all();
    return FVV_OK;
}

int32_t fvv_server_stop(fvv_ctx *c)
{
    if (!c) return FVV_E_ARG;
    if (!c->server) return fail(c, FVV_E_STATE, "server not running");
    server_teardown(c);
    return FVV_OK;
}

int32_t fvv_submit(fvv_ctx *c, const fvv_camera *virt, const fvv_synth_params *params, void *out_dev,
                   int64_t out_pitch, uint64_t *ticket)
{
    if (!c || !virt || !out_dev || !ticket) return FVV_E_ARG;
    Request r;
    Server *S;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        S = c->server;
        if (!S) return fail(c, FVV_E_STATE, "server not running");
        int32_t rc = resolve_params(c, params, r.P);
        if (rc) return rc;
        if ((rc = check_camera(c, *virt, false, "virtual camera"))) return rc;
        if (out_pitch < (int64_t)virt->width * 3) return fail(c, FVV_E_ARG, "out_pitch too small");
        if (r.P.path == FVV_PATH_LAYERED && !c->has_bg)
            return fail(c, FVV_E_STATE, "layered synthesis needs background models");
        request_bounds(c, *virt, r.P.k_nearest, r.P.path == FVV_PATH_LEARNED, r.P.path == FVV_PATH_LAYERED,
                       r.bytes, r.tiles);
    }
    r.cam = *virt;
    r.out = out_dev;
    r.pitch = out_pitch;
    r.arrive = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->qmu);
        S->recent.emplace_back(r.arrive, *virt);
        if (S->recent.size() > 4096) S->recent.pop_front();
        if (S->stop) return FVV_E_STATE;
        if (S->pending.size() >= 65536) return FVV_E_AGAIN;
        r.ticket = S->next_ticket++;
        {
            std::lock_guard<std::mutex> d(S->dmu);
            S->results[r.ticket] = Result();
        }
        S->pending.push_back(r);
    }
    S->qcv.notify_all();
    *ticket = r.ticket;
    return FVV_OK;
}

int32_t fvv_poll(fvv_ctx *c, uint64_t ticket, double *latency_s)
{
    if (!c || !c->server) return FVV_E_STATE;
    Server *S = c->server;
    std::lock_guard<std::mutex> lk(S->dmu);
    auto it = S->results.find(ticket);
    if (it == S->results.end()) return FVV_E_ARG;
    if (!it->second.done) return FVV_E_AGAIN;
    const int32_t st = it->second.status;
    if (latency_s) *latency_s = it->second.latency;
    S->results.erase(it);
    return st;
}

int32_t fvv_server_tx_cameras(fvv_ctx *c, int32_t n_tx, double window_s, uint32_t *mask)
{
    if (!c || !mask || n_tx < 1 || !(window_s >= 0.0)) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->server) return fail(c, FVV_E_STATE, "server not running");
    Server *S = c->server;
    std::vector<fvv_camera> views;
    {
        std::lock_guard<std::mutex> q(S->qmu);
        const Clock::time_point now = Clock::now();
        for (const auto &e : S->recent)
            if (std::chrono::duration<double>(now - e.first).count() <= window_s) views.push_back(e.second);
    }
    uint32_t m = 0;
    for (const auto &v : views) tx_union(c->rig.data(), (int)c->rig.size(), v, n_tx, m);
    *mask = m;
    return popcount32(m);
}

int32_t fvv_server_stats(fvv_ctx *c, uint64_t *out6)
{
    if (!c || !out6) return FVV_E_ARG;
    if (!c->server) return FVV_E_STATE;
    Server *S = c->server;
    std::lock_guard<std::mutex> lk(S->dmu);
    out6[0] = S->n_steps;
    out6[1] = S->n_done;
    out6[2] = S->n_failed;
    out6[3] = S->pixels;
    out6[4] = S->batch_sum;
    out6[5] = (uint64_t)(S->busy_s * 1e6);
    return FVV_OK;
}

// ---------------------------------------------------------------- learned path
uint64_t fvv_net_param_count(void) { return (uint64_t)unet_param_floats(); }

int32_t fvv_net_layer_info(int32_t layer, int32_t *out4)
{
    const unet_layer *l = unet_layer_info(layer);
    if (!l || !out4) return FVV_E_ARG;
    out4[0] = l->kind;
    out4[1] = l->cin;
    out4[2] = l->cout;
    out4[3] = l->kind == 0 ? 3 : (l->kind == 1 ? 2 : 1);
    return FVV_OK;
}

const char *fvv_net_layer_name(int32_t layer)
{
    const unet_layer *l = unet_layer_info(layer);
    return l ? l->name : nullptr;
}

int32_t fvv_net_load(fvv_ctx *c, const float *params, uint64_t n)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!params || n != unet_param_floats())
        return fail(c, FVV_E_ARG, "need %zu parameters, got %llu", unet_param_floats(), (unsigned long long)n);
    for (uint64_t e = 0; e < n; ++e)
        if (!std::isfinite(params[e])) return fail(c, FVV_E_ARG, "parameter %llu is not finite", (unsigned long long)e);
    DeviceGuard g(c->device);
    if (!c->net) {
        const size_t wb = unet_weight_bytes();
        if (c->budget && c->allocated + wb > c->budget)
            return fail(c, FVV_E_NOMEM, "device memory budget exceeded by the network weights (%zu bytes)", wb);
        c->net = unet_new();
        c->act = unet_act_new();
        if (!c->net || !c->act) return fail(c, FVV_E_NOMEM, "out of host memory");
        c->allocated += wb;
        c->net_bytes += wb;
    }
    HIPCHECK(c, hipDeviceSynchronize());
    HIPCHECK(c, unet_set_params(c->net, params, nullptr));
    return FVV_OK;
}

int32_t fvv_net_read(fvv_ctx *c, int32_t what, float *out, uint64_t n)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->net || !unet_loaded(c->net)) return fail(c, FVV_E_STATE, "no network loaded");
    if (!out || n != unet_param_floats())
        return fail(c, FVV_E_ARG, "need room for %zu parameters", unet_param_floats());
    DeviceGuard g(c->device);
    HIPCHECK(c, hipDeviceSynchronize());
    if (what == FVV_NET_PARAMS) HIPCHECK(c, unet_get_params(c->net, out, nullptr));
    else if (what == FVV_NET_GRADS) HIPCHECK(c, unet_get_grads(c->net, out, nullptr));
    else return fail(c, FVV_E_ARG, "unknown selector %d", what);
    return FVV_OK;
}

int32_t fvv_make_stack(fvv_ctx *c, const fvv_camera *virts, int32_t n_views, const fvv_synth_params *params,
                       void *stack_dev, void *stream)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!virts || !params || !stack_dev || n_views < 1) return fail(c, FVV_E_ARG, "null argument or n_views < 1");
    if (((uintptr_t)stack_dev & 15) != 0) return fail(c, FVV_E_ARG, "stack_dev must be 16-byte aligned");
    if (c->rig.empty()) return fail(c, FVV_E_STATE, "no rig set");
    std::vector<fvv_synth_params> Ps(n_views);
    int32_t rc;
    for (int v = 0; v < n_views; ++v) {
        if ((rc = resolve_params(c, &params[v], Ps[v]))) return rc;
        Ps[v].path = FVV_PATH_LEARNED;
        if ((rc = check_camera(c, virts[v], false, "virtual camera"))) return rc;
        if (virts[v].width != virts[0].width || virts[v].height != virts[0].height)
            return fail(c, FVV_E_ARG, "all views of a stack call must share one size");
    }
    DeviceGuard g(c->device);
    LearnedIO lio;
    lio.stack_out = (uint16_t *)stack_dev;
    lio.scratch_out = true;
    const hipStream_t s = (hipStream_t)stream;
    if ((rc = order_direct(c, s))) return rc;
    rc = launch_views(c, c->user, virts, Ps.data(), n_views, nullptr, nullptr, false, s, true, false, lio);
    const int32_t rm = mark_direct(c, s);
    return rc ? rc : rm;
}

int32_t fvv_net_forward(fvv_ctx *c, const void *stack_dev, int32_t n, int32_t height, int32_t width, float *out_dev,
                        void *stream)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->net || !unet_loaded(c->net)) return fail(c, FVV_E_STATE, "no network loaded");
    if (!stack_dev || !out_dev || n < 1 || height < 1 || width < 1 || height % UNET_ALIGN || width % UNET_ALIGN)
        return fail(c, FVV_E_ARG, "bad network input (sizes must be multiples of %d)", UNET_ALIGN);
    DeviceGuard g(c->device);
    const size_t px = (size_t)n * height * width;
    int32_t rc = reserve_act(c, c->act, px, false);
    if (rc) return rc;
    const hipStream_t s = (hipStream_t)stream;
    if ((rc = order_direct(c, s))) return rc;
    std::string err;
    hipEvent_t e0;
    fvv_prof *prof = c->profiling ? &c->prof : nullptr;
    fvv_prof_begin(prof, s, e0);
    const hipError_t e = unet_forward(c->net, c->act, (const uint16_t *)stack_dev, n, height, width, out_dev, nullptr,
                                      0, 0, 0, 0, s, err, c->debug);
    fvv_prof_end(prof, s, FVV_ST_NET, e0);
    const int32_t rm = mark_direct(c, s);
    rc = net_status(c, e, err, "network forward");
    return rc ? rc : rm;
}

int32_t fvv_net_train_step(fvv_ctx *c, const void *stack_dev, const float *target_dev, int32_t n, int32_t height,
                           int32_t width, int32_t valid_rows, float lr, int32_t apply, float *loss_out, void *stream)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->net || !unet_loaded(c->net)) return fail(c, FVV_E_STATE, "no network loaded");
    if (!stack_dev || !target_dev || n < 1 || height < 1 || width < 1 || height % UNET_ALIGN || width % UNET_ALIGN ||
        valid_rows < 1 || valid_rows > height)
        return fail(c, FVV_E_ARG, "bad training batch (sizes must be multiples of %d, 1 <= valid_rows <= height)",
                    UNET_ALIGN);
    if (!std::isfinite(lr) || lr < 0.f) return fail(c, FVV_E_ARG, "learning rate must be finite and >= 0");
    // the server's steps read the weights on their own streams while they run
    if (c->server) return fail(c, FVV_E_STATE, "stop the server before training");
    DeviceGuard g(c->device);
    int32_t rc = reserve_act(c, c->act, (size_t)n * height * width, true);
    if (rc) return rc;
    const hipStream_t s = (hipStream_t)stream;
    if ((rc = order_direct(c, s))) return rc;
    std::string err;
    hipEvent_t e0;
    fvv_prof *prof = c->profiling ? &c->prof : nullptr;
    fvv_prof_begin(prof, s, e0);
    const hipError_t e = unet_train(c->net, c->act, (const uint16_t *)stack_dev, target_dev, n, height, width,
                                    valid_rows, lr, apply, loss_out, s, err);
    fvv_prof_end(prof, s, FVV_ST_TRAIN, e0);
    const int32_t rm = mark_direct(c, s);
    rc = net_status(c, e, err, "training step");
    return rc ? rc : rm;
}

int32_t fvv_net_read_act(fvv_ctx *c, int32_t layer, void *host_out, int64_t bytes)
{
    if (!c) return FVV_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->act || !host_out || bytes < 0) return fail(c, FVV_E_STATE, "no network activations");
    DeviceGuard g(c->device);
    HIPCHECK(c, hipDeviceSynchronize());
    const hipError_t e = unet_read_act(c->act, layer, host_out, (size_t)bytes, nullptr);
    if (e != hipSuccess)
        return fail(c, FVV_E_ARG, "layer %d: wrong layer or byte count, or an output the last forward did not keep "
                    "(debug taps off)", layer);
    return FVV_OK;
}

uint64_t fvv_net_device_bytes(fvv_ctx *c) { return c ? c->net_bytes : 0; }

}  // extern "C"
