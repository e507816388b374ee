/*
 * fvv.h -- C ABI of the MI355X (gfx950) view-synthesis library libfvv.so.
 *
 * The library renders a virtual view from multiview-plus-depth (MVD) frames
 * of N calibrated cameras by depth-image-based rendering, the edge-server
 * stage of FVV Live (arXiv 2007.00558, Section VI "View synthesis"):
 * the input is colour plus depth from calibrated cameras (Sections III-IV),
 * the user moves a virtual camera continuously (Section VIII), and the output
 * is the image that camera sees, built from the few nearest reference
 * cameras (Section VI).
 *
 * Conventions
 *  - Every function returns an int32_t status: FVV_OK (0) or a negative
 *    FVV_E_* code; fvv_last_error() then describes the failure.  No C++
 *    exception crosses this boundary.
 *  - Pinhole cameras without distortion, OpenCV axes (x right, y down,
 *    z forward), world -> camera X_c = R X_w + t, pixel centres at integer
 *    coordinates, depth = Z-depth along the optical axis in millimetres
 *    (uint16, 0 = no depth).
 *  - Colour is packed RGB8 (3 bytes per pixel, R first).  Pitches are in
 *    bytes and must be at least width*3 (colour) or width*2 (depth).
 *  - Pointers marked "host or device" are interpreted according to the
 *    mem_kind argument of the call.  Device pointers must be addresses in
 *    the context's GPU (for example a torch tensor's data_ptr()).
 *  - stream is a hipStream_t (NULL = the default stream).  Device-memory
 *    calls are asynchronous on that stream: the caller keeps its buffers
 *    alive and unchanged until the stream has passed the call.  Host-memory
 *    calls return after the data has been consumed (upload) or written
 *    (synthesis).
 *  - A context is used by one host thread at a time, except fvv_submit and
 *    fvv_poll, which any thread may call while the server runs.
 *  - The direct device calls of a context (fvv_synthesize,
 *    fvv_synthesize_batch, fvv_make_stack, fvv_net_forward,
 *    fvv_net_train_step) share its workspace, network activations and debug
 *    taps.  A call on a stream other than the previous direct call's first
 *    waits, on the device, for that call's work, so calls may alternate
 *    streams freely; their results are those of the calls run one at a
 *    time.  The server's steps use workspaces of their own.
 */
#ifndef FVV_H
#define FVV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FVV_ABI_VERSION 10

/* status codes */
enum {
    FVV_OK = 0,
    FVV_E_ARG = -1,          /* null / short / out-of-range argument */
    FVV_E_STATE = -2,        /* call out of order: no rig, no frame, stale version */
    FVV_E_NOMEM = -3,        /* device allocation failed or memory budget exceeded */
    FVV_E_DEVICE = -4,       /* HIP runtime error (text in fvv_last_error) */
    FVV_E_AGAIN = -5,        /* not ready yet / admission refused; retry later */
    FVV_E_UNSUPPORTED = -6   /* valid request this build does not implement */
};

enum { FVV_MEM_HOST = 0, FVV_MEM_DEVICE = 1 };
enum { FVV_FILL_BG = 0, FVV_FILL_NONE = 1 };
enum { FVV_PATH_PLAIN = 0, FVV_PATH_LEARNED = 1, FVV_PATH_LAYERED = 2 };

#define FVV_BG_MM 0xFFFF             /* background signal in millimetre depth maps */

/* limits */
#define FVV_MAX_CAMERAS 32          /* rig size; the camera index fits 5 key bits */
#define FVV_MAX_K 8                 /* cameras blended per view */
#define FVV_MAX_SRC_PIXELS (1 << 27) /* width*height of a source camera (27 key bits) */
#define FVV_MAX_OUT_DIM 8192        /* output width and height */

typedef struct fvv_ctx fvv_ctx;

/* One calibrated camera (Section VII: multi-camera calibration).
 * depth_alpha / depth_beta are the per-camera depth-correction coefficients of
 * Eq. (1), z_post = (alpha z + beta) z; (0, 1) leaves depth unchanged.  They
 * are ignored for virtual cameras. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];     /* row-major rotation, world -> camera */
    float t[3];     /* translation, metres */
    float depth_alpha, depth_beta;
} fvv_camera;

/* One camera's MVD frame.  rgb: height rows of width*3 bytes; depth_mm:
 * height rows of width uint16 millimetres (0 = no depth; FVV_BG_MM = the
 * background signal: the pixel shows the static background, whose depth
 * the layered synthesis takes from the background model), or, once the
 * context's depth format is FVV_DEPTH_Y12, the 12-bit coded I420 image of
 * fvv_depth_encode_y12 with depth_pitch as its luma pitch.  Both NULL marks
 * the camera as absent from this frame set: it is then never selected. */
typedef struct {
    const void *rgb;
    int64_t rgb_pitch;
    const void *depth_mm;
    int64_t depth_pitch;
} fvv_view;

/* Synthesis parameters.  Zero-initialised fields take the defaults shown. */
typedef struct {
    int32_t k_nearest;      /* cameras blended per view (default 3, Section VI:
                               typically three; at most FVV_MAX_K) */
    float tau_rel;          /* relative depth tolerance of the consistency tests
                               (default 0.05) */
    float max_footprint;    /* splat footprint cap in output pixels (default 4) */
    int32_t fill_mode;      /* FVV_FILL_BG (default) or FVV_FILL_NONE (holes
                               stay black, as in the paper's system, Section IX) */
    int32_t path;           /* FVV_PATH_PLAIN; FVV_PATH_LEARNED: the network
                               loaded with fvv_net_load replaces the blend and
                               hole fill (plain result where no network is
                               loaded or its output is not finite);
                               FVV_PATH_LAYERED: foreground and background
                               layers (fvv_set_bg_model), k_nearest <= 4 */
    uint32_t exclude_mask;  /* rig cameras c with bit c set are not selected
                               (leave-one-camera-out evaluation); 0 = none */
    uint64_t frame_version; /* 0 = latest uploaded frame set, else that version
                               if it is still resident (the two most recent) */
} fvv_synth_params;

/* ABI version of the loaded library (FVV_ABI_VERSION it was built with). */
int32_t fvv_abi_version(void);

/* Create a context on HIP device hip_device.  mem_budget_bytes caps the
 * device memory the context may allocate (0 = no cap).  *out receives the
 * context; it owns every device buffer it allocates (frame store, per-view
 * workspaces). */
int32_t fvv_create(int32_t hip_device, uint64_t mem_budget_bytes, fvv_ctx **out);

/* Destroy a context; waits for its outstanding work.  NULL is a no-op. */
void fvv_destroy(fvv_ctx *ctx);

/* Text of the last failure on ctx (or, when ctx is NULL, of the calling
 * thread's last failed fvv_create or codec call).  Valid until the next call
 * on ctx. */
const char *fvv_last_error(const fvv_ctx *ctx);

/* Set the camera rig: n (1..FVV_MAX_CAMERAS) calibrated cameras.  Copies the
 * array.  Rejects non-finite values, fx/fy <= 0, R not orthonormal within
 * 1e-4, width*height outside 1..FVV_MAX_SRC_PIXELS.  Changing the rig drops
 * resident frame sets (FVV_E_STATE until the next upload). */
int32_t fvv_set_rig(fvv_ctx *ctx, const fvv_camera *cams, int32_t n);

/* Upload one MVD frame set: views[c] for every rig camera c (n must equal the
 * rig size).  mem_kind says whether the view pointers are host or device
 * memory.  The data are copied into the context's frame store (double
 * buffered: the two most recent sets stay resident), colour repacked to
 * 4-byte texels and depth decoded with the camera's Eq. (1) correction.
 * *out_version (may be NULL) receives the new set's version (1, 2, ...). */
int32_t fvv_upload_mvd(fvv_ctx *ctx, const fvv_view *views, int32_t n, int32_t mem_kind,
                       void *stream, uint64_t *out_version);

/* 12-bit depth coding for 8-bit YUV420 video codecs (Section V-A).
 * The capture side quantises depth to 12-bit codes (Eq. 2, linear in 1/z
 * between the clipping planes z_near and z_far, metres):
 *   code = round(4093 (1/z - 1/z_far) / (1/z_near - 1/z_far) + 2),
 * evaluated in double precision and rounded half up; 1 = no depth (0 mm) or
 * a rounded code outside 2..4095; 0 = the background signal (FVV_BG_MM).
 * Each 2x2 block p11 p12 / p21 p22 of codes becomes
 * one 2x2 block of an I420 image: Y = the code's 8 LSBs, mirrored to
 * 255 - LSBs when its 4 MSBs are odd (Eq. 3); U = the MSBs of p11 on the
 * even bits and of p12 on the odd bits; V = the same for p21 and p22.
 * Decoding inverts both steps and returns whole millimetres,
 * round(1000 / ((code - 2)/4093 (1/z_near - 1/z_far) + 1/z_far)),
 * FVV_BG_MM for code 0 and 0 for code 1.
 *
 * I420 layout (yuv): height rows of y_pitch bytes (Y), then U and V, each
 * height/2 rows of y_pitch/2 bytes.  y_pitch even and >= width; width and
 * height even, >= 2, width*height <= FVV_MAX_SRC_PIXELS, height <= 65536.
 * depth rows: depth_pitch bytes (even, >= 2*width), 2-byte aligned.
 * Both buffers are device memory; the work is enqueued on stream (HIP
 * stream, NULL = default) of the current device and the call returns at
 * once.  FVV_E_ARG for bad sizes, pitches or planes (0 < z_near < z_far,
 * finite); FVV_E_DEVICE if the launch fails. */
int32_t fvv_depth_encode_y12(const void *depth_mm, int64_t depth_pitch, int32_t width, int32_t height,
                             float z_near, float z_far, void *yuv, int64_t y_pitch, void *stream);
int32_t fvv_depth_decode_y12(const void *yuv, int64_t y_pitch, int32_t width, int32_t height, float z_near,
                             float z_far, void *depth_mm, int64_t depth_pitch, void *stream);

/* The same coding for n (1..FVV_MAX_CAMERAS) images of one size and one pair
 * of clipping planes in a single launch (a capture server coding all of its
 * cameras' depth maps).  depth_mm, depth_pitch, yuv and y_pitch are host
 * arrays of n entries (read during the call only); entry i follows the
 * single-image rules above.  The images must not overlap.  Same errors; on
 * any bad entry nothing is enqueued. */
int32_t fvv_depth_encode_y12_batch(int32_t n, const void *const *depth_mm, const int64_t *depth_pitch,
                                   int32_t width, int32_t height, float z_near, float z_far, void *const *yuv,
                                   const int64_t *y_pitch, void *stream);
int32_t fvv_depth_decode_y12_batch(int32_t n, const void *const *yuv, const int64_t *y_pitch, int32_t width,
                                   int32_t height, float z_near, float z_far, void *const *depth_mm,
                                   const int64_t *depth_pitch, void *stream);

/* Depth format of the following uploads on ctx: FVV_DEPTH_MM16 (default,
 * uint16 millimetres) or FVV_DEPTH_Y12 (the I420 image above, decoded to
 * millimetres by the ingest kernel; every camera's width and height even).
 * Eq. (1) is then applied to the decoded millimetres as for the 16-bit
 * format.  z_near / z_far are read for FVV_DEPTH_Y12 only.  Resident frame
 * sets are not affected. */
enum { FVV_DEPTH_MM16 = 0, FVV_DEPTH_Y12 = 1 };
int32_t fvv_set_depth_format(fvv_ctx *ctx, int32_t format, float z_near, float z_far);

/* Background models of the layered synthesis (Section VI): per rig camera,
 * the depth of the static background in uint16 millimetres (height rows of
 * width values, pitches[c] bytes per row; 0 = no background there), computed
 * at calibration; depth_mm[c] NULL = no model for camera c (its background
 * layer stays empty); depth_mm NULL clears every model.  Copied into the
 * context (host or device memory per mem_kind; the call returns when the
 * copy is done).  The models are calibrated geometry: Eq. (1) is not
 * applied to them.  Frame sets uploaded afterwards carry, per camera, a
 * foreground layer (live depth where it is not FVV_BG_MM) and a background
 * layer (the model's depth under the live colour of FVV_BG_MM pixels); the
 * call drops resident frame sets (FVV_E_STATE until the next upload).  The
 * layered synthesis warps, filters and mixes each layer over the same
 * selected cameras and stacks the foreground layer over the background
 * layer before the hole fill.  FVV_E_STATE while the server runs or
 * without a rig; a rig change clears the models. */
int32_t fvv_set_bg_model(fvv_ctx *ctx, const void *const *depth_mm, const int64_t *pitches, int32_t n,
                         int32_t mem_kind, void *stream);

/* Joint bilateral pre-filter of the live depth at ingest (Section VI: small
 * holes and gaps around object edges are closed before warping; the paper
 * gives no parameters).  With enable != 0, following uploads fill every
 * pixel without depth (0 mm; background-signalled pixels are neither filled
 * nor used) with the bilateral mean of the valid depths in its
 * (2 radius + 1)^2 window: weight = ws * wc with
 *   ws = floor(4096 exp(-(dx^2 + dy^2) / (2 sigma_s^2)) + 0.5)   (pixels)
 *   wc = floor(4096 exp(-d^2 / (2 sigma_c^2)) + 0.5)              (d = L1
 *        distance of the two RGB8 colours),
 * depth = floor((sum w D + floor(sum w / 2)) / sum w) millimetres, when at
 * least min_valid neighbours have w > 0 (else the pixel stays a hole).  One
 * pass over the transmitted millimetres (coded depth decoded first), before
 * the Eq. (1) decode.  radius 1..3, sigmas finite and > 0, min_valid in
 * 1..(2 radius + 1)^2 - 1 (suggested: 2, 1.5, 24, 5); enable == 0 turns the
 * filter off.  Resident frame sets are not affected. */
int32_t fvv_set_prefilter(fvv_ctx *ctx, int32_t enable, int32_t radius, float sigma_s, float sigma_c,
                          int32_t min_valid);

/* Copy camera cam's decoded depth plane of a resident frame set (version 0 =
 * latest) to host memory: width*height float32 metres after the pre-filter
 * and Eq. (1), bits 0xFFFFFFFF where there is no depth; layer 0 = live
 * (foreground) depth, 1 = the background layer of a layered frame set.
 * bytes must equal width*height*4.  For inspection and tests; synchronises
 * the device. */
int32_t fvv_read_frame_depth(fvv_ctx *ctx, int32_t cam, int32_t layer, uint64_t version, void *host_out,
                             int64_t bytes);

/* Render one virtual camera into out_rgb8 (height rows of width*3 bytes,
 * pitch out_pitch; host or device per mem_kind).  Steps, all on the GPU:
 * select the k nearest cameras and their distance weights, forward-splat
 * their valid pixels into a z-buffer of packed (depth, camera, pixel) keys,
 * 3x3 crack/speckle filter, depth-consistent backward colour fetch and
 * view-weighted blend, hole fill (Section VI). */
int32_t fvv_synthesize(fvv_ctx *ctx, const fvv_camera *virt, const fvv_synth_params *params,
                       void *out_rgb8, int64_t out_pitch, int32_t mem_kind, void *stream);

/* Render n_views virtual cameras against the same frame set in one batched
 * launch sequence.  outs[v] / pitches[v] as out_rgb8 / out_pitch above. */
int32_t fvv_synthesize_batch(fvv_ctx *ctx, const fvv_camera *virts, int32_t n_views,
                             const fvv_synth_params *params, void *const *outs,
                             const int64_t *pitches, int32_t mem_kind, void *stream);

/* For callers that cannot allocate memory -- code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation: render one virtual
 * camera exactly as fvv_synthesize does (device output, byte-identical
 * result) with every temporary buffer of the synthesis (view descriptor,
 * tile counters, bin lists and block ranges, splat records, slot plane,
 * tile summaries, open-hole list) in one fixed device array of
 * FVV_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  The call allocates no device and no pinned host
 * memory (no hipMalloc, hipFree or hipHostMalloc).
 *  - out_dev: device memory, height rows of width*3 bytes, pitch out_pitch;
 *    enqueued on stream, returns at once.
 *  - Paths FVV_PATH_PLAIN and FVV_PATH_LAYERED; FVV_PATH_LEARNED needs the
 *    network's activation memory: FVV_E_UNSUPPORTED.
 *  - FVV_E_NOMEM, with nothing enqueued, when the view's buffers exceed the
 *    array (a 1920x1080 view drawing on three 1280x720 cameras needs about
 *    34 MB, layered about 58 MB); other errors as fvv_synthesize.
 *  - Every call on one GPU, from any context and on any stream, shares that
 *    GPU's array and leaves its contents there; each call clears what must
 *    start at zero itself.  Calls whose device work overlaps race: the
 *    caller orders them (for example by issuing them on one stream). */
#define FVV_NOALLOC_SCRATCH_BYTES (64ull << 20)
int32_t fvv_synthesize_noalloc(fvv_ctx *ctx, const fvv_camera *virt, const fvv_synth_params *params,
                               void *out_dev, int64_t out_pitch, void *stream);

/* Host-only helpers (no device, no context): the camera selection and the
 * float32 pair matrices the kernels use, exposed for inspection and tests.
 * fvv_select_cameras: rank the present cameras (present may be NULL = all) by
 * centre distance to virt, write up to k rig indices to idx and their weights
 * 1/distance to w; a virtual camera within 1e-6 m of a source selects that
 * source alone with weight 1.  Returns the count (>= 0) or FVV_E_ARG.
 * fvv_pair_matrices: out[26] = A[9] a[3] B[9] b[3] sx sy, the forward
 * (source pixel -> virtual) and backward maps of the pinhole pair. */
int32_t fvv_select_cameras(const fvv_camera *rig, const int32_t *present, int32_t n,
                           const fvv_camera *virt, int32_t k, int32_t *idx, float *w);
int32_t fvv_pair_matrices(const fvv_camera *src, const fvv_camera *virt, float *out26);

/* Adaptive view transmission (Section V-C): only the n_tx cameras nearest
 * to a client's viewpoint are transmitted (five for one client, two more
 * than the three rendered, so a moving viewpoint always finds its cameras);
 * with several clients, the union.  Writes the set as a bit mask (bit c =
 * rig camera c) to *mask and returns its size, or FVV_E_ARG.  The ranking is
 * that of fvv_select_cameras (centre distance, ties to the lower index)
 * without the coincident-camera shortcut, so for n_tx >= k every camera the
 * synthesis selects for these viewpoints is in the set, and uploading only
 * the set renders those viewpoints exactly as uploading every camera.
 * Host-only. */
int32_t fvv_tx_cameras(const fvv_camera *rig, int32_t n, const fvv_camera *views, int32_t n_views,
                       int32_t n_tx, uint32_t *mask);

/* Debug taps for stage-by-stage checking.  fvv_set_debug(ctx, 1) makes the
 * following direct syntheses keep, for one view of each call (view 0, or
 * the index set with fvv_set_debug_view; a call with fewer views keeps
 * none), the raw and filtered z-buffers, the blend result before hole
 * filling and the bin-list load of every tile; fvv_debug_read copies one of
 * them to host memory (bytes must equal the tap's size):
 *   FVV_TAP_Z_RAW, FVV_TAP_Z_FILT: uint64 key per output pixel,
 *     key = float32 depth bits << 32 | camera << 27 | source pixel index,
 *     0xFFFFFFFFFFFFFFFF = empty;
 *   FVV_TAP_BLEND: uint32 RGBA8 per pixel, A = 255 covered, 0 hole;
 *   FVV_TAP_DEPTH: float32 depth per pixel (0 for holes);
 *   FVV_TAP_BG_Z_RAW, FVV_TAP_BG_Z_FILT (layered synthesis only): the
 *     background layer's key maps; the first two taps then hold the
 *     foreground layer's, BLEND and DEPTH the composite;
 *   FVV_TAP_TILES: two int32 per 32x32 output tile (row-major over the
 *     tile grid): the source-block entries the binning appended to the
 *     tile's list and the list's capacity; a tile with more entries than
 *     capacity tested every source block's tile range instead.
 * fvv_set_debug_view: the index of the tapped view (>= 0; FVV_E_ARG). */
enum { FVV_TAP_Z_RAW = 0, FVV_TAP_Z_FILT = 1, FVV_TAP_BLEND = 2, FVV_TAP_DEPTH = 3, FVV_TAP_BG_Z_RAW = 4,
       FVV_TAP_BG_Z_FILT = 5, FVV_TAP_TILES = 6 };
int32_t fvv_set_debug(fvv_ctx *ctx, int32_t enable);
int32_t fvv_set_debug_view(fvv_ctx *ctx, int32_t view);
int32_t fvv_debug_read(fvv_ctx *ctx, int32_t tap, void *host_out, int64_t bytes);

/* Measured peaks of device hip_device for the roofline of the plain path
 * (the operations the binning and the tile kernel are built from), each the
 * best of five timed launches after a warm-up, on the null stream (the call
 * synchronises the device and allocates 2 GiB for its duration):
 *   out[0] HBM copy bandwidth, GB/s of bytes read plus written (1 GiB copy);
 *   out[1] global 64-bit atomicMin per second, every lane its own word;
 *   out[2] the same with the 64 lanes of a wave on one word;
 *   out[3] LDS 64-bit atomicMin per second, conflict-free words;
 *   out[4] LDS 64-bit atomicMin per second, pseudo-random words of a 34x34
 *          window shared by eight waves (the splat's z-buffer).
 * Returns FVV_PEAKS (the count written) or an error (text in
 * fvv_last_error(NULL)); n must be >= FVV_PEAKS. */
#define FVV_PEAKS 5
int32_t fvv_measure_peaks(int32_t hip_device, double *out, int32_t n);

/* Self-check of the division the kernels use for every projected depth
 * (Section VI: the warps divide by the projected depth; the float32 reading
 * takes correctly rounded quotients): the reciprocal formed from the hardware
 * estimate and one Newton step, and the quotients derived from it, against
 * correctly rounded division, for every significand of the divisors
 * 2^e (1 + m 2^-23), e_lo <= e <= e_hi (-125 <= e_lo <= e_hi <= 125), two
 * dividends per divisor.  Writes the number of mismatching results to
 * *mismatches (host memory; 0 expected).  Synchronous on hip_device; returns
 * FVV_OK or an error (text in fvv_last_error(NULL)). */
int32_t fvv_check_reciprocal(int32_t hip_device, int32_t e_lo, int32_t e_hi, uint64_t *mismatches);

/* Self-check of the network's bfloat16 rounding (every stored tensor of the
 * learned path is rounded to bfloat16, round to nearest even): the
 * hardware conversion the kernels use against the rounding written out on
 * the bit pattern, for all 2^32 float32 patterns but the NaNs.  Writes the
 * number of mismatches to *mismatches (host memory; 0 expected).
 * Synchronous on hip_device; returns FVV_OK or an error. */
int32_t fvv_check_bf16(int32_t hip_device, uint64_t *mismatches);

/* Stage timing (tracing).  With profiling on, every kernel the context
 * launches is bracketed by HIP events on the caller's stream (this adds a
 * little launch overhead).  fvv_profile_read synchronises on the recorded
 * events and writes, per stage, the summed kernel time in milliseconds and
 * the number of launches since the last reset (n >= fvv_stage_count()).
 * fvv_stage_name gives a stage's name (NULL if out of range). */
int32_t fvv_set_profiling(fvv_ctx *ctx, int32_t enable);
int32_t fvv_stage_count(void);
const char *fvv_stage_name(int32_t stage);
int32_t fvv_profile_read(fvv_ctx *ctx, double *total_ms, int64_t *launches, int32_t n, int32_t reset);

/* Transmission set of the served clients: fvv_tx_cameras over the
 * viewpoints of the requests submitted in the last window_s seconds (at most
 * the last 4096 requests).  The edge server asks the capture side for these
 * cameras and uploads only them.  FVV_E_STATE if the server is not running. */
int32_t fvv_server_tx_cameras(fvv_ctx *ctx, int32_t n_tx, double window_s, uint32_t *mask);

/* Continuous-batching server: many users' viewpoint requests of any output
 * size rendered against the device-resident frame store (the edge server
 * serves each client's viewpoint, Section VIII).  A scheduler thread admits
 * pending requests in arrival order into the next step while step slots
 * (max_slots) and step workspace memory (step_bytes; 0 = room for max_slots
 * 1920x1080 views) last, and launches each step as one batched synthesis on
 * one of two streams with separate workspaces, so a new step starts while the
 * previous one still runs.  Results are written to the caller's device
 * buffers; their content is identical to fvv_synthesize of the same request
 * on the same frame version.  Uploads (fvv_upload_mvd) may continue while the
 * server runs; each step reads the latest version at its launch unless the
 * request names one.  The rig cannot change while the server runs.
 * fvv_server_start: FVV_E_STATE without a rig or if already running;
 *   device memory for both step workspaces is allocated here (FVV_E_NOMEM).
 * fvv_server_pause: paused != 0 holds new steps (requests keep queueing;
 *   steps already launched complete); 0 resumes.  Stopping ignores a pause.
 * fvv_server_stop: drains every pending request, joins the threads.
 * fvv_submit: thread-safe; copies the camera and parameters, stamps the
 *   arrival time and returns a ticket; out_dev (height rows of width*3
 *   bytes, pitch out_pitch) must have no pending work on any stream when
 *   submitted (the server's streams do not wait for the caller's) and must
 *   stay valid until the ticket completes;
 *   FVV_E_AGAIN when 65536 requests are already pending.
 * fvv_poll: FVV_OK once the request has completed (then *latency_s =
 *   completion - submission in seconds, host clock, and the ticket is
 *   released), FVV_E_AGAIN while pending, the request's error code if it
 *   failed (FVV_E_NOMEM: larger than a whole step), FVV_E_ARG for an unknown
 *   ticket.
 * fvv_server_stats: out6 = {steps, completed, failed, output pixels, sum of
 *   step sizes, microseconds between step launch and completion}. */
int32_t fvv_server_start(fvv_ctx *ctx, int32_t max_slots, uint64_t step_bytes);
int32_t fvv_server_pause(fvv_ctx *ctx, int32_t paused);
int32_t fvv_server_stop(fvv_ctx *ctx);
int32_t fvv_submit(fvv_ctx *ctx, const fvv_camera *virt, const fvv_synth_params *params, void *out_dev,
                   int64_t out_pitch, uint64_t *ticket);
int32_t fvv_poll(fvv_ctx *ctx, uint64_t ticket, double *latency_s);
int32_t fvv_server_stats(fvv_ctx *ctx, uint64_t *out6);

/* Learned blend/inpaint network (the learned path).  The paper mixes the
 * warped reference cameras with fixed weights by camera distance and leaves
 * disocclusions unfilled (Sections VI, IX); this path hands the same
 * per-camera evidence to a small U-Net that predicts the output colour.
 *  - Network: 3x3 convolutions + ReLU at widths 32/64/128/256 with 2x2
 *    max-pooling, 2x2 transposed convolutions with skip concatenation
 *    [up, skip], a 1x1 head + sigmoid; bfloat16 weights and activations,
 *    float32 accumulation; float32 master weights and Adam (0.9, 0.999,
 *    1e-8) for training.  fvv_net_layer_info(i, out4) gives layer i's kind
 *    (0 conv3x3+ReLU, 1 convT2x2, 2 head), C_in, C_out, kernel size;
 *    fvv_net_layer_name its name.
 *  - Parameters: fvv_net_param_count() float32 values, layer by layer, each
 *    layer's weights (C_out, kh, kw, C_in) then its bias (C_out); a transposed
 *    convolution maps input (y, x) to output (2y+kh, 2x+kw).
 *  - Stack (network input): bfloat16 [n][Hp][Wp][16], Hp and Wp the output
 *    height and width rounded up to multiples of 8.  Per pixel and for each
 *    of the first three selected cameras (selection order): the camera's
 *    depth-consistent bilinear colour R, G, B / 255, 0.5 / (its depth in that
 *    camera) capped at 1, and 1; zeros where the camera gives no sample, at
 *    pixels without a filtered point and in the padding; channel 15 zero.
 * fvv_net_load: host float32 parameters; resets the optimiser state.
 * fvv_net_read: host copy of the parameters (FVV_NET_PARAMS) or of the last
 *   training step's gradient (FVV_NET_GRADS).
 * fvv_make_stack: the stacks of n_views views of one size (params: one entry
 *   per view) into stack_dev (device, 16-byte aligned), asynchronously.
 * fvv_net_forward: out_dev (device float32 [n][height][width][3]) = the
 *   network's sigmoid output for n stacks of height x width (multiples of 8).
 * fvv_net_train_step: forward, L1 loss mean |out - target| over the first
 *   valid_rows rows of every image and 3 channels (target_dev device float32
 *   [n][height][width][3] in [0, 1]), backward; apply != 0 then takes one Adam
 *   step with learning rate lr.  *loss_out (host, may be NULL) receives the
 *   loss, which synchronises the stream.  The weight gradient is reduced in
 *   a fixed order (no float atomics): a step is bit-reproducible.
 *   FVV_E_STATE while the server runs (its steps read the weights).
 * fvv_net_read_act: host copy of one layer's output of the last forward,
 *   bfloat16 NHWC (bytes must be pixels at that layer's resolution x C_out x 2).
 *   With debug taps on (fvv_set_debug) a forward keeps every layer's output;
 *   with them off it may compute the finest transposed convolution inside
 *   the convolution that reads it (large batches) and the head inside the
 *   last convolution, whose output is then not stored either; reading such a
 *   layer then fails with FVV_E_ARG.  The network's results are the same
 *   bytes either way.
 * fvv_net_device_bytes: device memory held by the network and its
 *   activation sets (part of the context's budget). */
enum { FVV_NET_PARAMS = 0, FVV_NET_GRADS = 1 };
uint64_t fvv_net_param_count(void);
int32_t fvv_net_layer_info(int32_t layer, int32_t *out4);
const char *fvv_net_layer_name(int32_t layer);
int32_t fvv_net_load(fvv_ctx *ctx, const float *params, uint64_t n);
int32_t fvv_net_read(fvv_ctx *ctx, int32_t what, float *out, uint64_t n);
int32_t fvv_make_stack(fvv_ctx *ctx, const fvv_camera *virts, int32_t n_views, const fvv_synth_params *params,
                       void *stack_dev, void *stream);
int32_t fvv_net_forward(fvv_ctx *ctx, const void *stack_dev, int32_t n, int32_t height, int32_t width,
                        float *out_dev, void *stream);
int32_t fvv_net_train_step(fvv_ctx *ctx, const void *stack_dev, const float *target_dev, int32_t n,
                           int32_t height, int32_t width, int32_t valid_rows, float lr, int32_t apply,
                           float *loss_out, void *stream);
int32_t fvv_net_read_act(fvv_ctx *ctx, int32_t layer, void *host_out, int64_t bytes);
uint64_t fvv_net_device_bytes(fvv_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FVV_H */
