/*
 * fvv_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, single-threaded CPU reference of the depth-image-based
 * rendering (DIBR) view-synthesis path of FVV Live (arXiv 2007.00558,
 * Section VI "View synthesis").  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the HIP path never
 * links, includes or calls it, and it shares no code with the HIP path.
 *
 * The paper describes its renderer at block-diagram level only (Section VI):
 * each reference pixel plus its depth is a 3D point projected into the
 * virtual camera; cracks are handled by backward warping combined with image
 * filtering; disocclusions are covered by several reference cameras whose
 * contributions are mixed according to their distance to the virtual camera
 * (typically three cameras).  Every constant, tie-break and filter the paper
 * leaves open is fixed here as an explicit reading (see the step comments);
 * this file is the definition the GPU path must reproduce.
 *
 * Precision.  The paper fixes none.  Where floating point decides a discrete
 * outcome (which pixel a point lands on, which key wins the z-buffer, whether
 * a tap is depth-consistent, whether a pixel is a hole) the decision is taken
 * in IEEE float32, op by op, without fused multiply-add and with correctly
 * rounded division -- the precision of the kernels, so both sides decide
 * identically.  Pure value arithmetic (the bilinear and view-weighted colour
 * blend) is carried in double.  Build: gcc -O2 -ffp-contract=off
 * -fno-fast-math.
 *
 * Steps (names used throughout):
 *   O1 camera selection and view weights      (Section V-D, Section VI)
 *   O2 pair matrices                          (Section VI, pinhole geometry)
 *   O3 depth decode with correction           (Eq. 1, Section IV-A)
 *   O4 forward splat into a packed-key z-buffer (Section VI, 3D warping)
 *   O5 3x3 crack / speckle depth filter       (Section VI, "image filtering")
 *   O6 backward colour fetch and blend        (Section VI, backward warping and mixing)
 *   O7 background-directed hole fill          (Section VI disocclusions; the
 *                                              paper leaves them black, Section IX)
 *
 * Parity status: O1-O4, O6 and O7 are pinned by closed forms, invariants and
 * brute force in the CPU test suite.  The O5 filter rule, tau_rel, the
 * footprint cap and the hole-fill preference are definitions of this build
 * ("parity unpinned" for their quality: only their stated behaviour on
 * hand-built cases is checked).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_EMPTY 0xFFFFFFFFFFFFFFFFull
#define REF_MAXK 8

typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];   /* row-major, world -> camera: X_c = R X_w + t */
    float t[3];
    float depth_alpha, depth_beta;
} ref_camera;

/* pair record for one (source, virtual) camera pair, all float32:
 *   A[9], a[3]  forward  source pixel (i,j,z) -> virtual homogeneous point
 *   B[9], b[3]  backward virtual pixel (x,y,z) -> source homogeneous point
 *   sx, sy      focal-length ratios virtual / source                       */
typedef struct {
    float A[9], a[3], B[9], b[3], sx, sy;
} ref_pair;

/* ------------------------------------------------------------------------ */
/* O1: camera selection and view weights.
 * The paper transmits the N_Tx cameras closest to the virtual viewpoint
 * (Section V-D) and renders from typically three of them, mixing their
 * contributions by distance to the virtual camera (Section VI).
 * Reading: distance = Euclidean distance between camera centres C = -R^T t
 * in double; stable order by (distance, rig index); weight = 1/distance; if
 * the nearest centre is closer than 1e-6 m the virtual camera coincides with
 * that source and only it is used, with weight 1.
 * present[c] == 0 removes camera c from the ranking.
 * Returns the number of selected cameras K (0 if none). */
static void ref_center(const ref_camera *c, double C[3])
{
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k)
            s += (double)c->R[k * 3 + r] * (double)c->t[k];
        C[r] = -s;
    }
}

int fvv_ref_select(const ref_camera *rig, const int32_t *present, int32_t n,
                   const ref_camera *virt, int32_t k_sel,
                   int32_t *idx_out, double *w_out)
{
    double Cv[3], d[64];
    int order[64], m = 0;
    if (n > 64) return -1;
    ref_center(virt, Cv);
    for (int c = 0; c < n; ++c) {
        double Cc[3];
        if (present && !present[c]) continue;
        ref_center(&rig[c], Cc);
        double dx = Cc[0] - Cv[0], dy = Cc[1] - Cv[1], dz = Cc[2] - Cv[2];
        d[c] = sqrt(dx * dx + dy * dy + dz * dz);
        order[m++] = c;
    }
    /* insertion sort: stable, ties keep the lower rig index first */
    for (int a = 1; a < m; ++a) {
        int v = order[a], b = a - 1;
        while (b >= 0 && d[order[b]] > d[v]) {
            order[b + 1] = order[b];
            --b;
        }
        order[b + 1] = v;
    }
    int K = m < k_sel ? m : k_sel;
    if (K > REF_MAXK) K = REF_MAXK;
    if (K > 0 && d[order[0]] < 1e-6) {
        idx_out[0] = order[0];
        w_out[0] = 1.0;
        return 1;
    }
    for (int k = 0; k < K; ++k) {
        idx_out[k] = order[k];
        w_out[k] = 1.0 / d[order[k]];
    }
    return K;
}

/* OT: adaptive view transmission (Section V-C).  Only the N_Tx cameras
 * closest to a client's viewpoint are transmitted; with several clients the
 * edge server needs the union over their viewpoints.  Reading: the ranking
 * is O1's (centre distance in double, ties to the lower rig index) without
 * the coincident-camera shortcut, since the spare cameras are there for
 * viewpoints that move.  mask bit c = transmit camera c; returns the count. */
int32_t fvv_ref_tx_cameras(const ref_camera *rig, int32_t n, const ref_camera *views, int32_t n_views,
                           int32_t n_tx, uint32_t *mask)
{
    if (n > 32 || n < 1 || n_tx < 1) return -1;
    uint32_t m = 0;
    for (int v = 0; v < n_views; ++v) {
        double Cv[3], d[32];
        int order[32];
        ref_center(&views[v], Cv);
        for (int c = 0; c < n; ++c) {
            double Cc[3];
            ref_center(&rig[c], Cc);
            double dx = Cc[0] - Cv[0], dy = Cc[1] - Cv[1], dz = Cc[2] - Cv[2];
            d[c] = sqrt(dx * dx + dy * dy + dz * dz);
            order[c] = c;
        }
        for (int a = 1; a < n; ++a) {
            int x = order[a], b = a - 1;
            while (b >= 0 && d[order[b]] > d[x]) {
                order[b + 1] = order[b];
                --b;
            }
            order[b + 1] = x;
        }
        for (int e = 0; e < n_tx && e < n; ++e) m |= 1u << order[e];
    }
    *mask = m;
    int cnt = 0;
    for (int c = 0; c < n; ++c) cnt += (m >> c) & 1u;
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* O2: pair matrices.
 * Pinhole model (Section VI: a pixel is a ray, its depth fixes the point).
 * With X_c = z K_c^-1 [i,j,1]^T (z = Z-depth) and X_v = R_v R_c^T (X_c - t_c) + t_v:
 *   K_v X_v = z A [i,j,1]^T + a,  A = K_v R_v R_c^T K_c^-1,  a = K_v (t_v - R_v R_c^T t_c)
 * and the third component is the depth seen by the virtual camera.  The
 * backward pair swaps the roles.  Computed in double in a fixed order
 * (relative rotation, then times K^-1 on the right, then K on the left),
 * each entry rounded once to float32. */
static void ref_kmat(const ref_camera *c, double K[9])
{
    K[0] = c->fx; K[1] = 0.0;   K[2] = c->cx;
    K[3] = 0.0;   K[4] = c->fy; K[5] = c->cy;
    K[6] = 0.0;   K[7] = 0.0;   K[8] = 1.0;
}

static void ref_kinv(const ref_camera *c, double Ki[9])
{
    double fx = c->fx, fy = c->fy;
    Ki[0] = 1.0 / fx; Ki[1] = 0.0;      Ki[2] = -(double)c->cx / fx;
    Ki[3] = 0.0;      Ki[4] = 1.0 / fy; Ki[5] = -(double)c->cy / fy;
    Ki[6] = 0.0;      Ki[7] = 0.0;      Ki[8] = 1.0;
}

static void ref_mm(const double X[9], const double Y[9], double Z[9])
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k)
                s += X[r * 3 + k] * Y[k * 3 + c];
            Z[r * 3 + c] = s;
        }
}

/* from camera s (source of the points) to camera d (destination image) */
static void ref_pair_dir(const ref_camera *s, const ref_camera *d, float M[9], float m[3])
{
    double Rrel[9], Ks_inv[9], Kd[9], T1[9], T2[9], trel[3], out[3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)   /* (R_d R_s^T)[r][c] = sum_k R_d[r][k] R_s[c][k] */
                acc += (double)d->R[r * 3 + k] * (double)s->R[c * 3 + k];
            Rrel[r * 3 + c] = acc;
        }
    ref_kinv(s, Ks_inv);
    ref_kmat(d, Kd);
    ref_mm(Rrel, Ks_inv, T1);
    ref_mm(Kd, T1, T2);
    for (int r = 0; r < 3; ++r) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
            acc += Rrel[r * 3 + k] * (double)s->t[k];
        trel[r] = (double)d->t[r] - acc;
    }
    for (int r = 0; r < 3; ++r) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
            acc += Kd[r * 3 + k] * trel[k];
        out[r] = acc;
    }
    for (int e = 0; e < 9; ++e) M[e] = (float)T2[e];
    for (int e = 0; e < 3; ++e) m[e] = (float)out[e];
}

void fvv_ref_pair(const ref_camera *src, const ref_camera *virt, ref_pair *p)
{
    ref_pair_dir(src, virt, p->A, p->a);
    ref_pair_dir(virt, src, p->B, p->b);
    p->sx = (float)((double)virt->fx / (double)src->fx);
    p->sy = (float)((double)virt->fy / (double)src->fy);
}

/* ------------------------------------------------------------------------ */
/* O3: depth decode.  Millimetres -> metres (float32 division by 1000), then
 * the quadratic correction of Eq. 1, z_post = (alpha z + beta) z, in that
 * operation order.  (0, 1) is an exact identity.  Two values carry no live
 * depth: 0 (no depth, e.g. object boundaries) and 0xFFFF, the background
 * signal (the capture side removes background depth from the live stream,
 * Section IV-B; the layered synthesis takes it from the background model). */
#define REF_BG_MM 0xFFFFu
static inline int ref_has_depth(uint16_t d) { return d != 0 && d != REF_BG_MM; }

float fvv_ref_decode_depth(uint16_t d, float alpha, float beta)
{
    float z = (float)d / 1000.0f;
    float s = alpha * z;
    s = s + beta;
    return s * z;
}

/* O3 over a plane: float32 bits of the decoded depth, 0xFFFFFFFF where the
 * millimetre value carries no depth */
void fvv_ref_decode_plane(const uint16_t *mm, int64_t n, float alpha, float beta, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t b = 0xFFFFFFFFu;
        if (ref_has_depth(mm[i])) {
            float z = fvv_ref_decode_depth(mm[i], alpha, beta);
            memcpy(&b, &z, 4);
        }
        out[i] = b;
    }
}

static inline uint32_t ref_fbits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

static inline float ref_bitsf(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}

/* float32 projection of one pixel: p_r = ((M_r0 i + M_r1 j) + M_r2) z + m_r */
static inline void ref_project(const float M[9], const float m[3], float i, float j,
                               float z, float p[3])
{
    for (int r = 0; r < 3; ++r) {
        float s = M[r * 3 + 0] * i;
        float s2 = M[r * 3 + 1] * j;
        s = s + s2;
        s = s + M[r * 3 + 2];
        s = s * z;
        p[r] = s + m[r];
    }
}

/* ------------------------------------------------------------------------ */
/* O4: forward splat (3D warping of every valid reference pixel into the
 * virtual view, Section VI) into a z-buffer of packed 64-bit keys
 *   key = bits32(virtual depth) << 32 | camera rig index << 27 | source pixel index
 * Smaller key wins: nearer depth first (positive float32 bit patterns order
 * like the values), then lower camera index, then lower source pixel index.
 * Footprint (reading): each point covers the pixel centres x with
 * u - mx/2 <= x < u + mx/2 (same for rows), where mx = clamp((sx z)/p2, 1,
 * max_fp) is the point's own magnification; a fronto-parallel surface is then
 * tiled without cracks or overlaps.  In float32 with correctly rounded
 * division: u = p0/p2, v = p1/p2, mx = (sx z)/p2, my = (sy z)/p2.  Points
 * with p2 <= 0.01 m or non-finite image coordinates are dropped.
 * Z must hold W*H keys; it is initialised here. */
typedef struct {
    const uint16_t *depth;    /* source depth, millimetres */
    int64_t depth_pitch;      /* in elements */
    int32_t W, H, rig_index;
    float alpha, beta;
    const ref_pair *pair;
} ref_src;

void fvv_ref_splat(const ref_src *src, int32_t K, int32_t W, int32_t H,
                   float max_fp, uint64_t *Z)
{
    const float zclip = 0.01f;
    for (int64_t e = 0; e < (int64_t)W * H; ++e) Z[e] = REF_EMPTY;
    for (int k = 0; k < K; ++k) {
        const ref_src *s = &src[k];
        const ref_pair *p = s->pair;
        for (int j = 0; j < s->H; ++j) {
            for (int i = 0; i < s->W; ++i) {
                uint16_t d = s->depth[(int64_t)j * s->depth_pitch + i];
                if (!ref_has_depth(d)) continue;
                float z = fvv_ref_decode_depth(d, s->alpha, s->beta);
                float q[3];
                ref_project(p->A, p->a, (float)i, (float)j, z, q);
                if (!(q[2] > zclip)) continue;
                float u = q[0] / q[2];
                float v = q[1] / q[2];
                if (!isfinite(u) || !isfinite(v)) continue;
                float mx = (p->sx * z) / q[2];
                float my = (p->sy * z) / q[2];
                mx = fminf(fmaxf(mx, 1.0f), max_fp);
                my = fminf(fmaxf(my, 1.0f), max_fp);
                float hx = 0.5f * mx, hy = 0.5f * my;
                float x0f = ceilf(u - hx), x1f = ceilf(u + hx) - 1.0f;
                float y0f = ceilf(v - hy), y1f = ceilf(v + hy) - 1.0f;
                x0f = fmaxf(x0f, 0.0f);
                y0f = fmaxf(y0f, 0.0f);
                x1f = fminf(x1f, (float)(W - 1));
                y1f = fminf(y1f, (float)(H - 1));
                if (x0f > x1f || y0f > y1f) continue;
                uint64_t key = ((uint64_t)ref_fbits(q[2]) << 32)
                             | ((uint64_t)(uint32_t)s->rig_index << 27)
                             | (uint64_t)((int64_t)j * s->W + i);
                for (int y = (int)y0f; y <= (int)y1f; ++y)
                    for (int x = (int)x0f; x <= (int)x1f; ++x) {
                        uint64_t *cell = &Z[(int64_t)y * W + x];
                        if (key < *cell) *cell = key;
                    }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* O5: 3x3 depth filter on the key map (the "image filtering" that goes with
 * backward warping against cracks, Section VI).  Reads Z only.
 * V = valid keys among the 8 neighbours (outside the image counts as absent),
 * z(k) = the float32 depth in the key's upper half.
 *  (a) crack fill: an empty pixel with |V| >= 5 takes the lower median of V
 *      (element floor((|V|-1)/2) of V sorted by key);
 *  (b) speckle removal: a valid pixel with |V| >= 5 none of which satisfies
 *      |z(k) - z0| <= tau z0 takes the lower median of V;
 *  otherwise the key is kept. */
static uint64_t ref_lower_median(uint64_t *v, int n)
{
    for (int a = 1; a < n; ++a) {
        uint64_t x = v[a];
        int b = a - 1;
        while (b >= 0 && v[b] > x) {
            v[b + 1] = v[b];
            --b;
        }
        v[b + 1] = x;
    }
    return v[(n - 1) / 2];
}

void fvv_ref_filter(const uint64_t *Z, int32_t W, int32_t H, float tau, uint64_t *Zf)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            uint64_t c = Z[(int64_t)y * W + x];
            uint64_t v[8];
            int n = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    int xx = x + dx, yy = y + dy;
                    if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
                    uint64_t k = Z[(int64_t)yy * W + xx];
                    if (k != REF_EMPTY) v[n++] = k;
                }
            uint64_t out = c;
            if (n >= 5) {
                if (c == REF_EMPTY) {
                    out = ref_lower_median(v, n);
                } else {
                    float z0 = ref_bitsf((uint32_t)(c >> 32));
                    float lim = tau * z0;
                    int near = 0;
                    for (int e = 0; e < n; ++e) {
                        float zk = ref_bitsf((uint32_t)(v[e] >> 32));
                        if (fabsf(zk - z0) <= lim) near = 1;
                    }
                    if (!near) out = ref_lower_median(v, n);
                }
            }
            Zf[(int64_t)y * W + x] = out;
        }
}

/* ------------------------------------------------------------------------ */
/* O6: backward colour fetch, per-camera depth consistency, view-weighted
 * blend (backward warping, Section VI; mixing by camera distance).
 * For each output pixel with a valid filtered key at depth zf, and each
 * selected camera in selection order:
 *   q = B [x,y,1] zf + b (float32, as O4), require q2 > 0.01,
 *   u = q0/q2, v = q1/q2 (float32), require -0.5 <= u <= W_c - 0.5 and the
 *   same for v
 *   (the sample lies on the source image's pixel area),
 *   i0 = floor(u), j0 = floor(v), fu = u - i0, fv = v - j0;
 *   taps (i0,j0) (i0+1,j0) (i0,j0+1) (i0+1,j0+1) with bilinear weights
 *   (1-fu)(1-fv), fu(1-fv), (1-fu)fv, fu fv;
 *   a tap is valid iff it lies inside the image, has depth, and its decoded
 *   depth zs satisfies |zs - q2| <= tau q2 (float32);
 *   col_c = sum w_n rgb_n / sum w_n over valid taps (double); the camera is
 *   dropped when the sum of weights is 0.
 * out = sum w_c col_c / sum w_c over surviving cameras (double), rounded
 * half up and capped at 255; no surviving camera => hole.
 * Outputs: rgb (W*H*3), hole flags (1 = hole), depth (zf, 0 for holes). */
typedef struct {
    const uint8_t *rgb;       /* source colour, 3 bytes per pixel */
    int64_t rgb_pitch;        /* bytes */
    const uint16_t *depth;
    int64_t depth_pitch;      /* elements */
    int32_t W, H;
    float alpha, beta;
    const ref_pair *pair;
    double weight;
} ref_tex;

void fvv_ref_blend(const uint64_t *Zf, int32_t W, int32_t H, const ref_tex *tex,
                   int32_t K, float tau, uint8_t *rgb, uint8_t *hole, float *depth_out)
{
    const float zclip = 0.01f;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t o = (int64_t)y * W + x;
            uint64_t key = Zf[o];
            rgb[o * 3 + 0] = rgb[o * 3 + 1] = rgb[o * 3 + 2] = 0;
            hole[o] = 1;
            depth_out[o] = 0.0f;
            if (key == REF_EMPTY) continue;
            float zf = ref_bitsf((uint32_t)(key >> 32));
            double acc[3] = {0.0, 0.0, 0.0}, wsum = 0.0;
            for (int k = 0; k < K; ++k) {
                const ref_tex *t = &tex[k];
                float q[3];
                ref_project(t->pair->B, t->pair->b, (float)x, (float)y, zf, q);
                if (!(q[2] > zclip)) continue;
                float u = q[0] / q[2];
                float v = q[1] / q[2];
                if (!(u >= -0.5f && u <= (float)t->W - 0.5f)) continue;
                if (!(v >= -0.5f && v <= (float)t->H - 0.5f)) continue;
                float fi0 = floorf(u), fj0 = floorf(v);
                float fu = u - fi0, fv = v - fj0;
                int i0 = (int)fi0, j0 = (int)fj0;
                float lim = tau * q[2];
                double wt[4] = {(1.0 - fu) * (1.0 - fv), fu * (1.0 - (double)fv),
                                (1.0 - fu) * (double)fv, (double)fu * (double)fv};
                int ti[4] = {i0, i0 + 1, i0, i0 + 1};
                int tj[4] = {j0, j0, j0 + 1, j0 + 1};
                double cacc[3] = {0.0, 0.0, 0.0}, csum = 0.0;
                for (int n = 0; n < 4; ++n) {
                    if (ti[n] < 0 || tj[n] < 0 || ti[n] >= t->W || tj[n] >= t->H) continue;
                    uint16_t d = t->depth[(int64_t)tj[n] * t->depth_pitch + ti[n]];
                    if (!ref_has_depth(d)) continue;
                    float zs = fvv_ref_decode_depth(d, t->alpha, t->beta);
                    if (!(fabsf(zs - q[2]) <= lim)) continue;
                    const uint8_t *px = t->rgb + (int64_t)tj[n] * t->rgb_pitch + (int64_t)ti[n] * 3;
                    for (int ch = 0; ch < 3; ++ch) cacc[ch] += wt[n] * (double)px[ch];
                    csum += wt[n];
                }
                if (!(csum > 0.0)) continue;
                for (int ch = 0; ch < 3; ++ch) acc[ch] += t->weight * (cacc[ch] / csum);
                wsum += t->weight;
            }
            if (!(wsum > 0.0)) continue;
            for (int ch = 0; ch < 3; ++ch) {
                double val = floor(acc[ch] / wsum + 0.5);
                if (val > 255.0) val = 255.0;
                if (val < 0.0) val = 0.0;
                rgb[o * 3 + ch] = (uint8_t)val;
            }
            hole[o] = 0;
            depth_out[o] = zf;
        }
}

/* ------------------------------------------------------------------------ */
/* O6': input of the learned blend/inpaint network (reading: the paper mixes
 * the warped cameras with fixed distance weights, Section VI; the learned
 * path hands the same per-camera evidence to a network instead).  For every
 * pixel whose filtered z-buffer holds a point, and for each selected camera
 * slot k (selection order), the depth-consistent bilinear colour of that
 * camera -- the same sample O6 mixes -- gives five values: R, G, B divided
 * by 255, the inverse source-camera depth 0.5 / q_z (fp32, capped at 1) and
 * a validity flag 1.  Cameras that give no sample, unused slots and pixels
 * without a point give zeros.  Output: H*W*15 doubles, pixel-major. */
void fvv_ref_stack(const uint64_t *Zf, int32_t W, int32_t H, const ref_tex *tex,
                   int32_t K, float tau, double *stack)
{
    const float zclip = 0.01f;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t o = (int64_t)y * W + x;
            double *st = stack + o * 15;
            for (int c = 0; c < 15; ++c) st[c] = 0.0;
            uint64_t key = Zf[o];
            if (key == REF_EMPTY) continue;
            float zf = ref_bitsf((uint32_t)(key >> 32));
            for (int k = 0; k < K && k < 3; ++k) {
                const ref_tex *t = &tex[k];
                float q[3];
                ref_project(t->pair->B, t->pair->b, (float)x, (float)y, zf, q);
                if (!(q[2] > zclip)) continue;
                float u = q[0] / q[2];
                float v = q[1] / q[2];
                if (!(u >= -0.5f && u <= (float)t->W - 0.5f)) continue;
                if (!(v >= -0.5f && v <= (float)t->H - 0.5f)) continue;
                float fi0 = floorf(u), fj0 = floorf(v);
                float fu = u - fi0, fv = v - fj0;
                int i0 = (int)fi0, j0 = (int)fj0;
                float lim = tau * q[2];
                double wt[4] = {(1.0 - fu) * (1.0 - fv), fu * (1.0 - (double)fv),
                                (1.0 - fu) * (double)fv, (double)fu * (double)fv};
                double cacc[3] = {0.0, 0.0, 0.0}, csum = 0.0;
                for (int n = 0; n < 4; ++n) {
                    int ii = i0 + (n & 1), jj = j0 + (n >> 1);
                    if (ii < 0 || jj < 0 || ii >= t->W || jj >= t->H) continue;
                    uint16_t d = t->depth[(int64_t)jj * t->depth_pitch + ii];
                    if (!ref_has_depth(d)) continue;
                    float zs = fvv_ref_decode_depth(d, t->alpha, t->beta);
                    if (!(fabsf(zs - q[2]) <= lim)) continue;
                    const uint8_t *px = t->rgb + (int64_t)jj * t->rgb_pitch + (int64_t)ii * 3;
                    for (int ch = 0; ch < 3; ++ch) cacc[ch] += wt[n] * (double)px[ch];
                    csum += wt[n];
                }
                if (!(csum > 0.0)) continue;
                for (int ch = 0; ch < 3; ++ch) st[5 * k + ch] = cacc[ch] / csum / 255.0;
                float inv = 0.5f / q[2];
                st[5 * k + 3] = inv < 1.0f ? (double)inv : 1.0;
                st[5 * k + 4] = 1.0;
            }
        }
}

/* ------------------------------------------------------------------------ */
/* O7: hole fill.  The paper leaves areas no camera sees black (Section IX);
 * mode 1 reproduces that.  Mode 0 (reading; disocclusions uncover
 * background): for every hole, the nearest non-hole pixel to the left,
 * right, up and down of the blend output; the candidate with the largest
 * depth wins, then the nearest, then the order left, right, up, down; its
 * colour is copied.  No candidate => black.  Reads the blend output only. */
void fvv_ref_fill(const uint8_t *rgb, const uint8_t *hole, const float *depth,
                  int32_t W, int32_t H, int32_t mode, uint8_t *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t o = (int64_t)y * W + x;
            if (!hole[o]) {
                memcpy(out + o * 3, rgb + o * 3, 3);
                continue;
            }
            out[o * 3 + 0] = out[o * 3 + 1] = out[o * 3 + 2] = 0;
            if (mode != 0) continue;
            int best = -1, best_dist = 0;
            float best_z = 0.0f;
            int64_t best_o = 0;
            const int dxs[4] = {-1, 1, 0, 0}, dys[4] = {0, 0, -1, 1};
            for (int dir = 0; dir < 4; ++dir) {
                int xx = x, yy = y, dist = 0;
                for (;;) {
                    xx += dxs[dir];
                    yy += dys[dir];
                    ++dist;
                    if (xx < 0 || yy < 0 || xx >= W || yy >= H) { dist = -1; break; }
                    if (!hole[(int64_t)yy * W + xx]) break;
                }
                if (dist < 0) continue;
                int64_t co = (int64_t)yy * W + xx;
                float cz = depth[co];
                int better = 0;
                if (best < 0) better = 1;
                else if (cz > best_z) better = 1;
                else if (cz == best_z && dist < best_dist) better = 1;
                if (better) {
                    best = dir;
                    best_z = cz;
                    best_dist = dist;
                    best_o = co;
                }
            }
            if (best >= 0) memcpy(out + o * 3, rgb + best_o * 3, 3);
        }
}

/* ------------------------------------------------------------------------ */
/* Whole path: O1 .. O7 for one virtual view.
 * views_rgb[c] / views_depth[c] may be NULL for a camera absent from the
 * frame set.  Optional taps (may be NULL): Z (raw splat), Zf (filtered),
 * blend rgb / hole / depth before the fill.  Returns K (selected cameras) or
 * a negative number on bad arguments. */
int32_t fvv_ref_synthesize(const ref_camera *rig, int32_t n,
                           const uint8_t *const *views_rgb, const int64_t *rgb_pitch,
                           const uint16_t *const *views_depth, const int64_t *depth_pitch,
                           const ref_camera *virt, int32_t k_sel, float tau, float max_fp,
                           int32_t fill_mode, uint8_t *out_rgb,
                           uint64_t *tap_z, uint64_t *tap_zf, uint8_t *tap_rgb,
                           uint8_t *tap_hole, float *tap_depth,
                           int32_t *sel_out, double *w_out)
{
    if (n < 1 || n > 32 || k_sel < 1) return -1;
    int32_t present[64], idx[REF_MAXK];
    double w[REF_MAXK];
    for (int c = 0; c < n; ++c) present[c] = views_rgb[c] != NULL && views_depth[c] != NULL;
    int K = fvv_ref_select(rig, present, n, virt, k_sel, idx, w);
    int32_t W = virt->width, H = virt->height;
    int64_t npx = (int64_t)W * H;
    uint64_t *Z = tap_z ? tap_z : (uint64_t *)malloc(npx * 8);
    uint64_t *Zf = tap_zf ? tap_zf : (uint64_t *)malloc(npx * 8);
    uint8_t *rgb = tap_rgb ? tap_rgb : (uint8_t *)malloc(npx * 3);
    uint8_t *hole = tap_hole ? tap_hole : (uint8_t *)malloc(npx);
    float *dep = tap_depth ? tap_depth : (float *)malloc(npx * 4);
    ref_pair pairs[REF_MAXK];
    ref_src srcs[REF_MAXK];
    ref_tex texs[REF_MAXK];
    for (int k = 0; k < K; ++k) {
        const ref_camera *c = &rig[idx[k]];
        fvv_ref_pair(c, virt, &pairs[k]);
        srcs[k].depth = views_depth[idx[k]];
        srcs[k].depth_pitch = depth_pitch[idx[k]];
        srcs[k].W = c->width;
        srcs[k].H = c->height;
        srcs[k].rig_index = idx[k];
        srcs[k].alpha = c->depth_alpha;
        srcs[k].beta = c->depth_beta;
        srcs[k].pair = &pairs[k];
        texs[k].rgb = views_rgb[idx[k]];
        texs[k].rgb_pitch = rgb_pitch[idx[k]];
        texs[k].depth = views_depth[idx[k]];
        texs[k].depth_pitch = depth_pitch[idx[k]];
        texs[k].W = c->width;
        texs[k].H = c->height;
        texs[k].alpha = c->depth_alpha;
        texs[k].beta = c->depth_beta;
        texs[k].pair = &pairs[k];
        texs[k].weight = w[k];
        if (sel_out) sel_out[k] = idx[k];
        if (w_out) w_out[k] = w[k];
    }
    fvv_ref_splat(srcs, K, W, H, max_fp, Z);
    fvv_ref_filter(Z, W, H, tau, Zf);
    fvv_ref_blend(Zf, W, H, texs, K, tau, rgb, hole, dep);
    fvv_ref_fill(rgb, hole, dep, W, H, fill_mode, out_rgb);
    if (!tap_z) free(Z);
    if (!tap_zf) free(Zf);
    if (!tap_rgb) free(rgb);
    if (!tap_hole) free(hole);
    if (!tap_depth) free(dep);
    return K;
}

/* Timing mode (the benchmark's CPU baseline): fvv_ref_synthesize for
 * n_views virtual cameras of one frame set, views spread over `threads`
 * OpenMP threads (dynamic schedule).  Each view is computed exactly as a
 * call of fvv_ref_synthesize alone computes it (the views share only
 * read-only inputs), so the outputs equal those of the single-threaded
 * calls; outs[v] receives view v's RGB8.  Returns the number of views whose
 * arguments were rejected (0 on success). */
int32_t fvv_ref_synthesize_views(const ref_camera *rig, int32_t n,
                                 const uint8_t *const *views_rgb, const int64_t *rgb_pitch,
                                 const uint16_t *const *views_depth, const int64_t *depth_pitch,
                                 const ref_camera *virts, int32_t n_views, int32_t k_sel, float tau,
                                 float max_fp, int32_t fill_mode, uint8_t *const *outs, int32_t threads)
{
    int32_t bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) reduction(+ : bad)
    for (int32_t v = 0; v < n_views; ++v) {
        const int32_t K = fvv_ref_synthesize(rig, n, views_rgb, rgb_pitch, views_depth, depth_pitch, &virts[v],
                                             k_sel, tau, max_fp, fill_mode, outs[v], NULL, NULL, NULL, NULL,
                                             NULL, NULL, NULL);
        bad += K < 0;
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* OC: 12-bit depth coding for 8-bit YUV420 codecs (Section V-A).
 * Quantisation, Eq. 2: Y = (2^12 - 3)(1/z - 1/z_far)/(1/z_near - 1/z_far) + 2
 * (reading: double precision in that operation order, rounded half up);
 * code 1 = no depth, or out of range, read as a rounded value outside
 * 2..4095 (so a depth within half a code of a clipping plane keeps the end
 * code whatever the float32 rounding of the plane); code 0 = the background
 * signal, 0xFFFF in millimetre maps (O3).
 * Bit re-arrangement of each 2x2 block (p11 p12 / p21 p22) onto I420 planes:
 * Y of each pixel = its 8 LSBs, flipped to 255 - LSBs when its 4 MSBs are
 * odd (Eq. 3); U = the MSBs of p11 and p12 bit-interleaved, V = those of p21
 * and p22.  Reading of the missing figure: bit 2k of U is bit k of p11's
 * MSBs, bit 2k+1 is bit k of p12's (the most variable bits, the low ones,
 * land lowest).
 * Decoding inverts both steps; code 0 becomes 0xFFFF, code 1 becomes 0, and
 * a code >= 2 becomes
 * z = 1 / ((Y - 2)/4093 (1/z_near - 1/z_far) + 1/z_far) (double) and then
 * whole millimetres, floor(1000 z + 0.5) clamped to [1, 65535]. */
static inline uint8_t ref_interleave4(uint32_t a, uint32_t b)
{
    uint32_t v = 0;
    for (int k = 0; k < 4; ++k) v |= ((a >> k) & 1u) << (2 * k) | ((b >> k) & 1u) << (2 * k + 1);
    return (uint8_t)v;
}

uint16_t fvv_ref_depth_code(uint16_t mm, float z_near, float z_far)
{
    if (mm == REF_BG_MM) return 0;
    if (mm == 0) return 1;
    double z = (double)mm / 1000.0;
    double zn = (double)z_near, zf = (double)z_far;
    double a = 1.0 / z - 1.0 / zf;
    double b = 1.0 / zn - 1.0 / zf;
    double y = 4093.0 * a / b + 2.0;
    double r = floor(y + 0.5);
    if (!(r >= 2.0 && r <= 4095.0)) return 1;
    return (uint16_t)r;
}

uint16_t fvv_ref_code_depth(uint16_t code, float z_near, float z_far)
{
    if (code == 0) return REF_BG_MM;
    if (code == 1) return 0;
    double zn = (double)z_near, zf = (double)z_far;
    double t = (double)(code - 2) / 4093.0;
    double inv = t * (1.0 / zn - 1.0 / zf) + 1.0 / zf;
    double z = 1.0 / inv;
    double mm = floor(z * 1000.0 + 0.5);
    if (mm < 1.0) mm = 1.0;
    if (mm > 65535.0) mm = 65535.0;
    return (uint16_t)mm;
}

/* Eq. 2 over a plane: mm (pitch in elements) -> codes (W per row) */
void fvv_ref_depth_codes(const uint16_t *mm, int64_t pitch, int32_t W, int32_t H, float z_near, float z_far,
                         uint16_t *codes)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            codes[(int64_t)y * W + x] = fvv_ref_depth_code(mm[(int64_t)y * pitch + x], z_near, z_far);
}

void fvv_ref_codes_depth(const uint16_t *codes, int32_t W, int32_t H, float z_near, float z_far, uint16_t *mm)
{
    for (int64_t i = 0; i < (int64_t)W * H; ++i) mm[i] = fvv_ref_code_depth(codes[i], z_near, z_far);
}

/* codes (H x W, W and H even) -> I420 planes */
void fvv_ref_pack_y12(const uint16_t *codes, int32_t W, int32_t H, uint8_t *Y, uint8_t *U, uint8_t *V)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            uint32_t c = codes[(int64_t)y * W + x] & 0xFFFu;
            uint32_t msb = c >> 8, lsb = c & 0xFFu;
            Y[(int64_t)y * W + x] = (uint8_t)((msb & 1u) ? 255u - lsb : lsb);
        }
    for (int r = 0; r < H / 2; ++r)
        for (int c = 0; c < W / 2; ++c) {
            const uint16_t *p1 = codes + (int64_t)(2 * r) * W + 2 * c;
            const uint16_t *p2 = p1 + W;
            U[(int64_t)r * (W / 2) + c] = ref_interleave4(p1[0] >> 8, p1[1] >> 8);
            V[(int64_t)r * (W / 2) + c] = ref_interleave4(p2[0] >> 8, p2[1] >> 8);
        }
}

/* I420 planes -> codes */
void fvv_ref_unpack_y12(const uint8_t *Y, const uint8_t *U, const uint8_t *V, int32_t W, int32_t H, uint16_t *codes)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            uint32_t uv = (y & 1) ? V[(int64_t)(y / 2) * (W / 2) + x / 2] : U[(int64_t)(y / 2) * (W / 2) + x / 2];
            uint32_t msb = 0;
            for (int k = 0; k < 4; ++k) msb |= ((uv >> (2 * k + (x & 1))) & 1u) << k;
            uint32_t yv = Y[(int64_t)y * W + x];
            uint32_t lsb = (msb & 1u) ? 255u - yv : yv;
            codes[(int64_t)y * W + x] = (uint16_t)(msb << 8 | lsb);
        }
}

/* ------------------------------------------------------------------------ */
/* OJ: joint bilateral pre-filter of the live depth (Section VI: small holes
 * and gaps at object edges are closed before warping with a joint bilateral
 * filter; the paper states no parameters).  Readings:
 *  - it fills holes only: a pixel without depth (0) takes the bilateral
 *    mean of the valid depths in its (2r+1)^2 window, guided by the live
 *    colour; measured depths are left as they are, and background-signalled
 *    pixels (0xFFFF) are neither filled nor used;
 *  - weights are a spatial Gaussian (sigma_s, pixels) times a range Gaussian
 *    of the L1 colour distance (sigma_c, 8-bit levels), each rounded to a
 *    12-bit integer, exp in double: ws = floor(4096 exp(-(dx^2+dy^2) /
 *    (2 sigma_s^2)) + 0.5), wc = floor(4096 exp(-d^2 / (2 sigma_c^2)) + 0.5),
 *    w = ws wc;
 *  - a hole is filled when at least min_valid neighbours have w > 0; the
 *    filled depth is floor((sum w D + floor(sum w / 2)) / sum w) in integer
 *    arithmetic, millimetres;
 *  - one pass over the original map (filled values are not reused);
 *  - it runs on the transmitted millimetres, before the Eq. 1 decode. */
static void ref_jbf_tables(int32_t radius, float sigma_s, float sigma_c, uint32_t *ws, uint32_t *wc)
{
    const int n = 2 * radius + 1;
    for (int dy = -radius; dy <= radius; ++dy)
        for (int dx = -radius; dx <= radius; ++dx) {
            double e = exp(-(double)(dx * dx + dy * dy) / (2.0 * (double)sigma_s * (double)sigma_s));
            ws[(dy + radius) * n + dx + radius] = (uint32_t)floor(4096.0 * e + 0.5);
        }
    for (int d = 0; d <= 765; ++d) {
        double e = exp(-(double)d * (double)d / (2.0 * (double)sigma_c * (double)sigma_c));
        wc[d] = (uint32_t)floor(4096.0 * e + 0.5);
    }
}

void fvv_ref_prefilter(const uint8_t *rgb, int64_t rgb_pitch, const uint16_t *depth, int64_t depth_pitch,
                       int32_t W, int32_t H, int32_t radius, float sigma_s, float sigma_c, int32_t min_valid,
                       uint16_t *out)
{
    uint32_t ws[49], wc[766];
    ref_jbf_tables(radius, sigma_s, sigma_c, ws, wc);
    const int n = 2 * radius + 1;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const uint16_t d = depth[(int64_t)y * depth_pitch + x];
            uint16_t res = d;
            if (d == 0) {
                const uint8_t *cp = rgb + (int64_t)y * rgb_pitch + (int64_t)x * 3;
                uint64_t sw = 0, swd = 0;
                int cnt = 0;
                for (int dy = -radius; dy <= radius; ++dy)
                    for (int dx = -radius; dx <= radius; ++dx) {
                        const int xx = x + dx, yy = y + dy;
                        if ((dx == 0 && dy == 0) || xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
                        const uint16_t q = depth[(int64_t)yy * depth_pitch + xx];
                        if (!ref_has_depth(q)) continue;
                        const uint8_t *cq = rgb + (int64_t)yy * rgb_pitch + (int64_t)xx * 3;
                        const int dist = abs((int)cp[0] - (int)cq[0]) + abs((int)cp[1] - (int)cq[1]) +
                                         abs((int)cp[2] - (int)cq[2]);
                        const uint64_t w = (uint64_t)ws[(dy + radius) * n + dx + radius] * wc[dist];
                        if (w == 0) continue;
                        sw += w;
                        swd += w * q;
                        ++cnt;
                    }
                if (cnt >= min_valid && sw > 0) res = (uint16_t)((swd + sw / 2) / sw);
            }
            out[(int64_t)y * W + x] = res;
        }
}
