/*
 * FP64 CPU oracle for the semantic Gaussian rasterizer and view scorer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or constant with
 * the HIP library.
 *
 * What it computes (paper: "Understanding while Exploring: Semantics-driven
 * Active Mapping", arXiv 2506.00225):
 *   - the per-pixel front-to-back alpha compositing of Eq. 1 (colour, depth,
 *     silhouette) and Eq. 3 (sparse top-k semantics scattered into a full
 *     class map), Sec. 3.1 "Gaussian Mapping" / "Semantic Rendering";
 *   - its analytic gradient (Sec. 3.1 says the renderer is differentiable
 *     and that the semantic loss only reaches semantic attributes);
 *   - the per-view scores behind Eq. 5 (count of pixels with zero
 *     silhouette) and Eq. 6 (summed per-pixel entropy, Eq. 4, after the
 *     clip-to-[0.001,1] and renormalisation of Sec. 3.2).
 *
 * The paper does not spell out f_i(p); it is read as the EWA splat
 * o * exp(-1/2 d^T Sigma2^-1 d) with an opacity clamp alpha_max, a 1/255
 * cutoff and a 1e-4 transmittance stop (readings listed in the design
 * notes).  Everything here is plain double precision, one pixel at a time,
 * in the order the equations state; the only acceleration is that a pixel's
 * candidate list is read from a per-row list of Gaussians whose pixel
 * rectangle covers that row (a pure filter: outside its rectangle a
 * Gaussian's alpha is below the cutoff by construction), and "brute" mode
 * drops even that.
 *
 * Where single and double precision may legitimately decide a threshold
 * test differently (alpha near alpha_min, T (1 - alpha) near t_min), the
 * pixel walk can take the other outcome of each such "flagged" decision
 * (a per-pixel branch word), so a comparison can follow the outcome the
 * single-precision path took and still check every value exactly.
 *
 * Parity status: every function here is pinned by the CPU tests (closed
 * forms, textbook over-compositing, invariants, brute force, central finite
 * differences, the tight rectangle by numerical search, flipped decisions
 * against closed forms and against the threshold moved across them).  None
 * is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* camera: R[9] (world->camera, row-major), t[3], fx, fy, cx, cy, W, H */
enum { CAM_R = 0, CAM_T = 9, CAM_FX = 12, CAM_FY = 13, CAM_CX = 14, CAM_CY = 15, CAM_W = 16, CAM_H = 17 };
/* config: alpha_min, alpha_max, t_min, z_near, lowpass, tile_w, tile_h,
 *         sem_grad_to_geometry, margin_alpha, margin_t */
enum { CF_AMIN = 0, CF_AMAX, CF_TMIN, CF_ZNEAR, CF_LOWPASS, CF_TW, CF_TH, CF_SEMGEO, CF_MA, CF_MT };

static uint32_t f32_bits(double z) {
    float f = (float)z;
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* Quaternion (w,x,y,z), normalised, to a rotation matrix (row-major). */
static void quat_to_rot(const double *q, double *R, double *qn_out, double *norm_out) {
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
    if (qn_out) { qn_out[0] = w; qn_out[1] = x; qn_out[2] = y; qn_out[3] = z; }
    if (norm_out) *norm_out = n;
}

/*
 * Projection of every Gaussian into one camera (Sec. 3.1: transform to
 * camera space, project to the image plane).  EWA: Sigma2 = J W Sigma3 W^T
 * J^T + lowpass*I with Sigma3 = Rq diag(s^2) Rq^T.  Culling: z <= z_near,
 * det(Sigma2) <= 0, opacity below the alpha cutoff, an empty pixel
 * rectangle, or a projected mean beyond 2^30 px.  The rectangle is the exact axis-aligned box of the set where
 * o*exp(-Q/2) >= alpha_min, i.e. Q <= 2 ln(o/alpha_min), with pixel centres
 * at (col+0.5, row+0.5).
 */
int oracle_project(int64_t n, const double *means, const double *scales, const double *quats,
                   const double *opacity, const double *cam, const double *cfg,
                   double *mean2d, double *conic, double *cov2d, double *pcam,
                   int32_t *rect, uint32_t *zbits, int32_t *visible) {
    const double *W = cam + CAM_R, *t = cam + CAM_T;
    const double fx = cam[CAM_FX], fy = cam[CAM_FY], cx = cam[CAM_CX], cy = cam[CAM_CY];
    const int width = (int)cam[CAM_W], height = (int)cam[CAM_H];
    const double amin = cfg[CF_AMIN], znear = cfg[CF_ZNEAR], lp = cfg[CF_LOWPASS];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const double *m = means + 3 * i;
        double p[3];
        for (int r = 0; r < 3; r++) p[r] = W[3 * r + 0] * m[0] + W[3 * r + 1] * m[1] + W[3 * r + 2] * m[2] + t[r];
        pcam[3 * i + 0] = p[0]; pcam[3 * i + 1] = p[1]; pcam[3 * i + 2] = p[2];
        visible[i] = 0;
        rect[4 * i + 0] = rect[4 * i + 1] = rect[4 * i + 2] = rect[4 * i + 3] = -1;
        mean2d[2 * i] = mean2d[2 * i + 1] = 0;
        conic[3 * i] = conic[3 * i + 1] = conic[3 * i + 2] = 0;
        cov2d[3 * i] = cov2d[3 * i + 1] = cov2d[3 * i + 2] = 0;
        zbits[i] = f32_bits(p[2]);
        if (!(p[2] > znear)) continue;
        /* Sigma3 = Rq diag(s^2) Rq^T */
        double Rq[9];
        quat_to_rot(quats + 4 * i, Rq, NULL, NULL);
        const double *s = scales + 3 * i;
        double S3[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0;
                for (int c = 0; c < 3; c++) acc += Rq[3 * a + c] * s[c] * s[c] * Rq[3 * b + c];
                S3[3 * a + b] = acc;
            }
        /* J (2x3), T = J W (2x3) */
        const double z = p[2];
        double J[6] = {fx / z, 0, -fx * p[0] / (z * z), 0, fy / z, -fy * p[1] / (z * z)};
        double T[6];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0;
                for (int c = 0; c < 3; c++) acc += J[3 * a + c] * W[3 * c + b];
                T[3 * a + b] = acc;
            }
        /* Sigma2 = T S3 T^T + lp I */
        double S2[4];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                double acc = 0;
                for (int c = 0; c < 3; c++)
                    for (int d = 0; d < 3; d++) acc += T[3 * a + c] * S3[3 * c + d] * T[3 * b + d];
                S2[2 * a + b] = acc;
            }
        S2[0] += lp; S2[3] += lp;
        const double sxx = S2[0], sxy = 0.5 * (S2[1] + S2[2]), syy = S2[3];
        cov2d[3 * i + 0] = sxx; cov2d[3 * i + 1] = sxy; cov2d[3 * i + 2] = syy;
        const double det = sxx * syy - sxy * sxy;
        if (!(det > 0)) continue;
        conic[3 * i + 0] = syy / det;
        conic[3 * i + 1] = -sxy / det;
        conic[3 * i + 2] = sxx / det;
        const double mx = fx * p[0] / z + cx, my = fy * p[1] / z + cy;
        mean2d[2 * i + 0] = mx; mean2d[2 * i + 1] = my;
        const double o = opacity[i];
        if (!(o >= amin)) continue;
        const double qmax = 2.0 * log(o / amin);
        const double ex = sqrt(qmax * sxx), ey = sqrt(qmax * syy);
        double clo = ceil(mx - ex - 0.5), chi = floor(mx + ex - 0.5);
        double rlo = ceil(my - ey - 0.5), rhi = floor(my + ey - 0.5);
        if (clo < 0) clo = 0;
        if (chi > width - 1) chi = width - 1;
        if (rlo < 0) rlo = 0;
        if (rhi > height - 1) rhi = height - 1;
        if (!(clo <= chi) || !(rlo <= rhi)) continue;
        /* Reading: a projected mean farther than 2^30 px from the image
         * origin (on either axis) is culled.  Such a point lies outside what
         * a pixel-space record can hold; it reaches the image only through
         * a footprint of the same astronomical size. */
        if (!(fabs(mx) < 1073741824.0) || !(fabs(my) < 1073741824.0)) continue;
        rect[4 * i + 0] = (int32_t)clo; rect[4 * i + 1] = (int32_t)chi;
        rect[4 * i + 2] = (int32_t)rlo; rect[4 * i + 3] = (int32_t)rhi;
        visible[i] = 1;
    }
    return 0;
}

/* ---- front-to-back order: (fp32 depth bits, id) ascending ---- */
static const uint32_t *g_sort_z;
static int cmp_depth(const void *a, const void *b) {
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    if (g_sort_z[i] != g_sort_z[j]) return g_sort_z[i] < g_sort_z[j] ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

static int64_t depth_order(int64_t n, const uint32_t *zbits, const int32_t *visible, int64_t **out) {
    int64_t nv = 0;
    for (int64_t i = 0; i < n; i++) nv += visible[i] != 0;
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (nv > 0 ? nv : 1));
    int64_t c = 0;
    for (int64_t i = 0; i < n; i++)
        if (visible[i]) ord[c++] = i;
    g_sort_z = zbits;
    qsort(ord, (size_t)nv, sizeof(int64_t), cmp_depth);
    *out = ord;
    return nv;
}

/* Per-row candidate lists (ids in front-to-back order) whose rectangle covers
 * the row.  In brute mode every visible Gaussian is a candidate of every row. */
typedef struct { int64_t *ids; int64_t *start; } rowlists;

static void build_rowlists(int64_t nv, const int64_t *ord, const int32_t *rect, int height, int brute, rowlists *rl) {
    rl->start = (int64_t *)calloc((size_t)height + 1, sizeof(int64_t));
    if (brute) {
        rl->ids = (int64_t *)malloc(sizeof(int64_t) * (nv > 0 ? nv : 1));
        memcpy(rl->ids, ord, sizeof(int64_t) * nv);
        return;
    }
    for (int64_t a = 0; a < nv; a++) {
        const int32_t *r = rect + 4 * ord[a];
        for (int y = r[2]; y <= r[3]; y++) rl->start[y + 1]++;
    }
    for (int y = 0; y < height; y++) rl->start[y + 1] += rl->start[y];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (height + 1));
    memcpy(fill, rl->start, sizeof(int64_t) * (height + 1));
    rl->ids = (int64_t *)malloc(sizeof(int64_t) * (rl->start[height] > 0 ? rl->start[height] : 1));
    for (int64_t a = 0; a < nv; a++) {
        const int32_t *r = rect + 4 * ord[a];
        for (int y = r[2]; y <= r[3]; y++) rl->ids[fill[y]++] = ord[a];
    }
    free(fill);
}

/* The projected scene of one view as the compositing reads it. */
typedef struct {
    const double *mean2d, *conic, *depth, *opacity;
    const int32_t *rect;
    int32_t width, height, brute;
    double amin, amax, tmin, ma, mt;
    int64_t nv;
    int64_t *ord;
    rowlists rl;
} view_scene;

static void scene_open(view_scene *s, int64_t n, const double *mean2d, const double *conic, const double *depth,
                       const double *opacity, const int32_t *rect, const uint32_t *zbits, const int32_t *visible,
                       int32_t width, int32_t height, const double *cfg, int32_t brute) {
    s->mean2d = mean2d; s->conic = conic; s->depth = depth; s->opacity = opacity; s->rect = rect;
    s->width = width; s->height = height; s->brute = brute;
    s->amin = cfg[CF_AMIN]; s->amax = cfg[CF_AMAX]; s->tmin = cfg[CF_TMIN];
    s->ma = cfg[CF_MA]; s->mt = cfg[CF_MT];
    s->nv = depth_order(n, zbits, visible, &s->ord);
    build_rowlists(s->nv, s->ord, rect, height, brute, &s->rl);
}

static void scene_close(view_scene *s) {
    free(s->ord);
    free(s->rl.ids);
    free(s->rl.start);
}

/* One blend step's record, kept for the reverse walk. */
typedef struct { int64_t id; double alpha, G, T; int clamped; double dx, dy; } blendrec;
typedef struct { blendrec *r; int64_t cap; } blendbuf;

static void buf_push(blendbuf *b, int64_t nb, const blendrec *x) {
    if (nb == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 64;
        b->r = (blendrec *)realloc(b->r, sizeof(blendrec) * b->cap);
    }
    b->r[nb] = *x;
}

static uint64_t mix64(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
    return h;
}

/* What a pixel's walk reports besides its blends. */
typedef struct {
    double T;        /* final transmittance */
    int flags;       /* bit 0: an alpha near alpha_min; bit 1: a T(1 - alpha) near t_min */
    int nflagged;    /* decisions met within the margins, in walk order */
    uint64_t sig;    /* hash of every candidate's decision (finite differences) */
} walk_info;

/*
 * The front-to-back walk of Eq. 1 at the centre of pixel (x, y): for each
 * candidate in (depth, id) order, alpha = min(alpha_max, o G) with
 * G = exp(-Q/2), Q = d^T A d; skip it when alpha < alpha_min; stop, without
 * blending it, when T (1 - alpha) < t_min; otherwise record the blend (its
 * alpha, G and the transmittance T in front of it) and multiply T by
 * (1 - alpha).
 *
 * A decision is "flagged" when alpha lies within the relative margin
 * margin_alpha of alpha_min, or T (1 - alpha) within margin_t of t_min:
 * there single and double precision may legitimately decide differently.
 * Bit j of `branch` takes the other outcome of the j-th flagged decision met
 * on the walk (j < 32); branch = 0 is the plain definition.
 */
static int64_t walk_pixel(const view_scene *s, int x, int y, uint32_t branch, blendbuf *buf, walk_info *info) {
    const double px = x + 0.5, py = y + 0.5;
    int64_t lb, le;
    if (s->brute) { lb = 0; le = s->nv; }
    else { lb = s->rl.start[y]; le = s->rl.start[y + 1]; }
    double T = 1.0;
    int64_t nb = 0;
    int flags = 0, nfl = 0;
    uint64_t sig = 0;
    for (int64_t a = lb; a < le; a++) {
        const int64_t i = s->rl.ids[a];
        if (!s->brute) {
            const int32_t *r = s->rect + 4 * i;
            if (x < r[0] || x > r[1]) continue;
        }
        const double dx = px - s->mean2d[2 * i], dy = py - s->mean2d[2 * i + 1];
        const double A = s->conic[3 * i], B = s->conic[3 * i + 1], Cc = s->conic[3 * i + 2];
        const double Q = A * dx * dx + 2.0 * B * dx * dy + Cc * dy * dy;
        const double G = exp(-0.5 * Q);
        const double og = s->opacity[i] * G;
        const int clamped = og >= s->amax;
        const double alpha = clamped ? s->amax : og;
        int skip = alpha < s->amin;
        if (fabs(alpha / s->amin - 1.0) < s->ma) {
            flags |= 1;
            if (nfl < 32 && (branch >> nfl) & 1u) skip = !skip;
            nfl++;
        }
        if (skip) {
            sig = mix64(sig, (uint64_t)i * 4 + 0);
            continue;
        }
        const double Tn = T * (1.0 - alpha);
        int stop = Tn < s->tmin;
        if (fabs(Tn / s->tmin - 1.0) < s->mt) {
            flags |= 2;
            if (nfl < 32 && (branch >> nfl) & 1u) stop = !stop;
            nfl++;
        }
        if (stop) {
            sig = mix64(sig, (uint64_t)i * 4 + 3);
            break;
        }
        blendrec rec = {i, alpha, G, T, clamped, dx, dy};
        buf_push(buf, nb, &rec);
        nb++;
        T = Tn;
        sig = mix64(sig, (uint64_t)i * 4 + (clamped ? 2 : 1));
    }
    info->T = T;
    info->flags = flags;
    info->nflagged = nfl;
    info->sig = sig;
    return nb;
}

/* Eq. 1 and Eq. 3 over one pixel's blends: C = sum c_i w_i, D = sum z_i w_i,
 * S = sum w_i and P[idx_ij] += v_ij w_i, with w_i = alpha_i T_i. */
static void accumulate_pixel(const blendbuf *buf, int64_t nb, const double *depth, const double *rgb,
                             const double *sem_val, const int32_t *sem_idx, int32_t k, int32_t C,
                             double *out_c, double *out_d, double *out_s, double *out_p) {
    double Cc[3] = {0, 0, 0}, Dd = 0, Ss = 0;
    for (int m = 0; m < C; m++) out_p[m] = 0;
    for (int64_t b = 0; b < nb; b++) {
        const int64_t i = buf->r[b].id;
        const double w = buf->r[b].alpha * buf->r[b].T;
        for (int c = 0; c < 3; c++) Cc[c] += rgb[3 * i + c] * w;
        Dd += depth[i] * w;
        Ss += w;
        for (int j = 0; j < k; j++) out_p[sem_idx[(int64_t)i * k + j]] += sem_val[(int64_t)i * k + j] * w;
    }
    for (int c = 0; c < 3; c++) out_c[c] = Cc[c];
    *out_d = Dd;
    *out_s = Ss;
}

/*
 * Eq. 1 and Eq. 3, one pixel at a time (walk_pixel, then accumulate_pixel).
 * `branch` (may be NULL: all zero) picks, per pixel, the outcomes of its
 * flagged decisions.  Also reports, per pixel, the flag word and the
 * decision signature of walk_pixel.
 */
int oracle_render(int64_t n, const double *mean2d, const double *conic, const double *depth,
                  const double *opacity, const double *rgb, const double *sem_val, const int32_t *sem_idx,
                  int32_t k, int32_t C, const int32_t *rect, const uint32_t *zbits, const int32_t *visible,
                  int32_t width, int32_t height, const double *cfg, int32_t brute, const uint32_t *branch,
                  double *out_rgb, double *out_depth, double *out_sil, double *out_sem, double *out_tfinal,
                  int32_t *out_ncontrib, int32_t *out_flags, uint64_t *out_sig) {
    view_scene s;
    scene_open(&s, n, mean2d, conic, depth, opacity, rect, zbits, visible, width, height, cfg, brute);
#pragma omp parallel
    {
        blendbuf buf = {NULL, 0};
#pragma omp for schedule(dynamic, 1)
        for (int y = 0; y < height; y++) {
            for (int x = 0; x < width; x++) {
                const int64_t pix = (int64_t)y * width + x;
                walk_info info;
                const int64_t nb = walk_pixel(&s, x, y, branch ? branch[pix] : 0u, &buf, &info);
                accumulate_pixel(&buf, nb, depth, rgb, sem_val, sem_idx, k, C, out_rgb + 3 * pix, out_depth + pix,
                                 out_sil + pix, out_sem + pix * C);
                out_tfinal[pix] = info.T;
                out_ncontrib[pix] = (int32_t)nb;
                if (out_flags) out_flags[pix] = info.flags;
                if (out_sig) out_sig[pix] = info.sig;
            }
        }
        free(buf.r);
    }
    scene_close(&s);
    return 0;
}

/*
 * Every outcome of the flagged decisions of the listed pixels (pix[2 q] = x,
 * pix[2 q + 1] = y): for branch word b in [0, 2^nbits), the maps of pixel q
 * under walk_pixel(.., b, ..), stored at row q * 2^nbits + b of the outputs.
 * out_nflag gives, per row, the flagged decisions that walk met: a walk
 * that met more than nbits of them has outcomes this enumeration leaves out.
 */
int oracle_render_branches(int64_t n, const double *mean2d, const double *conic, const double *depth,
                           const double *opacity, const double *rgb, const double *sem_val, const int32_t *sem_idx,
                           int32_t k, int32_t C, const int32_t *rect, const uint32_t *zbits, const int32_t *visible,
                           int32_t width, int32_t height, const double *cfg, int64_t npix, const int32_t *pix,
                           int32_t nbits, double *out_rgb, double *out_depth, double *out_sil, double *out_sem,
                           double *out_tfinal, int32_t *out_ncontrib, int32_t *out_nflag) {
    if (nbits < 0 || nbits > 16) return 1;
    const int64_t nb_rows = (int64_t)1 << nbits;
    view_scene s;
    scene_open(&s, n, mean2d, conic, depth, opacity, rect, zbits, visible, width, height, cfg, 0);
#pragma omp parallel
    {
        blendbuf buf = {NULL, 0};
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < npix; q++) {
            const int x = pix[2 * q], y = pix[2 * q + 1];
            for (int64_t b = 0; b < nb_rows; b++) {
                const int64_t row = q * nb_rows + b;
                walk_info info;
                const int64_t nb = walk_pixel(&s, x, y, (uint32_t)b, &buf, &info);
                accumulate_pixel(&buf, nb, depth, rgb, sem_val, sem_idx, k, C, out_rgb + 3 * row, out_depth + row,
                                 out_sil + row, out_sem + row * C);
                out_tfinal[row] = info.T;
                out_ncontrib[row] = (int32_t)nb;
                out_nflag[row] = info.nflagged;
            }
        }
        free(buf.r);
    }
    scene_close(&s);
    return 0;
}

/*
 * Analytic gradient of  L = sum_p <g(p), maps(p)>  with respect to each
 * Gaussian's 2D parameters: mean2d (2), conic (a, b, c with Q = a dx^2 +
 * 2 b dx dy + c dy^2), opacity, rgb (3), depth value z, and the k semantic
 * values.  Reverse walk over each pixel's blends (walk_pixel, with the
 * pixel's `branch` word, may be NULL):
 *   w_i = alpha_i T_i;  dL/dz_i^ch = w_i g_ch;
 *   dL/dalpha_i = T_i e_i - R_i / (1 - alpha_i),  e_i = sum_ch z_i^ch g_ch,
 *   R_i = sum_{l>i} e_l w_l;
 * the semantic channels enter e_i only when sem_grad_to_geometry is set
 * (Sec. 3.1: the semantic loss updates only semantic attributes).  alpha =
 * min(alpha_max, o G) has zero derivative where it is clamped.
 */
int oracle_render_backward(int64_t n, const double *mean2d, const double *conic, const double *depth,
                           const double *opacity, const double *rgb, const double *sem_val,
                           const int32_t *sem_idx, int32_t k, int32_t C, const int32_t *rect,
                           const uint32_t *zbits, const int32_t *visible, int32_t width, int32_t height,
                           const double *cfg, const uint32_t *branch, const double *g_rgb, const double *g_depth,
                           const double *g_sil, const double *g_sem,
                           double *d_mean2d, double *d_conic, double *d_opacity, double *d_rgb,
                           double *d_depth, double *d_sem) {
    const int semgeo = cfg[CF_SEMGEO] != 0;
    view_scene s;
    scene_open(&s, n, mean2d, conic, depth, opacity, rect, zbits, visible, width, height, cfg, 0);
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    const int64_t stride = 10 + k; /* mean2d 2, conic 3, opacity 1, rgb 3, depth 1, sem k */
    double *acc = (double *)calloc((size_t)nthreads * n * stride, sizeof(double));
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *my = acc + (int64_t)tid * n * stride;
        blendbuf buf = {NULL, 0};
#pragma omp for schedule(static)
        for (int y = 0; y < height; y++) {
            for (int x = 0; x < width; x++) {
                const int64_t pix = (int64_t)y * width + x;
                walk_info info;
                const int64_t nb = walk_pixel(&s, x, y, branch ? branch[pix] : 0u, &buf, &info);
                const double *gC = g_rgb + 3 * pix;
                const double gD = g_depth[pix], gS = g_sil[pix];
                const double *gP = g_sem + pix * C;
                double R = 0.0;
                for (int64_t b = nb - 1; b >= 0; b--) {
                    const blendrec *rb = buf.r + b;
                    const int64_t i = rb->id;
                    const double alpha = rb->alpha, Ti = rb->T, w = alpha * Ti;
                    double *gi = my + i * stride;
                    double e = gD * depth[i] + gS;
                    for (int c = 0; c < 3; c++) {
                        gi[6 + c] += w * gC[c];
                        e += rgb[3 * i + c] * gC[c];
                    }
                    gi[9] += w * gD;
                    double es = 0;
                    for (int j = 0; j < k; j++) {
                        const double gp = gP[sem_idx[i * k + j]];
                        gi[10 + j] += w * gp;
                        es += sem_val[i * k + j] * gp;
                    }
                    if (semgeo) e += es;
                    const double dalpha = Ti * e - R / (1.0 - alpha);
                    R += e * w;
                    if (rb->clamped) continue;
                    gi[5] += dalpha * rb->G;
                    const double dQ = dalpha * (-0.5 * alpha);
                    const double dx = rb->dx, dy = rb->dy;
                    const double ca = conic[3 * i], cb = conic[3 * i + 1], cc = conic[3 * i + 2];
                    gi[2] += dQ * dx * dx;
                    gi[3] += dQ * 2.0 * dx * dy;
                    gi[4] += dQ * dy * dy;
                    gi[0] += dQ * (-2.0) * (ca * dx + cb * dy);
                    gi[1] += dQ * (-2.0) * (cb * dx + cc * dy);
                }
            }
        }
        free(buf.r);
    }
    for (int64_t i = 0; i < n; i++) {
        double sm[64];
        for (int64_t v = 0; v < stride; v++) sm[v] = 0;
        for (int th = 0; th < nthreads; th++) {
            const double *src = acc + ((int64_t)th * n + i) * stride;
            for (int64_t v = 0; v < stride; v++) sm[v] += src[v];
        }
        d_mean2d[2 * i] = sm[0]; d_mean2d[2 * i + 1] = sm[1];
        d_conic[3 * i] = sm[2]; d_conic[3 * i + 1] = sm[3]; d_conic[3 * i + 2] = sm[4];
        d_opacity[i] = sm[5];
        d_rgb[3 * i] = sm[6]; d_rgb[3 * i + 1] = sm[7]; d_rgb[3 * i + 2] = sm[8];
        d_depth[i] = sm[9];
        for (int j = 0; j < k; j++) d_sem[i * k + j] = sm[10 + j];
    }
    free(acc);
    scene_close(&s);
    return 0;
}

/*
 * Chain rule from the 2D parameters (mean2d, conic, camera-space depth) to
 * the 3D ones (means, scales, quaternions), for one camera.  Only visible
 * Gaussians receive gradient.  Steps, in reverse of oracle_project:
 *   A = Sigma2^-1          -> dSigma2 = -A dA A
 *   Sigma2 = T S3 T^T + lI -> dS3 = T^T dSigma2 T,  dT = 2 dSigma2 T S3
 *   T = J W                -> dJ = dT W^T, then J(p) -> dp
 *   mean2d(p), depth = p_z -> dp
 *   p = W mu + t           -> dmu = W^T dp
 *   S3 = M M^T, M = Rq diag(s) -> dM = 2 dS3 M -> ds, dRq -> dq_hat -> dq
 */
int oracle_project_backward(int64_t n, const double *means, const double *scales, const double *quats,
                            const double *cam, const int32_t *visible, const double *conic,
                            const double *d_mean2d, const double *d_conic, const double *d_depth,
                            double *d_means, double *d_scales, double *d_quats) {
    const double *W = cam + CAM_R, *t = cam + CAM_T;
    const double fx = cam[CAM_FX], fy = cam[CAM_FY];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        for (int c = 0; c < 3; c++) { d_means[3 * i + c] = 0; d_scales[3 * i + c] = 0; }
        for (int c = 0; c < 4; c++) d_quats[4 * i + c] = 0;
        if (!visible[i]) continue;
        const double *m = means + 3 * i;
        double p[3];
        for (int r = 0; r < 3; r++) p[r] = W[3 * r + 0] * m[0] + W[3 * r + 1] * m[1] + W[3 * r + 2] * m[2] + t[r];
        const double x = p[0], y = p[1], z = p[2];
        double Rq[9], qn[4], qnorm;
        quat_to_rot(quats + 4 * i, Rq, qn, &qnorm);
        const double *s = scales + 3 * i;
        double M[9], S3[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) M[3 * a + b] = Rq[3 * a + b] * s[b];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0;
                for (int c = 0; c < 3; c++) acc += M[3 * a + c] * M[3 * b + c];
                S3[3 * a + b] = acc;
            }
        double J[6] = {fx / z, 0, -fx * x / (z * z), 0, fy / z, -fy * y / (z * z)};
        double T[6];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0;
                for (int c = 0; c < 3; c++) acc += J[3 * a + c] * W[3 * c + b];
                T[3 * a + b] = acc;
            }
        /* dA as a symmetric matrix: the off-diagonal parameter b appears twice */
        const double A[4] = {conic[3 * i], conic[3 * i + 1], conic[3 * i + 1], conic[3 * i + 2]};
        const double dA[4] = {d_conic[3 * i], 0.5 * d_conic[3 * i + 1], 0.5 * d_conic[3 * i + 1], d_conic[3 * i + 2]};
        double tmp[4], dS2[4];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) tmp[2 * a + b] = A[2 * a] * dA[b] + A[2 * a + 1] * dA[2 + b];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) dS2[2 * a + b] = -(tmp[2 * a] * A[b] + tmp[2 * a + 1] * A[2 + b]);
        /* dS3 = T^T dS2 T ; dT = 2 dS2 T S3 */
        double dS3[9], dT[6], TS3[6];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0;
                for (int c = 0; c < 2; c++)
                    for (int d = 0; d < 2; d++) acc += T[3 * c + a] * dS2[2 * c + d] * T[3 * d + b];
                dS3[3 * a + b] = acc;
            }
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0;
                for (int c = 0; c < 3; c++) acc += T[3 * a + c] * S3[3 * c + b];
                TS3[3 * a + b] = acc;
            }
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 3; b++) dT[3 * a + b] = 2.0 * (dS2[2 * a] * TS3[b] + dS2[2 * a + 1] * TS3[3 + b]);
        /* dJ = dT W^T */
        double dJ[6];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0;
                for (int c = 0; c < 3; c++) acc += dT[3 * a + c] * W[3 * b + c];
                dJ[3 * a + b] = acc;
            }
        double dp[3] = {0, 0, 0};
        const double z2 = z * z, z3 = z2 * z;
        dp[0] += dJ[2] * (-fx / z2);
        dp[1] += dJ[5] * (-fy / z2);
        dp[2] += dJ[0] * (-fx / z2) + dJ[2] * (2.0 * fx * x / z3) + dJ[4] * (-fy / z2) + dJ[5] * (2.0 * fy * y / z3);
        const double gmx = d_mean2d[2 * i], gmy = d_mean2d[2 * i + 1];
        dp[0] += gmx * fx / z;
        dp[1] += gmy * fy / z;
        dp[2] += -gmx * fx * x / z2 - gmy * fy * y / z2;
        dp[2] += d_depth[i];
        for (int c = 0; c < 3; c++) d_means[3 * i + c] = W[c] * dp[0] + W[3 + c] * dp[1] + W[6 + c] * dp[2];
        /* dM = 2 dS3 M ; ds_b = sum_a dM_ab Rq_ab ; dRq_ab = dM_ab s_b */
        double dM[9], dR[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0;
                for (int c = 0; c < 3; c++) acc += dS3[3 * a + c] * M[3 * c + b];
                dM[3 * a + b] = 2.0 * acc;
            }
        for (int b = 0; b < 3; b++) {
            double acc = 0;
            for (int a = 0; a < 3; a++) acc += dM[3 * a + b] * Rq[3 * a + b];
            d_scales[3 * i + b] = acc;
        }
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) dR[3 * a + b] = dM[3 * a + b] * s[b];
        const double w = qn[0], qx = qn[1], qy = qn[2], qz = qn[3];
        double dq[4];
        dq[0] = 2.0 * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
        dq[1] = 2.0 * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.0 * qx * dR[4] - w * dR[5] + qz * dR[6] + w * dR[7] - 2.0 * qx * dR[8]);
        dq[2] = 2.0 * (-2.0 * qy * dR[0] + qx * dR[1] + w * dR[2] + qx * dR[3] + qz * dR[5] - w * dR[6] + qz * dR[7] - 2.0 * qy * dR[8]);
        dq[3] = 2.0 * (-2.0 * qz * dR[0] - w * dR[1] + qx * dR[2] + w * dR[3] - 2.0 * qz * dR[4] + qy * dR[5] + qx * dR[6] + qy * dR[7]);
        const double dot = dq[0] * qn[0] + dq[1] * qn[1] + dq[2] * qn[2] + dq[3] * qn[3];
        for (int c = 0; c < 4; c++) d_quats[4 * i + c] = (dq[c] - qn[c] * dot) / qnorm;
    }
    return 0;
}

/*
 * Per-view scores behind Eq. 5 and Eq. 6: n_empty counts pixels with zero
 * silhouette (no Gaussian blended: n_contrib == 0); entropy_sum adds, in
 * pixel order, H(p) = -sum_m q_m ln q_m with q = clip(P, 0.001, 1)
 * renormalised over all C classes (Eq. 4 with the clip of Sec. 3.2).
 */
int oracle_score(int32_t width, int32_t height, int32_t C, const double *sem, const int32_t *ncontrib,
                 int64_t *n_empty, double *entropy_sum, double *out_h) {
    const int64_t P = (int64_t)width * height;
    int64_t ne = 0;
    double hs = 0;
    for (int64_t p = 0; p < P; p++) {
        if (ncontrib[p] == 0) ne++;
        const double *v = sem + p * C;
        double Z = 0;
        for (int m = 0; m < C; m++) {
            double q = v[m];
            if (q < 0.001) q = 0.001;
            if (q > 1.0) q = 1.0;
            Z += q;
        }
        double h = 0;
        for (int m = 0; m < C; m++) {
            double q = v[m];
            if (q < 0.001) q = 0.001;
            if (q > 1.0) q = 1.0;
            q /= Z;
            h -= q * log(q);
        }
        if (out_h) out_h[p] = h;
        hs += h;
    }
    *n_empty = ne;
    *entropy_sum = hs;
    return 0;
}
