/*
 * sgr.h -- C ABI of the MI355X semantic Gaussian rasterizer and view scorer.
 *
 * The operations follow "Understanding while Exploring: Semantics-driven
 * Active Mapping" (arXiv 2506.00225):
 *   - Sec. 3.1 "Gaussian Mapping": Gaussians are transformed into camera
 *     space, sorted front to back, projected and alpha-composited (Eq. 1)
 *     into colour C, depth D and silhouette S;
 *   - Sec. 3.1 "Sparse Semantic Representation" / "Semantic Rendering":
 *     each Gaussian carries k (class index, probability) pairs whose values
 *     are composited into a full C-class map (Eq. 3);
 *   - Sec. 3.1: the renderer is differentiable; the semantic loss reaches
 *     only the semantic attributes;
 *   - Sec. 3.2: candidate views are scored by the number of pixels with
 *     zero silhouette (Eq. 5) and by the summed per-pixel entropy (Eq. 4,
 *     Eq. 6) of the clipped, renormalised semantic map.
 *
 * Conventions (all calls):
 *   - Every array pointer is a DEVICE pointer owned by the caller, unless
 *     it is documented as a host pointer.  `cams` and every struct passed
 *     by pointer are HOST memory, read during the call only.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is
 *     the default stream).  Errors found on the host are returned before
 *     anything is enqueued.  Errors found on the device (key capacity) are
 *     recorded in a status word inside the workspace; read it with
 *     sgr_read_status (which synchronises the stream).
 *   - The library allocates no device memory.  All scratch lives in the
 *     caller's workspace, whose size is sgr_workspace_size(...).  Its
 *     layout is a pure function of (n, cams' sizes, num_views, cfg,
 *     key_capacity): the calls of one frame must receive the same values.
 *   - Calls on one workspace must be ordered on one stream; two frames in
 *     flight need two workspaces.
 *   - Gaussian parameters are post-activation: scales are linear metres,
 *     opacity in (0,1), quaternions (w,x,y,z) need not be normalised
 *     (they are normalised inside sgr_project and the gradient includes
 *     the normalisation).
 *   - Camera: R is world->camera, row-major; camera x right, y down, z
 *     forward; pixel (col,row) has its centre at (col+0.5, row+0.5).
 *   - Images are channel-last, row-major: rgb [H][W][3], depth/sil/t_final/
 *     n_contrib [H][W], sem [H][W][C].
 */
#ifndef SGR_H
#define SGR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGR_OK = 0,
    SGR_EINVAL = 1,       /* invalid argument, detected on the host */
    SGR_ECAPACITY = 2,    /* more tile keys than key_capacity (device-side) */
    SGR_EHIP = 3,         /* a HIP runtime call failed */
    SGR_EUNSUPPORTED = 4  /* valid but unsupported (e.g. tile size) */
} sgr_status;

typedef struct {
    float R[9];        /* world -> camera rotation, row-major */
    float t[3];        /* world -> camera translation */
    float fx, fy, cx, cy;
    int32_t width, height;
} sgr_camera;

typedef struct {
    float alpha_min;   /* skip a Gaussian whose alpha is below this (1/255) */
    float alpha_max;   /* opacity clamp (0.99) */
    float t_min;       /* stop before transmittance would drop below this (1e-4) */
    float z_near;      /* cull Gaussians whose camera-space z is <= this (0.2 m) */
    float lowpass;     /* screen-space low-pass added to the 2D covariance (0.3 px^2) */
    int32_t num_classes;          /* C, 1..256 */
    int32_t top_k;                /* k, 1..32 */
    int32_t sem_grad_to_geometry; /* 0: semantic channels do not reach alpha (Sec. 3.1) */
    int32_t tile_w, tile_h;       /* 0 or 16 (the only supported tile) */
    int32_t sem_accumulators;     /* where the forward and scoring kernels keep the per-pixel
                                     class sums: SGR_ACC_AUTO (LDS when it fits), SGR_ACC_LDS
                                     or SGR_ACC_REGISTERS (C <= 128).  A speed choice only:
                                     every output is bitwise the same. */
    int32_t tile_order;           /* which tile a workgroup takes: SGR_TILES_AUTO or
                                     SGR_TILES_XCD (each of the 8 XCDs walks one contiguous
                                     run of tiles, sharing its L2) or SGR_TILES_LINEAR. */
    int32_t score_workgroups;     /* workgroups of the persistent scoring launch; 0 = as many
                                     as are resident at once.  Speed only. */
    int32_t sem_passes;           /* LDS class sums only: 0 = automatic, or 1..4 class ranges
                                     composited one after another (a tile's geometry is
                                     recomposited per range; a workgroup needs 1/passes of the
                                     class-sum LDS, so more fit on a CU).  Speed only.  The fused
                                     loss uses one pass whenever a view has a dense semantic
                                     target or asks for the dense semantic gradient. */
    int32_t bwd_batch;            /* keys the backward stages per batch (k = 16 only): 0 = 44,
                                     or 32, 44, 56 (less LDS per workgroup, so more of them
                                     per CU, against more barriers per key).  Speed only. */
    int32_t radix_bits;           /* widest digit of the radix sorts: 0 = 8, or 6 or 8 (the
                                     key bits are spread evenly over the passes this needs).
                                     Speed only: the sorts are stable, so the order is the same. */
} sgr_config;

enum { SGR_ACC_AUTO = 0, SGR_ACC_LDS = 1, SGR_ACC_REGISTERS = 2 };
enum { SGR_TILES_AUTO = 0, SGR_TILES_XCD = 1, SGR_TILES_LINEAR = 2 };

typedef struct {
    int64_t n;
    const float *means;    /* [n][3] */
    const float *scales;   /* [n][3] */
    const float *quats;    /* [n][4] (w,x,y,z) */
    const float *opacity;  /* [n] */
    const float *rgb;      /* [n][3] */
    const float *sem_val;  /* [n][k] */
    const uint8_t *sem_idx;/* [n][k] class indices < C */
} sgr_gaussians;

/* Per-view output maps of sgr_render_forward.  Any pointer may be NULL to
 * skip that output (t_final and n_contrib are still kept internally for the
 * backward pass). */
typedef struct {
    float *rgb, *depth, *sil, *sem, *t_final;
    int32_t *n_contrib;
} sgr_maps;

/* Per-view incoming gradients dL/d(map) for sgr_render_backward.  A NULL
 * pointer means a zero gradient for that map.  The semantic gradient is
 * either dense (sem, [H][W][C]) or, when sem is NULL, one class per pixel:
 * dL/dP is sem_at_label[p] at class sem_label[p] and zero elsewhere (the
 * shape of a cross-entropy gradient; a label outside [0, C) has none). */
typedef struct {
    const float *rgb, *depth, *sil, *sem;
    const int32_t *sem_label;    /* [H][W] */
    const float *sem_at_label;   /* [H][W] */
} sgr_map_grads;

/* Gradient outputs (same layouts as sgr_gaussians), overwritten, summed over
 * views.  A NULL pointer skips that output. */
typedef struct {
    float *means, *scales, *quats, *opacity, *rgb, *sem_val;
} sgr_grads;

/* Byte offsets of named arrays inside the workspace (for inspection and
 * tests).  Counts are element capacities. */
typedef struct {
    size_t total_bytes;
    size_t counters;        /* uint32: [0] status, [1] visible, [2] keys, ... */
    size_t views;           /* per-view device table */
    size_t proj_count;      /* uint32 [V*n]: tiles touched per (view, Gaussian); 0 = culled */
    size_t proj_zbits;      /* uint32 [V*n]: bits of fp32 camera-space z */
    size_t pair_rec;        /* 3 x float4 [V*n]: compositing record of each visible pair; records are
                               numbered in (view, Gaussian id) order */
    size_t pair_lin;        /* uint32 [V*n]: (view*n + id) of each record */
    size_t order;           /* uint32 [V*n]: record of each visible pair, front to back (depth rank) */
    size_t sorted_keys;     /* uint32 [key_capacity]: global tile id, sorted */
    size_t sorted_vals;     /* uint32 [key_capacity]: emission index of each sorted key */
    size_t key_owner;       /* uint32 [key_capacity]: record of the pair that emitted key e
                               (sorted key s belongs to record key_owner[sorted_vals[s]]) */
    size_t ranges;          /* uint32 [num_tiles][2]: [start, end) per global tile */
    size_t tile_offsets;    /* uint32 [V*n]: first emission index of each visible pair, by depth rank */
    int64_t num_tiles;      /* sum over views of tiles_x * tiles_y */
    int64_t num_pixels;     /* sum over views of W * H */
    int64_t vn;             /* V * n */
} sgr_layout;

/* Workspace size in bytes for a frame; 0 if the arguments are invalid. */
size_t sgr_workspace_size(int64_t n, const sgr_camera *cams, int32_t num_views, const sgr_config *cfg,
                          int64_t key_capacity);

/* Fills `out` with the workspace layout for these arguments. */
sgr_status sgr_workspace_layout(int64_t n, const sgr_camera *cams, int32_t num_views, const sgr_config *cfg,
                                int64_t key_capacity, sgr_layout *out);

/*
 * sgr_project -- Sec. 3.1 (camera transform, EWA projection to a 2D conic,
 * front-to-back depth order).  For every (view, Gaussian): camera-space
 * p = R mu + t; culled when p.z <= z_near, det(Sigma2) <= 0, opacity <
 * alpha_min or an empty pixel rectangle; Sigma2 = J R Sigma3 R^T J^T +
 * lowpass*I, Sigma3 = Rq diag(s^2) Rq^T; the pixel rectangle is the exact
 * axis-aligned box of {o exp(-Q/2) >= alpha_min}, Q = d^T Sigma2^-1 d,
 * computed in double precision.  Visible pairs are then sorted by (fp32 z
 * bits, Gaussian id) per view (their records are built in (view, Gaussian
 * id) order, and the sort orders record numbers).
 */
sgr_status sgr_project(const sgr_gaussians *g, const sgr_camera *cams, int32_t num_views, const sgr_config *cfg,
                       int64_t key_capacity, void *workspace, size_t workspace_bytes, void *stream);

/*
 * sgr_bin -- tile binning (Sec. 3.1: Gaussians are composited in depth
 * order, nearest first, here per tile).  Emits one key per (visible pair, 16x16 tile its pixel rectangle
 * touches), sorts the keys by (view, tile) with a stable on-device radix
 * sort so each tile's list stays front to back, and builds [start, end) per
 * tile.  If d_num_keys is not NULL the key count K is written there
 * (device int64).  K > key_capacity sets SGR_ECAPACITY in the status word
 * and the later calls of the frame do no work.
 */
sgr_status sgr_bin(const sgr_gaussians *g, const sgr_camera *cams, int32_t num_views, const sgr_config *cfg,
                   int64_t key_capacity, int64_t *d_num_keys, void *workspace, size_t workspace_bytes,
                   void *stream);

/*
 * sgr_render_forward -- Eq. 1 (colour, depth, silhouette) and Eq. 3
 * (semantics) per pixel, front to back: alpha = min(alpha_max, o G); skip
 * when alpha < alpha_min; stop, without blending, when T (1 - alpha) <
 * t_min; otherwise add z alpha T and set T <- T (1 - alpha).  `out` is an
 * array of num_views sgr_maps.  n_contrib counts blended Gaussians and
 * t_final is the final transmittance.
 */
sgr_status sgr_render_forward(const sgr_gaussians *g, const sgr_camera *cams, int32_t num_views,
                              const sgr_config *cfg, int64_t key_capacity, const sgr_maps *out,
                              void *workspace, size_t workspace_bytes, void *stream);

/*
 * sgr_render_forward_dense -- sgr_render_forward with a dense semantic
 * distribution per Gaussian: dense_sem[n][C] (device) takes the place of the
 * top-k lists in Eq. 3, so every blend updates all C class sums.  It is the
 * dense representation the sparse one is measured against (supplement
 * S.2.2's runtime comparison).  Follows sgr_project and sgr_bin on the same
 * workspace; g's top-k arrays are read by those calls only.
 */
sgr_status sgr_render_forward_dense(const sgr_gaussians *g, const float *dense_sem, const sgr_camera *cams,
                                    int32_t num_views, const sgr_config *cfg, int64_t key_capacity,
                                    const sgr_maps *out, void *workspace, size_t workspace_bytes, void *stream);

/*
 * sgr_render_backward -- gradient of sum_views sum_p <dL[v](p), maps[v](p)>
 * with respect to means, scales, quats, opacity, rgb and sem_val, walking
 * each pixel's blended list back to front from the saved final
 * transmittance.  With sem_grad_to_geometry = 0 the semantic maps reach
 * only sem_val (Sec. 3.1).  Must follow sgr_render_forward on the same
 * workspace.  `dL` is an array of num_views sgr_map_grads.  Gradients of
 * each tile are reduced inside the tile and summed per Gaussian in a fixed
 * order: the result is bitwise reproducible.
 */
sgr_status sgr_render_backward(const sgr_gaussians *g, const sgr_camera *cams, int32_t num_views,
                               const sgr_config *cfg, int64_t key_capacity, const sgr_map_grads *dL,
                               const sgr_grads *out, void *workspace, size_t workspace_bytes, void *stream);

/*
 * The two halves of sgr_render_backward, for callers that time or schedule
 * them apart; called in this order on the same workspace they give the same
 * bits as sgr_render_backward.
 *
 * sgr_render_backward_tiles -- the compositing part (Eq. 1 and Eq. 3
 * differentiated per pixel): every (view, tile) walks its list back to front
 * and writes, for each of its keys, the tile's summed gradient with respect
 * to the projected 2D mean, conic, opacity, colour, depth and top-k values
 * into that key's slot in the workspace (no atomics).  Must follow
 * sgr_render_forward.
 *
 * sgr_render_backward_gather -- sums each Gaussian's key slots in a fixed
 * order and chains the result through the EWA projection (Sec. 3.1's
 * splatting of 3D Gaussians) to means, scales (linear), quats (including
 * their normalisation), opacity, rgb and sem_val, summed over views.  `out`
 * is overwritten.  Must follow sgr_render_backward_tiles.
 */
sgr_status sgr_render_backward_tiles(const sgr_gaussians *g, const sgr_camera *cams, int32_t num_views,
                                     const sgr_config *cfg, int64_t key_capacity, const sgr_map_grads *dL,
                                     void *workspace, size_t workspace_bytes, void *stream);
sgr_status sgr_render_backward_gather(const sgr_gaussians *g, const sgr_camera *cams, int32_t num_views,
                                      const sgr_config *cfg, int64_t key_capacity, const sgr_grads *out,
                                      void *workspace, size_t workspace_bytes, void *stream);

/* Targets and gradient outputs of one view for sgr_render_forward_loss.
 * Any target may be NULL to drop its term; any output may be NULL. */
typedef struct {
    const float *rgb;      /* [H][W][3] target colour */
    const float *depth;    /* [H][W] target depth */
    const int32_t *label;  /* [H][W] class labels: cross-entropy term */
    const float *sem;      /* [H][W][C] pseudo-ground-truth class distribution: the
                              Hellinger + cosine term (used instead of label if both) */
    float *g_rgb, *g_depth, *g_sil, *g_sem;  /* dL/d(map), same layouts as sgr_maps */
    float *g_sem_at_label;                   /* [H][W]: with a label target, dL/dP at the label
                                                (zero at every other class), the sparse form
                                                sgr_map_grads takes; 0 where the label is invalid */
} sgr_loss_view;

/* Weights of the per-keyframe mapping loss (defaults in brackets). */
typedef struct {
    float w_depth, w_rgb, w_sil, w_sem;  /* [1, 0.5, 1, 1] */
    float sil_thresh;                    /* [0.99] colour and depth count where S > this */
    float ce_floor;                      /* [1e-6] cross-entropy uses ln max(P_label, floor) */
    float lambda_hd, lambda_cos;         /* [0.8, 0.2] Hellinger and cosine weights */
    float entropy_tau;                   /* [<= 0: ln k] supervise pixels whose target entropy is below */
    float sqrt_eps;                      /* [1e-8] inside the Hellinger square roots */
} sgr_loss_config;

/*
 * sgr_render_forward_loss -- sgr_render_forward with the mapping loss fused
 * into its epilogue, where each tile's per-pixel class sums are still in
 * LDS.  Per view, with P pixels:
 *   L = (1/P) sum_p [ m (w_depth |D - D*| + w_rgb sum_ch |C - C*|)
 *                     + w_sil |S - 1| + w_sem L_sem ],   m = [S > sil_thresh]
 * (the silhouette-masked depth and colour L1 of Sec. 3.1; m is not
 * differentiated).  L_sem is the semantic loss of Sec. 3.1: with a dense
 * target g, M_H (lambda_hd D_HD(g, P) + lambda_cos (1 - cos(g, P))) with the
 * entropy mask M_H = [H(g) < tau] and D_HD the Hellinger distance; with
 * labels, -ln max(P_label, ce_floor).  Writes dL/d(map) for every view
 * (ready for sgr_render_backward) and loss[v] (device, double).  `out` may
 * be NULL or name any subset of the maps to write as well.  The per-pixel
 * class sums never go to HBM unless out[v].sem asks for them.  Needs the
 * LDS class-sum placement (C <= 141): otherwise SGR_EUNSUPPORTED.
 */
sgr_status sgr_render_forward_loss(const sgr_gaussians *g, const sgr_camera *cams, int32_t num_views,
                                   const sgr_config *cfg, int64_t key_capacity, const sgr_maps *out,
                                   const sgr_loss_view *lv, const sgr_loss_config *lc, double *loss,
                                   void *workspace, size_t workspace_bytes, void *stream);

/*
 * sgr_score_views -- Sec. 3.2, Eq. 4-6: for each of num_views candidate
 * views (sizes may differ), render the silhouette and semantics without
 * writing maps and reduce per view: n_empty[v] = number of pixels where no
 * Gaussian is blended (S = 0), entropy_sum[v] = sum over pixels of
 * H = -sum_m q_m ln q_m with q = clip(P, 0.001, 1) renormalised over all C
 * classes.  Runs sgr_project and sgr_bin itself; the compositing of every
 * (view, tile) runs in one persistent launch.  n_empty, entropy_sum are
 * device arrays [num_views].
 */
sgr_status sgr_score_views(const sgr_gaussians *g, const sgr_camera *cams, int32_t num_views,
                           const sgr_config *cfg, int64_t key_capacity, uint32_t *n_empty, double *entropy_sum,
                           void *workspace, size_t workspace_bytes, void *stream);

/*
 * sgr_score_maps -- the same per-view reduction as sgr_score_views from an
 * already rendered dense map of one view (sem [H][W][C], n_contrib [H][W]);
 * writes n_empty[0] and entropy_sum[0] (device).  Used by the plain
 * one-view-per-launch path.  The workspace (sgr_score_maps_workspace_size
 * bytes, 256-byte aligned) holds per-block partial sums.
 */
size_t sgr_score_maps_workspace_size(int32_t width, int32_t height);
sgr_status sgr_score_maps(const float *sem, const int32_t *n_contrib, int32_t width, int32_t height,
                          int32_t num_classes, uint32_t *n_empty, double *entropy_sum, void *workspace,
                          size_t workspace_bytes, void *stream);

/*
 * sgr_score_maps_noalloc -- sgr_score_maps for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): it takes no workspace and allocates
 * nothing.  Its per-block partial sums live in a static device array of
 * SGR_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends, so it accepts at most SGR_NOALLOC_MAX_PIXELS
 * pixels (width * height); a larger view returns SGR_EUNSUPPORTED before
 * anything is enqueued.  Other arguments and outputs as sgr_score_maps
 * (device arrays; SGR_EINVAL for a bad argument; SGR_EHIP if the array's
 * device address cannot be found).  Every call on one GPU shares that
 * array: calls that overlap on one GPU (two streams, or two threads) race
 * and give wrong results; calls ordered on one stream are fine.
 */
#define SGR_NOALLOC_SCRATCH_BYTES (1u << 20)
#define SGR_NOALLOC_MAX_PIXELS (16 * 1024 * 1024)
sgr_status sgr_score_maps_noalloc(const float *sem, const int32_t *n_contrib, int32_t width, int32_t height,
                                  int32_t num_classes, uint32_t *n_empty, double *entropy_sum, void *stream);

/* ------------------------------------------------------------------------
 * Mapping-iteration helpers (used by a mapping step around the rasterizer).
 * ------------------------------------------------------------------------ */

/*
 * sgr_mapping_loss_grad -- gradient with respect to the rendered maps of
 *   L = (1/P) sum_p [ m(p) (w0 |D - D*| + w1 sum_ch |C - C*|) + w2 |S - 1|
 *                     - w3 ln max(P_label(p), 1e-6) ],   m(p) = [S(p) > w4],
 * the silhouette-masked depth + colour L1 of Sec. 3.1 (w0 = 1, w1 = 0.5,
 * w4 = 0.99) plus silhouette and cross-entropy terms.  The mask is not
 * differentiated.  weights is a HOST array {w0, w1, w2, w3, w4}.  Maps and
 * targets are device arrays of num_pixels pixels (rgb [P][3], sem [P][C],
 * label int32 [P] with values < num_classes); outputs are overwritten,
 * g_sem densely.  scratch is a device float array of num_pixels.
 */
sgr_status sgr_mapping_loss_grad(const float *rgb, const float *depth, const float *sil, const float *sem,
                                 const float *t_rgb, const float *t_depth, const int32_t *label, int64_t num_pixels,
                                 int32_t num_classes, const float *weights, float *g_rgb, float *g_depth, float *g_sil,
                                 float *g_sem, float *scratch, void *stream);

/* One Adam segment: parameters p, gradient g, moments m and v (device, n
 * floats each); after the update p is clamped to [lo, hi]. */
typedef struct {
    float *p;
    const float *g;
    float *m, *v;
    int64_t n;
    float lo, hi;
} sgr_adam_segment;

#define SGR_MAX_ADAM_SEGMENTS 8

/*
 * sgr_adam_step -- one fused Adam update (bias-corrected, step >= 1) of up
 * to SGR_MAX_ADAM_SEGMENTS segments in a single launch:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p = clamp(p - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), lo, hi).
 * `segments` is a HOST array.
 */
sgr_status sgr_adam_step(const sgr_adam_segment *segments, int32_t num_segments, float lr, float beta1, float beta2,
                         float eps, int32_t step, void *stream);

/*
 * sgr_render_backward_gather_adam -- sgr_render_backward_gather and then
 * one sgr_adam_step of the six parameter tensors, in one pass: each
 * Gaussian's gradient (the chain rule through the EWA projection of
 * Sec. 3.1, summed over views) updates its parameters where it is formed
 * and is never written out, so the gradient tensors' write and re-read are
 * saved.  The result is bitwise that of the two calls.  `segments` is a
 * HOST array of exactly 6 segments in the order means, scales, quats,
 * opacity, rgb, sem_val, with n = 3n, 3n, 4n, n, 3n and k n elements (the
 * Gaussians' n and the config's k), p the parameter tensor (it may be the
 * array the Gaussians struct points to: each element is read before it is
 * written, by the same thread), m and v its moments, lo/hi its clamp; their
 * g is ignored.  Adam arguments as sgr_adam_step.  Must follow
 * sgr_render_backward_tiles.
 */
sgr_status sgr_render_backward_gather_adam(const sgr_gaussians *g, const sgr_camera *cams, int32_t num_views,
                                           const sgr_config *cfg, int64_t key_capacity,
                                           const sgr_adam_segment *segments, float lr, float beta1, float beta2,
                                           float eps, int32_t step, void *workspace, size_t workspace_bytes,
                                           void *stream);

/* ------------------------------------------------------------------ sparse semantic state
 * Sec. 3.1, sparse semantic representation: a Gaussian keeps the top-k
 * classes of the distribution it is initialised from; later observations
 * update the kept values with the indices fixed. */

/*
 * sgr_topk_select -- for Gaussian i, the k classes with the highest
 * probability in row pixel[i] of dist ([rows][num_classes], device; pixel
 * NULL: row i), in decreasing order, equal values keeping the smaller class
 * first and NaN counting as -inf.  Writes sem_idx[n][k] and sem_val[n][k]
 * (the probabilities, -inf stored as 0; with renormalize != 0 divided by
 * their sum).  k <= num_classes <= 256, k <= 32.
 */
sgr_status sgr_topk_select(const float *dist, const int64_t *pixel, int64_t n, int32_t num_classes, int32_t k,
                           int32_t renormalize, uint8_t *sem_idx, float *sem_val, void *stream);

/*
 * sgr_topk_update -- fixed-index update of the kept values toward a new
 * observation: sem_val[i][m] = (1 - rate) sem_val[i][m]
 * + rate * dist[pixel[i]][sem_idx[i][m]] (an index >= num_classes reads 0).
 * 0 <= rate <= 1.
 */
sgr_status sgr_topk_update(const float *dist, const int64_t *pixel, int64_t n, int32_t num_classes, int32_t k,
                           const uint8_t *sem_idx, float rate, float *sem_val, void *stream);

/* ------------------------------------------------------------------ planning
 * Next-best-view selection (Sec. 3.2): candidate poses from the newly
 * observed voxels of the exploration map, their scores (sgr_score_poses,
 * Eq. 4-6) and the overall criterion with motion cost (Eq. 7). */

/* Exploration map: nx*ny*nz voxels of edge `voxel` from `origin`, one byte
 * per voxel (x fastest); 1 marks an observed free voxel. */
typedef struct {
    int32_t nx, ny, nz;
    float voxel;
    float origin[3];
} sgr_grid;

/* One sampling stage (coarse: step 1, 5 directions, one height; fine: step
 * 0.5, 15 directions, several heights). */
typedef struct {
    float step;          /* v1: spacing of candidate positions, rounded to whole voxels */
    int32_t directions;  /* v2: viewing directions per position (Fibonacci lattice on the sphere) */
    float z_min, z_max;  /* heights of the position layers (equal: one layer) */
} sgr_sampling;

/* Workspace bytes of sgr_generate_candidates for this grid and stage. */
size_t sgr_candidates_workspace_size(const sgr_grid *grid, const sgr_sampling *s);

/*
 * sgr_generate_candidates -- candidate poses (Sec. 3.2, exploration
 * strategy).  Positions are the centres of voxels that are free in
 * free_now and not in free_before (NULL: nothing was free), on a lattice of
 * round(step / voxel) voxels in x and y and on the layers
 * i0, i0 + s, ... whose centre height lies in [z_min - voxel/2,
 * z_max + voxel/2); order z, y, x.  Each position takes the `directions`
 * Fibonacci-lattice directions d_j, z_j = 1 - (2j+1)/n, azimuth j pi
 * (3 - sqrt 5); candidate v = position * directions + j.  Poses: 12 floats,
 * world-to-camera R (rows right, down, forward = d_j, with up +z, or +x
 * when |d_j . z| > 0.99) then t = -R p.  positions: [V][3].  The total V is
 * written to *d_count (device int64); entries past `capacity` are not
 * written.  All pointers are device pointers.
 */
sgr_status sgr_generate_candidates(const sgr_grid *grid, const uint8_t *free_now, const uint8_t *free_before,
                                   const sgr_sampling *s, int64_t capacity, float *poses, float *positions,
                                   int64_t *d_count, void *workspace, size_t workspace_bytes, void *stream);

/*
 * sgr_score_poses -- sgr_score_views for num_views cameras that share the
 * intrinsics and size of `intrinsics` (host; its R and t are ignored) and
 * take their R and t from the device array poses[num_views][12] (as written
 * by sgr_generate_candidates), so a planning step needs no host copy of
 * the poses.  Same workspace as sgr_score_views for these sizes.
 */
sgr_status sgr_score_poses(const sgr_gaussians *g, const sgr_camera *intrinsics, int32_t num_views, const float *poses,
                           const sgr_config *cfg, int64_t key_capacity, uint32_t *n_empty, double *entropy_sum,
                           void *workspace, size_t workspace_bytes, void *stream);

/*
 * sgr_combine_scores -- Eq. 5-7 over the candidate pool, in double
 * precision: I_geo = N_S / sum N_S (Eq. 5: softmax of log N_S), I_sem =
 * softmax of the entropy sums (Eq. 6), I = (1 - softmax(l)) I_geo I_sem with
 * l the distance from `current` (host, 3 floats) to each candidate position
 * (Eq. 7).  Candidates with N_S < prune_fraction * pixels are flagged in
 * pruned[]; *best is the unpruned candidate with the largest I (the first
 * on ties) or -1.  score: [V] double, pruned: [V] bytes, best: one int32;
 * device pointers.  If every N_S is 0, I_geo is 0.  One workgroup, fixed
 * reduction order: the result is reproducible bit for bit.
 */
sgr_status sgr_combine_scores(int32_t num_views, const uint32_t *n_empty, const double *entropy_sum,
                              const float *positions, const float *current, int64_t pixels, float prune_fraction,
                              double *score, uint8_t *pruned, int32_t *best, void *stream);

/* Synchronises `stream` and reads the status word, the visible-pair count
 * and the key count of the workspace (host outputs; any may be NULL). */
sgr_status sgr_read_status(const void *workspace, void *stream, int64_t *num_visible, int64_t *num_keys);

/* A static, NUL-terminated description of a status code; any int is
 * accepted (a value that is not an sgr_status gives "unknown status"). */
const char *sgr_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* SGR_H */
