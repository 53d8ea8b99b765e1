/*
 * hashpoint.h -- C ABI of the MI355X (gfx950) HashPoint hot path.
 *
 * HashPoint (arXiv 2404.14044) renders a neural point cloud by ray tracing.
 * Sec. 3.2 ("hashed-point searching") projects every point onto the image
 * plane (no z-buffer) and regroups the point list per pixel into a table whose
 * key is the pixel index and whose value is (first point, count); a ray then
 * visits the pixels of a window around its own and tests each listed point
 * by its distance to the ray.  Sec. 3.3 ("adaptive primary surface
 * sampling") projects the neighbours onto the ray as sample candidates,
 * scores each by the mean distance to its K nearest points (Eq. 4), turns it
 * into a confidence alpha = gamma exp(-d^2/beta^2), weights it by the
 * transmittance of the earlier candidates (Eq. 5) and keeps the candidates
 * near the first surface.  Sec. 3.4 decodes the kept samples with an MLP and
 * composites them by volume rendering (Eq. 2).
 *
 * The calls below are those steps:
 *   hp_build_table      - projection and pixel table        (Sec. 3.2, Fig. 2)
 *   hp_search_sample    - window search and sampling        (Sec. 3.2-3.3, Eq. 4-5)
 *   hp_render           - aggregation, MLP, compositing     (Sec. 3.4, Eq. 2)
 *   hp_render_backward  - gradient of the render            (Sec. 3.4, Eq. 2)
 *   hp_render_backward_samples - the same from kept samples
 *   hp_search_render    - search + sampling + render in one launch
 *   hp_knp_blend        - K nearest points to each ray, Eq. 1 blend (Sec. 3.1)
 *
 * General rules
 *  - All buffers are caller-owned.  Pointers documented "device" are HIP
 *    device memory; "host" pointers are read before the call returns.  The
 *    library allocates nothing and keeps no state between calls.
 *  - Calls are asynchronous on the given HIP stream (0 = the null stream).
 *    Arguments are validated on the host before any launch; a rejected call
 *    launches nothing and returns an error status.
 *  - Rays are numbered view-major, then row-major: ray = ray_base(view) +
 *    v * W + u, where ray_base(view) is the sum of W * H over earlier views.
 *  - Every discrete result (table order, neighbour lists, samples, nearest
 *    neighbours) is deterministic and identical run to run.
 */
#ifndef HASHPOINT_H
#define HASHPOINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hp_status;
enum {
    HP_OK = 0,
    HP_E_INVALID = 1,     /* bad argument (null pointer, out-of-range value) */
    HP_E_WORKSPACE = 2,   /* workspace pointer null or smaller than required */
    HP_E_UNSUPPORTED = 3, /* valid request this build does not implement      */
    HP_E_CAPACITY = 4,    /* an index would not fit in int32                   */
    HP_E_HIP = 5          /* a HIP runtime call failed; see hp_last_hip_error  */
};

enum { HP_FP32 = 0, HP_BF16 = 1 };                 /* decoder precision  */
/* Bucket order of the table (hp_params.layout); no result depends on it. */
enum {
    HP_LAYOUT_ROWMAJOR = 0, /* row-major over the guard-banded pixel grid         */
    HP_LAYOUT_TILED = 1,    /* 8x8-pixel tiles, row-major inside each tile        */
    HP_LAYOUT_MORTON = 2    /* 8x8-pixel tiles, Z-order (Morton) inside each tile */
};
/* Window of buckets a ray visits (hp_params.window_shape); both complete. */
enum {
    HP_WINDOW_DISC = 0,  /* buckets within the proven pixel radius of the ray */
    HP_WINDOW_SQUARE = 1 /* the square around that disc (fewer tests per bucket) */
};
/* Search radius laws (hp_params.radius_mode). */
enum {
    HP_RADIUS_LINEAR = 0, /* rho = radius * max(1, t * inv_tref)                     */
    HP_RADIUS_EQ3 = 1,    /* rho = kappa t, kappa per pixel from Eq. 3 as derived     */
    HP_RADIUS_EQ3_AF = 2, /* the same with the first small-angle step (AB ~ AF)      */
    HP_RADIUS_EQ3_AE = 3  /* the same with the second small-angle step (AB ~ AE)     */
};
/* Samplers (hp_params.sampler). */
enum {
    HP_SAMPLER_PS = 0, /* adaptive primary-surface sampling (Sec. 3.3, Eq. 4, Eq. 5) */
    HP_SAMPLER_MS = 1  /* uniform multi-surface sampling, the Sec. 3.5 baseline      */
};

#define HP_MAX_VIEWS 32
#define HP_MAX_K 32
#define HP_MAX_SAMPLES 64
#define HP_MAX_MCAP 64
#define HP_FEAT_DIM 32
#define HP_HIDDEN 64
/* device scratch of hp_render_backward_noalloc, per GPU (32 MiB) */
#define HP_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)

/* Pinhole camera (host).  OpenCV axes: +x right, +y down, +z forward.
 * Camera-space position of world point p is R (p - C); pixel (u, v) spans
 * [u, u+1) x [v, v+1) and its ray passes through (u + 0.5, v + 0.5). */
typedef struct hp_camera {
    int32_t W, H;
    float fx, fy, cx, cy;
    float R[9]; /* world -> camera rotation, row-major */
    float C[3]; /* camera centre, world coordinates     */
} hp_camera;

/* Run parameters (host).
 *  radius, inv_tref: in HP_RADIUS_LINEAR mode the search radius is
 *      rho(t) = radius * max(1, t * inv_tref); inv_tref = 0 gives a fixed
 *      radius, inv_tref = 1 / t_near a cone equal to radius at t_near
 *      (Sec. 3.2) without Eq. 3's per-pixel factor.  radius also bounds the
 *      depth summaries' search in every mode.
 *  t_near, t_far: range of the ray parameter t (0 < t_near <= t_far).
 *  K: points per pseudo-UDF (Eq. 4), 1..HP_MAX_K.
 *  n_samples: cap on samples per ray, 1..HP_MAX_SAMPLES.
 *  m_cap: cap on the per-ray neighbour list, 1..HP_MAX_MCAP.
 *  gamma, inv_beta2: alpha = gamma * exp(-d^2 * inv_beta2), 0 < gamma <= 1.
 *  eps_w: a candidate becomes a sample when its weight (Eq. 5) > eps_w.
 *  eps_idw: floor of the distance in the inverse-distance feature weights.
 *  delta_last: interval length of the last sample of a ray (Eq. 2).
 *  bg: background colour.
 *  layout: HP_LAYOUT_ROWMAJOR, HP_LAYOUT_TILED or HP_LAYOUT_MORTON (Sec. 3.2
 *      mentions a Z-order arrangement; read here as an order of buckets).
 *  flags: reserved, must be 0.
 *  search_chunk: rays a search workgroup takes at a time, 0 = default (4),
 *      at most 64; search_blocks: search grid (workgroups each taking
 *      chunks of rays in turn), 0 = default (65,536).
 *      Neither changes any result; an autotuner picks them per workload.
 *  radius_mode: HP_RADIUS_*.  In the Eq. 3 modes rho(t) = kappa t with, for
 *      the pixel centre E = (a, b, 1) on the image plane at unit focal
 *      length (L = |E|, |w| = sqrt(a^2 + b^2)), BF = rddot / L and
 *      kappa = BF / sqrt((|w| - rddot)^2 + 1) (EQ3), BF / (L - BF |w|)
 *      (EQ3_AF) or BF / L (EQ3_AE), each a fixed sequence of binary32
 *      operations (Sec. 3.2, Eq. 3, and the appendix's derivation).
 *  rddot: the kernel disc radius r'' on that image plane, 0 < rddot < 1;
 *      ignored (must be 0) in HP_RADIUS_LINEAR mode.
 *  sampler: HP_SAMPLER_PS, or HP_SAMPLER_MS: positions
 *      t_k = fma(k + 0.5, (t_far - t_near) / ms_steps, t_near), k < ms_steps,
 *      each a sample (in order, up to n_samples) when a point of the ray's
 *      neighbour list lies within rho(t_k) of it, with its K nearest listed
 *      points; primary = the nearest point of the first sample.  gamma,
 *      inv_beta2 and eps_w are then unused.
 *  ms_steps: 1..2^24 with HP_SAMPLER_MS, 0 otherwise.
 *  Launch shapes, none of which changes any result (an autotuner picks them
 *  per workload; 0 = default):
 *  search_band: consecutive rays dealt to one XCD at a time by the search
 *      kernels, 0 (1,600) or 64..2^24;
 *  window_shape: HP_WINDOW_DISC or HP_WINDOW_SQUARE;
 *  render_rays: rays a render wave composites at a time, 0 (16), 16, 32 or 64;
 *  render_blocks: render grid; a workgroup takes every render_blocks-th
 *      chunk of render_rays rays (persistent, loading the decoder weights
 *      once), 0 = one workgroup per chunk. */
typedef struct hp_params {
    float radius, inv_tref, t_near, t_far;
    int32_t K, n_samples, m_cap;
    float gamma, inv_beta2, eps_w, eps_idw, delta_last;
    float bg[3];
    int32_t layout, flags;
    int32_t search_chunk, search_blocks;
    int32_t radius_mode;
    float rddot;
    int32_t sampler, ms_steps;
    int32_t search_band, window_shape, render_rays, render_blocks;
} hp_params;

/* Per-view geometry of a table, filled by hp_build_table. */
typedef struct hp_view_info {
    int32_t W, H;         /* image size                                       */
    int32_t g;            /* guard band in pixels around the image            */
    int32_t Wg, Hg;       /* bucket grid, at least (W + 2g) x (H + 2g)         */
    int32_t bucket_base;  /* first bucket of the view in the table            */
    int32_t ray_base;     /* first ray of the view                            */
    float delta_max;      /* bound on a neighbour's pixel offset from its ray  */
} hp_view_info;

/* A built table (host struct of device pointers into the caller's workspace).
 *  offsets[b] .. offsets[b+1]: slots of bucket b; offsets has n_buckets + 1
 *      entries and offsets[n_buckets] is the number of inserted points.
 *  pts[4 * slot + 0..3]: camera-space x, y, z and the point index (as int32
 *      bits), ordered by bucket, then z, then point index.
 *  perm[slot]: the point index of each slot.
 *  pcam[4 * (view * n_points + i) + 0..3]: camera-space x, y, z of point i in
 *      that view and its index (as pts; only defined for inserted points),
 *      in point order: the search finds a listed point's coordinates here.
 *  bucket_z, cell_zmin: depth summaries used to bound each ray's window. */
typedef struct hp_table {
    int32_t n_views;
    int32_t layout;
    int64_t n_points;
    int64_t n_buckets;
    int64_t n_rays;
    int32_t *offsets;
    float *pts;
    int32_t *perm;
    float *pcam;
    float *bucket_z;      /* [n_buckets] depth of each bucket's first point, +inf if empty */
    uint32_t *cell_zmin;  /* [n_cells] min depth (binary32 bits) of 8x8-bucket cells      */
    int64_t n_cells;
    uint64_t build_key;   /* hash of the cameras and of the parameters the table
                             depends on (radius, inv_tref, t_near, radius_mode,
                             rddot, layout); calls on the table check it       */
    void *scratch;
    hp_view_info views[HP_MAX_VIEWS];
} hp_table;

/* Per-ray and per-sample outputs of hp_search_sample (device, caller-owned).
 *  Per ray r: n_sel[r] samples, primary[r] = point index of the first
 *      sample (-1 if none), n_nbr[r] = neighbours kept (<= m_cap),
 *      flags[r] bit 0 = more than m_cap neighbours were found.
 *  Per sample s < n_sel[r] (row = r * n_samples + s): t[row] is its ray
 *      parameter; knn_idx[row * K + k], knn_dist[row * K + k] are its nearest
 *      neighbours in increasing distance (ties by index), padded with -1 / 0.
 *      Rows s >= n_sel[r] are not written.
 *  nbr_idx, nbr_t (nullable, [R * m_cap]): the neighbour list in (t, index)
 *      order, padded with -1 / 0. */
typedef struct hp_samples {
    int32_t *n_sel;
    int32_t *primary;
    int32_t *n_nbr;
    uint32_t *flags;
    float *t;
    int32_t *knn_idx;
    float *knn_dist;
    int32_t *nbr_idx;
    float *nbr_t;
} hp_samples;

/* MLP 32 -> 64 -> 64 -> 4 with ReLU; colour = sigmoid(o0..2), density =
 * softplus(o3).  Weights W[out][in], FP32, device. */
typedef struct hp_mlp {
    float *W1, *b1, *W2, *b2, *W3, *b3;
} hp_mlp;

/* Element counts of the arrays of an hp_samples for R rays with these
 * parameters (host only, no GPU needed): n_rays for n_sel, primary, n_nbr and
 * flags; sample_rows = R * n_samples for t; knn_entries = sample_rows * K for
 * knn_idx and knn_dist; nbr_entries = R * m_cap for the optional nbr_idx and
 * nbr_t.  Returns HP_E_INVALID for R < 0 or invalid parameters and
 * HP_E_CAPACITY when a count would not fit in int64. */
typedef struct hp_shape {
    int64_t n_rays;
    int64_t sample_rows;
    int64_t knn_entries;
    int64_t nbr_entries;
} hp_shape;

hp_status hp_samples_shape(int64_t R, const hp_params *p, hp_shape *out);

/* Workspace bytes hp_build_table needs for n points and these views (host
 * only, no GPU needed).  Returns 0 and sets *status on invalid input. */
size_t hp_table_workspace(int64_t n, const hp_camera *cams, int32_t n_views,
                          const hp_params *p, hp_status *status);

/* Guard band and window bound of one view (host only).  The bound
 * delta = f rho L^2 / (t - rho |w|) on the pixel offset of a point within
 * rho(t) of a ray with normalised image coordinate w (L^2 = 1 + |w|^2) does
 * not grow with t, so its value at t_near and the image corner bounds every
 * neighbour; g = floor(0.5 + delta) + 1.  In the Eq. 3 modes
 * delta = f kappa L^2 / (1 - kappa |w|) for every t, and every variant has
 * kappa <= rddot / (1 - rddot^2 / 4), which with the corner's |w| bounds it. */
hp_status hp_view_bounds(const hp_camera *cam, const hp_params *p, int32_t *g, float *delta_max);

/* The paper's search-kernel size s = 2 ceil(rddot / rdot) + 1 for this view
 * (Sec. 3.2), rdot = sqrt(1 / (pi fx fy)) the radius of a disc of one pixel's
 * area on the unit-focal image plane; in HP_RADIUS_LINEAR mode rddot is
 * read as rho(t_near) / t_near.  Reported beside the guard band g, which is
 * what the search uses (host only). */
hp_status hp_paper_kernel_size(const hp_camera *cam, const hp_params *p, int32_t *s);

/* Build the pixel table (Sec. 3.2, Fig. 2) for n_views cameras.
 *  xyz: device, n x 3 FP32 world positions.  Non-finite points and points
 *      not in front of a camera (z <= 0) or projecting outside the image
 *      plus its guard band are not inserted for that camera.
 *  ws: device workspace of ws_bytes >= hp_table_workspace(...).  The table
 *      lives in it; keep it alive and unmodified while the table is used.
 *  out: host struct filled with pointers into ws and per-view geometry.
 * Errors: HP_E_INVALID (null pointers, bad camera or parameters),
 *  HP_E_WORKSPACE, HP_E_CAPACITY (n * n_views or bucket count >= 2^31). */
hp_status hp_build_table(const float *xyz, int64_t n, const hp_camera *cams, int32_t n_views,
                         const hp_params *p, void *ws, size_t ws_bytes, hp_table *out,
                         void *stream);

/* Search and sample every ray of every view of the table (Sec. 3.2-3.3).
 *  cams and p must be the ones the table was built with: cameras and the
 *  fields radius, inv_tref, t_near, radius_mode, rddot and layout must be
 *  equal (HP_E_INVALID otherwise); the other fields may differ.
 *  out: device arrays sized for R = tab->n_rays rays (see hp_samples).
 * Errors: HP_E_INVALID, HP_E_UNSUPPORTED (K > HP_MAX_K). */
hp_status hp_search_sample(const hp_table *tab, const hp_camera *cams, int32_t n_views,
                           const hp_params *p, hp_samples *out, void *stream);

/* Decode and composite (Sec. 3.4, Eq. 2).
 *  smp: samples from hp_search_sample for R rays.
 *  feat: device, n_points x C FP32 features; C must be HP_FEAT_DIM.
 *  precision: HP_FP32, or HP_BF16 (decoder operands rounded to bfloat16,
 *      FP32 accumulation; aggregation and compositing stay FP32).
 *  rgb (R x 3), depth (R), acc (R): device FP32 outputs.  depth and acc may
 *      be NULL.
 * Errors: HP_E_INVALID, HP_E_UNSUPPORTED (C != HP_FEAT_DIM). */
hp_status hp_render(const hp_samples *smp, int64_t R, const float *feat, int32_t C,
                    const hp_mlp *mlp, int32_t precision, const hp_params *p, float *rgb,
                    float *depth, float *acc, void *stream);

/* Search, sampling, aggregation, decoder and compositing in one launch
 * (Sec. 3.2-3.4): the same operations in the same order as
 * hp_search_sample followed by hp_render, so rgb, depth and acc are
 * identical, without writing the samples.  Requires n_samples <= 16 and
 * K <= 16 (the samples of a ray form one 16-wide decoder tile).
 *  rgb (R x 3), depth, acc (R, nullable), n_sel (R, nullable): device.
 * Errors: HP_E_INVALID, HP_E_UNSUPPORTED (C != HP_FEAT_DIM, n_samples > 16,
 *      K > 16). */
hp_status hp_search_render(const hp_table *tab, const hp_camera *cams, int32_t n_views,
                           const hp_params *p, const float *feat, int32_t C, const hp_mlp *mlp,
                           int32_t precision, float *rgb, float *depth, float *acc,
                           int32_t *n_sel, void *stream);

/* K-NP extraction and image-based blending (Sec. 3.1, Eq. 1) on the same
 * table and search: for every ray, the K points nearest to the ray among its
 * neighbours (points within rho(t) of it, t in [t_near, t_far]; all of them,
 * m_cap does not apply), ordered by (binary32 squared distance to the ray,
 * point index), and c(r) = sum_i w_i c_i / sum_i w_i with
 * w_i = 1 / max(e_i, eps_idw), e_i = sqrt of that squared distance, in FP32;
 * rays without a neighbour get bg.  The sampler fields of p are ignored.
 *  cams, n_views, p: as given to hp_build_table.  K: 1..HP_MAX_MCAP.
 *  colors: device, n_points x 3 FP32 per-point colours.
 *  rgb: device, R x 3 FP32 output (R = tab->n_rays).
 *  knp_cnt (R, nullable), knp_idx / knp_dist (R x K, both or neither):
 *      device outputs, the count min(K, neighbours) and the list (padded with
 *      -1 / 0).
 * Errors: HP_E_INVALID, HP_E_UNSUPPORTED (K out of range). */
hp_status hp_knp_blend(const hp_table *tab, const hp_camera *cams, int32_t n_views,
                       const hp_params *p, int32_t K, const float *colors, float *rgb,
                       int32_t *knp_cnt, int32_t *knp_idx, float *knp_dist, void *stream);

/* Workspace bytes hp_render_backward needs for this table and these
 * parameters (host only): per-workgroup decoder-gradient slices plus a ring
 * for the recomputed samples (as hp_samples, without the optional neighbour
 * lists) of one chunk of min(tab->n_rays, 262144) rays.  The workspace does not
 * grow with the rays beyond that; hp_render_backward accepts any workspace
 * that holds the slices and at least one ray, and recomputes the rays in
 * chunks of as many as it holds. */
size_t hp_backward_workspace(const hp_table *tab, const hp_params *p, hp_status *status);

/* Gradient of L with respect to the features and MLP parameters (Sec. 3.4,
 * Eq. 2 differentiated through the decoder and the inverse-distance
 * aggregation), given grad_rgb = dL/drgb (device, R x 3, R = tab->n_rays).
 * Search and sampling are recomputed from the table (samples depend on
 * geometry only) one chunk of rays at a time into the workspace's ring, and
 * each chunk's gradient is accumulated as in hp_render_backward_samples; the
 * result does not depend on the chunk size beyond the order of float atomics.
 *  cams, n_views, p: as given to hp_build_table; precision: the decoder
 *      precision of the forward render (the activations are replayed in it;
 *      the gradient itself is FP32 with FP32 weights).
 *  grad_feat (device, n_points x C) and every array of grad_mlp (device,
 *      FP32, shapes as hp_mlp) are ADDED to: zero them first for a plain
 *      gradient.  Feature gradients are accumulated with atomics, so results
 *      are reproducible to rounding only.
 *  ws: device workspace; hp_backward_workspace bytes, or any size that holds
 *      the gradient slices and the samples of one ray (larger: fewer chunks).
 * Errors: HP_E_INVALID, HP_E_WORKSPACE, HP_E_UNSUPPORTED (C != HP_FEAT_DIM,
 *      K > HP_MAX_K). */
hp_status hp_render_backward(const hp_table *tab, const hp_camera *cams, int32_t n_views,
                             const float *feat, int32_t C, const hp_mlp *mlp, int32_t precision,
                             const hp_params *p, const float *grad_rgb, float *grad_feat,
                             hp_mlp *grad_mlp, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes hp_render_backward_samples needs (host only). */
size_t hp_backward_samples_workspace(const hp_params *p, hp_status *status);

/* The same gradient from samples the caller kept (Sec. 3.4, Eq. 2): smp as
 * written by hp_search_sample for R rays with these parameters (only n_sel,
 * t, knn_idx and knn_dist are read).  Arguments otherwise as
 * hp_render_backward; ws: at least hp_backward_samples_workspace bytes.
 * Errors: HP_E_INVALID, HP_E_WORKSPACE, HP_E_UNSUPPORTED, HP_E_CAPACITY
 *      (R >= 2^31). */
hp_status hp_render_backward_samples(const hp_samples *smp, int64_t R, const float *feat,
                                     int32_t C, const hp_mlp *mlp, int32_t precision,
                                     const hp_params *p, const float *grad_rgb, float *grad_feat,
                                     hp_mlp *grad_mlp, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * recomputing gradient of hp_render_backward, with the same arguments and
 * results but no workspace.  Its decoder-gradient slices and recompute ring
 * live in a device array of HP_NOALLOC_SCRATCH_BYTES that the library holds
 * on each GPU it runs on until the process ends; the rays are recomputed in
 * chunks of as many as the ring holds after the slices (about 24,000 rays at
 * K = 8, S = 16), so any number of rays is accepted.  It calls no hipMalloc,
 * hipFree or allocating library routine.  Calls on one GPU share its array:
 * calls that overlap on one GPU (several streams or threads at once) race
 * and must be serialised by the caller.
 * Errors: as hp_render_backward, minus HP_E_WORKSPACE; HP_E_CAPACITY if the
 *      slices and one ray's samples do not fit the array (not reachable
 *      within HP_MAX_K and HP_MAX_SAMPLES); HP_E_HIP if the array's address
 *      cannot be obtained. */
hp_status hp_render_backward_noalloc(const hp_table *tab, const hp_camera *cams, int32_t n_views,
                                     const float *feat, int32_t C, const hp_mlp *mlp,
                                     int32_t precision, const hp_params *p, const float *grad_rgb,
                                     float *grad_feat, hp_mlp *grad_mlp, void *stream);

/* Evaluates on the device, element by element, the binary32 exponential
 * that decides the candidate confidences alpha = gamma exp(-d^2 / beta^2)
 * (Sec. 3.3): y[i] = E(x[i]) for the n values of x (device, FP32), written to
 * y (device, FP32, n entries, may not overlap x).  E is the fixed operation
 * sequence the search kernels use: x = k ln2 + r by a Cody-Waite reduction
 * with a 16-bit head of ln2 (k = rint(x / ln2), so that k times the head is
 * exact), the degree-7 Taylor polynomial of exp(r) in Horner form with fused
 * multiply-adds, then scaling by 2^k; it returns 0 for x < -86 and NaN and is
 * meant for x <= 0.  For tests of bit-reproducibility against other
 * implementations of that sequence.  Asynchronous on `stream`.
 * Errors: HP_E_INVALID (n < 0, null pointer with n > 0). */
hp_status hp_exp32_eval(const float *x, float *y, int64_t n, void *stream);

/* Evaluates on the device the rounding of binary32 values to bfloat16 that
 * the BF16 decoder applies to its operands (features, activations, weights;
 * round to nearest, ties to even, subnormals kept): y[i] = x[i] rounded, as
 * binary32 (n values, device; y may not overlap x).  For tests of
 * bit-reproducibility against the definition.  Asynchronous on `stream`.
 * Errors: HP_E_INVALID (n < 0, null pointer with n > 0). */
hp_status hp_bf16_eval(const float *x, float *y, int64_t n, void *stream);

/* Status text, and the last HIP error code seen by this thread. */
const char *hp_status_str(hp_status s);
int32_t hp_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HASHPOINT_H */
