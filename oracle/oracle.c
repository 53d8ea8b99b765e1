/*
 * CPU oracle for the HashPoint hot path (arXiv 2404.14044).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct
 * restatement of what the method computes.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load it; the product library
 * never links, calls or includes anything from here, and this file shares no
 * source with the GPU path.
 *
 * The neighbour search is brute force over every point (Sec. 3.5 names brute
 * force as the baseline that hashed-point searching accelerates, and Sec. 4.2
 * notes that all search structures must retrieve the same points), so the
 * table-based GPU search must reproduce it exactly.
 *
 * Two stages:
 *   exact stage (binary32): every discrete decision is a function of values
 *     produced by a fixed sequence of correctly rounded IEEE-754 binary32
 *     operations (+ - * / sqrt, rint, floor, and fmaf only where written).
 *     Built with -ffp-contract=off so the compiler adds no fused operations.
 *   continuous stage (binary64): feature aggregation, MLP, compositing (Eq. 2)
 *     and their gradients.
 *
 * Readings of the paper taken where it is silent are listed next to the code
 * that applies them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t W, H;
    float fx, fy, cx, cy;
    float R[9]; /* world -> camera rotation, row-major */
    float C[3]; /* camera centre, world coordinates */
} orc_camera;

typedef struct {
    float radius, inv_tref, t_near, t_far;
    int32_t K, n_samples, m_cap;
    float gamma, inv_beta2, eps_w, eps_idw, delta_last;
    float bg[3];
    int32_t radius_mode; /* 0: r max(1, t inv_tref); 1-3: Eq. 3 cone (below) */
    float rddot;         /* Eq. 3 kernel disc radius, image plane at unit focal length */
    int32_t sampler;     /* 0: adaptive primary-surface walk; 1: uniform multi-surface */
    int32_t ms_steps;    /* uniform positions along [t_near, t_far] (sampler 1)       */
} orc_params;

#define ORC_SAMPLER_PS 0
#define ORC_SAMPLER_MS 1

#define ORC_RADIUS_LINEAR 0
#define ORC_RADIUS_EQ3 1    /* Eq. 3 as derived (Appendix, similar triangles) */
#define ORC_RADIUS_EQ3_AF 2 /* Eq. 3 with AB replaced by AF (first small-angle step) */
#define ORC_RADIUS_EQ3_AE 3 /* Eq. 3 with AB replaced by AE (second step)         */

#define ORC_HID 64
#define ORC_OUT 4

/* ------------------------------------------------------------------------ */
/* exp for the confidence alpha = gamma * exp(-d^2 / beta^2) (Sec. 3.3).     */
/* Cody-Waite reduction x = k ln2 + r, |r| <= ln2/2, then the degree-7      */
/* Taylor polynomial of exp(r) in Horner form, then scaling by 2^k.          */
/* Constants are the FP64 values rounded once to binary32.                   */
/* ------------------------------------------------------------------------ */
float or_exp32(float x)
{
    if (!(x >= -86.0f)) return 0.0f; /* also maps NaN to 0 */
    const float inv_ln2 = (float)(1.0 / 0.69314718055994530942);
    const float ln2_hi = 0.693145751953125f; /* 45426 / 65536: 16 significant bits */
    const float ln2_lo = (float)(0.69314718055994530942 - 0.693145751953125);
    const float k = rintf(x * inv_ln2);
    float r = fmaf(-k, ln2_hi, x);
    r = fmaf(-k, ln2_lo, r);
    const float c[8] = {1.0f, 1.0f, (float)(1.0 / 2.0), (float)(1.0 / 6.0), (float)(1.0 / 24.0),
                        (float)(1.0 / 120.0), (float)(1.0 / 720.0), (float)(1.0 / 5040.0)};
    float p = c[7];
    for (int i = 6; i >= 0; --i) p = fmaf(p, r, c[i]);
    const int ki = (int)k;
    union { uint32_t u; float f; } s;
    s.u = (uint32_t)(ki + 127) << 23;
    return p * s.f;
}

void or_exp32_array(const float *x, float *y, int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = or_exp32(x[i]);
}

/* ------------------------------------------------------------------------ */
/* Search radius, linear mode: rho(t) = r * max(1, t * inv_tref).  With      */
/* inv_tref = 0 it is a fixed radius; with inv_tref = 1/t_near it is a cone  */
/* through the optical centre equal to the hyper-parameter radius at t_near  */
/* (Sec. 3.2), i.e. Eq. 3 without its per-pixel factor.                      */
/* ------------------------------------------------------------------------ */
static float rho_linear(const orc_params *p, float t)
{
    float s = t * p->inv_tref;
    float m = (s > 1.0f) ? s : 1.0f;
    return p->radius * m;
}

/* ------------------------------------------------------------------------ */
/* Per-pixel cone of Eq. 3.  With the image plane at unit distance (f = 1),  */
/* a pixel centre E = (a, b, 1) at distance AE = L = |E| from the optical    */
/* centre A and |w| = sqrt(a^2 + b^2) from the principal point G, and the    */
/* kernel disc of radius rddot around E, the appendix's construction gives   */
/*   BF = rddot AG / AE = rddot / L         (B: disc edge towards G),        */
/*   AB = sqrt((GE - rddot)^2 + AG^2) = sqrt((|w| - rddot)^2 + 1),           */
/*   r(t) = AD BF / AB with AD = t          (rho = t kappa, kappa = BF / AB). */
/* The small-angle variants replace AB by AF = AE - BF EG / AG = L - BF |w|  */
/* or by AE = L.  Reading: GE is taken as |w| (equal to sqrt(AE^2 - AG^2),   */
/* without its cancellation).                                                */
/* ------------------------------------------------------------------------ */
static float kappa_of(const orc_params *p, float a, float b, float L)
{
    if (p->radius_mode == ORC_RADIUS_LINEAR) return 0.0f;
    const float wn = sqrtf(a * a + b * b);
    const float bf = p->rddot / L;
    if (p->radius_mode == ORC_RADIUS_EQ3) {
        const float m = wn - p->rddot;
        return bf / sqrtf(fmaf(m, m, 1.0f));
    }
    if (p->radius_mode == ORC_RADIUS_EQ3_AF) return bf / fmaf(-bf, wn, L);
    return bf / L;
}

/* rho(t) of a ray with cone slope kappa (ignored in the linear mode). */
static float rho_of(const orc_params *p, float kappa, float t)
{
    return p->radius_mode == ORC_RADIUS_LINEAR ? rho_linear(p, t) : t * kappa;
}

float or_kappa(const orc_params *p, float a, float b, float L) { return kappa_of(p, a, b, L); }

/* Guard band g around the image (in pixels).  A point within rho(t) of a    */
/* ray at parameter t >= t_near projects at most                             */
/*   delta = f rho L^2 / (t - rho |w|)                                       */
/* pixels from that ray's pixel centre, where w is the ray's normalised image */
/* coordinate and L^2 = 1 + |w|^2; delta does not grow with t, so its value   */
/* at t_near and the image corner bounds every ray.  Returns -1 when the      */
/* bound does not exist (the radius swallows the near plane).                */
int32_t or_guard(const orc_camera *cam, const orc_params *p)
{
    double w2 = 0.0;
    for (int cu = 0; cu < 2; ++cu)
        for (int cv = 0; cv < 2; ++cv) {
            double u = cu ? (cam->W - 1) : 0, v = cv ? (cam->H - 1) : 0;
            double a = (u + 0.5 - cam->cx) / cam->fx, b = (v + 0.5 - cam->cy) / cam->fy;
            if (a * a + b * b > w2) w2 = a * a + b * b;
        }
    double f = cam->fx > cam->fy ? cam->fx : cam->fy;
    double delta;
    if (p->radius_mode == ORC_RADIUS_LINEAR) {
        double s = (double)p->t_near * p->inv_tref;
        double rho = (double)p->radius * (s > 1.0 ? s : 1.0);
        double den = p->t_near - rho * sqrt(w2);
        if (!(den > 0.0)) return -1;
        delta = f * rho * (1.0 + w2) / den;
    } else {
        /* rho = kappa t: delta = f kappa L^2 / (1 - kappa |w|) for every t; */
        /* every variant has kappa <= rddot / (1 - rddot^2 / 4)              */
        double k = (double)p->rddot / (1.0 - 0.25 * (double)p->rddot * p->rddot);
        double den = 1.0 - k * sqrt(w2);
        if (!(k > 0.0) || !(den > 0.0)) return -1;
        delta = f * k * (1.0 + w2) / den;
    }
    if (!(delta < 1e6)) return -1;
    return (int32_t)floor(0.5 + delta) + 1;
}

/* The paper's kernel size s = 2 ceil(rddot / rdot) + 1, rdot = sqrt(dx dy /  */
/* pi) the radius of the disc of one pixel's area (Sec. 3.2).  In the linear */
/* mode rddot is read as the radius at t_near over t_near.                   */
int32_t or_paper_s(const orc_camera *cam, const orc_params *p)
{
    double rdd = p->radius_mode == ORC_RADIUS_LINEAR
                     ? (double)rho_linear(p, p->t_near) / p->t_near
                     : (double)p->rddot;
    double rdot = sqrt(1.0 / ((double)cam->fx * cam->fy * 3.14159265358979323846));
    return 2 * (int32_t)ceil(rdd / rdot) + 1;
}

/* ------------------------------------------------------------------------ */
/* Camera transform (Sec. 3.2, projection of every point): p_c = R (p - C).  */
/* ------------------------------------------------------------------------ */
void or_to_camera(const float *xyz, int64_t n, const orc_camera *cam, float *pc)
{
    const float *R = cam->R;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        float qx = xyz[3 * i + 0] - cam->C[0];
        float qy = xyz[3 * i + 1] - cam->C[1];
        float qz = xyz[3 * i + 2] - cam->C[2];
        pc[3 * i + 0] = fmaf(R[2], qz, fmaf(R[1], qy, R[0] * qx));
        pc[3 * i + 1] = fmaf(R[5], qz, fmaf(R[4], qy, R[3] * qx));
        pc[3 * i + 2] = fmaf(R[8], qz, fmaf(R[7], qy, R[6] * qx));
    }
}

/* ------------------------------------------------------------------------ */
/* Pixel-keyed table (Sec. 3.2, Fig. 2): every point in front of the camera  */
/* is projected (no z-buffer) and assigned to the pixel it falls in; the     */
/* table lists, per pixel, the points of that pixel.  Reading: pixels form a */
/* grid widened by the guard band g on each side, the key is the row-major   */
/* pixel index of that grid, and points of one pixel are ordered by depth    */
/* z_c and then by point index.                                              */
/* key[i] = -1 for points that are not inserted.  order[0..n_in) lists the   */
/* inserted point indices sorted by (key, z_c, index).  Returns n_in.        */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t key; float z; int32_t idx; } tab_ent;

static int cmp_tab(const void *a, const void *b)
{
    const tab_ent *x = (const tab_ent *)a, *y = (const tab_ent *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->z != y->z) return x->z < y->z ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

int64_t or_table(const float *pc, int64_t n, const orc_camera *cam, int32_t g,
                 int32_t *key, int32_t *order)
{
    const int64_t Wg = (int64_t)cam->W + 2 * g;
    const float lo = (float)(-g), hiu = (float)(cam->W + g), hiv = (float)(cam->H + g);
    for (int64_t i = 0; i < n; ++i) {
        float x = pc[3 * i], y = pc[3 * i + 1], z = pc[3 * i + 2];
        key[i] = -1;
        if (!(z > 0.0f) || !isfinite(x) || !isfinite(y) || !isfinite(z)) continue;
        float uf = fmaf(cam->fx, x / z, cam->cx);
        float vf = fmaf(cam->fy, y / z, cam->cy);
        if (!(uf >= lo && uf < hiu && vf >= lo && vf < hiv)) continue;
        int64_t bu = (int64_t)floorf(uf) + g, bv = (int64_t)floorf(vf) + g;
        key[i] = (int32_t)(bv * Wg + bu);
    }
    int64_t n_in = 0;
    for (int64_t i = 0; i < n; ++i) n_in += key[i] >= 0;
    tab_ent *e = (tab_ent *)malloc((size_t)(n_in ? n_in : 1) * sizeof(tab_ent));
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (key[i] >= 0) { e[k].key = key[i]; e[k].z = pc[3 * i + 2]; e[k].idx = (int32_t)i; ++k; }
    qsort(e, (size_t)n_in, sizeof(tab_ent), cmp_tab);
    for (int64_t j = 0; j < n_in; ++j) order[j] = e[j].idx;
    free(e);
    return n_in;
}

/* ------------------------------------------------------------------------ */
/* Ray of pixel (u, v): from the optical centre through the pixel centre     */
/* (u + 0.5, v + 0.5), unit length, camera coordinates.                      */
/* ------------------------------------------------------------------------ */
static void ray_abl(const orc_camera *cam, int32_t u, int32_t v, float *a, float *b, float *L)
{
    *a = (((float)u + 0.5f) - cam->cx) / cam->fx;
    *b = (((float)v + 0.5f) - cam->cy) / cam->fy;
    *L = sqrtf(fmaf(*b, *b, fmaf(*a, *a, 1.0f)));
}

void or_ray_dir(const orc_camera *cam, int32_t u, int32_t v, float d[3])
{
    float a, b, L;
    ray_abl(cam, u, v, &a, &b, &L);
    d[0] = a / L;
    d[1] = b / L;
    d[2] = 1.0f / L;
}

/* Cone slope kappa of pixel (u, v) (0 in the linear mode). */
float or_ray_kappa(const orc_camera *cam, const orc_params *p, int32_t u, int32_t v)
{
    float a, b, L;
    ray_abl(cam, u, v, &a, &b, &L);
    return kappa_of(p, a, b, L);
}

/* Projection parameter t of camera-space point x on ray d, and the squared  */
/* distance between x and the ray point at parameter s.                      */
static float ray_t(const float *x, const float *d)
{
    return fmaf(x[2], d[2], fmaf(x[1], d[1], x[0] * d[0]));
}

static float dist2_at(const float *x, const float *d, float s)
{
    float ex = fmaf(-s, d[0], x[0]);
    float ey = fmaf(-s, d[1], x[1]);
    float ez = fmaf(-s, d[2], x[2]);
    return fmaf(ez, ez, fmaf(ey, ey, ex * ex));
}

typedef struct { float key; int32_t idx; int32_t aux; } kv_ent;

static int cmp_kv(const void *a, const void *b)
{
    const kv_ent *x = (const kv_ent *)a, *y = (const kv_ent *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* ------------------------------------------------------------------------ */
/* Exact stage for a list of rays (pixel indices v*W + u of one camera).     */
/*                                                                           */
/* Search (Sec. 3.2): the neighbours of a ray are the points whose distance  */
/* to the ray is at most rho(t) at their projection parameter t, with t in   */
/* [t_near, t_far].  Brute force over all n points.  N(ray) is the           */
/* neighbour list ordered by (t, index) and cut to its first m_cap entries;  */
/* flags bit 0 records that the cut dropped some.                            */
/*                                                                           */
/* Sampling (Sec. 3.3, Eq. 4, Eq. 5): every neighbour, projected onto the    */
/* ray, is a sample candidate; candidates are visited in depth order.  For   */
/* candidate j at t_j with R_j = rho(t_j): its K neighbouring points are the */
/* K entries of N(ray) nearest to the candidate (ties by index) among those  */
/* within R_j; missing ones count as distance R_j (reading: an isolated      */
/* candidate then scores as far from any surface).  Pseudo-UDF d_j is their */
/* mean distance (Eq. 4), alpha_j = gamma exp(-d_j^2 / beta^2), and the      */
/* occlusion-aware weight is w_j = alpha_j prod_{k<j} (1 - alpha_k) over all */
/* earlier candidates (Eq. 5).  A candidate becomes a sample when            */
/* w_j > eps_w (reading of "larger than zero"), up to n_samples per ray.     */
/* The primary surface is the point of the first sample, or -1.              */
/*                                                                           */
/* Outputs, per ray r (M = m_cap, S = n_samples):                            */
/*   n_nbr[r], flags[r], nbr_idx/nbr_t[r*M + j] (j < n_nbr; rest -1 / 0),    */
/*   n_sel[r], primary[r], smp_t[r*S + s], knn_cnt[r*S + s],                 */
/*   knn_idx/knn_dist[(r*S + s)*K + k] (k < knn_cnt; rest -1 / 0).           */
/* Optional per-candidate diagnostics (may be NULL), [r*M + j]:              */
/*   cand_d (d_j), cand_alpha, cand_w, cand_T (transmittance before j).      */
/* ------------------------------------------------------------------------ */
void or_exact(const float *pc, int64_t n, const orc_camera *cam, const orc_params *p,
              const int32_t *pix, int64_t n_rays,
              int32_t *n_nbr, uint32_t *flags, int32_t *nbr_idx, float *nbr_t,
              int32_t *n_sel, int32_t *primary, float *smp_t, int32_t *knn_idx,
              float *knn_dist, int32_t *knn_cnt,
              float *cand_d, float *cand_alpha, float *cand_w, float *cand_T)
{
    const int M = p->m_cap, S = p->n_samples, K = p->K;
#pragma omp parallel
    {
        uint8_t *pass = (uint8_t *)malloc((size_t)(n ? n : 1));
        float *tv = (float *)malloc((size_t)(n ? n : 1) * sizeof(float));
        int64_t cap = 1024;
        kv_ent *nb = (kv_ent *)malloc((size_t)cap * sizeof(kv_ent));
        int64_t kn_cap = M > 0 ? M : 1;
        kv_ent *kn = (kv_ent *)malloc((size_t)kn_cap * sizeof(kv_ent));
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < n_rays; ++r) {
            const int32_t u = pix[r] % cam->W, v = pix[r] / cam->W;
            float d[3];
            or_ray_dir(cam, u, v, d);
            const float kap = or_ray_kappa(cam, p, u, v);
            /* brute-force predicate over all points */
            for (int64_t i = 0; i < n; ++i) {
                const float *x = pc + 3 * i;
                float t = ray_t(x, d);
                float e2 = dist2_at(x, d, t);
                float rho = rho_of(p, kap, t);
                tv[i] = t;
                pass[i] = (uint8_t)((x[2] > 0.0f) & (t >= p->t_near) & (t <= p->t_far) &
                                    (e2 <= rho * rho));
            }
            int64_t cnt = 0;
            for (int64_t i = 0; i < n; ++i) {
                if (!pass[i]) continue;
                if (cnt == cap) {
                    cap *= 2;
                    nb = (kv_ent *)realloc(nb, (size_t)cap * sizeof(kv_ent));
                }
                nb[cnt].key = tv[i];
                nb[cnt].idx = (int32_t)i;
                nb[cnt].aux = 0;
                ++cnt;
            }
            qsort(nb, (size_t)cnt, sizeof(kv_ent), cmp_kv);
            const int m = (int)(cnt < M ? cnt : M);
            n_nbr[r] = m;
            flags[r] = (cnt > M) ? 1u : 0u;
            for (int j = 0; j < M; ++j) {
                nbr_idx[r * M + j] = j < m ? nb[j].idx : -1;
                nbr_t[r * M + j] = j < m ? nb[j].key : 0.0f;
            }
            float T = 1.0f;
            int sel = 0;
            primary[r] = -1;
            if (p->sampler == ORC_SAMPLER_MS) {
                /* Multi-surface sampling (Sec. 3.5, the volume-rendering baseline */
                /* it is compared with): uniform positions t_k = t_near + (k + 1/2) */
                /* step along the ray, each with a radius search around it: a      */
                /* position lies on a surface when some neighbour of the ray (any  */
                /* of them: the m_cap cut of N(ray) does not apply) is within      */
                /* R_k = rho(t_k) of it, and every such position becomes a sample  */
                /* (in depth order, up to n_samples) with its K nearest such        */
                /* neighbours.  Reading: the primary surface is the nearest point  */
                /* of the first sample.                                             */
                const float step = (p->t_far - p->t_near) / (float)p->ms_steps;
                if (cnt > kn_cap) {
                    kn_cap = cnt;
                    kn = (kv_ent *)realloc(kn, (size_t)kn_cap * sizeof(kv_ent));
                }
                for (int k = 0; k < p->ms_steps && sel < S; ++k) {
                    const float tk = fmaf((float)k + 0.5f, step, p->t_near);
                    const float Rk = rho_of(p, kap, tk);
                    const float R2 = Rk * Rk;
                    int64_t kc = 0;
                    for (int64_t i = 0; i < cnt; ++i) {
                        float dd = dist2_at(pc + 3 * (int64_t)nb[i].idx, d, tk);
                        if (dd <= R2) { kn[kc].key = dd; kn[kc].idx = nb[i].idx; ++kc; }
                    }
                    if (kc == 0) continue;
                    qsort(kn, (size_t)kc, sizeof(kv_ent), cmp_kv);
                    const int kj = kc < K ? (int)kc : K;
                    const int64_t row = r * S + sel;
                    smp_t[row] = tk;
                    knn_cnt[row] = kj;
                    for (int q = 0; q < K; ++q) {
                        knn_idx[row * K + q] = q < kj ? kn[q].idx : -1;
                        knn_dist[row * K + q] = q < kj ? sqrtf(kn[q].key) : 0.0f;
                    }
                    if (sel == 0) primary[r] = kn[0].idx;
                    ++sel;
                }
            }
            /* candidate walk in depth order */
            for (int j = 0; j < (p->sampler == ORC_SAMPLER_MS ? 0 : m); ++j) {
                const float tj = nb[j].key;
                const float Rj = rho_of(p, kap, tj);
                const float R2 = Rj * Rj;
                int kc = 0;
                for (int i = 0; i < m; ++i) {
                    float dd = dist2_at(pc + 3 * (int64_t)nb[i].idx, d, tj);
                    if (dd <= R2) { kn[kc].key = dd; kn[kc].idx = nb[i].idx; ++kc; }
                }
                qsort(kn, (size_t)kc, sizeof(kv_ent), cmp_kv);
                const int kj = kc < K ? kc : K;
                float sum = 0.0f;
                for (int k = 0; k < kj; ++k) sum = sum + sqrtf(kn[k].key);
                const float dj = (sum + (float)(K - kj) * Rj) / (float)K;
                const float uj = (dj * dj) * p->inv_beta2;
                const float aj = p->gamma * or_exp32(-uj);
                const float wj = aj * T;
                if (cand_d) cand_d[r * M + j] = dj;
                if (cand_alpha) cand_alpha[r * M + j] = aj;
                if (cand_w) cand_w[r * M + j] = wj;
                if (cand_T) cand_T[r * M + j] = T;
                if (wj > p->eps_w && sel < S) {
                    const int64_t row = r * S + sel;
                    smp_t[row] = tj;
                    knn_cnt[row] = kj;
                    for (int k = 0; k < K; ++k) {
                        knn_idx[row * K + k] = k < kj ? kn[k].idx : -1;
                        knn_dist[row * K + k] = k < kj ? sqrtf(kn[k].key) : 0.0f;
                    }
                    if (sel == 0) primary[r] = nb[j].idx;
                    ++sel;
                }
                T = T * (1.0f - aj);
            }
            n_sel[r] = sel;
            for (int s = sel; s < S; ++s) {
                smp_t[r * S + s] = 0.0f;
                knn_cnt[r * S + s] = 0;
                for (int k = 0; k < K; ++k) {
                    knn_idx[(r * S + s) * K + k] = -1;
                    knn_dist[(r * S + s) * K + k] = 0.0f;
                }
            }
            if (cand_d)
                for (int j = (p->sampler == ORC_SAMPLER_MS ? 0 : m); j < M; ++j) {
                    cand_d[r * M + j] = 0.0f;
                    if (cand_alpha) cand_alpha[r * M + j] = 0.0f;
                    if (cand_w) cand_w[r * M + j] = 0.0f;
                    if (cand_T) cand_T[r * M + j] = 0.0f;
                }
        }
        free(pass);
        free(tv);
        free(nb);
        free(kn);
    }
}

/* ------------------------------------------------------------------------ */
/* K-NP extraction and image-based blending (Sec. 3.1, Eq. 1), the other    */
/* consumer of the neighbour search: the K points nearest to the ray among  */
/* its neighbours (points within rho(t) of it, t in [t_near, t_far]),        */
/* ordered by (squared distance to the ray e^2, index), with geometric       */
/* blending weights.  Reading: w_i = 1 / max(e_i, eps_idw), normalised, and  */
/* per-point colours c_i; a ray without neighbours returns bg.  Selection   */
/* is exact binary32 (e^2 as in the search); blending in binary64.          */
/* Outputs per ray r: knp_cnt[r], knp_idx/knp_dist[r*K + k] (k < cnt;       */
/* rest -1 / 0), rgb[3r..3r+2].                                              */
/* ------------------------------------------------------------------------ */
void or_knp(const float *pc, int64_t n, const orc_camera *cam, const orc_params *p,
            const int32_t *pix, int64_t n_rays, int32_t K, const float *colors,
            int32_t *knp_cnt, int32_t *knp_idx, float *knp_dist, double *rgb)
{
#pragma omp parallel
    {
        int64_t cap = 1024;
        kv_ent *nb = (kv_ent *)malloc((size_t)cap * sizeof(kv_ent));
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < n_rays; ++r) {
            const int32_t u = pix[r] % cam->W, v = pix[r] / cam->W;
            float d[3];
            or_ray_dir(cam, u, v, d);
            const float kap = or_ray_kappa(cam, p, u, v);
            int64_t cnt = 0;
            for (int64_t i = 0; i < n; ++i) {
                const float *x = pc + 3 * i;
                float t = ray_t(x, d);
                float e2 = dist2_at(x, d, t);
                float rho = rho_of(p, kap, t);
                if (!((x[2] > 0.0f) & (t >= p->t_near) & (t <= p->t_far) & (e2 <= rho * rho))) continue;
                if (cnt == cap) {
                    cap *= 2;
                    nb = (kv_ent *)realloc(nb, (size_t)cap * sizeof(kv_ent));
                }
                nb[cnt].key = e2;
                nb[cnt].idx = (int32_t)i;
                nb[cnt].aux = 0;
                ++cnt;
            }
            qsort(nb, (size_t)cnt, sizeof(kv_ent), cmp_kv);
            const int kk = (int)(cnt < K ? cnt : K);
            knp_cnt[r] = kk;
            double ws = 0.0, c0 = 0.0, c1 = 0.0, c2 = 0.0;
            for (int k = 0; k < K; ++k) {
                knp_idx[r * K + k] = k < kk ? nb[k].idx : -1;
                knp_dist[r * K + k] = k < kk ? sqrtf(nb[k].key) : 0.0f;
                if (k >= kk) continue;
                const double e = sqrt((double)nb[k].key);
                const double w = 1.0 / (e > p->eps_idw ? e : (double)p->eps_idw);
                const float *c = colors + 3 * (int64_t)nb[k].idx;
                ws += w;
                c0 += w * c[0];
                c1 += w * c[1];
                c2 += w * c[2];
            }
            rgb[3 * r + 0] = kk ? c0 / ws : p->bg[0];
            rgb[3 * r + 1] = kk ? c1 / ws : p->bg[1];
            rgb[3 * r + 2] = kk ? c2 / ws : p->bg[2];
        }
        free(nb);
    }
}

/* ------------------------------------------------------------------------ */
/* Continuous stage in binary64.                                             */
/*                                                                           */
/* Feature at a sample (Sec. 3.4: features of the sample's neighbouring      */
/* points are aggregated; reading: inverse-distance weights                  */
/* 1 / max(dist, eps_idw), normalised), an MLP 32 -> 64 -> 64 -> 4 with ReLU */
/* giving colour c = sigmoid(o_0..2) and density sigma = softplus(o_3), and  */
/* volume rendering (Eq. 2): transmittance tau_j = exp(-sum_{k<j} sigma_k    */
/* Delta_k), weight tau_j (1 - exp(-sigma_j Delta_j)), with Delta_j the gap  */
/* to the next sample and delta_last for the last one.  Outputs colour       */
/* sum w c + (1 - sum w) bg, depth sum w t and opacity sum w.                */
/* Geometry (t_j, ray direction, point positions) is the exact stage's       */
/* binary32 values, widened exactly.                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
} orc_mlp;

static double sigm(double x) { return x >= 0 ? 1.0 / (1.0 + exp(-x)) : exp(x) / (1.0 + exp(x)); }
static double softplus(double x) { return (x > 0 ? x : 0.0) + log1p(exp(-fabs(x))); }

/* ------------------------------------------------------------------------ */
/* Decoder precision (reading R22 of the BF16 decoder).  quant = 0: every   */
/* operand is used as it is.  quant = 1: the decoder's operands -- the      */
/* aggregated feature, the two hidden activations and the three weight      */
/* matrices -- are rounded to bfloat16 (8 significant bits, round to         */
/* nearest, ties to even); biases, the products' sums, the activations     */
/* themselves, aggregation and compositing are not.  quant = 2: the same    */
/* function with each rounding replaced by its offset bf16(x) - x recorded  */
/* by a quant = 1 call, held fixed: x -> x + offset.  At the recording      */
/* point the two agree exactly; quant = 2 is smooth in every input (away    */
/* from ReLU kinks), so its central differences check the analytic         */
/* gradient below, which for quant = 1 and 2 treats every rounding as       */
/* x -> x + (fixed offset), i.e. as the identity.                           */
/* ------------------------------------------------------------------------ */
#define ORC_ACT_OFF(C) ((C) + 2 * ORC_HID) /* offsets per sample: f, h1, h2 */

double or_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    const double ax = fabs(x);
    if (ax < 0x1p-126) return nearbyint(x * 0x1p133) * 0x1p-133; /* subnormal spacing 2^-133 */
    int e;
    frexp(x, &e); /* |x| = m 2^e, m in [0.5, 1) */
    return ldexp(nearbyint(ldexp(x, 8 - e)), e - 8);
}

/* or_bf16 over an array of binary32 values, each result rounded to binary32 */
/* (a value that rounds past the largest bfloat16 gives infinity).           */
void or_bf16_array(const float *x, float *y, int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = (float)or_bf16((double)x[i]);
}

typedef struct {
    int32_t mode;         /* 0, 1 or 2 (above)                                 */
    double *w_off;        /* [n_w1 + n_w2 + n_w3] weight offsets: written by   */
                          /* mode 1 when not NULL, read by mode 2              */
    double *act_off;      /* [rays * S * ORC_ACT_OFF(C)] per-sample offsets of */
                          /* (f, h1, h2): the same                             */
} orc_quant;

/* Effective decoder weights: W + offset (mode 1: the offset that rounds W). */
typedef struct {
    double *W1, *W2, *W3;
} orc_wq;

static int wq_make(const orc_mlp *mlp, int C, const orc_quant *q, orc_wq *w)
{
    const int n1 = ORC_HID * C, n2 = ORC_HID * ORC_HID, n3 = ORC_OUT * ORC_HID;
    w->W1 = (double *)malloc((size_t)(n1 + n2 + n3) * sizeof(double));
    if (!w->W1) return 0;
    w->W2 = w->W1 + n1;
    w->W3 = w->W2 + n2;
    const float *src[3] = {mlp->W1, mlp->W2, mlp->W3};
    double *dst[3] = {w->W1, w->W2, w->W3};
    const int cnt[3] = {n1, n2, n3};
    int base = 0;
    for (int m = 0; m < 3; ++m) {
        for (int i = 0; i < cnt[m]; ++i) {
            const double x = src[m][i];
            double off = 0.0;
            if (q && q->mode == 1) {
                off = or_bf16(x) - x;
                if (q->w_off) q->w_off[base + i] = off;
            } else if (q && q->mode == 2) {
                off = q->w_off[base + i];
            }
            dst[m][i] = x + off;
        }
        base += cnt[m];
    }
    return 1;
}

/* x -> its decoder operand under q (off: this value's offset slot). */
static double operand(const orc_quant *q, double x, double *off)
{
    if (!q || q->mode == 0) return x;
    if (q->mode == 1) {
        const double o = or_bf16(x) - x;
        if (off) *off = o;
        return x + o;
    }
    return x + *off;
}

/* per-sample forward; keeps activations for the backward pass */
typedef struct {
    double f[64], fq[64];          /* aggregated feature, its decoder operand */
    double z1[ORC_HID], h1q[ORC_HID], z2[ORC_HID], h2q[ORC_HID], o[ORC_OUT];
    double wsum, w[64];
} smp_state;

static void sample_forward(const float *pc, const float *feat, int C, const orc_mlp *mlp,
                           const orc_wq *wq, const orc_quant *q, double *off,
                           const float *d, float t, const int32_t *idx, int K, float eps_idw,
                           smp_state *st)
{
    double xs[3] = {(double)t * d[0], (double)t * d[1], (double)t * d[2]};
    for (int c = 0; c < C; ++c) st->f[c] = 0.0;
    st->wsum = 0.0;
    for (int k = 0; k < K; ++k) {
        st->w[k] = 0.0;
        if (idx[k] < 0) continue;
        const float *x = pc + 3 * (int64_t)idx[k];
        double dx = x[0] - xs[0], dy = x[1] - xs[1], dz = x[2] - xs[2];
        double dist = sqrt(dx * dx + dy * dy + dz * dz);
        double wk = 1.0 / (dist > eps_idw ? dist : (double)eps_idw);
        st->w[k] = wk;
        st->wsum += wk;
        for (int c = 0; c < C; ++c) st->f[c] += wk * feat[(int64_t)idx[k] * C + c];
    }
    for (int c = 0; c < C; ++c) {
        st->f[c] /= st->wsum;
        st->fq[c] = operand(q, st->f[c], off ? off + c : NULL);
    }
    for (int o = 0; o < ORC_HID; ++o) {
        double a = mlp->b1[o];
        for (int c = 0; c < C; ++c) a += wq->W1[o * C + c] * st->fq[c];
        st->z1[o] = a;
        st->h1q[o] = operand(q, a > 0 ? a : 0.0, off ? off + C + o : NULL);
    }
    for (int o = 0; o < ORC_HID; ++o) {
        double a = mlp->b2[o];
        for (int c = 0; c < ORC_HID; ++c) a += wq->W2[o * ORC_HID + c] * st->h1q[c];
        st->z2[o] = a;
        st->h2q[o] = operand(q, a > 0 ? a : 0.0, off ? off + C + ORC_HID + o : NULL);
    }
    for (int o = 0; o < ORC_OUT; ++o) {
        double a = mlp->b3[o];
        for (int c = 0; c < ORC_HID; ++c) a += wq->W3[o * ORC_HID + c] * st->h2q[c];
        st->o[o] = a;
    }
}

static double *sample_offsets(const orc_quant *q, int64_t row, int C)
{
    if (!q || q->mode == 0 || !q->act_off) return NULL;
    return q->act_off + row * ORC_ACT_OFF(C);
}

/* Render (Eq. 2) of the exact stage's samples, binary64; decoder operands */
/* under quant (0: none, 1: bfloat16, 2: recorded offsets; see above).     */
void or_render64q(const float *pc, const float *feat, int32_t C,
                  const float *W1, const float *b1, const float *W2, const float *b2,
                  const float *W3, const float *b3,
                  const orc_camera *cam, const orc_params *p, const int32_t *pix, int64_t n_rays,
                  const int32_t *n_sel, const float *smp_t, const int32_t *knn_idx,
                  int32_t quant, double *w_off, double *act_off,
                  double *rgb, double *depth, double *acc)
{
    const orc_mlp mlp = {W1, b1, W2, b2, W3, b3};
    const orc_quant q = {quant, w_off, act_off};
    orc_wq wq;
    if (!wq_make(&mlp, C, &q, &wq)) return;
    const int S = p->n_samples, K = p->K;
#pragma omp parallel
    {
        smp_state *st = (smp_state *)malloc(sizeof(smp_state));
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n_rays; ++r) {
            float d[3];
            or_ray_dir(cam, pix[r] % cam->W, pix[r] / cam->W, d);
            double T = 1.0, col[3] = {0, 0, 0}, dep = 0.0, ws = 0.0;
            const int ns = n_sel[r];
            for (int s = 0; s < ns; ++s) {
                const int64_t row = r * S + s;
                sample_forward(pc, feat, C, &mlp, &wq, &q, sample_offsets(&q, row, C), d,
                               smp_t[row], knn_idx + row * K, K, p->eps_idw, st);
                double sigma = softplus(st->o[3]);
                double delta = (s + 1 < ns) ? (double)smp_t[row + 1] - (double)smp_t[row]
                                            : (double)p->delta_last;
                double a = -expm1(-sigma * delta);
                double w = T * a;
                for (int c = 0; c < 3; ++c) col[c] += w * sigm(st->o[c]);
                dep += w * smp_t[row];
                ws += w;
                T = T * exp(-sigma * delta);
            }
            for (int c = 0; c < 3; ++c) rgb[3 * r + c] = col[c] + (1.0 - ws) * p->bg[c];
            depth[r] = dep;
            acc[r] = ws;
        }
        free(st);
    }
    free(wq.W1);
}

void or_render64(const float *pc, const float *feat, int32_t C,
                 const float *W1, const float *b1, const float *W2, const float *b2,
                 const float *W3, const float *b3,
                 const orc_camera *cam, const orc_params *p, const int32_t *pix, int64_t n_rays,
                 const int32_t *n_sel, const float *smp_t, const int32_t *knn_idx,
                 double *rgb, double *depth, double *acc)
{
    or_render64q(pc, feat, C, W1, b1, W2, b2, W3, b3, cam, p, pix, n_rays, n_sel, smp_t, knn_idx,
                 0, NULL, NULL, rgb, depth, acc);
}

/* ------------------------------------------------------------------------ */
/* Gradient of sum_r grad_rgb[r] . rgb[r] with respect to the features and  */
/* the MLP parameters, for the render above (analytic, binary64).  The      */
/* samples are functions of geometry only, so they stay fixed.  With quant  */
/* 1 or 2 every rounding of a decoder operand counts as x -> x + (fixed     */
/* offset): the products use the rounded operands (weights and activations) */
/* and the ReLU masks the unrounded pre-activations.  Results are ADDED to  */
/* g_feat (n x C) and g_W1..g_b3.                                           */
/* ------------------------------------------------------------------------ */
void or_grad64q(const float *pc, const float *feat, int32_t C,
                const float *W1, const float *b1, const float *W2, const float *b2,
                const float *W3, const float *b3,
                const orc_camera *cam, const orc_params *p, const int32_t *pix, int64_t n_rays,
                const int32_t *n_sel, const float *smp_t, const int32_t *knn_idx,
                int32_t quant, double *w_off, double *act_off,
                const double *grad_rgb, double *g_feat,
                double *g_W1, double *g_b1, double *g_W2, double *g_b2, double *g_W3, double *g_b3)
{
    const orc_mlp mlp = {W1, b1, W2, b2, W3, b3};
    const orc_quant q = {quant, w_off, act_off};
    orc_wq wq;
    if (!wq_make(&mlp, C, &q, &wq)) return;
    const int S = p->n_samples, K = p->K;
    const int n_w1 = ORC_HID * C, n_w2 = ORC_HID * ORC_HID, n_w3 = ORC_OUT * ORC_HID;
    const int n_par = n_w1 + ORC_HID + n_w2 + ORC_HID + n_w3 + ORC_OUT;
    int n_thr = 1;
#ifdef _OPENMP
    n_thr = omp_get_max_threads();
#endif
    double *gpar = (double *)calloc((size_t)n_thr * n_par, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gw1 = gpar + (size_t)tid * n_par, *gb1 = gw1 + n_w1, *gw2 = gb1 + ORC_HID,
               *gb2 = gw2 + n_w2, *gw3 = gb2 + ORC_HID, *gb3 = gw3 + n_w3;
        int Smax = S > 0 ? S : 1;
        smp_state *st = (smp_state *)malloc((size_t)Smax * sizeof(smp_state));
        double *a = (double *)malloc((size_t)Smax * sizeof(double));
        double *Tj = (double *)malloc((size_t)Smax * sizeof(double));
        double *delta = (double *)malloc((size_t)Smax * sizeof(double));
        double *sigma = (double *)malloc((size_t)Smax * sizeof(double));
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n_rays; ++r) {
            const int ns = n_sel[r];
            if (ns == 0) continue;
            float d[3];
            or_ray_dir(cam, pix[r] % cam->W, pix[r] / cam->W, d);
            double T = 1.0;
            for (int s = 0; s < ns; ++s) {
                const int64_t row = r * S + s;
                sample_forward(pc, feat, C, &mlp, &wq, &q, sample_offsets(&q, row, C), d,
                               smp_t[row], knn_idx + row * K, K, p->eps_idw, &st[s]);
                sigma[s] = softplus(st[s].o[3]);
                delta[s] = (s + 1 < ns) ? (double)smp_t[row + 1] - (double)smp_t[row]
                                        : (double)p->delta_last;
                a[s] = -expm1(-sigma[s] * delta[s]);
                Tj[s] = T;
                T = T * exp(-sigma[s] * delta[s]);
            }
            const double *g = grad_rgb + 3 * r;
            double U[3] = {0, 0, 0}, P = 1.0;
            for (int s = ns - 1; s >= 0; --s) {
                double c[3], dLda = 0.0;
                for (int k = 0; k < 3; ++k) c[k] = sigm(st[s].o[k]);
                for (int k = 0; k < 3; ++k)
                    dLda += g[k] * (Tj[s] * (c[k] - U[k]) - p->bg[k] * Tj[s] * P);
                double dLdsig = dLda * delta[s] * exp(-sigma[s] * delta[s]);
                double go[ORC_OUT];
                for (int k = 0; k < 3; ++k) go[k] = g[k] * Tj[s] * a[s] * c[k] * (1.0 - c[k]);
                go[3] = dLdsig * sigm(st[s].o[3]);
                for (int k = 0; k < 3; ++k) U[k] = a[s] * c[k] + (1.0 - a[s]) * U[k];
                P = (1.0 - a[s]) * P;
                /* MLP backward */
                double gz2[ORC_HID], gz1[ORC_HID], gf[64];
                for (int o = 0; o < ORC_OUT; ++o) {
                    gb3[o] += go[o];
                    for (int c2 = 0; c2 < ORC_HID; ++c2) gw3[o * ORC_HID + c2] += go[o] * st[s].h2q[c2];
                }
                for (int c2 = 0; c2 < ORC_HID; ++c2) {
                    double acc2 = 0.0;
                    for (int o = 0; o < ORC_OUT; ++o) acc2 += wq.W3[o * ORC_HID + c2] * go[o];
                    gz2[c2] = st[s].z2[c2] > 0 ? acc2 : 0.0;
                }
                for (int o = 0; o < ORC_HID; ++o) {
                    gb2[o] += gz2[o];
                    for (int c1 = 0; c1 < ORC_HID; ++c1) gw2[o * ORC_HID + c1] += gz2[o] * st[s].h1q[c1];
                }
                for (int c1 = 0; c1 < ORC_HID; ++c1) {
                    double acc1 = 0.0;
                    for (int o = 0; o < ORC_HID; ++o) acc1 += wq.W2[o * ORC_HID + c1] * gz2[o];
                    gz1[c1] = st[s].z1[c1] > 0 ? acc1 : 0.0;
                }
                for (int o = 0; o < ORC_HID; ++o) {
                    gb1[o] += gz1[o];
                    for (int c0 = 0; c0 < C; ++c0) gw1[o * C + c0] += gz1[o] * st[s].fq[c0];
                }
                for (int c0 = 0; c0 < C; ++c0) {
                    double acc0 = 0.0;
                    for (int o = 0; o < ORC_HID; ++o) acc0 += wq.W1[o * C + c0] * gz1[o];
                    gf[c0] = acc0;
                }
                /* inverse-distance aggregation backward */
                const int32_t *idx = knn_idx + (r * S + s) * K;
                for (int k = 0; k < K; ++k) {
                    if (idx[k] < 0) continue;
                    double wk = st[s].w[k] / st[s].wsum;
                    for (int c0 = 0; c0 < C; ++c0) {
#pragma omp atomic
                        g_feat[(int64_t)idx[k] * C + c0] += wk * gf[c0];
                    }
                }
            }
        }
        free(st);
        free(a);
        free(Tj);
        free(delta);
        free(sigma);
    }
    for (int t = 0; t < n_thr; ++t) {
        const double *gw1 = gpar + (size_t)t * n_par, *gb1 = gw1 + n_w1, *gw2 = gb1 + ORC_HID,
                     *gb2 = gw2 + n_w2, *gw3 = gb2 + ORC_HID, *gb3 = gw3 + n_w3;
        for (int i = 0; i < n_w1; ++i) g_W1[i] += gw1[i];
        for (int i = 0; i < ORC_HID; ++i) g_b1[i] += gb1[i];
        for (int i = 0; i < n_w2; ++i) g_W2[i] += gw2[i];
        for (int i = 0; i < ORC_HID; ++i) g_b2[i] += gb2[i];
        for (int i = 0; i < n_w3; ++i) g_W3[i] += gw3[i];
        for (int i = 0; i < ORC_OUT; ++i) g_b3[i] += gb3[i];
    }
    free(gpar);
    free(wq.W1);
}

void or_grad64(const float *pc, const float *feat, int32_t C,
               const float *W1, const float *b1, const float *W2, const float *b2,
               const float *W3, const float *b3,
               const orc_camera *cam, const orc_params *p, const int32_t *pix, int64_t n_rays,
               const int32_t *n_sel, const float *smp_t, const int32_t *knn_idx,
               const double *grad_rgb, double *g_feat,
               double *g_W1, double *g_b1, double *g_W2, double *g_b2, double *g_W3, double *g_b3)
{
    or_grad64q(pc, feat, C, W1, b1, W2, b2, W3, b3, cam, p, pix, n_rays, n_sel, smp_t, knn_idx,
               0, NULL, NULL, grad_rgb, g_feat, g_W1, g_b1, g_W2, g_b2, g_W3, g_b3);
}

void or_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
