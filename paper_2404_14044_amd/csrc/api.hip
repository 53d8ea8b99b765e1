// C ABI of the HashPoint library: host-side validation, workspace layout and
// kernel launches.  No allocation; the only global state is the per-device
// address of the allocation-free backward's scratch array.
#include <math.h>
#include <string.h>

#include <mutex>

#include "hp_backward.hpp"
#include "hp_device.hpp"
#include "hp_kernels.hpp"
#include "hp_search.hpp"
#include "hp_table_ws.hpp"

namespace {

thread_local int32_t g_last_hip_error = 0;

hp_status hip_fail(hipError_t e)
{
    g_last_hip_error = (int32_t)e;
    return HP_E_HIP;
}

bool finite_f(float x) { return isfinite(x) != 0; }

bool valid_camera(const hp_camera &c)
{
    if (c.W < 1 || c.H < 1) return false;
    if (!(c.fx > 0.0f) || !(c.fy > 0.0f) || !finite_f(c.fx) || !finite_f(c.fy)) return false;
    if (!finite_f(c.cx) || !finite_f(c.cy)) return false;
    for (int i = 0; i < 9; ++i)
        if (!finite_f(c.R[i])) return false;
    for (int i = 0; i < 3; ++i)
        if (!finite_f(c.C[i])) return false;
    return true;
}

bool valid_params(const hp_params &p)
{
    if (!(p.radius > 0.0f) || !finite_f(p.radius)) return false;
    if (!(p.inv_tref >= 0.0f) || !finite_f(p.inv_tref)) return false;
    if (!(p.t_near > 0.0f) || !(p.t_far >= p.t_near) || !finite_f(p.t_far)) return false;
    if (p.K < 1 || p.n_samples < 1 || p.n_samples > HP_MAX_SAMPLES) return false;
    if (p.m_cap < 1 || p.m_cap > HP_MAX_MCAP) return false;
    if (!(p.gamma > 0.0f) || !(p.gamma <= 1.0f)) return false;
    if (!(p.inv_beta2 >= 0.0f) || !finite_f(p.inv_beta2)) return false;
    if (!(p.eps_w >= 0.0f) || !finite_f(p.eps_w)) return false;
    if (!(p.eps_idw > 0.0f) || !finite_f(p.eps_idw)) return false;
    if (!(p.delta_last > 0.0f) || !finite_f(p.delta_last)) return false;
    for (int i = 0; i < 3; ++i)
        if (!finite_f(p.bg[i])) return false;
    if (p.layout != HP_LAYOUT_ROWMAJOR && p.layout != HP_LAYOUT_TILED &&
        p.layout != HP_LAYOUT_MORTON)
        return false;
    if (p.search_band != 0 && (p.search_band < 64 || p.search_band > (1 << 24))) return false;
    if (p.window_shape != HP_WINDOW_DISC && p.window_shape != HP_WINDOW_SQUARE) return false;
    if (p.render_rays != 0 && p.render_rays != 16 && p.render_rays != 32 && p.render_rays != 64)
        return false;
    if (p.render_blocks < 0) return false;
    if (p.flags != 0) return false;
    if (p.search_chunk < 0 || p.search_chunk > 64 || p.search_blocks < 0) return false;
    if (p.sampler == HP_SAMPLER_PS) {
        if (p.ms_steps != 0) return false;
    } else if (p.sampler == HP_SAMPLER_MS) {
        if (p.ms_steps < 1 || p.ms_steps > (1 << 24)) return false;
    } else {
        return false;
    }
    if (p.radius_mode == HP_RADIUS_LINEAR) return p.rddot == 0.0f;
    if (p.radius_mode != HP_RADIUS_EQ3 && p.radius_mode != HP_RADIUS_EQ3_AF &&
        p.radius_mode != HP_RADIUS_EQ3_AE)
        return false;
    return p.rddot > 0.0f && p.rddot < 1.0f;
}

// Pixel-offset bound of a neighbour (see hashpoint.h, hp_view_bounds).
bool view_bound(const hp_camera &c, const hp_params &p, double &delta)
{
    double w2max = 0.0;
    const double us[2] = {0.5, c.W - 0.5}, vs[2] = {0.5, c.H - 0.5};
    for (double u : us)
        for (double v : vs) {
            const double a = (u - c.cx) / c.fx, b = (v - c.cy) / c.fy;
            w2max = fmax(w2max, a * a + b * b);
        }
    const double f = fmax((double)c.fx, (double)c.fy);
    if (p.radius_mode == HP_RADIUS_LINEAR) {
        const double rho = (double)p.radius * fmax(1.0, (double)p.t_near * p.inv_tref);
        const double den = (double)p.t_near - rho * sqrt(w2max);
        if (!(den > 0.0)) return false;
        delta = f * rho * (1.0 + w2max) / den;
    } else {
        const double k = (double)p.rddot / (1.0 - 0.25 * (double)p.rddot * p.rddot);
        const double den = 1.0 - k * sqrt(w2max);
        if (!(den > 0.0)) return false;
        delta = f * k * (1.0 + w2max) / den;
    }
    return isfinite(delta) != 0 && delta < 1e6;
}

struct Geometry {
    hp::ViewSet vs;
    int64_t n_buckets = 0, n_rays = 0, n_cells = 0;
};

hp_status plan_views(const hp_camera *cams, int32_t n_views, const hp_params &p, Geometry &geo,
                     hp_view_info *info)
{
    memset(&geo.vs, 0, sizeof(geo.vs));
    geo.vs.n = n_views;
    geo.vs.layout = p.layout;
    int64_t nb = 0, nr = 0, nc = 0;
    for (int i = 0; i < n_views; ++i) {
        const hp_camera &c = cams[i];
        if (!valid_camera(c)) return HP_E_INVALID;
        double delta;
        if (!view_bound(c, p, delta)) return HP_E_INVALID;
        const int32_t g = (int32_t)floor(0.5 + delta) + 1;
        int64_t Wg = (int64_t)c.W + 2 * g, Hg = (int64_t)c.H + 2 * g;
        if (p.layout != HP_LAYOUT_ROWMAJOR) {  // whole 8x8 tiles
            Wg = (Wg + 7) / 8 * 8;
            Hg = (Hg + 7) / 8 * 8;
        }
        if (Wg * Hg >= ((int64_t)1 << 31) - nb - 1) return HP_E_CAPACITY;
        hp::ViewK &V = geo.vs.v[i];
        V.fx = c.fx;
        V.fy = c.fy;
        V.cx = c.cx;
        V.cy = c.cy;
        memcpy(V.R, c.R, sizeof(V.R));
        memcpy(V.C, c.C, sizeof(V.C));
        V.W = c.W;
        V.H = c.H;
        V.g = g;
        V.Wg = (int32_t)Wg;
        V.Hg = (int32_t)Hg;
        V.bucket_base = (int32_t)nb;
        V.ray_base = (int32_t)nr;
        V.dmax = (float)(delta * (1.0 + 1e-5) + 1e-3);
        V.slot_base = 0;
        V.cell_base = (int32_t)nc;
        V.ncx = (int32_t)((Wg + hp::CELL - 1) / hp::CELL);
        nc += (int64_t)V.ncx * ((Hg + hp::CELL - 1) / hp::CELL);
        if (info) {
            info[i].W = c.W;
            info[i].H = c.H;
            info[i].g = g;
            info[i].Wg = V.Wg;
            info[i].Hg = V.Hg;
            info[i].bucket_base = V.bucket_base;
            info[i].ray_base = V.ray_base;
            info[i].delta_max = (float)delta;
        }
        nb += Wg * Hg;
        nr += (int64_t)c.W * c.H;
        if (nr >= ((int64_t)1 << 31)) return HP_E_CAPACITY;
    }
    geo.n_buckets = nb;
    geo.n_rays = nr;
    geo.n_cells = nc;
    return HP_OK;
}

int knn_template(int K) { return K <= 4 ? 4 : K <= 8 ? 8 : K <= 16 ? 16 : 32; }

// FNV-1a over the cameras and the parameters a table depends on (its guard
// band, window bounds and bucket layout): a search with other values would
// use bounds that no longer cover every neighbour.
uint64_t table_key(const hp_camera *cams, int32_t n_views, const hp_params &p)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *data, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(data);
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    };
    mix(&n_views, sizeof(n_views));
    mix(cams, sizeof(hp_camera) * (size_t)n_views);
    mix(&p.radius, sizeof(p.radius));
    mix(&p.inv_tref, sizeof(p.inv_tref));
    mix(&p.t_near, sizeof(p.t_near));
    mix(&p.radius_mode, sizeof(p.radius_mode));
    mix(&p.rddot, sizeof(p.rddot));
    mix(&p.layout, sizeof(p.layout));
    return h;
}

}  // namespace

extern "C" {

const char *hp_status_str(hp_status s)
{
    switch (s) {
    case HP_OK: return "ok";
    case HP_E_INVALID: return "invalid argument";
    case HP_E_WORKSPACE: return "workspace missing or too small";
    case HP_E_UNSUPPORTED: return "unsupported request";
    case HP_E_CAPACITY: return "index capacity exceeded (int32)";
    case HP_E_HIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

int32_t hp_last_hip_error(void) { return g_last_hip_error; }

hp_status hp_view_bounds(const hp_camera *cam, const hp_params *p, int32_t *g, float *delta_max)
{
    if (!cam || !p || !valid_camera(*cam) || !valid_params(*p)) return HP_E_INVALID;
    double delta;
    if (!view_bound(*cam, *p, delta)) return HP_E_INVALID;
    if (g) *g = (int32_t)floor(0.5 + delta) + 1;
    if (delta_max) *delta_max = (float)delta;
    return HP_OK;
}

hp_status hp_paper_kernel_size(const hp_camera *cam, const hp_params *p, int32_t *s)
{
    if (!cam || !p || !s || !valid_camera(*cam) || !valid_params(*p)) return HP_E_INVALID;
    double rdd = p->rddot;
    if (p->radius_mode == HP_RADIUS_LINEAR) {
        const float m = p->t_near * p->inv_tref;
        rdd = (double)(p->radius * (m > 1.0f ? m : 1.0f)) / p->t_near;
    }
    const double rdot = sqrt(1.0 / ((double)cam->fx * cam->fy * 3.14159265358979323846));
    const double half = ceil(rdd / rdot);
    if (!(half < 1e6)) return HP_E_INVALID;
    *s = 2 * (int32_t)half + 1;
    return HP_OK;
}

hp_status hp_samples_shape(int64_t R, const hp_params *p, hp_shape *out)
{
    if (!p || !out || R < 0 || !valid_params(*p)) return HP_E_INVALID;
    const int64_t lim = (int64_t)1 << 62;
    const int64_t S = p->n_samples, K = p->K, M = p->m_cap;
    if (R > lim / S || R * S > lim / K || R > lim / M) return HP_E_CAPACITY;
    out->n_rays = R;
    out->sample_rows = R * S;
    out->knn_entries = R * S * K;
    out->nbr_entries = R * M;
    return HP_OK;
}

size_t hp_table_workspace(int64_t n, const hp_camera *cams, int32_t n_views, const hp_params *p,
                          hp_status *status)
{
    hp_status st = HP_OK;
    Geometry geo;
    if (!cams || !p || n < 0 || n_views < 1 || n_views > HP_MAX_VIEWS || !valid_params(*p)) st = HP_E_INVALID;
    else if (n * n_views >= ((int64_t)1 << 31)) st = HP_E_CAPACITY;
    else st = plan_views(cams, n_views, *p, geo, nullptr);
    if (status) *status = st;
    if (st != HP_OK) return 0;
    return hp::table_ws_layout(nullptr, n, n_views, geo.n_buckets, geo.n_cells).bytes;
}

hp_status hp_build_table(const float *xyz, int64_t n, const hp_camera *cams, int32_t n_views,
                         const hp_params *p, void *ws, size_t ws_bytes, hp_table *out, void *stream)
{
    if (!cams || !p || !out || n < 0 || n_views < 1 || n_views > HP_MAX_VIEWS) return HP_E_INVALID;
    if (n > 0 && !xyz) return HP_E_INVALID;
    if (!valid_params(*p)) return HP_E_INVALID;
    if (n * n_views >= ((int64_t)1 << 31)) return HP_E_CAPACITY;
    Geometry geo;
    hp_view_info info[HP_MAX_VIEWS];
    const hp_status st = plan_views(cams, n_views, *p, geo, info);
    if (st != HP_OK) return st;
    const hp::TableWs tw = hp::table_ws_layout(ws, n, n_views, geo.n_buckets, geo.n_cells);
    if (!ws || ws_bytes < tw.bytes) return HP_E_WORKSPACE;

    const hipError_t e =
        hp::launch_build(xyz, n, geo.vs, geo.n_buckets, geo.n_cells, tw, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);

    memset(out, 0, sizeof(*out));
    out->n_views = n_views;
    out->layout = p->layout;
    out->n_points = n;
    out->n_buckets = geo.n_buckets;
    out->n_rays = geo.n_rays;
    out->offsets = tw.offsets;
    out->pts = reinterpret_cast<float *>(tw.pts);
    out->perm = tw.perm;
    out->pcam = reinterpret_cast<float *>(tw.pcam);
    out->bucket_z = tw.bucket_z;
    out->cell_zmin = tw.cell_zmin;
    out->n_cells = geo.n_cells;
    out->build_key = table_key(cams, n_views, *p);
    out->scratch = tw.views;
    memcpy(out->views, info, sizeof(hp_view_info) * n_views);
    return HP_OK;
}

static hp_status make_ctx(const hp_table *tab, const hp_camera *cams, int32_t n_views,
                          const hp_params *p, hp::SearchCtx &c)
{
    if (!tab || !cams || !p || n_views != tab->n_views || !valid_params(*p)) return HP_E_INVALID;
    if (p->layout != tab->layout || table_key(cams, n_views, *p) != tab->build_key)
        return HP_E_INVALID;
    if (p->K > HP_MAX_K) return HP_E_UNSUPPORTED;
    if (!tab->offsets || !tab->pts || !tab->pcam || !tab->scratch || !tab->bucket_z ||
        !tab->cell_zmin)
        return HP_E_INVALID;
    Geometry geo;
    const hp_status st = plan_views(cams, n_views, *p, geo, nullptr);
    if (st != HP_OK) return st;
    if (geo.n_rays != tab->n_rays || geo.n_buckets != tab->n_buckets) return HP_E_INVALID;
    for (int i = 0; i < n_views; ++i)
        if (tab->views[i].g != geo.vs.v[i].g || tab->views[i].W != cams[i].W ||
            tab->views[i].H != cams[i].H)
            return HP_E_INVALID;
    c.offsets = tab->offsets;
    c.pts = reinterpret_cast<const float4 *>(tab->pts);
    c.pcam = reinterpret_cast<const float4 *>(tab->pcam);
    c.bucket_z = tab->bucket_z;
    c.cell_zmin = tab->cell_zmin;
    c.views = reinterpret_cast<const hp::ViewK *>(tab->scratch);
    c.n_views = n_views;
    c.layout = tab->layout;
    c.n_points = tab->n_points;
    c.ray0 = 0;
    c.n_rays = tab->n_rays;
    c.radius = p->radius;
    c.inv_tref = p->inv_tref;
    c.t_near = p->t_near;
    c.t_far = p->t_far;
    c.gamma = p->gamma;
    c.inv_beta2 = p->inv_beta2;
    c.eps_w = p->eps_w;
    c.K = p->K;
    c.S = p->n_samples;
    c.M = p->m_cap;
    c.chunk = p->search_chunk > 0 ? p->search_chunk : 4;
    c.band = p->search_band > 0 ? p->search_band : hp::BAND_RAYS;
    c.window = p->window_shape;
    c.blocks = p->search_blocks;
    c.rmode = p->radius_mode;
    c.rddot = p->rddot;
    c.sampler = p->sampler;
    c.ms_steps = p->ms_steps;
    return HP_OK;
}

hp_status hp_search_sample(const hp_table *tab, const hp_camera *cams, int32_t n_views,
                           const hp_params *p, hp_samples *out, void *stream)
{
    hp::SearchCtx c;
    const hp_status st = make_ctx(tab, cams, n_views, p, c);
    if (st != HP_OK) return st;
    if (!out || !out->n_sel || !out->primary || !out->n_nbr || !out->flags || !out->t ||
        !out->knn_idx || !out->knn_dist)
        return HP_E_INVALID;
    if ((out->nbr_idx == nullptr) != (out->nbr_t == nullptr)) return HP_E_INVALID;
    hp::SampleOut o{out->n_sel, out->primary, out->n_nbr, out->flags, out->t,
                    out->knn_idx, out->knn_dist, out->nbr_idx, out->nbr_t};
    const hipError_t e = hp::launch_search_sample(c, o, knn_template(p->K), (hipStream_t)stream);
    return e == hipSuccess ? HP_OK : hip_fail(e);
}

hp_status hp_knp_blend(const hp_table *tab, const hp_camera *cams, int32_t n_views,
                       const hp_params *p, int32_t K, const float *colors, float *rgb,
                       int32_t *knp_cnt, int32_t *knp_idx, float *knp_dist, void *stream)
{
    hp::SearchCtx c;
    const hp_status st = make_ctx(tab, cams, n_views, p, c);
    if (st != HP_OK) return st;
    if (K < 1 || K > HP_MAX_MCAP) return HP_E_UNSUPPORTED;
    if (!colors || !rgb || ((knp_idx == nullptr) != (knp_dist == nullptr))) return HP_E_INVALID;
    hp::KnpArgs a;
    a.colors = colors;
    a.K = K;
    a.eps_idw = p->eps_idw;
    for (int i = 0; i < 3; ++i) a.bg[i] = p->bg[i];
    a.rgb = rgb;
    a.cnt = knp_cnt;
    a.idx = knp_idx;
    a.dist = knp_dist;
    const hipError_t e = hp::launch_knp(c, a, (hipStream_t)stream);
    return e == hipSuccess ? HP_OK : hip_fail(e);
}

hp_status hp_search_render(const hp_table *tab, const hp_camera *cams, int32_t n_views,
                           const hp_params *p, const float *feat, int32_t C, const hp_mlp *mlp,
                           int32_t precision, float *rgb, float *depth, float *acc,
                           int32_t *n_sel, void *stream)
{
    hp::SearchCtx c;
    const hp_status st = make_ctx(tab, cams, n_views, p, c);
    if (st != HP_OK) return st;
    if (C != HP_FEAT_DIM) return HP_E_UNSUPPORTED;
    if (p->n_samples > hp::fused_max_samples() || p->K > 16) return HP_E_UNSUPPORTED;
    if (precision != HP_FP32 && precision != HP_BF16) return HP_E_INVALID;
    if (!feat || !mlp || !rgb) return HP_E_INVALID;
    if (!mlp->W1 || !mlp->b1 || !mlp->W2 || !mlp->b2 || !mlp->W3 || !mlp->b3) return HP_E_INVALID;
    hp::FusedArgs a;
    a.feat = feat;
    a.w = hp::MlpWeights{mlp->W1, mlp->b1, mlp->W2, mlp->b2, mlp->W3, mlp->b3};
    a.eps_idw = p->eps_idw;
    a.delta_last = p->delta_last;
    for (int i = 0; i < 3; ++i) a.bg[i] = p->bg[i];
    a.rgb = rgb;
    a.depth = depth;
    a.acc = acc;
    a.n_sel = n_sel;
    a.K = p->K;
    const hipError_t e =
        hp::launch_fused(c, a, knn_template(p->K), precision, (hipStream_t)stream);
    return e == hipSuccess ? HP_OK : hip_fail(e);
}

hp_status hp_exp32_eval(const float *x, float *y, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!x || !y))) return HP_E_INVALID;
    const hipError_t e = hp::launch_exp_neg(x, y, n, (hipStream_t)stream);
    return e == hipSuccess ? HP_OK : hip_fail(e);
}

hp_status hp_bf16_eval(const float *x, float *y, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!x || !y))) return HP_E_INVALID;
    const hipError_t e = hp::launch_bf16_round(x, y, n, (hipStream_t)stream);
    return e == hipSuccess ? HP_OK : hip_fail(e);
}

hp_status hp_render(const hp_samples *smp, int64_t R, const float *feat, int32_t C,
                    const hp_mlp *mlp, int32_t precision, const hp_params *p, float *rgb,
                    float *depth, float *acc, void *stream)
{
    if (!smp || !mlp || !p || R < 0 || !valid_params(*p)) return HP_E_INVALID;
    if (C != HP_FEAT_DIM) return HP_E_UNSUPPORTED;
    if (precision != HP_FP32 && precision != HP_BF16) return HP_E_INVALID;
    if (p->K > HP_MAX_K) return HP_E_UNSUPPORTED;
    if (R >= ((int64_t)1 << 31)) return HP_E_CAPACITY;
    if (R > 0 && (!smp->n_sel || !smp->t || !smp->knn_idx || !smp->knn_dist || !feat || !rgb))
        return HP_E_INVALID;
    if (!mlp->W1 || !mlp->b1 || !mlp->W2 || !mlp->b2 || !mlp->W3 || !mlp->b3) return HP_E_INVALID;
    hp::RenderArgs a;
    a.n_sel = smp->n_sel;
    a.t = smp->t;
    a.knn_idx = smp->knn_idx;
    a.knn_dist = smp->knn_dist;
    a.n_rays = R;
    a.feat = feat;
    a.W1 = mlp->W1;
    a.b1 = mlp->b1;
    a.W2 = mlp->W2;
    a.b2 = mlp->b2;
    a.W3 = mlp->W3;
    a.b3 = mlp->b3;
    a.K = p->K;
    a.S = p->n_samples;
    a.eps_idw = p->eps_idw;
    a.delta_last = p->delta_last;
    for (int i = 0; i < 3; ++i) a.bg[i] = p->bg[i];
    a.rgb = rgb;
    a.depth = depth;
    a.acc = acc;
    a.rpw = p->render_rays > 0 ? p->render_rays : 16;
    a.blocks = p->render_blocks;
    const hipError_t e = hp::launch_render(a, precision, (hipStream_t)stream);
    return e == hipSuccess ? HP_OK : hip_fail(e);
}

}  // extern "C"

// Backward workspace: decoder-gradient slices, then (for the recomputing
// entry point) a ring holding the recomputed samples of one chunk of rays,
// each array 256-byte aligned.  The chunk is as many rays as the workspace
// holds (at most all of them), so the workspace need not grow with the rays.
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr int64_t BWD_DEFAULT_CHUNK_RAYS = 262144;

struct BwdWsLayout {
    size_t partial, n_sel, primary, n_nbr, flags, t, knn_idx, knn_dist, bytes;
};

static BwdWsLayout bwd_ws_layout(int64_t chunk_rays, const hp_params &p)
{
    BwdWsLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align256(bytes);
        return at;
    };
    const size_t R = (size_t)chunk_rays;
    const size_t RS = R * (size_t)p.n_samples;
    L.partial = take(hp::backward_partial_bytes());
    L.n_sel = take(R * 4);
    L.primary = take(R * 4);
    L.n_nbr = take(R * 4);
    L.flags = take(R * 4);
    L.t = take(RS * 4);
    L.knn_idx = take(RS * (size_t)p.K * 4);
    L.knn_dist = take(RS * (size_t)p.K * 4);
    L.bytes = off;
    return L;
}

// Rays per recompute chunk that ws_bytes holds (0: not even one), at most R.
static int64_t bwd_chunk_rays(size_t ws_bytes, int64_t R, const hp_params &p)
{
    if (ws_bytes < bwd_ws_layout(1, p).bytes) return 0;
    const size_t per_ray = 16 + (size_t)p.n_samples * (4 + 8 * (size_t)p.K);
    const size_t fixed = align256(hp::backward_partial_bytes()) + 7 * 256;
    int64_t n = ws_bytes > fixed ? (int64_t)((ws_bytes - fixed) / per_ray) : 1;
    const int64_t cap = R > 0 ? R : 1;
    if (n > cap) n = cap;
    if (n < 1) n = 1;
    while (n > 1 && bwd_ws_layout(n, p).bytes > ws_bytes) --n;
    return n;
}

static hp_status check_backward_args(const float *feat, int32_t C, const hp_mlp *mlp,
                                     int32_t precision, const hp_params *p, const float *grad_rgb,
                                     float *grad_feat, const hp_mlp *grad_mlp)
{
    if (!p || !valid_params(*p)) return HP_E_INVALID;
    if (C != HP_FEAT_DIM) return HP_E_UNSUPPORTED;
    if (p->K > HP_MAX_K) return HP_E_UNSUPPORTED;
    if (precision != HP_FP32 && precision != HP_BF16) return HP_E_INVALID;
    if (!feat || !mlp || !grad_rgb || !grad_feat || !grad_mlp) return HP_E_INVALID;
    if (!mlp->W1 || !mlp->b1 || !mlp->W2 || !mlp->b2 || !mlp->W3 || !mlp->b3) return HP_E_INVALID;
    if (!grad_mlp->W1 || !grad_mlp->b1 || !grad_mlp->W2 || !grad_mlp->b2 || !grad_mlp->W3 ||
        !grad_mlp->b3)
        return HP_E_INVALID;
    return HP_OK;
}

static hp::BwdArgs backward_args(const int32_t *n_sel, const float *t, const int32_t *knn_idx,
                                  const float *knn_dist, int64_t R, const float *feat,
                                  const hp_mlp *mlp, const hp_params *p, const float *grad_rgb,
                                  float *grad_feat, float *partial)
{
    hp::BwdArgs A;
    A.n_sel = n_sel;
    A.t = t;
    A.knn_idx = knn_idx;
    A.knn_dist = knn_dist;
    A.n_rays = R;
    A.K = p->K;
    A.S = p->n_samples;
    A.rpw = hp::backward_rays_per_wave(p->n_samples);
    A.feat = feat;
    A.w = hp::MlpWeights{mlp->W1, mlp->b1, mlp->W2, mlp->b2, mlp->W3, mlp->b3};
    A.eps_idw = p->eps_idw;
    A.delta_last = p->delta_last;
    for (int i = 0; i < 3; ++i) A.bg[i] = p->bg[i];
    A.grad_rgb = grad_rgb;
    A.grad_feat = grad_feat;
    A.partial = partial;
    A.queue = nullptr;  // (set by backward_accumulate)
    return A;
}

static hp::MlpGrad mlp_grad(const hp_mlp *g)
{
    return hp::MlpGrad{g->W1, g->b1, g->W2, g->b2, g->W3, g->b3};
}

// Recompute the samples of the table's rays chunk by chunk into the ring at
// `base` (layout L, chunk_rays rays) and accumulate each chunk's gradient.
static hp_status backward_recompute(const hp::SearchCtx &c0, const hp_params *p, const float *feat,
                                    const hp_mlp *mlp, int32_t precision, const float *grad_rgb,
                                    float *grad_feat, hp_mlp *grad_mlp, char *base,
                                    const BwdWsLayout &L, int64_t chunk_rays, hipStream_t stream)
{
    float *partial = reinterpret_cast<float *>(base + L.partial);
    hipError_t e = hp::backward_zero(partial, stream);
    if (e != hipSuccess) return hip_fail(e);
    hp::SampleOut o{reinterpret_cast<int32_t *>(base + L.n_sel),
                    reinterpret_cast<int32_t *>(base + L.primary),
                    reinterpret_cast<int32_t *>(base + L.n_nbr),
                    reinterpret_cast<uint32_t *>(base + L.flags),
                    reinterpret_cast<float *>(base + L.t),
                    reinterpret_cast<int32_t *>(base + L.knn_idx),
                    reinterpret_cast<float *>(base + L.knn_dist),
                    nullptr,
                    nullptr};
    const int kt = knn_template(p->K);
    for (int64_t r0 = 0; r0 < c0.n_rays; r0 += chunk_rays) {
        hp::SearchCtx c = c0;
        c.ray0 = r0;
        c.n_rays = (c0.n_rays - r0) < chunk_rays ? c0.n_rays - r0 : chunk_rays;
        e = hp::launch_search_sample(c, o, kt, stream);
        if (e != hipSuccess) return hip_fail(e);
        const hp::BwdArgs A = backward_args(o.n_sel, o.t, o.knn_idx, o.knn_dist, c.n_rays, feat, mlp,
                                            p, grad_rgb + 3 * r0, grad_feat, partial);
        e = hp::backward_accumulate(A, precision, stream);
        if (e != hipSuccess) return hip_fail(e);
    }
    e = hp::backward_reduce(partial, mlp_grad(grad_mlp), stream);
    return e == hipSuccess ? HP_OK : hip_fail(e);
}

extern "C" {

size_t hp_backward_workspace(const hp_table *tab, const hp_params *p, hp_status *status)
{
    const hp_status st = (tab && p && valid_params(*p) && tab->n_rays >= 0) ? HP_OK : HP_E_INVALID;
    if (status) *status = st;
    if (st != HP_OK) return 0;
    int64_t n = tab->n_rays < BWD_DEFAULT_CHUNK_RAYS ? tab->n_rays : BWD_DEFAULT_CHUNK_RAYS;
    return bwd_ws_layout(n > 0 ? n : 1, *p).bytes;
}

size_t hp_backward_samples_workspace(const hp_params *p, hp_status *status)
{
    const hp_status st = (p && valid_params(*p)) ? HP_OK : HP_E_INVALID;
    if (status) *status = st;
    return st == HP_OK ? align256(hp::backward_partial_bytes()) : 0;
}

hp_status hp_render_backward(const hp_table *tab, const hp_camera *cams, int32_t n_views,
                             const float *feat, int32_t C, const hp_mlp *mlp, int32_t precision,
                             const hp_params *p, const float *grad_rgb, float *grad_feat,
                             hp_mlp *grad_mlp, void *ws, size_t ws_bytes, void *stream)
{
    hp::SearchCtx c;
    hp_status st = make_ctx(tab, cams, n_views, p, c);
    if (st != HP_OK) return st;
    st = check_backward_args(feat, C, mlp, precision, p, grad_rgb, grad_feat, grad_mlp);
    if (st != HP_OK) return st;
    const int64_t chunk = bwd_chunk_rays(ws ? ws_bytes : 0, tab->n_rays, *p);
    if (!ws || chunk < 1) return HP_E_WORKSPACE;
    return backward_recompute(c, p, feat, mlp, precision, grad_rgb, grad_feat, grad_mlp,
                              static_cast<char *>(ws), bwd_ws_layout(chunk, *p), chunk,
                              (hipStream_t)stream);
}

hp_status hp_render_backward_samples(const hp_samples *smp, int64_t R, const float *feat,
                                     int32_t C, const hp_mlp *mlp, int32_t precision,
                                     const hp_params *p, const float *grad_rgb, float *grad_feat,
                                     hp_mlp *grad_mlp, void *ws, size_t ws_bytes, void *stream)
{
    if (!smp || R < 0) return HP_E_INVALID;
    const hp_status st = check_backward_args(feat, C, mlp, precision, p, grad_rgb, grad_feat, grad_mlp);
    if (st != HP_OK) return st;
    if (R >= ((int64_t)1 << 31)) return HP_E_CAPACITY;
    if (R > 0 && (!smp->n_sel || !smp->t || !smp->knn_idx || !smp->knn_dist)) return HP_E_INVALID;
    if (!ws || ws_bytes < align256(hp::backward_partial_bytes())) return HP_E_WORKSPACE;
    float *partial = static_cast<float *>(ws);
    hipError_t e = hp::backward_zero(partial, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    const hp::BwdArgs A = backward_args(smp->n_sel, smp->t, smp->knn_idx, smp->knn_dist, R, feat, mlp,
                                        p, grad_rgb, grad_feat, partial);
    e = hp::backward_accumulate(A, precision, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    e = hp::backward_reduce(partial, mlp_grad(grad_mlp), (hipStream_t)stream);
    return e == hipSuccess ? HP_OK : hip_fail(e);
}

}  // extern "C"

// Allocation-free backward.  Its decoder-gradient slices and recompute ring
// live in `scratch`, a device array that the code object brings with it (each
// GPU that loads the library holds its own copy until the process ends).  In
// host code the array's name stands for a host-side shadow, not a device
// address, so the kernels only ever receive the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device and kept.  Every call on a GPU reuses that GPU's array: the slices
// are cleared by a fill kernel at the start of each call, the ring is fully
// rewritten by each chunk's search; calls that overlap on one GPU race.
static __device__ __align__(256) unsigned char scratch[HP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[SCRATCH_MAX_DEVICES];

// Device address of the current device's scratch array (looked up on the
// first call on each device).
hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

hp_status hp_render_backward_noalloc(const hp_table *tab, const hp_camera *cams, int32_t n_views,
                                     const float *feat, int32_t C, const hp_mlp *mlp,
                                     int32_t precision, const hp_params *p, const float *grad_rgb,
                                     float *grad_feat, hp_mlp *grad_mlp, void *stream)
{
    hp::SearchCtx c;
    hp_status st = make_ctx(tab, cams, n_views, p, c);
    if (st != HP_OK) return st;
    st = check_backward_args(feat, C, mlp, precision, p, grad_rgb, grad_feat, grad_mlp);
    if (st != HP_OK) return st;
    // the slices and the samples of at least one ray must fit the array
    const int64_t chunk = bwd_chunk_rays(HP_NOALLOC_SCRATCH_BYTES, tab->n_rays, *p);
    if (chunk < 1) return HP_E_CAPACITY;
    void *base = nullptr;
    const hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return hip_fail(e);
    return backward_recompute(c, p, feat, mlp, precision, grad_rgb, grad_feat, grad_mlp,
                              static_cast<char *>(base), bwd_ws_layout(chunk, *p), chunk,
                              (hipStream_t)stream);
}

}  // extern "C"
