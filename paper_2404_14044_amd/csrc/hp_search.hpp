// Per-ray hashed-point search (Sec. 3.2) and adaptive primary-surface sampling
// (Sec. 3.3, Eq. 4, Eq. 5), one wave per ray.  Shared by the forward kernel
// and the backward kernel, which recomputes the samples instead of storing them.
//
// Search.  A neighbour of the ray is a point within rho(t) of it at its own
// parameter t in [t_near, t_far].  Such a point projects at most
//     delta(t) = f rho(t) L^2 / (t - rho(t) |w|)
// pixels from the ray's pixel centre (w: normalised image coordinate of the
// ray, L^2 = 1 + |w|^2, f = max(fx, fy)), and delta does not grow with t.  So
// the wave visits the buckets of a disc of radius delta(t_near) around the
// pixel, and inside a bucket at distance D from the pixel centre it only needs
// points with t <= f r L^2 / D + r |w|, i.e. with camera depth
//     z <= (f r L^2 / D + 2 r |w|) / L        (fixed-radius branch of rho),
// and since buckets are ordered by z a bucket whose first point is deeper is
// skipped whole.  These cuts are widened by relative margins far above binary32
// rounding; the exact predicate decides.
//
// Lanes first sweep the window buckets (one bucket per lane), compact the
// non-empty survivors into an LDS list, then sweep the points of the listed
// buckets (one point per lane, located by binary search over the list's
// prefix sums), apply the exact predicate and append the keys
// (t bits << 32 | point index) of passing points to a pending buffer.  Every
// 64 pending keys are sorted across the wave and merged into a running
// ascending top-64, whose largest key then filters later appends.
//
// Sampling.  Lane j takes candidate j (the j-th neighbour in (t, index)
// order).  Its K nearest neighbours among N(ray) within R_j = rho(t_j) can only
// lie in a window |t_i - t_j| <= R_j of the sorted list, found by binary
// search; the lane keeps a sorted register list of (dist^2 bits << 32 | index).
// Then the wave walks the candidates in order accumulating the transmittance
// of Eq. 5 and stops once no later candidate can pass eps_w (alpha <= gamma,
// so w_j <= gamma T).
#pragma once

#include "hp_device.hpp"

namespace hp {

struct SearchCtx {
    const int32_t *offsets;
    const float4 *pts;
    const int32_t *slot_of;
    const ViewK *views;
    int32_t n_views, layout;
    int64_t n_points, n_rays;
    float radius, inv_tref, t_near, t_far, gamma, inv_beta2, eps_w;
    int32_t K, S, M;
};

constexpr int BL_CAP = 128;

struct SearchLds {
    int32_t bl_start[BL_CAP];
    int32_t bl_cnt[BL_CAP];
    int32_t bl_pre[BL_CAP];
    float bl_zmax[BL_CAP];
    uint64_t pend[2 * WAVE];
    float4 nb_p[WAVE];
    float nb_t[WAVE];
};

// Ray geometry, uniform across the wave.
struct RayGeom {
    int vi, u, v;
    float dx, dy, dz, a, b, L, wn;
};

__device__ __forceinline__ void lds_sync() { __syncthreads(); }

__device__ __forceinline__ RayGeom ray_geometry(const SearchCtx &c, int64_t ray)
{
    RayGeom r;
    int vi = 0;
    while (vi + 1 < c.n_views && c.views[vi + 1].ray_base <= ray) ++vi;
    const ViewK &V = c.views[vi];
    const int local = (int)(ray - V.ray_base);
    r.vi = vi;
    r.u = local % V.W;
    r.v = local / V.W;
    ray_dir(V, r.u, r.v, r.dx, r.dy, r.dz, r.a, r.b, r.L);
    r.wn = __builtin_sqrtf(r.a * r.a + r.b * r.b);
    return r;
}

// Find the index of the last prefix entry <= q among pre[0..n).
__device__ __forceinline__ int find_bucket(const int32_t *pre, int n, int q)
{
    int lo = 0, hi = n;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Search one ray.  Returns, in `top` (one key per lane, ascending), the
// 64 smallest (t, index) keys of the ray's neighbours (missing = ~0), and
// the total neighbour count.
__device__ __forceinline__ void search_neighbours(const SearchCtx &c, const RayGeom &g,
                                                  SearchLds &sh, uint64_t &top, int &count)
{
    const int l = lane_id();
    const ViewK &V = c.views[g.vi];
    const float L2 = fma_rn(g.wn, g.wn, 1.0f);
    const float f = V.fx > V.fy ? V.fx : V.fy;
    const float rho_n = search_radius(c.radius, c.inv_tref, c.t_near);
    const float rho_f = search_radius(c.radius, c.inv_tref, c.t_far);
    const float z_lo = ((c.t_near - g.wn * rho_n) / g.L) * 0.999f - 1e-6f;
    const float z_hi = ((c.t_far + g.wn * rho_f) / g.L) * 1.001f + 1e-6f;
    // pixel offset bound once rho has reached its linear branch
    float dinf = 0.0f;
    if (c.inv_tref > 0.0f) {
        const float k = c.radius * c.inv_tref;
        const float den = 1.0f - k * g.wn;
        dinf = den > 0.0f ? (f * k * L2 / den) * 1.001f + 0.01f : __builtin_inff();
    }
    const float frL2 = f * c.radius * L2;
    const float two_rw = 2.0f * c.radius * g.wn;
    const float Dmax = V.dmax;
    int h = (int)__builtin_floorf(Dmax + 0.5f);
    if (h > V.g) h = V.g;
    const int Wd = 2 * h + 1;
    const int total = Wd * Wd;
    const int gx = g.u + V.g, gy = g.v + V.g;

    top = ~0ull;
    uint64_t tau = ~0ull;
    count = 0;
    int npend = 0;
    int nbl = 0;

    auto flush = [&](int take) {
        // merge pend[0..take) (take <= 64) into top; keep the rest pending
        lds_sync();
        uint64_t x = (l < take) ? sh.pend[l] : ~0ull;
        const int rem = npend - take;
        const uint64_t y = (l < rem) ? sh.pend[take + l] : 0ull;
        lds_sync();
        if (l < rem) sh.pend[l] = y;
        npend = rem;
        x = wave_sort_u64(x);
        top = wave_merge_low_u64(top, x);
        tau = shfl_u64(top, WAVE - 1);
        lds_sync();
    };

    auto sweep_points = [&](int nb) {
        // prefix sums of the listed bucket sizes
        lds_sync();
        const int c0 = (l < nb) ? sh.bl_cnt[l] : 0;
        const int i0 = wave_incl_scan_i32(c0);
        const int c1 = (WAVE + l < nb) ? sh.bl_cnt[WAVE + l] : 0;
        const int i1 = wave_incl_scan_i32(c1) + readlane_i32(i0, WAVE - 1);
        sh.bl_pre[l] = i0 - c0;
        sh.bl_pre[WAVE + l] = i1 - c1;
        const int totp = readlane_i32(i1, WAVE - 1);
        lds_sync();
        for (int p0 = 0; p0 < totp; p0 += WAVE) {
            const int p = p0 + l;
            bool pass = false;
            uint64_t key = 0;
            if (p < totp) {
                const int bsel = find_bucket(sh.bl_pre, nb, p);
                const int slot = sh.bl_start[bsel] + (p - sh.bl_pre[bsel]);
                const float4 P = c.pts[slot];
                if (P.z <= sh.bl_zmax[bsel] && P.z >= z_lo) {
                    const float t = ray_param(P.x, P.y, P.z, g.dx, g.dy, g.dz);
                    const float e2 = dist2_at(P.x, P.y, P.z, g.dx, g.dy, g.dz, t);
                    const float rho = search_radius(c.radius, c.inv_tref, t);
                    pass = (P.z > 0.0f) & (t >= c.t_near) & (t <= c.t_far) & (e2 <= rho * rho);
                    key = ((uint64_t)__float_as_uint(t) << 32) | __float_as_uint(P.w);
                }
            }
            count += popc64(ballot(pass));
            const bool keep = pass && key < tau;
            const uint64_t km = ballot(keep);
            if (keep) sh.pend[npend + rank_below(km)] = key;
            npend += popc64(km);
            if (npend >= WAVE) flush(WAVE);
        }
    };

    for (int q0 = 0; q0 < total; q0 += WAVE) {
        const int q = q0 + l;
        bool ok = q < total;
        int st = 0, cnt = 0;
        float zmax = z_hi;
        if (ok) {
            const int qy = q / Wd;
            const int dyi = qy - h, dxi = q - qy * Wd - h;
            const int bx = gx + dxi, by = gy + dyi;
            ok = bx >= 0 && bx < V.Wg && by >= 0 && by < V.Hg;
            const float ex = __builtin_fmaxf(0.0f, __builtin_fabsf((float)dxi) - 0.5f);
            const float ey = __builtin_fmaxf(0.0f, __builtin_fabsf((float)dyi) - 0.5f);
            const float D = __builtin_sqrtf(ex * ex + ey * ey);
            ok = ok && D <= Dmax;
            const float Dp = D - 0.01f;
            if (Dp > 0.0f && Dp > dinf) {
                const float zc = ((frL2 / Dp + two_rw) / g.L) * 1.001f + 1e-5f;
                zmax = zc < z_hi ? zc : z_hi;
            }
            if (ok) {
                const int key = bucket_of(V, c.layout, bx, by);
                st = c.offsets[key];
                cnt = c.offsets[key + 1] - st;
                ok = cnt > 0;
                if (ok) ok = c.pts[st].z <= zmax;
            }
        }
        const uint64_t m = ballot(ok);
        if (ok) {
            const int pos = nbl + rank_below(m);
            sh.bl_start[pos] = st;
            sh.bl_cnt[pos] = cnt;
            sh.bl_zmax[pos] = zmax;
        }
        nbl += popc64(m);
        if (nbl >= WAVE || (q0 + WAVE >= total && nbl > 0)) {
            sweep_points(nbl);
            nbl = 0;
        }
    }
    if (npend > 0) flush(npend);
}

// Candidate walk.  On return lane j < m holds candidate j: its t, point index,
// its K nearest neighbours `kd` (ascending (dist^2 bits, index), ~0 = none),
// their number kc, and alpha.  selmask has bit j set for selected candidates.
template <int KT>
__device__ __forceinline__ void walk_candidates(const SearchCtx &c, const RayGeom &g, SearchLds &sh,
                                                uint64_t top, int m, float &tj, int &idxj,
                                                uint64_t (&kd)[KT], int &kc, float &alpha,
                                                uint64_t &selmask, int &n_sel)
{
    const int l = lane_id();
    const bool cand = l < m;
    tj = __uint_as_float((uint32_t)(top >> 32));
    idxj = (int)(uint32_t)top;
    lds_sync();
    if (cand) {
        const int slot = c.slot_of[(int64_t)g.vi * c.n_points + idxj];
        sh.nb_p[l] = c.pts[slot];
        sh.nb_t[l] = tj;
    }
    lds_sync();
#pragma unroll
    for (int k = 0; k < KT; ++k) kd[k] = ~0ull;
    int lo = 0, hi = 0;
    float Rj = 0.0f, R2 = 0.0f;
    if (cand) {
        Rj = search_radius(c.radius, c.inv_tref, tj);
        R2 = Rj * Rj;
        const float span = Rj * 1.001f + tj * 4e-6f + 1e-7f;
        const float tlo = tj - span, thi = tj + span;
        int a = 0, b = m;  // first index with nb_t >= tlo
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (sh.nb_t[mid] < tlo) a = mid + 1;
            else b = mid;
        }
        lo = a;
        b = m;  // first index with nb_t > thi
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (sh.nb_t[mid] <= thi) a = mid + 1;
            else b = mid;
        }
        hi = a;
    }
    int span_n = hi - lo;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const int y = __shfl_xor(span_n, o, WAVE);
        span_n = span_n > y ? span_n : y;
    }
    for (int it = 0; it < span_n; ++it) {
        const int i = lo + it;
        bool ins = false;
        uint64_t key = ~0ull;
        if (i < hi) {
            const float4 P = sh.nb_p[i];
            const float d2 = dist2_at(P.x, P.y, P.z, g.dx, g.dy, g.dz, tj);
            key = ((uint64_t)__float_as_uint(d2) << 32) | __float_as_uint(P.w);
            ins = (d2 <= R2) && (key < kd[KT - 1]);
        }
        if (ballot(ins)) {
            if (ins) {
                uint64_t x = key;
#pragma unroll
                for (int k = 0; k < KT; ++k) {
                    const uint64_t lo64 = umin64(kd[k], x);
                    x = umax64(kd[k], x);
                    kd[k] = lo64;
                }
            }
        }
    }
    kc = 0;
    float sum = 0.0f;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        if (k < c.K && kd[k] != ~0ull) {
            sum = sum + __builtin_sqrtf(__uint_as_float((uint32_t)(kd[k] >> 32)));
            ++kc;
        }
    }
    alpha = 0.0f;
    if (cand) {
        const float dj = (sum + (float)(c.K - kc) * Rj) / (float)c.K;
        const float uj = (dj * dj) * c.inv_beta2;
        alpha = c.gamma * exp_neg(-uj);
    }
    // transmittance walk in candidate order (Eq. 5)
    float T = 1.0f;
    int sel = 0;
    uint64_t smask = 0;
    for (int j = 0; j < m; ++j) {
        const float aj = readlane_f32(alpha, j);
        const float wj = aj * T;
        if (wj > c.eps_w && sel < c.S) {
            smask |= 1ull << j;
            ++sel;
        }
        T = T * (1.0f - aj);
        if (sel == c.S || c.gamma * T <= c.eps_w) break;
    }
    selmask = smask;
    n_sel = sel;
}

}  // namespace hp
