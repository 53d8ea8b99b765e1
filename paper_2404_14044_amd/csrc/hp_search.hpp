// Per-ray hashed-point search (Sec. 3.2) and adaptive primary-surface sampling
// (Sec. 3.3, Eq. 4, Eq. 5), one wave per ray.  Shared by the search + sampling
// kernels (also run by the backward pass to recompute its samples), the K-NP
// kernel and the fused search + render kernel.
//
// Search.  A neighbour of the ray is a point within rho(t) of it at its own
// parameter t in [t_near, t_far].  Such a point projects at most
//     delta(t) = f rho(t) L^2 / (t - rho(t) |w|)
// pixels from the ray's pixel centre (w: normalised image coordinate of the
// ray, L^2 = 1 + |w|^2, f = max(fx, fy)), and delta does not grow with t.
// Its depth z also bounds t from below, t >= (L z - |w| r) / (1 + |w| r
// inv_tref).  So
//   1. the minimum depth of the 8x8-bucket cells around the pixel is read; if
//      they are all empty the ray has no neighbour, else the smallest depth
//      bounds t and thus the window radius delta(t) (two rounds, each over the
//      cells of the previous radius; four lanes per ray do this for up to
//      sixteen rays at once, ray_setup);
//   2. the wave visits the buckets of that disc, and inside a bucket at distance D from
//      the pixel centre only needs points with t <= f r L^2 / D + r |w|, i.e.
//      z <= (f r L^2 / D + 2 r |w|) / L (fixed-radius branch of rho); buckets
//      are ordered by z, so a bucket whose first point is deeper is skipped.
// Every bound is widened by relative margins far above binary32 rounding; the
// exact predicate decides.
//
// Lanes first sweep the window buckets (one bucket per lane), compact the
// non-empty survivors into an LDS list, then sweep the points of the listed
// buckets (one point per lane, its bucket found by a prefix maximum over the
// bucket heads), apply the exact predicate and append the keys
// (t bits << 32 | point index) of passing points to a pending buffer.  Every
// 64 pending keys are sorted across the wave and merged into a running
// ascending top-64, whose largest key then filters later appends.
//
// Sampling.  Candidates are the neighbours in (t, index) order.  The K
// nearest neighbours of candidate j within R_j = rho(t_j) lie in the window
// |t_i - t_j| <= R_j of the sorted list (distance >= |t_i - t_j| up to
// rounding), found by binary search.  Sixteen candidates are served at once,
// four lanes each: the lanes split the window, keep sorted register lists of
// (dist^2 bits << 32 | index) and merge them across the quad.  The wave then
// walks those candidates in order accumulating the transmittance of Eq. 5 and
// stops once no later candidate can pass eps_w (alpha <= gamma, so
// w_j <= gamma T), which usually happens within the first sixteen.
#pragma once
#include "hp_device.hpp"

namespace hp {

struct SearchCtx {
    const int32_t *offsets;
    const float4 *pts;
    const float4 *pcam;    // camera-space points in point order, per view
    const float *bucket_z;
    const uint32_t *cell_zmin;
    const ViewK *views;
    int32_t n_views, layout;
    int64_t n_points;
    int64_t ray0, n_rays;   // rays ray0 .. ray0 + n_rays - 1 of the table's views
    float radius, inv_tref, t_near, t_far, gamma, inv_beta2, eps_w;
    int32_t K, S, M;
    int32_t chunk, blocks;  // rays per work chunk, persistent grid (0 = default)
    int32_t rmode;          // HP_RADIUS_*
    float rddot;            // Eq. 3 kernel disc radius (unit focal length)
    int32_t sampler;        // HP_SAMPLER_*
    int32_t ms_steps;       // uniform positions of the multi-surface sampler
    int32_t band;           // consecutive rays per XCD band (BAND_RAYS by default)
    int32_t window;         // HP_WINDOW_*: disc of buckets, or the square around it
};

// One ray's geometry and search bounds, uniform across the wave that
// searches it (computed once per ray by one lane, see ray_setup).
struct RayGeom {
    int32_t vi, gx, gy;  // view, pixel position in the padded bucket grid
    int32_t h;           // window half-width in buckets; -1: nothing can be near
    float dx, dy, dz;    // unit direction (camera frame)
    float wn;            // |w|, the norm of the normalised image coordinate
    float kappa;         // Eq. 3 cone slope of this pixel (rho = kappa t), 0 in the linear mode
    float inv_L;         // 1 / L
    float z_lo, z_hi;    // depth range of possible neighbours
    float dinf;          // window radius once rho is on its linear branch
    float frL2, two_rw;  // f r L^2 and 2 r |w| of the per-bucket depth bound
    float Dmax;          // window radius in pixels
};

constexpr int BL_CAP = 128;
constexpr int RS_CAP = 16;              // rays whose set-up one pass computes
constexpr int RS_LANES = WAVE / RS_CAP;  // lanes per ray in that pass

struct SearchLds {
    RayGeom rs[RS_CAP];
    int32_t bl_start[BL_CAP];
    int32_t bl_cnt[BL_CAP];
    int32_t bl_pre[WAVE];  // (indexed by flat point offset within a sweep step)
    float bl_zmax[BL_CAP];
    uint64_t pend[2 * WAVE];
    float4 nb_p[WAVE];
    float nb_t[WAVE];
};
// 32 one-wave workgroups (8 waves per SIMD) share a CU's 160 KB of LDS
static_assert(sizeof(SearchLds) <= 5120, "search LDS above 5120 B halves occupancy");

// Rays per XCD band: two image rows of an 800-pixel-wide view (object view
// 0.568 ms with bands of 12,800 rays, 0.545 with 3,200, 0.532 with 1,600,
// 0.534 with 800; room view 3.09, 2.83, 2.81, 2.81 ms).
constexpr int64_t BAND_RAYS = 1600;

// Default grid of the search launches: 65,536 one-wave workgroups (on the
// object view, 640k rays, 2.4 chunks of 4 rays each), eight times what the
// GPU keeps resident, so workgroups that drew empty chunks are replaced as
// they finish (measured: 8,192 resident-sized persistent workgroups
// 0.631 ms, 65,536 0.56 ms; room view 4.04 vs 3.69 ms; one workgroup per
// chunk 0.58 / 3.91 ms).
constexpr int64_t DEFAULT_SEARCH_BLOCKS = 65536;

// Grid for the banded launches: at most `cap` workgroups, a multiple of 8.
inline int64_t banded_grid(const SearchCtx &c, int64_t cap)
{
    const int64_t chunks = (c.n_rays + c.chunk - 1) / c.chunk;
    int64_t blocks = chunks < cap ? chunks : cap;
    if (blocks == 0) return 0;
    return blocks < 8 ? 8 : (blocks & ~(int64_t)7);
}

// Search radius of a ray at parameter t.
__device__ __forceinline__ float rho_at(const SearchCtx &c, const RayGeom &g, float t)
{
    return c.rmode == HP_RADIUS_LINEAR ? search_radius(c.radius, c.inv_tref, t) : t * g.kappa;
}

__device__ __forceinline__ void lds_sync() { wave_lds_sync(); }

// ---------------------------------------------------------------------------
// cross-lane exchange: lane l receives lane l ^ j's value.  DPP for j < 16
// (row rotations act inside rows of 16 lanes), swizzle for 16, permute for 32.
// The last two run on the LDS crossbar, off the vector ALU, which bounds the
// search kernels (the gfx950 permlane swaps measured slower here for that).
// ---------------------------------------------------------------------------
template <int J>
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t v)
{
    // (mov_dpp with every row and bank enabled writes all lanes: no old value)
    const int x = (int)v;
    if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);
    if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);
    if constexpr (J == 4) {
        const int down = __builtin_amdgcn_mov_dpp(x, 0x124, 0xF, 0xF, false);  // from l - 4
        const int up = __builtin_amdgcn_mov_dpp(x, 0x12C, 0xF, 0xF, false);    // from l + 4
        return (uint32_t)((lane_id() & 4) ? down : up);
    }
    if constexpr (J == 8) return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, false);
    if constexpr (J == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle(x, 0x401F);
    return (uint32_t)__shfl_xor(x, J, WAVE);
}

template <int J>
__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t v)
{
    const uint32_t lo = xor_lane_u32<J>((uint32_t)v);
    const uint32_t hi = xor_lane_u32<J>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// The lanes whose index has bit k set, as a 64-bit lane mask.
constexpr uint64_t lane_bit_mask(int k)
{
    return k == 0   ? 0xAAAAAAAAAAAAAAAAull
           : k == 1 ? 0xCCCCCCCCCCCCCCCCull
           : k == 2 ? 0xF0F0F0F0F0F0F0F0ull
           : k == 3 ? 0xFF00FF00FF00FF00ull
           : k == 4 ? 0xFFFF0000FFFF0000ull
                    : 0xFFFFFFFF00000000ull;
}

// Per-lane predicate "bit i of mask M" from a constant mask: the compiler
// builds the mask with two scalar moves where it is used, where a lane-index
// test was kept in a scalar register pair for the whole kernel (six of them
// for the sorts) and pushed other scalars out to vector lanes.
template <uint64_t M>
__device__ __forceinline__ bool lanes_in(void)
{
    return __builtin_amdgcn_inverse_ballot_w64(M);
}

constexpr int log2_lane(int j) { return j == 1 ? 0 : j == 2 ? 1 : j == 4 ? 2 : j == 8 ? 3 : j == 16 ? 4 : 5; }

// One compare-exchange stage in which every block ascends: lanes l and l ^ J
// keep the minimum in the lower lane (one 64-bit compare, two selects).
template <int J>
__device__ __forceinline__ uint64_t cx_stage(uint64_t x, int)
{
    const uint64_t y = xor_lane_u64<J>(x);
    const bool take = (y < x) != lanes_in<lane_bit_mask(log2_lane(J))>();
    return take ? y : x;
}

template <int J>
__device__ __forceinline__ uint64_t cx_merge(uint64_t x, int l)
{
    x = cx_stage<J>(x, l);
    if constexpr (J > 1) x = cx_merge<J / 2>(x, l);
    return x;
}

// Inverts the keys of the lanes whose lane-index bits A and B differ (B = -1:
// bit A alone): bitwise NOT reverses the order of keys.
template <int A, int B>
__device__ __forceinline__ uint64_t flip_keys(uint64_t x)
{
    constexpr uint64_t m = lane_bit_mask(A) ^ (B >= 0 ? lane_bit_mask(B) : 0ull);
    return lanes_in<m>() ? ~x : x;
}

// Bitonic sort of one key per lane across the wave.  In the merge of blocks
// of K lanes, the blocks that must descend hold inverted keys, so that every
// stage is the same ascending compare-exchange; the keys are re-inverted
// between block sizes as the block directions change.
template <bool DESC>
__device__ __forceinline__ uint64_t wave_sort_dir(uint64_t x)
{
    const int l = lane_id();
    x = flip_keys<1, -1>(x);  // K = 2 blocks descend where lane bit 1 is set
    if constexpr (DESC) x = ~x;
    x = cx_merge<1>(x, l);
    x = flip_keys<1, 2>(x);
    x = cx_merge<2>(x, l);
    x = flip_keys<2, 3>(x);
    x = cx_merge<4>(x, l);
    x = flip_keys<3, 4>(x);
    x = cx_merge<8>(x, l);
    x = flip_keys<4, 5>(x);
    x = cx_merge<16>(x, l);
    x = flip_keys<5, -1>(x);  // one block of 64: ascends (descends with DESC)
    x = cx_merge<32>(x, l);
    if constexpr (DESC) x = ~x;
    return x;
}

__device__ __forceinline__ uint64_t wave_sort_fast(uint64_t x) { return wave_sort_dir<false>(x); }
__device__ __forceinline__ uint64_t wave_sort_desc(uint64_t x) { return wave_sort_dir<true>(x); }

// Keep the 64 smallest of an ascending and a descending wave-sorted list,
// ascending: their lane-wise minimum is bitonic and holds the 64 smallest;
// half-cleaners then sort it.
__device__ __forceinline__ uint64_t wave_merge_low_fast(uint64_t asc, uint64_t desc)
{
    return cx_merge<WAVE / 2>(umin64(asc, desc), lane_id());
}

// Lane p of each quad's value, on all four lanes (p a constant after unrolling).
__device__ __forceinline__ uint32_t quad_bcast_u32(uint32_t v, int p)
{
    const int x = (int)v;
    switch (p) {
    case 0: return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x00, 0xF, 0xF, false);
    case 1: return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x55, 0xF, 0xF, false);
    case 2: return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xAA, 0xF, 0xF, false);
    default: return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xFF, 0xF, 0xF, false);
    }
}

__device__ __forceinline__ uint64_t quad_bcast_u64(uint64_t v, int p)
{
    return ((uint64_t)quad_bcast_u32((uint32_t)(v >> 32), p) << 32) | quad_bcast_u32((uint32_t)v, p);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive prefix maximum across the wave (row shifts, then row broadcasts).
// Lanes without a source read INT_MIN, the identity of max, which lets the
// compiler fold each shift into its max instruction.
__device__ __forceinline__ int wave_prefix_max_i32(int v)
{
    constexpr int I = (int)0x80000000;
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x111, 0xF, 0xF, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x112, 0xF, 0xF, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x113, 0xF, 0xF, false));  // row_shr:3
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x114, 0xF, 0xE, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x118, 0xF, 0xC, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(I, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return v;
}

// Minimum depth over the depth cells holding the buckets within h of grid
// position (gx, gy) (+inf if they are all empty), by the RS_LANES lanes of a
// group (sub = lane within the group; every lane of the group returns it).
__device__ __forceinline__ float group_cells_zmin(const SearchCtx &c, const ViewK &V, int gx, int gy,
                                                  int h, int sub)
{
    const int cx0 = max(gx - h, 0) >> CELL_SHIFT, cx1 = min(gx + h, V.Wg - 1) >> CELL_SHIFT;
    const int cy0 = max(gy - h, 0) >> CELL_SHIFT, cy1 = min(gy + h, V.Hg - 1) >> CELL_SHIFT;
    float z = __builtin_inff();
    // cells in row-major order, cell sub, sub + RS_LANES, ... of the block to
    // this lane, four loads in flight at a time (a load per step of a nested
    // loop waited for each in turn); the minimum does not depend on the order
    const int nx = cx1 - cx0 + 1, ny = cy1 - cy0 + 1;
    const int ncell = (nx > 0 && ny > 0) ? nx * ny : 0;  // (nx >= 1 below)
    int cx = cx0 + sub, cy = cy0;
    if (ncell > 0)
        while (cx > cx1 && cy <= cy1) cx -= nx, ++cy;
    for (int ci = sub; ci < ncell; ci += 4 * RS_LANES) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = ci + j * RS_LANES < ncell ? __uint_as_float(c.cell_zmin[V.cell_base + cy * V.ncx + cx])
                                             : __builtin_inff();
            cx += RS_LANES;
            while (cx > cx1 && cy <= cy1) cx -= nx, ++cy;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) z = __builtin_fminf(z, v[j]);
    }
    static_assert(RS_LANES == 4 || RS_LANES == 8, "groups of four or eight lanes");
    z = __builtin_fminf(z, __uint_as_float(xor_lane_u32<1>(__float_as_uint(z))));
    z = __builtin_fminf(z, __uint_as_float(xor_lane_u32<2>(__float_as_uint(z))));
    if constexpr (RS_LANES == 8)
        z = __builtin_fminf(z, __uint_as_float(xor_lane_u32<4>(__float_as_uint(z))));
    return z;
}

// Reciprocal for the search bounds only (within a few ulp: every bound
// carries a relative margin of at least 1e-4; the exact predicate decides).
__device__ __forceinline__ float bound_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Window radius (pixels) for neighbours whose depth is at least zmin.
__device__ __forceinline__ float radius_for_depth(const SearchCtx &c, float kappa, float L, float wn,
                                                  float f, float L2, float zmin, float dcap,
                                                  float dinf)
{
    // a pure cone projects to a disc whose radius does not depend on depth
    if (c.rmode != HP_RADIUS_LINEAR) return dinf < dcap ? dinf : dcap;
    const float k = c.radius * c.inv_tref;
    float t = (L * zmin - wn * c.radius) * bound_rcp(1.0f + wn * k);
    t = t * 0.9999f - 1e-6f;
    if (!(t > c.t_near)) t = c.t_near;
    const float rho = search_radius(c.radius, c.inv_tref, t);
    const float den = t - rho * wn;
    if (!(den > 0.0f)) return dcap;
    const float d = (f * rho * L2 * bound_rcp(den)) * 1.0001f + 0.01f;
    return d < dcap ? d : dcap;
}

// Geometry and search bounds of one ray, computed by a group of RS_LANES
// lanes (sub = lane within the group), which share the depth-cell rounds.  The window:
// a neighbour projects at most delta(t) = f rho L^2 / (t - rho |w|) pixels
// from the pixel centre, and delta does not grow with t; the smallest depth
// of the depth cells around the pixel bounds t from below, so two rounds
// (each over the cells of the previous radius) shrink the window from the
// view-wide bound.  If every such cell is empty, no point is near the ray.
__device__ __forceinline__ int ray_view(const SearchCtx &c, int64_t ray)
{
    // bisection over the views' first rays (a walk along the list waits for
    // each load in turn): views[lo].ray_base <= ray < views[hi].ray_base
    int lo = 0, hi = c.n_views;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (c.views[mid].ray_base <= ray) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Window half-width of the first depth-cell round: the view-wide bound.
__device__ __forceinline__ int first_round_h(const ViewK &V)
{
    return min((int)__builtin_floorf(V.dmax + 0.5f), V.g);
}

// Minimum depth of the cells within the view-wide window of a ray (+inf:
// no point can be near it), by a group of RS_LANES lanes.
__device__ __forceinline__ float ray_first_zmin(const SearchCtx &c, int64_t ray, int sub)
{
    const int vi = ray_view(c, ray);
    const ViewK &V = c.views[vi];
    const int local = (int)(ray - V.ray_base);
    return group_cells_zmin(c, V, local % V.W + V.g, local / V.W + V.g, first_round_h(V), sub);
}

// (zmin1: the first round's minimum depth, ray_first_zmin, already taken)
__device__ __forceinline__ RayGeom ray_setup(const SearchCtx &c, int64_t ray, int sub, float zmin1)
{
    RayGeom g;
    const int vi = ray_view(c, ray);
    const ViewK &V = c.views[vi];
    const int local = (int)(ray - V.ray_base);
    const int u = local % V.W, v = local / V.W;
    float a, b, L;
    ray_dir(V, u, v, g.dx, g.dy, g.dz, a, b, L);
    g.vi = vi;
    g.wn = __builtin_sqrtf(a * a + b * b);
    // Eq. 3 on the unit-focal image plane: BF = rddot / L over AB, AF or AE
    g.kappa = 0.0f;
    if (c.rmode != HP_RADIUS_LINEAR) {
        const float bf = c.rddot / L;
        if (c.rmode == HP_RADIUS_EQ3) {
            const float m = g.wn - c.rddot;
            g.kappa = bf / __builtin_sqrtf(fma_rn(m, m, 1.0f));
        } else if (c.rmode == HP_RADIUS_EQ3_AF) {
            g.kappa = bf / fma_rn(-bf, g.wn, L);
        } else {
            g.kappa = bf / L;
        }
    }
    const float L2 = fma_rn(g.wn, g.wn, 1.0f);
    const float f = V.fx > V.fy ? V.fx : V.fy;
    const float rho_n = rho_at(c, g, c.t_near);
    const float rho_f = rho_at(c, g, c.t_far);
    g.inv_L = bound_rcp(L);
    g.z_lo = ((c.t_near - g.wn * rho_n) * g.inv_L) * 0.999f - 1e-6f;
    g.z_hi = ((c.t_far + g.wn * rho_f) * g.inv_L) * 1.001f + 1e-6f;
    // pixel offset bound once rho has reached its linear branch
    g.dinf = 0.0f;
    const float klin = c.rmode == HP_RADIUS_LINEAR ? c.radius * c.inv_tref : g.kappa;
    if (klin > 0.0f) {
        const float den = 1.0f - klin * g.wn;
        g.dinf = den > 0.0f ? (f * klin * L2 * bound_rcp(den)) * 1.001f + 0.01f : __builtin_inff();
    }
    g.frL2 = f * c.radius * L2;
    g.two_rw = 2.0f * c.radius * g.wn;
    g.gx = u + V.g;
    g.gy = v + V.g;
    float Dmax = V.dmax;
    int h = first_round_h(V);
    for (int round = 0; round < 2; ++round) {
        const float zmin = round == 0 ? zmin1 : group_cells_zmin(c, V, g.gx, g.gy, h, sub);
        if (!(zmin < __builtin_inff())) {
            h = -1;  // no point anywhere near this ray
            break;
        }
        Dmax = radius_for_depth(c, g.kappa, L, g.wn, f, L2, zmin, Dmax, g.dinf);
        h = min((int)__builtin_floorf(Dmax + 0.5f), V.g);
    }
    g.h = h;
    g.Dmax = Dmax;
    return g;
}

__device__ __forceinline__ float uniform_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A ray's set-up as the whole wave reads it back from the LDS.  A ray with
// nothing near it (h < 0) needs no more than h.
__device__ __forceinline__ RayGeom load_ray(const RayGeom &src)
{
    RayGeom g;
    g.h = uniform_i32(src.h);
    if (g.h < 0) {
        g.vi = g.gx = g.gy = 0;
        g.dx = g.dy = g.dz = g.wn = g.kappa = g.inv_L = 0.0f;
        g.z_lo = g.z_hi = g.dinf = g.frL2 = g.two_rw = g.Dmax = 0.0f;
        return g;
    }
    g.vi = uniform_i32(src.vi);
    g.gx = uniform_i32(src.gx);
    g.gy = uniform_i32(src.gy);
    g.dx = uniform_f32(src.dx);
    g.dy = uniform_f32(src.dy);
    g.dz = uniform_f32(src.dz);
    g.wn = uniform_f32(src.wn);
    g.kappa = uniform_f32(src.kappa);
    g.inv_L = uniform_f32(src.inv_L);
    g.z_lo = uniform_f32(src.z_lo);
    g.z_hi = uniform_f32(src.z_hi);
    g.dinf = uniform_f32(src.dinf);
    g.frL2 = uniform_f32(src.frL2);
    g.two_rw = uniform_f32(src.two_rw);
    g.Dmax = uniform_f32(src.Dmax);
    return g;
}

// Persistent iteration over the rays of a launch, one ray at a time per
// workgroup, body(ray, geometry).  Workgroups take chunks of c.chunk
// consecutive rays (neighbouring pixels share table buckets).  They are dealt
// to the eight XCDs round-robin (workgroup b runs on XCD b % 8), each with its
// own L2, so the chunks are grouped into bands of BAND_RAYS consecutive rays
// and XCD x takes bands x, x + 8, ...: the rays one XCD's workgroups search at
// a time are then neighbours and share that L2's table lines.  Within its
// bands an XCD's workgroups stride by their number, so each still sees a mix
// of empty and busy regions.  The grid must be a multiple of 8.
// The per-ray set-up (divisions, square roots, the depth-cell rounds) is
// uniform work that a whole wave would repeat on every lane; groups of lanes
// instead compute it for up to RS_CAP rays of the chunk at once into the LDS.
// The first depth-cell round goes first: a ray whose view-wide window holds
// no point (most rays of a view that an object does not fill) is finished
// there by empty(ray), called on one lane per such ray, and neither gets the
// rest of the set-up nor a pass of the wave.
template <typename Body, typename Empty>
__device__ __forceinline__ void for_each_ray_banded(const SearchCtx &c, RayGeom *rs, Body body,
                                                    Empty empty)
{
    const int l = lane_id();
    // (chunk, band and slot numbers in 32 bits: a launch has fewer than 2^31
    // rays, so every chunk number below fits an unsigned 32-bit integer, and
    // 64-bit ones held scalar registers that the body then spilled)
    const uint32_t n_chunks = (uint32_t)((c.n_rays + c.chunk - 1) / c.chunk);
    // chunks per band (fewer when the launch has fewer than eight full bands,
    // so that every XCD gets a share)
    uint32_t band = (uint32_t)(((int64_t)c.band + c.chunk - 1) / c.chunk);
    if ((uint64_t)band * 8 > n_chunks) band = (n_chunks + 7) / 8 > 0 ? (n_chunks + 7) / 8 : 1;
    const uint32_t xcd = blockIdx.x & 7;
    const uint32_t slot = blockIdx.x >> 3, n_slots = gridDim.x >> 3;
    const uint32_t n_bands = (n_chunks + band - 1) / band;
    const uint32_t my_chunks = (n_bands > xcd ? (n_bands - xcd + 7) / 8 : 0) * band;
    // first ray (relative to c.ray0) and ray count of this workgroup's li-th chunk
    auto chunk_rays = [&](uint32_t li, uint32_t &r0, int &n) {
        n = 0;
        r0 = 0;
        if (li >= my_chunks) return;
        const uint32_t ch = (xcd + 8 * (li / band)) * band + li % band;
        if (ch >= n_chunks) return;
        r0 = ch * (uint32_t)c.chunk;
        n = (int)min((int64_t)c.chunk, c.n_rays - (int64_t)r0);
    };
    // four chunks per set-up pass (the chunks themselves stay small, for balance)
    for (uint32_t li = slot; li < my_chunks; li += 4 * n_slots) {
        uint32_t ra, rb, rc, rd;
        int na, nb, nc, nd;
        chunk_rays(li, ra, na);
        chunk_rays(li + n_slots, rb, nb);
        chunk_rays(li + 2 * n_slots, rc, nc);
        chunk_rays(li + 3 * n_slots, rd, nd);
        const int nab = na + nb, nabc = nab + nc, ntot = nabc + nd;
        auto ray_at = [&](int i) -> int64_t {
            const uint32_t r = i < na ? ra + i : i < nab ? rb + (i - na) : i < nabc ? rc + (i - nab) : rd + (i - nabc);
            return c.ray0 + (int64_t)r;
        };
        for (int s0 = 0; s0 < ntot; s0 += RS_CAP) {
            const int n = min(RS_CAP, ntot - s0);
            // lanes 4 k .. 4 k + 3 set up ray s0 + k (lanes past the batch
            // repeat its last ray)
            const int k = l / RS_LANES, sub = l % RS_LANES;
            const int64_t rk = ray_at(s0 + (k < n ? k : n - 1));
            const float z1 = ray_first_zmin(c, rk, sub);
            const bool lead = sub == 0 && k < n;
            const uint64_t near = ballot(lead && z1 < __builtin_inff());  // bit RS_LANES k
            if (lead && !(z1 < __builtin_inff())) empty(rk);
            if (near == 0) continue;
            lds_sync();
            const RayGeom gk = ray_setup(c, rk, sub, z1);
            if (lead) rs[k] = gk;
            lds_sync();
            for (int i = 0; i < n; ++i)
                if ((near >> (RS_LANES * i)) & 1ull) body(ray_at(s0 + i), load_ray(rs[i]));
        }
    }
}

// Search one ray.  Returns, in `top` (one key per lane, ascending), the
// 64 smallest (t, index) keys of the ray's neighbours (missing = ~0), and
// the total neighbour count; with `lo`, only the keys >= lo count (the
// multi-surface sampler walks a ray's neighbours 64 at a time this way).
// BY_E2 orders the kept neighbours by (squared distance to the ray, index)
// instead of (t, index): the K nearest points to the ray (K-NP, Eq. 1).
template <bool BY_E2 = false>
__device__ __forceinline__ void search_neighbours(const SearchCtx &c, const RayGeom &g,
                                                  SearchLds &sh, uint64_t &top, int &count,
                                                  uint64_t lo = 0)
{
    const int l = lane_id();
    const ViewK &V = c.views[g.vi];
    const float z_lo = g.z_lo, z_hi = g.z_hi, dinf = g.dinf;
    const float frL2 = g.frL2, two_rw = g.two_rw, inv_L = g.inv_L, Dmax = g.Dmax;
    const int gx = g.gx, gy = g.gy, h = g.h;
    // (the square window also visits the corners beyond the proven radius)
    const bool square = c.window == HP_WINDOW_SQUARE;

    top = ~0ull;
    count = 0;
    if (h < 0) return;  // no point anywhere near this ray
    // the view's grid, read once (the loops below would reload it after
    // every store they cannot prove unrelated)
    ViewK Vg;
    Vg.Wg = V.Wg;
    Vg.Hg = V.Hg;
    Vg.bucket_base = V.bucket_base;
    const int Wg = Vg.Wg, Hg = Vg.Hg, cell_base = V.cell_base, ncx = V.ncx;

    uint64_t tau = ~0ull;
    bool have_top = false;
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
        // the first flush sorts straight into the (empty) top list; later ones
        // sort descending (ascending on inverted keys) and merge
        const uint64_t inv = have_top ? ~0ull : 0ull;
        x = wave_sort_fast(x ^ inv) ^ inv;
        if (have_top) top = wave_merge_low_fast(top, x);
        else top = x;
        have_top = true;
        tau = readlane_u64(top, WAVE - 1);
        lds_sync();
    };

    auto sweep_points = [&](int nb) {
        // points of the listed buckets, flattened; each lane finds its bucket
        // by a prefix maximum over the bucket heads that fall in its chunk
        lds_sync();
        const int c0 = (l < nb) ? sh.bl_cnt[l] : 0;
        const int i0 = wave_incl_scan_i32(c0);
        const int c1 = (WAVE + l < nb) ? sh.bl_cnt[WAVE + l] : 0;
        const int i1 = wave_incl_scan_i32(c1) + readlane_i32(i0, WAVE - 1);
        const int pre0 = i0 - c0, pre1 = i1 - c1;  // first flat index of buckets l, 64 + l
        const int totp = readlane_i32(i1, WAVE - 1);
        int carry = 0;
        for (int p0 = 0; p0 < totp; p0 += WAVE) {
            sh.bl_pre[l] = -1;
            lds_sync();
            if (l < nb && pre0 >= p0 && pre0 < p0 + WAVE) sh.bl_pre[pre0 - p0] = l;
            if (WAVE + l < nb && pre1 >= p0 && pre1 < p0 + WAVE) sh.bl_pre[pre1 - p0] = WAVE + l;
            lds_sync();
            int own = sh.bl_pre[l];
            if (l == 0 && own < 0) own = carry;
            own = wave_prefix_max_i32(own);
            carry = readlane_i32(own, WAVE - 1);
            const int p = p0 + l;
            const int pa = __shfl(pre0, own & (WAVE - 1), WAVE);
            const int pb = __shfl(pre1, own & (WAVE - 1), WAVE);
            bool pass = false;
            uint64_t key = 0;
            if (p < totp) {
                const int bpre = (own < WAVE) ? pa : pb;
                const int slot = sh.bl_start[own] + (p - bpre);
                float4 P = c.pts[slot];
                // one 16-byte load: otherwise the compiler loads (z, w) first
                // and (x, y) only for points that pass the depth test, two
                // dependent loads in place of one
                asm volatile("" : "+v"(P.x), "+v"(P.y), "+v"(P.z), "+v"(P.w));
                if (P.z <= sh.bl_zmax[own] && P.z >= z_lo) {
                    const float t = ray_param(P.x, P.y, P.z, g.dx, g.dy, g.dz);
                    const float e2 = dist2_at(P.x, P.y, P.z, g.dx, g.dy, g.dz, t);
                    const float rho = rho_at(c, g, t);
                    pass = (P.z > 0.0f) & (t >= c.t_near) & (t <= c.t_far) & (e2 <= rho * rho);
                    key = ((uint64_t)__float_as_uint(BY_E2 ? e2 : t) << 32) | __float_as_uint(P.w);
                }
            }
            const bool live = pass && key >= lo;
            count += popc64(ballot(live));
            const bool keep = live && key < tau;
            const uint64_t km = ballot(keep);
            if (keep) sh.pend[npend + rank_below(km)] = key;
            npend += popc64(km);
            if (npend >= WAVE) flush(WAVE);
            lds_sync();
        }
    };

    // one window bucket at offset (dxi, dyi) from the pixel's bucket: returns
    // whether it may hold a neighbour, and its slots
    auto zmax_at = [&](float D) -> float {
        // bounds only (margins of 1e-3 px and 0.1% dwarf 1-ulp approximations)
        const float Dp = D - 0.01f;
        if (Dp > 0.0f && Dp > dinf) {
            const float zc = ((frL2 * __builtin_amdgcn_rcpf(Dp) + two_rw) * inv_L) * 1.001f + 1e-5f;
            return zc < z_hi ? zc : z_hi;
        }
        return z_hi;
    };
    auto offset_D = [](int adx, int ady) -> float {
        const float ex = __builtin_fmaxf(0.0f, (float)adx - 0.5f);
        const float ey = __builtin_fmaxf(0.0f, (float)ady - 0.5f);
        return __builtin_amdgcn_sqrtf(ex * ex + ey * ey);
    };
    auto probe = [&](bool valid, int dxi, int dyi, int &st, int &cnt, float &zmax) -> bool {
        zmax = z_hi;
        st = cnt = 0;
        if (!valid) return false;
        const int bx = gx + dxi, by = gy + dyi;
        const float D = offset_D(dxi < 0 ? -dxi : dxi, dyi < 0 ? -dyi : dyi);
        if (!(bx >= 0 && bx < Wg && by >= 0 && by < Hg && (square || D <= Dmax))) return false;
        zmax = zmax_at(D);
        const int key = bucket_of(Vg, c.layout, bx, by);
        st = c.offsets[key];
        cnt = c.offsets[key + 1] - st;
        // the first depth is loaded with the offsets, not after them
        const float z0 = c.bucket_z[key];
        return cnt > 0 && z0 <= zmax;
    };
    auto append = [&](bool ok, int st, int cnt, float zmax) {
        const uint64_t m = ballot(ok);
        if (ok) {
            const int pos = nbl + rank_below(m);
            sh.bl_start[pos] = st;
            sh.bl_cnt[pos] = cnt;
            sh.bl_zmax[pos] = zmax;
        }
        nbl += popc64(m);
        if (nbl >= WAVE) {
            sweep_points(nbl);
            nbl = 0;
        }
    };
    // Larger windows: the buckets are culled by 8x8-bucket cells first: a cell whose
    // nearest window bucket is at distance D is skipped when its minimum
    // depth exceeds the depth bound at D (the bound only falls with D).
    // Surviving cells are listed (up to 64 at a time, in the LDS the walk
    // uses later) with the prefix of their window-bucket counts; each cell's
    // buckets then go to one chunk of lanes, four cells per step.
    // Small windows (most rays of object-scale scenes) skip the cell pass.
    const int Wd = 2 * h + 1;
    if (Wd * Wd <= 4 * WAVE) {
        // (q + 0.5) / Wd is at least 0.5 / Wd from an integer, far more than
        // the error of a float reciprocal, so the row index below is exact.
        const float inv_wd = 1.0f / (float)Wd;
        for (int q0 = 0; q0 < Wd * Wd; q0 += 2 * WAVE) {
            const int qa = q0 + l, qb = q0 + WAVE + l;
            const int ya = (int)(((float)qa + 0.5f) * inv_wd), yb = (int)(((float)qb + 0.5f) * inv_wd);
            int stA, cntA, stB, cntB;
            float zA, zB;
            const bool okA = probe(qa < Wd * Wd, qa - ya * Wd - h, ya - h, stA, cntA, zA);
            const bool okB = probe(qb < Wd * Wd, qb - yb * Wd - h, yb - h, stB, cntB, zB);
            append(okA, stA, cntA, zA);
            append(okB, stB, cntB, zB);
        }
        if (nbl > 0) sweep_points(nbl);
        if (npend > 0) flush(npend);
        return;
    }
    int4 *const cl = reinterpret_cast<int4 *>(sh.nb_p);  // (bx0, by0, width, prefix)
    const int wx0 = max(gx - h, 0), wx1 = min(gx + h, Wg - 1);
    const int wy0 = max(gy - h, 0), wy1 = min(gy + h, Hg - 1);
    const int cx0 = wx0 >> CELL_SHIFT, cy0 = wy0 >> CELL_SHIFT;
    const int ncw = (wx1 >> CELL_SHIFT) - cx0 + 1;
    const int ncell = ncw * ((wy1 >> CELL_SHIFT) - cy0 + 1);
    for (int c0 = 0; c0 < ncell; c0 += WAVE) {
        const int ci = c0 + l;
        bool keep = false;
        int bx0 = 0, by0 = 0, bw = 0, nbk = 0;
        if (ci < ncell) {
            const int cyy = cy0 + ci / ncw, cxx = cx0 + ci % ncw;
            bx0 = max(cxx << CELL_SHIFT, wx0);
            by0 = max(cyy << CELL_SHIFT, wy0);
            const int bx1 = min((cxx << CELL_SHIFT) + CELL - 1, wx1);
            const int by1 = min((cyy << CELL_SHIFT) + CELL - 1, wy1);
            bw = bx1 - bx0 + 1;
            nbk = bw * (by1 - by0 + 1);
            const int adx = gx < bx0 ? bx0 - gx : (gx > bx1 ? gx - bx1 : 0);
            const int ady = gy < by0 ? by0 - gy : (gy > by1 ? gy - by1 : 0);
            const float D = offset_D(adx, ady);
            const float cz = __uint_as_float(c.cell_zmin[cell_base + cyy * ncx + cxx]);
            keep = (square || D <= Dmax) && cz <= zmax_at(D);
        }
        const uint64_t km = ballot(keep);
        if (km == 0) continue;
        const int nk = keep ? nbk : 0;
        const int inc = wave_incl_scan_i32(nk);
        const int total = readlane_i32(inc, WAVE - 1);
        lds_sync();
        if (keep) cl[rank_below(km)] = make_int4(bx0, by0, bw, inc - nk);
        lds_sync();
        const int ncl = popc64(km);
        // one listed cell per chunk of lanes (a cell holds at most 64
        // buckets), four cells per step so that their loads overlap; the
        // order in which buckets are appended does not change the kept keys
        for (int k0 = 0; k0 < ncl; k0 += 4) {
            bool v[4], ok[4];
            int dx[4], dy[4], st[4], cnt[4];
            float zm[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v[u] = false;
                dx[u] = dy[u] = 0;
                if (k0 + u < ncl) {
                    const int4 e = cl[k0 + u];
                    const int nin = (k0 + u + 1 < ncl ? cl[k0 + u + 1].w : total) - e.w;
                    if (l < nin) {
                        const int ry = (int)(((float)l + 0.5f) * __builtin_amdgcn_rcpf((float)e.z));
                        dx[u] = e.x + (l - ry * e.z) - gx;
                        dy[u] = e.y + ry - gy;
                        v[u] = true;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) ok[u] = probe(v[u], dx[u], dy[u], st[u], cnt[u], zm[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) append(ok[u], st[u], cnt[u], zm[u]);
        }
    }
    if (nbl > 0) sweep_points(nbl);
    if (npend > 0) flush(npend);
}

// Merge two ascending KT-lists and keep the KT smallest, ascending: the
// element-wise minimum of a and reversed b is a bitonic sequence holding the
// KT smallest, which half-cleaners then sort.
template <int KT>
__device__ __forceinline__ void merge_low(uint64_t (&a)[KT], const uint64_t (&b)[KT])
{
#pragma unroll
    for (int k = 0; k < KT; ++k) a[k] = kmin(a[k], b[KT - 1 - k]);
#pragma unroll
    for (int j = KT / 2; j > 0; j >>= 1) {
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            if ((k & j) == 0) kswap(a[k], a[k + j]);
        }
    }
}

// Ascending sort of eight keys on the 19-comparator network for n = 8.
__device__ __forceinline__ void sort8(uint64_t (&x)[8])
{
    kswap(x[0], x[2]); kswap(x[1], x[3]); kswap(x[4], x[6]); kswap(x[5], x[7]);
    kswap(x[0], x[4]); kswap(x[1], x[5]); kswap(x[2], x[6]); kswap(x[3], x[7]);
    kswap(x[0], x[1]); kswap(x[2], x[3]); kswap(x[4], x[5]); kswap(x[6], x[7]);
    kswap(x[2], x[4]); kswap(x[3], x[5]);
    kswap(x[1], x[4]); kswap(x[3], x[6]);
    kswap(x[1], x[2]); kswap(x[3], x[4]); kswap(x[5], x[6]);
}

// Quad-split nearest neighbours of the ray point at tq among the sorted-list
// entries [lo, hi) within R2: lane q of each quad takes entries lo + q,
// lo + q + 4, ... into an ascending register list of (dist^2 bits << 32 |
// index); the quad then merges its four lists (DPP within the quad).
template <int KT>
__device__ __forceinline__ void knn_window(const RayGeom &g, const SearchLds &sh, float tq, float R2,
                                           int lo, int hi, uint64_t (&kd)[KT])
{
    const int q = lane_id() & 3;
#pragma unroll
    for (int k = 0; k < KT; ++k) kd[k] = KEY_NONE;
    int n_it = (hi - lo - q + 3) >> 2;
    n_it = n_it > 0 ? n_it : 0;
    n_it = max(n_it, (int)xor_lane_u32<4>((uint32_t)n_it));
    n_it = max(n_it, (int)xor_lane_u32<8>((uint32_t)n_it));
    n_it = max(n_it, (int)xor_lane_u32<16>((uint32_t)n_it));
    n_it = max(n_it, (int)xor_lane_u32<32>((uint32_t)n_it));
    // (n_it is now the maximum over the lanes with this lane's q; the
    // quad-gather path below reads the other lanes of the quad, so all lanes
    // must take it together: its test uses the maximum over the whole wave)
    int n_all = max(n_it, (int)xor_lane_u32<1>((uint32_t)n_it));
    n_all = max(n_all, (int)xor_lane_u32<2>((uint32_t)n_all));
    if constexpr (KT >= 8) {
        if (n_all <= 2) {
            // at most two entries per lane: the quad's union fits eight; sort
            // each lane's pair, gather the quad's four pairs on every lane and
            // merge the sorted runs 2 -> 4 -> 8
            uint64_t x[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int i = lo + q + 4 * e;
                x[e] = KEY_NONE;
                if (e < n_it && i < hi) {
                    const float4 P = sh.nb_p[i];
                    const float d2 = dist2_at(P.x, P.y, P.z, g.dx, g.dy, g.dz, tq);
                    if (d2 <= R2) x[e] = ((uint64_t)__float_as_uint(d2) << 32) | __float_as_uint(P.w);
                }
            }
            kswap(x[0], x[1]);
            uint64_t v[8];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                v[2 * p] = quad_bcast_u64(x[0], p);
                v[2 * p + 1] = quad_bcast_u64(x[1], p);
            }
            // (each merge reverses its second run, making the pair of runs
            // bitonic, then half-cleaners sort it)
#pragma unroll
            for (int r0 = 0; r0 < 8; r0 += 4) {
                uint64_t *w = v + r0;
                const uint64_t t = w[2];
                w[2] = w[3];
                w[3] = t;
                kswap(w[0], w[2]);
                kswap(w[1], w[3]);
                kswap(w[0], w[1]);
                kswap(w[2], w[3]);
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const uint64_t t = v[4 + k];
                v[4 + k] = v[7 - k];
                v[7 - k] = t;
            }
#pragma unroll
            for (int j = 4; j > 0; j >>= 1)
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if ((k & j) == 0) kswap(v[k], v[k + j]);
#pragma unroll
            for (int k = 0; k < KT; ++k) kd[k] = k < 8 ? v[k < 8 ? k : 0] : KEY_NONE;
            return;
        }
    }
    if constexpr (KT >= 16) {
        if (n_all <= 4) {
            // every lane holds at most four entries, so the quad's union fits
            // sixteen: sort each lane's four, gather the quad's sixteen keys
            // on every lane and merge the four sorted runs (no list merges)
            uint64_t x[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = lo + q + 4 * e;
                x[e] = KEY_NONE;
                if (e < n_it && i < hi) {
                    const float4 P = sh.nb_p[i];
                    const float d2 = dist2_at(P.x, P.y, P.z, g.dx, g.dy, g.dz, tq);
                    if (d2 <= R2) x[e] = ((uint64_t)__float_as_uint(d2) << 32) | __float_as_uint(P.w);
                }
            }
            kswap(x[0], x[1]);
            kswap(x[2], x[3]);
            kswap(x[0], x[2]);
            kswap(x[1], x[3]);
            kswap(x[1], x[2]);
            uint64_t v[16];
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int e = 0; e < 4; ++e) v[4 * p + e] = quad_bcast_u64(x[e], p);
            // runs of 4 -> 8 -> 16: the second run reversed makes a bitonic
            // sequence, which half-cleaners sort
#pragma unroll
            for (int r0 = 0; r0 < 16; r0 += 8) {
                uint64_t *w = v + r0;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const uint64_t t = w[4 + k];
                    w[4 + k] = w[7 - k];
                    w[7 - k] = t;
                }
#pragma unroll
                for (int j = 4; j > 0; j >>= 1)
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        if ((k & j) == 0) kswap(w[k], w[k + j]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint64_t t = v[8 + k];
                v[8 + k] = v[15 - k];
                v[15 - k] = t;
            }
#pragma unroll
            for (int j = 8; j > 0; j >>= 1)
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    if ((k & j) == 0) kswap(v[k], v[k + j]);
#pragma unroll
            for (int k = 0; k < KT; ++k) kd[k] = k < 16 ? v[k < 16 ? k : 0] : KEY_NONE;
            return;
        }
    }
    // longer windows: the first eight entries are sorted outright (19
    // compare-exchanges) and their smallest KT are the list (the test is
    // wave-uniform: n_all is the maximum over the wave)
    int it0 = 0;
    if (n_all > 4) {
        it0 = 8;
        uint64_t x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int i = lo + q + 4 * e;
            x[e] = KEY_NONE;
            if (e < n_it && i < hi) {
                const float4 P = sh.nb_p[i];
                const float d2 = dist2_at(P.x, P.y, P.z, g.dx, g.dy, g.dz, tq);
                if (d2 <= R2) x[e] = ((uint64_t)__float_as_uint(d2) << 32) | __float_as_uint(P.w);
            }
        }
        sort8(x);
#pragma unroll
        for (int k = 0; k < KT && k < 8; ++k) kd[k] = x[k];
    }
    // later entries four at a time: sort the four keys (five
    // compare-exchanges), then merge them into the list as the upper half of
    // a bitonic sequence
    for (int it = it0; it < n_it; it += 4) {
        uint64_t x[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = lo + q + 4 * (it + e);
            x[e] = KEY_NONE;
            if (i < hi) {
                const float4 P = sh.nb_p[i];
                const float d2 = dist2_at(P.x, P.y, P.z, g.dx, g.dy, g.dz, tq);
                if (d2 <= R2) x[e] = ((uint64_t)__float_as_uint(d2) << 32) | __float_as_uint(P.w);
            }
        }
        kswap(x[0], x[1]);
        kswap(x[2], x[3]);
        kswap(x[0], x[2]);
        kswap(x[1], x[3]);
        kswap(x[1], x[2]);
        static_assert(KT >= 4, "lists of at least four");
#pragma unroll
        for (int e = 0; e < 4; ++e) kd[KT - 4 + e] = kmin(kd[KT - 4 + e], x[3 - e]);
        // kd is now bitonic and holds the KT smallest: half-cleaners sort it
#pragma unroll
        for (int j = KT / 2; j > 0; j >>= 1) {
#pragma unroll
            for (int k = 0; k < KT; ++k)
                if ((k & j) == 0) kswap(kd[k], kd[k + j]);
        }
    }
    uint64_t other[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) other[k] = xor_lane_u64<1>(kd[k]);
    merge_low<KT>(kd, other);
#pragma unroll
    for (int k = 0; k < KT; ++k) other[k] = xor_lane_u64<2>(kd[k]);
    merge_low<KT>(kd, other);
}

// Nearest neighbours of 16 candidates at once.  Lane l = 4 g + q serves
// candidate c0 + g; its four lanes split the candidate's t-window of the
// sorted list (entries within R_j in t), each keeping an ascending register
// list, merged across the quad.  On return every lane of the quad holds the
// candidate's KT smallest keys (KEY_NONE = none).
template <int KT>
__device__ __forceinline__ void knn_quad(const SearchCtx &c, const RayGeom &g, const SearchLds &sh,
                                         int j, int m, uint64_t (&kd)[KT])
{
    const bool active = j < m;
    float tj = 0.0f, R2 = 0.0f;
    int lo = 0, hi = 0;
    if (active) {
        tj = sh.nb_t[j];
        const float Rj = rho_at(c, g, tj);
        R2 = Rj * Rj;
        // |t_i - t_j| > span implies dist^2 > R_j^2 (margins above rounding)
        const float span = Rj * 1.001f + tj * 4e-6f + 1e-7f;
        const float tlo = tj - span, thi = tj + span;
        int a = 0, b = j;  // first index with t >= tlo
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (sh.nb_t[mid] < tlo) a = mid + 1;
            else b = mid;
        }
        lo = a;
        a = j + 1;
        b = m;  // first index with t > thi
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (sh.nb_t[mid] <= thi) a = mid + 1;
            else b = mid;
        }
        hi = a;
    }
    knn_window<KT>(g, sh, tj, R2, lo, hi, kd);
}

// Distances of a quad's list entries split over its lanes: lane q takes the
// correctly rounded square roots of entries k = q, q + 4, ... (dq[e] for
// k = 4 e + q), so no lane computes more than KT / 4 of them.  Lane-local
// (every lane of a quad holds the same list).
template <int KT>
__device__ __forceinline__ uint64_t quad_entry(const uint64_t (&kd)[KT], int e)
{
    const int q = lane_id() & 3;
    uint64_t k0 = kd[4 * e], k1 = kd[4 * e + 1], k2 = kd[4 * e + 2], k3 = kd[4 * e + 3];
    // (an empty asm hides where the values came from: a select between
    // list elements would otherwise become a variable index into the list,
    // which then lives in scratch memory instead of registers)
    asm("" : "+v"(k0), "+v"(k1), "+v"(k2), "+v"(k3));
    return (q & 2) ? ((q & 1) ? k3 : k2) : ((q & 1) ? k1 : k0);
}

template <int KT>
__device__ __forceinline__ void quad_list_sqrt(const uint64_t (&kd)[KT], float (&dq)[KT / 4])
{
#pragma unroll
    for (int e = 0; e < KT / 4; ++e)
        dq[e] = __builtin_sqrtf(__uint_as_float((uint32_t)(quad_entry<KT>(kd, e) >> 32)));
}

// Candidate walk.  Candidates (the neighbours in (t, index) order) are
// processed 16 at a time, candidate c0 + g on lanes 4 g .. 4 g + 3.  After a
// chunk's transmittance walk, emit(s, q, tj, kd, kc) is called on the four
// lanes (q = 0..3) of every candidate that became sample s, with its K nearest
// neighbours kd (ascending (dist^2 bits, index), KEY_NONE = none), their number kc
// and the lane's share dq of their distances (quad_list_sqrt).  Returns the sample count and sets first_idx to the primary point.
template <int KT, typename Emit>
__device__ __forceinline__ int walk_candidates(const SearchCtx &c, const RayGeom &g, SearchLds &sh,
                                               uint64_t top, int m, int &first_idx, Emit emit)
{
    const int l = lane_id();
    lds_sync();
    if (l < m) {
        const int idxj = (int)(uint32_t)top;
        sh.nb_p[l] = c.pcam[(int64_t)g.vi * c.n_points + idxj];
        sh.nb_t[l] = __uint_as_float((uint32_t)(top >> 32));
    }
    lds_sync();
    float T = 1.0f;
    int sel = 0;
    first_idx = -1;
    bool done = false;
    for (int c0 = 0; c0 < m && !done; c0 += 16) {
        const int j = c0 + (l >> 2);
        uint64_t kd[KT];
        knn_quad<KT>(c, g, sh, j, m, kd);
        // each lane takes a quarter of the square roots; the quad then shares
        // them so that every lane sums all of them in list order
        float dq[KT / 4], dist[KT];
        quad_list_sqrt<KT>(kd, dq);
#pragma unroll
        for (int k = 0; k < KT; ++k)
            dist[k] = __uint_as_float(quad_bcast_u32(__float_as_uint(dq[k >> 2]), k & 3));
        // the list's valid entries (key != ~0) form a prefix; the first K count
        int kc = 0;
#pragma unroll
        for (int k = 0; k < KT; ++k) kc += kd[k] != KEY_NONE ? 1 : 0;
        kc = min(kc, c.K);
        float alpha = 0.0f, tj = 0.0f;
        if (j < m) {
            tj = sh.nb_t[j];
            const float Rj = rho_at(c, g, tj);
            float sum = 0.0f;  // (adding +0 past the prefix leaves it unchanged)
#pragma unroll
            for (int k = 0; k < KT; ++k) sum = sum + (k < kc ? dist[k] : 0.0f);
            const float dj = (sum + (float)(c.K - kc) * Rj) / (float)c.K;
            const float uj = (dj * dj) * c.inv_beta2;
            alpha = c.gamma * exp_neg(-uj);
        }
        // transmittance walk over this chunk (Eq. 5).  The transmittance in
        // front of each candidate is the running product of (1 - alpha) in
        // candidate order, one binary32 multiply after another as a sequential
        // walk takes them (candidates past the list have alpha = 0, a factor
        // of exactly 1); the value in front of each candidate reaches its quad
        // through the LDS.
        const int gl = l >> 2;
        const int ncand = min(c0 + 16, m) - c0;
        const int sel0 = sel;
        float *const tb = reinterpret_cast<float *>(sh.pend);  // (free during the walk)
#pragma unroll
        for (int gg = 0; gg < 16; ++gg) {
            const float aj = readlane_f32(alpha, 4 * gg);
            if (l == 0) tb[gg] = T;
            T = T * (1.0f - aj);
        }
        lds_sync();
        const float Tb = tb[gl];
        // the sequential walk's decisions, one candidate per quad leader:
        // selected when its weight passes eps_w while fewer than S samples
        // are taken; it stops after the S-th sample or once gamma T <= eps_w
        const float wq = alpha * Tb;
        const float Ta = Tb * (1.0f - alpha);
        const bool lead = (l & 3) == 0 && gl < ncand;
        const uint64_t pm = ballot(lead && wq > c.eps_w);         // bit 4 g
        const uint64_t dm = ballot(lead && c.gamma * Ta <= c.eps_w);
        int stop = dm ? __builtin_ctzll(dm) : WAVE;
        const int room = c.S - sel0;
        if (popc64(pm) >= room) {
            uint64_t x = pm;
            for (int k = 1; k < room; ++k) x &= x - 1ull;
            stop = min(stop, __builtin_ctzll(x));
        }
        if (stop < WAVE) done = true;
        const uint64_t smask = stop < WAVE ? pm & ((2ull << stop) - 1ull) : pm;
        sel += popc64(smask);
        if (smask) {
            if (sel0 == 0) {
                const int gsel = __builtin_ctzll(smask) >> 2;
                first_idx = __float_as_int(sh.nb_p[c0 + gsel].w);
            }
            // (the rank from the lane's own position: a per-lane mask would be
            // kept, and spilled, for the whole kernel)
            if ((smask >> (l & ~3)) & 1ull)
                emit(sel0 + rank_below(smask) - ((l & 3) ? 1 : 0), l & 3, tj, kd, dq, kc);
        }
    }
    return sel;
}

__device__ __forceinline__ int wave_min_i32(int v)
{
    v = min(v, (int)xor_lane_u32<1>((uint32_t)v));
    v = min(v, (int)xor_lane_u32<2>((uint32_t)v));
    v = min(v, (int)xor_lane_u32<4>((uint32_t)v));
    v = min(v, (int)xor_lane_u32<8>((uint32_t)v));
    v = min(v, (int)xor_lane_u32<16>((uint32_t)v));
    v = min(v, (int)xor_lane_u32<32>((uint32_t)v));
    return v;
}

// Uniform multi-surface sampling (the baseline of Sec. 3.5): positions
// t_k = t_near + (k + 1/2) step, k < ms_steps, each with a radius search: a
// position is a sample when some neighbour of the ray (any of them, not only
// the first m_cap) lies within R_k = rho(t_k) of it (the exact test), in
// depth order up to S, with its K nearest such neighbours.  The neighbours
// are walked in depth order 64 at a time: a slab is the 64 smallest keys at
// or above a bound (search_neighbours with `lo`), kept sorted in the LDS.
// Positions go 16 at a time, one per quad (lanes 4 g .. 4 g + 3), each
// keeping its K nearest over the slabs that reach its window |t - t_k| <= R_k
// (distance >= |t_i - t_k| up to rounding); a batch starts from the slab of
// keys at or above its first window and jumps over positions that no
// neighbour can reach.  emit() as for the candidate walk; first_idx is the
// nearest point of the first sample.  top, count: the ray's first slab and
// neighbour count, as search_neighbours returned them.
template <int KT, typename Emit>
__device__ __forceinline__ int uniform_samples(const SearchCtx &c, const RayGeom &g, SearchLds &sh,
                                               uint64_t top, int count, int &first_idx, Emit emit)
{
    const int l = lane_id();
    first_idx = -1;
    if (count == 0) return 0;
    const int nk = c.ms_steps;
    const float step = (c.t_far - c.t_near) / (float)nk;
    auto pos_t = [&](int k) { return fma_rn((float)k + 0.5f, step, c.t_near); };
    // |t_i - t_k| > span implies dist^2 > R_k^2 (margins above rounding)
    auto pos_span = [&](float tk) { return rho_at(c, g, tk) * 1.001f + tk * 4e-6f + 1e-7f; };
    // every window ends within smax of its position (rho grows with t)
    const float smax = pos_span(c.t_far);
    // a position before this one cannot reach a key at t (one spare)
    auto first_reaching = [&](float t) -> int {
        float f = (t - smax - c.t_near) / step - 0.5f;
        f = __builtin_fminf(__builtin_fmaxf(f, -2.0f), (float)nk + 2.0f);
        return max((int)__builtin_floorf(f) - 1, 0);
    };
    uint64_t keys = top;  // the current slab, one key per lane
    int n = count < WAVE ? count : WAVE, rest = count;
    auto load_slab = [&]() {
        lds_sync();
        if (l < n) {
            const int idxj = (int)(uint32_t)keys;
            sh.nb_p[l] = c.pcam[(int64_t)g.vi * c.n_points + idxj];
            sh.nb_t[l] = __uint_as_float((uint32_t)(keys >> 32));
        }
        lds_sync();
    };
    // first slab entry with t >= tlo (n if none)
    auto slab_lower = [&](float tlo) {
        int a = 0, e = n;
        while (a < e) {
            const int mid = (a + e) >> 1;
            if (sh.nb_t[mid] < tlo) a = mid + 1;
            else e = mid;
        }
        return a;
    };
    load_slab();
    int sel = 0;
    const int gp = l >> 2;
    int b = first_reaching(sh.nb_t[0]);
    while (b < nk && sel < c.S) {
        const int k = b + gp;
        const bool active = k < nk;
        float tk = 0.0f, R2 = 0.0f, span = 0.0f;
        if (active) {
            tk = pos_t(k);
            const float Rk = rho_at(c, g, tk);
            R2 = Rk * Rk;
            span = pos_span(tk);
        }
        const float tl = pos_t(min(b + 15, nk - 1));
        const float t_end = tl + pos_span(tl);  // where the batch's last window ends
        uint64_t kd[KT];
#pragma unroll
        for (int q = 0; q < KT; ++q) kd[q] = KEY_NONE;
        for (;;) {
            int wlo = 0, whi = 0;
            if (active) {
                wlo = slab_lower(tk - span);
                whi = wlo;
                int e = n;  // first entry with t > tk + span
                while (whi < e) {
                    const int mid = (whi + e) >> 1;
                    if (sh.nb_t[mid] <= tk + span) whi = mid + 1;
                    else e = mid;
                }
            }
            uint64_t part[KT];
            knn_window<KT>(g, sh, tk, R2, wlo, whi, part);
            merge_low<KT>(kd, part);
            // the next slab, unless this one held every remaining key or
            // ends beyond the last window of the batch
            if (rest <= n || sh.nb_t[n - 1] > t_end) break;
            const uint64_t last = readlane_u64(keys, n - 1);
            search_neighbours(c, g, sh, keys, rest, last + 1ull);
            n = rest < WAVE ? rest : WAVE;
            load_slab();
        }
        const bool kept = active && kd[0] != KEY_NONE;
        const uint64_t km = ballot(kept && (l & 3) == 0);  // bit 4 p: position b + p kept
        const int room = c.S - sel;
        const int rank = popc64(km & ((1ull << (4 * gp)) - 1ull));
        if (km) {
            if (sel == 0) first_idx = readlane_i32((int)(uint32_t)kd[0], __builtin_ctzll(km));
            if (kept && rank < room) {
                int kc = 0;
#pragma unroll
                for (int q = 0; q < KT; ++q) kc += (q < c.K && kd[q] != KEY_NONE) ? 1 : 0;
                float dq[KT / 4];
                quad_list_sqrt<KT>(kd, dq);
                emit(sel + rank, l & 3, tk, kd, dq, kc);
            }
            const int nkept = popc64(km);
            sel += nkept < room ? nkept : room;
        }
        // the next batch starts from the keys at or above its first window
        b += 16;
        if (b >= nk || sel >= c.S) break;
        const float tb = pos_t(b);
        const float tlo = tb - pos_span(tb);
        if (!(sh.nb_t[0] <= tlo && rest <= n)) {
            // (the current slab does not hold every key from tlo on)
            const uint64_t lo_key = tlo > 0.0f ? ((uint64_t)__float_as_uint(tlo) << 32) : 0ull;
            search_neighbours(c, g, sh, keys, rest, lo_key);
            if (rest == 0) break;
            n = rest < WAVE ? rest : WAVE;
            load_slab();
        }
        const int j = slab_lower(tlo);
        if (j >= n) break;  // no key at or beyond the next window
        b = max(b, first_reaching(sh.nb_t[j]));
    }
    return sel;
}

}  // namespace hp
