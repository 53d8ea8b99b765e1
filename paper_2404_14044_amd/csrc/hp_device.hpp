// Device-side building blocks shared by the HashPoint kernels (gfx950, wave64).
//
// Everything that decides a discrete result (which bucket a point falls in,
// whether a point is a neighbour of a ray, which neighbours are nearest, which
// candidates become samples) is written as one fixed sequence of correctly
// rounded binary32 operations, with fused multiply-adds only where __fmaf_rn
// is spelled out.  The library is compiled with -ffp-contract=off so the
// compiler adds none, and with correctly rounded division and square root.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hashpoint.h"

namespace hp {

constexpr int WAVE = 64;

// Per-view constants, stored once per table in device memory.
struct ViewK {
    float fx, fy, cx, cy;
    float R[9];
    float C[3];
    int32_t W, H, g, Wg, Hg;
    int32_t bucket_base, ray_base;
    float dmax;        // window radius in pixels, with margin
    int32_t slot_base; // first slot of the view (written on the device)
    int32_t cell_base; // first depth cell of the view
    int32_t ncx;       // depth cells per grid row (cells are CELL x CELL buckets)
    int32_t pad;
};

// Depth cells: blocks of CELL x CELL buckets whose minimum camera depth the
// table keeps, so a ray can bound the depth of anything near it cheaply.
constexpr int CELL_SHIFT = 3;
constexpr int CELL = 1 << CELL_SHIFT;

struct ViewSet {
    int32_t n;
    int32_t layout;
    ViewK v[HP_MAX_VIEWS];
};

__device__ __forceinline__ float fma_rn(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Camera-space position p_c = R (p - C).
__device__ __forceinline__ void to_camera(const ViewK &V, float px, float py, float pz, float &x,
                                          float &y, float &z)
{
    const float qx = px - V.C[0], qy = py - V.C[1], qz = pz - V.C[2];
    x = fma_rn(V.R[2], qz, fma_rn(V.R[1], qy, V.R[0] * qx));
    y = fma_rn(V.R[5], qz, fma_rn(V.R[4], qy, V.R[3] * qx));
    z = fma_rn(V.R[8], qz, fma_rn(V.R[7], qy, V.R[6] * qx));
}

// Bucket of grid cell (bx, by) of a view.  Row-major, or 8x8 tiles stored
// row-major with the cells inside each tile row-major (TILED) or in Z-order
// (MORTON: the bits of x and y interleaved, x in the even bits).
__device__ __forceinline__ int32_t bucket_of(const ViewK &V, int layout, int bx, int by)
{
    if (layout != HP_LAYOUT_ROWMAJOR) {
        const int ntx = V.Wg >> 3;
        const int tile = V.bucket_base + ((((by >> 3) * ntx) + (bx >> 3)) << 6);
        const int x = bx & 7, y = by & 7;
        if (layout == HP_LAYOUT_TILED) return tile + (y << 3) + x;
        return tile + ((x & 1) | ((y & 1) << 1) | ((x & 2) << 1) | ((y & 2) << 2) | ((x & 4) << 2) |
                       ((y & 4) << 3));
    }
    return V.bucket_base + by * V.Wg + bx;
}

// Unit ray through the centre of pixel (u, v), camera coordinates; also the
// normalised image coordinates (a, b) and L = sqrt(1 + a^2 + b^2).
__device__ __forceinline__ void ray_dir(const ViewK &V, int u, int v, float &dx, float &dy,
                                        float &dz, float &a, float &b, float &L)
{
    a = (((float)u + 0.5f) - V.cx) / V.fx;
    b = (((float)v + 0.5f) - V.cy) / V.fy;
    L = __builtin_sqrtf(fma_rn(b, b, fma_rn(a, a, 1.0f)));
    dx = a / L;
    dy = b / L;
    dz = 1.0f / L;
}

// rho(t) = radius * max(1, t * inv_tref)
__device__ __forceinline__ float search_radius(float radius, float inv_tref, float t)
{
    const float s = t * inv_tref;
    return radius * (s > 1.0f ? s : 1.0f);
}

// Ray parameter of camera-space point x on unit ray d.
__device__ __forceinline__ float ray_param(float x, float y, float z, float dx, float dy, float dz)
{
    return fma_rn(z, dz, fma_rn(y, dy, x * dx));
}

// Squared distance between point x and the ray point s * d.
__device__ __forceinline__ float dist2_at(float x, float y, float z, float dx, float dy, float dz,
                                          float s)
{
    const float ex = fma_rn(-s, dx, x);
    const float ey = fma_rn(-s, dy, y);
    const float ez = fma_rn(-s, dz, z);
    return fma_rn(ez, ez, fma_rn(ey, ey, ex * ex));
}

// exp(x) for x <= 0 in binary32, bit-reproducible: x = k ln2 + r with
// ln2 split in a 16-bit head (k * head exact) and a tail, |r| <= ln2 / 2,
// exp(r) by its Taylor polynomial of degree 7 in Horner form (truncation
// below 1e-8 relative), then scaled by 2^k built from exponent bits.  Each
// constant is the binary64 value rounded once to binary32.  Returns 0 below
// -86 and for NaN.  Never exceeds 1.
__device__ __forceinline__ float exp_neg(float x)
{
    if (!(x >= -86.0f)) return 0.0f;
    constexpr float kInvLn2 = (float)(1.0 / 0.69314718055994530942);
    constexpr float kLn2Head = 0.693145751953125f;
    constexpr float kLn2Tail = (float)(0.69314718055994530942 - 0.693145751953125);
    const float k = __builtin_rintf(x * kInvLn2);
    float r = fma_rn(-k, kLn2Head, x);
    r = fma_rn(-k, kLn2Tail, r);
    float q = (float)(1.0 / 5040.0);
    q = fma_rn(q, r, (float)(1.0 / 720.0));
    q = fma_rn(q, r, (float)(1.0 / 120.0));
    q = fma_rn(q, r, (float)(1.0 / 24.0));
    q = fma_rn(q, r, (float)(1.0 / 6.0));
    q = fma_rn(q, r, 0.5f);
    q = fma_rn(q, r, 1.0f);
    q = fma_rn(q, r, 1.0f);
    const int ki = (int)k;
    return q * __uint_as_float((uint32_t)(ki + 127) << 23);
}

// Neighbours k0 .. k0 + 3 of a list of K: indices (-1 past the end) and
// distances (1 past the end).  With `vec` (K a multiple of 4, both arrays
// 16-byte aligned) each array takes one 16-byte load instead of four.
__device__ __forceinline__ bool nbr_vec_ok(const int32_t *ki, const float *kd, int K)
{
    return (K & 3) == 0 && ((((uintptr_t)ki) | ((uintptr_t)kd)) & 15) == 0;
}

__device__ __forceinline__ void load_nbr4(const int32_t *ki, const float *kd, int k0, int K, bool vec,
                                          int *idx, float *d)
{
    if (vec) {
        const int4 iv = *reinterpret_cast<const int4 *>(ki + k0);
        const float4 dv = *reinterpret_cast<const float4 *>(kd + k0);
        idx[0] = iv.x, idx[1] = iv.y, idx[2] = iv.z, idx[3] = iv.w;
        d[0] = dv.x, d[1] = dv.y, d[2] = dv.z, d[3] = dv.w;
        return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool in = k0 + j < K;
        idx[j] = in ? ki[k0 + j] : -1;
        d[j] = in ? kd[k0 + j] : 1.0f;
    }
}

// ---------------------------------------------------------------------------
// wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Orders this wave's LDS accesses.  A wave's LDS operations complete in
// program order, so a compiler barrier is enough for its lanes to see each
// other's writes; no workgroup barrier, as several independent waves may
// share a workgroup.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a < b ? b : a; }

// (a, b) <- (min, max) of the pair, on one compare: the empty asm keeps the
// compiler from seeing a minimum and a maximum, each with its own compare
__device__ __forceinline__ void cswap64(uint64_t &a, uint64_t &b)
{
    const bool s = b < a;
    asm("" : "+v"(a), "+v"(b));
    const uint64_t lo = s ? b : a;
    b = s ? a : b;
    a = lo;
}

// Keys (bits of a non-negative binary32 << 32 | index) read as binary64 are
// non-negative finite numbers, subnormal ones included, whose numeric order is
// the order of their bit patterns, so lane-local sorting networks order them
// with the binary64 minimum and maximum: one instruction each, where integer
// 64-bit keys take a compare and four selects.  (Subnormal binary64 values
// are kept by the kernels' floating-point mode; the keys are never NaN.)
// KEY_NONE, the largest finite binary64, marks an empty slot: a NaN would be
// dropped by the minimum and maximum.
constexpr uint64_t KEY_NONE = 0x7FEFFFFFFFFFFFFFull;

__device__ __forceinline__ double key_f64(uint64_t k) { return __longlong_as_double((long long)k); }
__device__ __forceinline__ uint64_t f64_key(double d) { return (uint64_t)__double_as_longlong(d); }

__device__ __forceinline__ uint64_t kmin(uint64_t a, uint64_t b)
{
    return f64_key(__builtin_fmin(key_f64(a), key_f64(b)));
}

// (a, b) <- (min, max) of two keys
__device__ __forceinline__ void kswap(uint64_t &a, uint64_t &b)
{
    const double x = key_f64(a), y = key_f64(b);
    a = f64_key(__builtin_fmin(x, y));
    b = f64_key(__builtin_fmax(x, y));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// number of set bits of m below this lane
__device__ __forceinline__ int rank_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ __forceinline__ int wave_incl_scan_i32(int v)
{
    // inside rows of 16 (lanes shifted in from outside the row add 0), then
    // the last lane of row 0 into rows 1, 3 and of row 1 into rows 2, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

__device__ __forceinline__ float readlane_f32(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ int readlane_i32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

}  // namespace hp
