// Pixel-table construction (Sec. 3.2, Fig. 2): project every point into every
// view, count points per bucket with atomics (the counter's old value is the
// point's rank in its bucket), scan the counts into bucket offsets, place each
// point at offset + rank, and order each bucket by depth.
//
// Passes (each a coalesced sweep except the scatter and the bucket sorts):
//   k_project      (view, point)  -> (bucket, z), the camera-space point (pcam),
//                  a per-bucket count and the point's arrival rank in its
//                  bucket (kept in perm until k_materialize overwrites it)
//   k_scan_*       counts         -> exclusive offsets, three passes
//   k_scatter      (view, point)  -> 64-bit key (z bits, point index) per slot
//   k_sort_small   one lane per bucket of at most 16 points, register network
//   k_sort_listed  one wave per bucket of 17..128 points, register bitonic;
//                  one workgroup per larger bucket, bitonic in LDS or global
//   k_materialize  one lane per slot: camera-space point and index (from pcam)
#include "hp_device.hpp"
#include "hp_kernels.hpp"
#include "hp_search.hpp"
#include "hp_table_ws.hpp"

namespace hp {

__global__ void k_fill_i32(int32_t *p, int32_t val, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

// The build's first launch: the views' constants to device memory (first
// workgroup), n counters cleared and nz depth-cell minima set to +inf (all
// of them).
__global__ void k_build_begin(ViewSet vs, ViewK *out, int32_t *p, int64_t n, uint32_t *z,
                              int64_t nz)
{
    if (blockIdx.x == 0 && threadIdx.x < vs.n) out[threadIdx.x] = vs.v[threadIdx.x];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nz;
         i += (int64_t)gridDim.x * blockDim.x)
        z[i] = 0x7f800000u;
}

// grid: (ceil(n / (256 PROJ_PER)), n_views).  Each thread takes PROJ_PER
// points strided by the workgroup size, so that its count atomics (whose
// returned rank the point needs) are in flight together: one at a time, the
// wave would wait out the device-scope round trip of each.
constexpr int PROJ_PER = 4;

__global__ void __launch_bounds__(256) k_project(const float *__restrict__ xyz, int64_t n,
                                                 const ViewK *__restrict__ views, int layout,
                                                 int2 *__restrict__ kz, float4 *__restrict__ pcam,
                                                 int32_t *__restrict__ count,
                                                 int32_t *__restrict__ rank)
{
    const int vi = blockIdx.y;
    const ViewK &V = views[vi];
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x * PROJ_PER + threadIdx.x;
    int32_t key[PROJ_PER];
    float zz[PROJ_PER];
#pragma unroll
    for (int j = 0; j < PROJ_PER; ++j) {
        const int64_t i = i0 + (int64_t)j * blockDim.x;
        key[j] = -1;
        zz[j] = 0.0f;
        if (i >= n) continue;
        float x, y, z;
        to_camera(V, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], x, y, z);
        pcam[(int64_t)vi * n + i] = make_float4(x, y, z, __int_as_float((int)i));
        zz[j] = z;
        if (z > 0.0f && __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z)) {
            const float uf = fma_rn(V.fx, x / z, V.cx);
            const float vf = fma_rn(V.fy, y / z, V.cy);
            const float lo = (float)(-V.g);
            if (uf >= lo && uf < (float)(V.W + V.g) && vf >= lo && vf < (float)(V.H + V.g)) {
                const int bx = (int)__builtin_floorf(uf) + V.g;
                const int by = (int)__builtin_floorf(vf) + V.g;
                key[j] = bucket_of(V, layout, bx, by);
            }
        }
    }
    int32_t r[PROJ_PER];
#pragma unroll
    for (int j = 0; j < PROJ_PER; ++j)
        r[j] = key[j] >= 0 ? atomicAdd(&count[key[j]], 1) : 0;  // arrival rank inside the bucket
#pragma unroll
    for (int j = 0; j < PROJ_PER; ++j) {
        const int64_t i = i0 + (int64_t)j * blockDim.x;
        if (i >= n) continue;
        kz[(int64_t)vi * n + i] = make_int2(key[j], __float_as_int(zz[j]));
        rank[(int64_t)vi * n + i] = r[j];
    }
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts -> offsets[n + 1]
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256;
constexpr int SCAN_PER = 16;
constexpr int SCAN_TILE = SCAN_T * SCAN_PER;

__device__ __forceinline__ int block_excl_scan(int v, int *sh_warp, int &total)
{
    const int l = lane_id();
    const int w = threadIdx.x / WAVE;
    const int inc = wave_incl_scan_i32(v);
    if (l == WAVE - 1) sh_warp[w] = inc;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_T / WAVE; ++k) {
        const int s = sh_warp[k];
        base += (k < w) ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_reduce(const int32_t *__restrict__ in, int64_t n,
                                                        int32_t *__restrict__ block_sums)
{
    __shared__ int sh[SCAN_T / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) s += (base + k < n) ? in[base + k] : 0;
    int total;
    block_excl_scan(s, sh, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// single workgroup: exclusive scan of the block sums in place
__global__ void __launch_bounds__(SCAN_T) k_scan_blocks(int32_t *__restrict__ sums, int64_t nb)
{
    __shared__ int sh[SCAN_T / WAVE];
    int carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_T) {
        const int64_t i = b0 + threadIdx.x;
        const int v = (i < nb) ? sums[i] : 0;
        int total;
        const int ex = block_excl_scan(v, sh, total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
}

__global__ void __launch_bounds__(SCAN_T) k_scan_apply(const int32_t *__restrict__ in, int64_t n,
                                                       const int32_t *__restrict__ block_base,
                                                       int32_t *__restrict__ out)
{
    __shared__ int sh[SCAN_T / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
    int v[SCAN_PER];
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int run = block_excl_scan(s, sh, total) + block_base[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = block_base[blockIdx.x] + total;
}

// ---------------------------------------------------------------------------
// scatter: one 64-bit key per slot, (z bits) << 32 | point index.  z > 0, so
// the bits of z order like z, and the key orders by (z, index).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_scatter(const int2 *__restrict__ kz,
                                                 const int32_t *__restrict__ rank, int64_t total,
                                                 int64_t n, const int32_t *__restrict__ offsets,
                                                 uint64_t *__restrict__ skey)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int2 e = kz[i];
    if (e.x < 0) return;
    const int64_t p = i % n;
    skey[offsets[e.x] + rank[i]] = ((uint64_t)(uint32_t)e.y << 32) | (uint32_t)p;
}

// ---------------------------------------------------------------------------
// per-bucket sort of the keys
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void sort_net(uint64_t (&k)[N])
{
    // bitonic network with all comparators ascending in the merge phase
#pragma unroll
    for (int s = 2; s <= N; s <<= 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int p = i ^ (s - 1);
            if (p > i) {
                const uint64_t a = k[i], b = k[p];
                k[i] = umin64(a, b);
                k[p] = umax64(a, b);
            }
        }
#pragma unroll
        for (int j = s >> 2; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int p = i ^ j;
                if (p > i) {
                    const uint64_t a = k[i], b = k[p];
                    k[i] = umin64(a, b);
                    k[p] = umax64(a, b);
                }
            }
        }
    }
}

template <int N>
__device__ __forceinline__ uint64_t sort_bucket_regs(uint64_t *__restrict__ skey, int start, int cnt)
{
    uint64_t k[N];
#pragma unroll
    for (int i = 0; i < N; ++i) k[i] = (i < cnt) ? skey[start + i] : ~0ull;
    sort_net<N>(k);
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i < cnt) skey[start + i] = k[i];
    return k[0];
}

constexpr int SMALL_MAX = 16;

// Buckets of more than SMALL_MAX points are listed for the wave and
// workgroup sorts: those of up to 128 points from the front of big_list
// (count big_n[0], sort_mid), larger ones from its back (count big_n[1],
// sort_big), so that neither role walks the other's entries.
__device__ __forceinline__ void list_big_bucket(int32_t *__restrict__ big_list,
                                                int32_t *__restrict__ big_n, int64_t cap, int b,
                                                int cnt)
{
    if (cnt <= 2 * WAVE) big_list[atomicAdd(&big_n[0], 1)] = b;
    else big_list[cap - 1 - atomicAdd(&big_n[1], 1)] = b;
}

__global__ void __launch_bounds__(256) k_sort_small(const int32_t *__restrict__ offsets, int64_t nb,
                                                    uint64_t *__restrict__ skey,
                                                    int32_t *__restrict__ big_list,
                                                    int32_t *__restrict__ big_n,
                                                    float *__restrict__ bucket_z)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int start = offsets[b];
    const int cnt = offsets[b + 1] - start;
    uint64_t first = ~0ull;
    if (cnt == 1) first = skey[start];
    else if (cnt > 1 && cnt <= 4) first = sort_bucket_regs<4>(skey, start, cnt);
    else if (cnt > 4 && cnt <= 8) first = sort_bucket_regs<8>(skey, start, cnt);
    else if (cnt > 8 && cnt <= SMALL_MAX) first = sort_bucket_regs<16>(skey, start, cnt);
    else if (cnt > SMALL_MAX) {
        list_big_bucket(big_list, big_n, nb, (int32_t)b, cnt);
        return;  // k_sort_listed writes bucket_z
    }
    bucket_z[b] = cnt > 0 ? __uint_as_float((uint32_t)(first >> 32)) : __builtin_inff();
}

// Where sorted slots also become table points: pts[slot] = the camera-space
// point of its index (pcam of the bucket's view) and perm[slot] = the index.
// pts == nullptr: the slots are materialised afterwards (k_materialize).
struct SlotOut {
    const float4 *pcam;
    int64_t n;
    const ViewK *views;
    int n_views;
    float4 *pts;
    int32_t *perm;
};

__device__ __forceinline__ const float4 *bucket_pcam(const SlotOut &o, int b)
{
    int vi = 0;
    while (vi + 1 < o.n_views && o.views[vi + 1].bucket_base <= b) ++vi;
    return o.pcam + (int64_t)vi * o.n;
}

__device__ __forceinline__ void put_slot(const SlotOut &o, const float4 *pc, int slot, uint64_t key)
{
    const int32_t idx = (int32_t)(uint32_t)key;
    o.pts[slot] = pc[idx];
    o.perm[slot] = idx;
}

template <int N>
__device__ __forceinline__ uint64_t sort_bucket_to_slots(const uint64_t *__restrict__ skey, int start,
                                                         int cnt, const SlotOut &so,
                                                         const float4 *pc)
{
    uint64_t k[N];
#pragma unroll
    for (int i = 0; i < N; ++i) k[i] = (i < cnt) ? skey[start + i] : ~0ull;
    sort_net<N>(k);
    // the points gathered before they are stored: the stores may alias the
    // gathered rows as far as the compiler knows, so put one by one each
    // load would wait for the previous store
    // (slots past the bucket's end gather its first point, unused; a plain
    // vector type, which the compiler keeps in registers, where an array of
    // float4 went to scratch memory)
    typedef float fx4 __attribute__((ext_vector_type(4)));
    const fx4 *src = reinterpret_cast<const fx4 *>(pc);
    fx4 *dst = reinterpret_cast<fx4 *>(so.pts);
    // (eight at a time, four beside the sixteen keys of the largest case:
    // at most 32 registers, so that three 512-thread workgroups share a CU
    // and one round of them covers the object view's superbuckets)
    constexpr int G = N < 8 ? N : (N == 16 ? 4 : 8);
#pragma unroll
    for (int i0 = 0; i0 < N; i0 += G) {
        fx4 v[G];
#pragma unroll
        for (int j = 0; j < G; ++j) v[j] = src[(int32_t)(uint32_t)(i0 + j < cnt ? k[i0 + j] : k[0])];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (i0 + j < cnt) {
                dst[start + i0 + j] = v[j];
                so.perm[start + i0 + j] = (int32_t)(uint32_t)k[i0 + j];
            }
        }
    }
    return k[0];
}

// ---------------------------------------------------------------------------
// Two-level build (views of up to SB_MAX superbuckets each).  Per-point atomics
// on the bucket counters cost the build most of its time: device-scope
// atomics whose returned value the point needs (its rank in the bucket)
// stall at the memory side, one per point.  Here buckets are grouped into
// superbuckets of SB consecutive keys; a workgroup counts its points per
// superbucket in LDS and makes one global atomic per superbucket it touches,
// which places its points' records contiguously by superbucket; then one
// workgroup per superbucket counts, scans, places and sorts the buckets of
// its SB keys with LDS atomics only.
// ---------------------------------------------------------------------------
constexpr int SB = 1 << SB_SHIFT;  // buckets per superbucket
constexpr int SB_PER = 8;          // points per thread of the projection passes
constexpr int SB_T = 256;

// superbuckets spanned by view V's buckets
__device__ __forceinline__ void view_superbuckets(const ViewK &V, int &lo, int &cnt)
{
    lo = V.bucket_base >> SB_SHIFT;
    cnt = ((V.bucket_base + V.Wg * V.Hg - 1) >> SB_SHIFT) - lo + 1;
}

// grid: (ceil(n / (SB_T SB_PER)), n_views).  Projection, bucket key and
// depth of each point; per-superbucket totals.
__global__ void __launch_bounds__(SB_T) k_project_sb(const float *__restrict__ xyz, int64_t n,
                                                     const ViewK *__restrict__ views, int layout,
                                                     int2 *__restrict__ kz,
                                                     float4 *__restrict__ pcam,
                                                     int32_t *__restrict__ sb_count)
{
    __shared__ int hist[SB_MAX];
    const int vi = blockIdx.y;
    const ViewK &V = views[vi];
    int sb_lo, nsb;
    view_superbuckets(V, sb_lo, nsb);
    for (int j = threadIdx.x; j < nsb; j += SB_T) hist[j] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * SB_T * SB_PER + threadIdx.x;
    // all of the thread's points loaded first, so that the loads are in
    // flight together (in one loop with the stores and the exit test below
    // they went one at a time)
    float px[SB_PER], py[SB_PER], pz[SB_PER];
#pragma unroll
    for (int j = 0; j < SB_PER; ++j) {
        const int64_t i = i0 + (int64_t)j * SB_T;
        px[j] = py[j] = pz[j] = 0.0f;
        if (i < n) {
            px[j] = xyz[3 * i];
            py[j] = xyz[3 * i + 1];
            pz[j] = xyz[3 * i + 2];
        }
    }
#pragma unroll
    for (int j = 0; j < SB_PER; ++j) {
        const int64_t i = i0 + (int64_t)j * SB_T;
        if (i >= n) break;
        float x, y, z;
        to_camera(V, px[j], py[j], pz[j], x, y, z);
        pcam[(int64_t)vi * n + i] = make_float4(x, y, z, __int_as_float((int)i));
        int32_t key = -1;
        if (z > 0.0f && __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z)) {
            const float uf = fma_rn(V.fx, x / z, V.cx);
            const float vf = fma_rn(V.fy, y / z, V.cy);
            const float lo = (float)(-V.g);
            if (uf >= lo && uf < (float)(V.W + V.g) && vf >= lo && vf < (float)(V.H + V.g)) {
                const int bx = (int)__builtin_floorf(uf) + V.g;
                const int by = (int)__builtin_floorf(vf) + V.g;
                key = bucket_of(V, layout, bx, by);
                atomicAdd(&hist[(key >> SB_SHIFT) - sb_lo], 1);
            }
        }
        kz[(int64_t)vi * n + i] = make_int2(key, __float_as_int(z));
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nsb; j += SB_T)
        if (hist[j]) atomicAdd(&sb_count[sb_lo + j], hist[j]);
}

// one workgroup: exclusive scan of the superbucket totals -> sb_off[0 .. nsb],
// and the table's last offset (points inserted)
__global__ void __launch_bounds__(1024) k_sb_scan(const int32_t *__restrict__ sb_count, int nsb,
                                                  int32_t *__restrict__ sb_off,
                                                  int32_t *__restrict__ offsets_end)
{
    __shared__ int sh[1024 / WAVE];
    const int l = lane_id(), w = threadIdx.x / WAVE;
    int carry = 0;
    for (int b0 = 0; b0 < nsb; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const int v = i < nsb ? sb_count[i] : 0;
        const int inc = wave_incl_scan_i32(v);
        if (l == WAVE - 1) sh[w] = inc;
        __syncthreads();
        int base = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < 1024 / WAVE; ++k) {
            base += k < w ? sh[k] : 0;
            tot += sh[k];
        }
        if (i < nsb) sb_off[i] = carry + base + inc - v;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sb_off[nsb] = carry;
        *offsets_end = carry;
    }
}

// Tables of at most SCAN_SB superbuckets in all skip the scan's launch: every
// workgroup of the scatter scans the totals itself (SCAN_SB / SB_T per
// thread) into LDS, and the first one also writes them out for the
// superbucket workgroups.
constexpr int SCAN_SB = 1024;

// grid as k_project_sb.  Each point's record (key, z bits, index) goes to its
// superbucket's range: rank among the workgroup's points of the superbucket
// (LDS atomic) plus the workgroup's share of the range (one global atomic per
// superbucket touched).  The order inside a superbucket does not matter: its
// buckets are sorted by (z, index) next.  With SCAN, the superbucket offsets
// are scanned here from the nsb_all totals (nsb_all <= SCAN_SB) instead of
// read from sb_off, which workgroup (0, 0) fills, with the table's last
// offset.
template <bool SCAN>
__global__ void __launch_bounds__(SB_T) k_scatter_sb(const int2 *__restrict__ kz, int64_t n,
                                                     const ViewK *__restrict__ views,
                                                     int32_t *__restrict__ sb_off,
                                                     int32_t *__restrict__ sb_cursor,
                                                     int4 *__restrict__ rec,
                                                     const int32_t *__restrict__ sb_count,
                                                     int nsb_all, int32_t *__restrict__ offsets_end)
{
    __shared__ int hist[SB_MAX];
    __shared__ int offs[SCAN ? SCAN_SB : 1];
    __shared__ int wsum[SB_T / WAVE];
    const int vi = blockIdx.y;
    const ViewK &V = views[vi];
    int sb_lo, nsb;
    view_superbuckets(V, sb_lo, nsb);
    for (int j = threadIdx.x; j < nsb; j += SB_T) hist[j] = 0;
    const int64_t i0 = (int64_t)blockIdx.x * SB_T * SB_PER + threadIdx.x;
    int2 e[SB_PER];
    int r[SB_PER];
    // loads first, then the LDS atomics (interleaved, each load waited)
#pragma unroll
    for (int j = 0; j < SB_PER; ++j) {
        const int64_t i = i0 + (int64_t)j * SB_T;
        e[j] = i < n ? kz[(int64_t)vi * n + i] : make_int2(-1, 0);
    }
    if constexpr (SCAN) {
        // exclusive scan of the totals, PER consecutive ones per thread
        constexpr int PER = SCAN_SB / SB_T;
        const int k0 = threadIdx.x * PER;
        int c[PER], t = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            c[q] = k0 + q < nsb_all ? sb_count[k0 + q] : 0;
            t += c[q];
        }
        const int l = lane_id(), w = threadIdx.x / WAVE;
        const int inc = wave_incl_scan_i32(t);
        if (l == WAVE - 1) wsum[w] = inc;
        __syncthreads();
        int run = inc - t, tot = 0;
#pragma unroll
        for (int k = 0; k < SB_T / WAVE; ++k) {
            run += k < w ? wsum[k] : 0;
            tot += wsum[k];
        }
        const bool first = blockIdx.x == 0 && blockIdx.y == 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            offs[k0 + q] = run;
            if (first && k0 + q < nsb_all) sb_off[k0 + q] = run;
            run += c[q];
        }
        if (first && threadIdx.x == 0) {
            sb_off[nsb_all] = tot;
            *offsets_end = tot;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SB_PER; ++j)
        r[j] = e[j].x >= 0 ? atomicAdd(&hist[(e[j].x >> SB_SHIFT) - sb_lo], 1) : 0;
    __syncthreads();
    for (int j = threadIdx.x; j < nsb; j += SB_T) {
        const int c = hist[j];
        const int base = SCAN ? offs[sb_lo + j] : sb_off[sb_lo + j];
        hist[j] = c ? base + atomicAdd(&sb_cursor[sb_lo + j], c) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SB_PER; ++j) {
        if (e[j].x < 0) continue;
        const int64_t i = i0 + (int64_t)j * SB_T;
        rec[hist[(e[j].x >> SB_SHIFT) - sb_lo] + r[j]] = make_int4(e[j].x, e[j].y, (int)i, vi);
    }
}

// One workgroup per superbucket: bucket counts (LDS atomics), their scan
// (the table's offsets for these SB keys), placement of every record, then
// each bucket of at most SMALL_MAX points sorted by (z, index) in registers
// (larger ones are listed for k_sort_listed) and its depth noted.  The
// depth cells' minima come from the records themselves (every point's depth,
// listed buckets included): a minimum per cell in the LDS for the cells from
// the first one of the superbucket's first cell row on, device atomics for
// any cell beyond those (a row-major grid wider than about 2,000 buckets, or
// a superbucket that reaches far into a second view).  Depths of binned
// points are positive and finite, so their bits order as the values do.
constexpr int FIN_T = 512;  // threads of a superbucket's workgroup
constexpr int FIN_CELLS = 512;

// depth cell of bucket b of a view (bucket_base, Wg, cell_base, ncx)
__device__ __forceinline__ int cell_of_bucket(int layout, int b, int base, int wg, int cbase, int ncx)
{
    const int local = b - base;
    if (layout != HP_LAYOUT_ROWMAJOR) return cbase + (local >> 6);  // cells are the 8x8 tiles
    const int by = local / wg, bx = local - by * wg;
    return cbase + (by >> CELL_SHIFT) * ncx + (bx >> CELL_SHIFT);
}

__global__ void __launch_bounds__(FIN_T) __attribute__((amdgpu_waves_per_eu(6, 8))) k_finalize_sb(const int4 *__restrict__ rec,
                                                      const int32_t *__restrict__ sb_off,
                                                      int64_t n_buckets,
                                                      int32_t *__restrict__ offsets,
                                                      uint64_t *__restrict__ skey,
                                                      int32_t *__restrict__ big_list,
                                                      int32_t *__restrict__ big_n,
                                                      float *__restrict__ bucket_z, SlotOut so,
                                                      int layout, uint32_t *__restrict__ cell_zmin)
{
    __shared__ int cnt[SB];
    __shared__ int cur[SB];
    __shared__ int sh[FIN_T / WAVE];
    __shared__ uint32_t zc[FIN_CELLS];
    const int sb = blockIdx.x;
    const int64_t key0 = (int64_t)sb << SB_SHIFT;
    const int nkeys = (int)min((int64_t)SB, n_buckets - key0);
    const int r0 = sb_off[sb], r1 = sb_off[sb + 1];
    // the view of the superbucket's first bucket, and the first cell of that
    // bucket's cell row (row-major) or its cell (tiles)
    int v0 = 0;
    while (v0 + 1 < so.n_views && so.views[v0 + 1].bucket_base <= key0) ++v0;
    const int base0 = so.views[v0].bucket_base, wg0 = so.views[v0].Wg;
    const int cbase0 = so.views[v0].cell_base, ncx0 = so.views[v0].ncx;
    const int end0 = base0 + wg0 * so.views[v0].Hg;
    const int cell_lo = layout != HP_LAYOUT_ROWMAJOR
                            ? cbase0 + (((int)key0 - base0) >> 6)
                            : cbase0 + ((((int)key0 - base0) / wg0) >> CELL_SHIFT) * ncx0;
    for (int k = threadIdx.x; k < SB; k += FIN_T) cnt[k] = 0;
    for (int k = threadIdx.x; k < FIN_CELLS; k += FIN_T) zc[k] = 0x7f800000u;
    __syncthreads();
    // records four at a time, their loads in flight together (the order in
    // which a bucket's records arrive does not matter: each bucket is sorted
    // by (z, index) below)
    constexpr int RB = 4;
    const int2 *rxy = reinterpret_cast<const int2 *>(rec);  // (bucket, depth bits) of record i at 2 i
    for (int i0 = r0 + threadIdx.x; i0 < r1; i0 += RB * FIN_T) {
        int2 x[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j)
            x[j] = i0 + j * FIN_T < r1 ? rxy[2 * (int64_t)(i0 + j * FIN_T)] : make_int2(-1, 0);
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const int b = x[j].x;
            if (b < 0) continue;
            atomicAdd(&cnt[b - (int)key0], 1);
            int cell;
            if (b < end0) {
                cell = cell_of_bucket(layout, b, base0, wg0, cbase0, ncx0);
            } else {
                const ViewK &Vr = so.views[rec[i0 + j * FIN_T].w];
                cell = cell_of_bucket(layout, b, Vr.bucket_base, Vr.Wg, Vr.cell_base, Vr.ncx);
            }
            const int rel = cell - cell_lo;
            if ((unsigned)rel < (unsigned)FIN_CELLS) atomicMin(&zc[rel], (uint32_t)x[j].y);
            else atomicMin(&cell_zmin[cell], (uint32_t)x[j].y);
        }
    }
    __syncthreads();
    // exclusive scan over the SB counts, SB / FIN_T consecutive ones per thread
    constexpr int PER = SB / FIN_T;
    const int k0 = threadIdx.x * PER;
    int c[PER], s = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        c[q] = cnt[k0 + q];
        s += c[q];
    }
    const int l = lane_id(), w = threadIdx.x / WAVE;
    const int inc = wave_incl_scan_i32(s);
    if (l == WAVE - 1) sh[w] = inc;
    __syncthreads();
    int run = r0 + inc - s;
#pragma unroll
    for (int k = 0; k < FIN_T / WAVE; ++k) run += k < w ? sh[k] : 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        cur[k0 + q] = run;
        if (k0 + q < nkeys) offsets[key0 + k0 + q] = run;
        run += c[q];
    }
    __syncthreads();
    for (int i0 = r0 + threadIdx.x; i0 < r1; i0 += RB * FIN_T) {
        int4 e[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) e[j] = i0 + j * FIN_T < r1 ? rec[i0 + j * FIN_T] : make_int4(-1, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            if (e[j].x >= 0) {
                const int slot = atomicAdd(&cur[e[j].x - (int)key0], 1);
                skey[slot] = ((uint64_t)(uint32_t)e[j].y << 32) | (uint32_t)e[j].z;
            }
        }
    }
    __syncthreads();  // (the placed keys are read back below by other threads)
    for (int k = threadIdx.x; k < FIN_CELLS; k += FIN_T)
        if (zc[k] != 0x7f800000u) atomicMin(&cell_zmin[cell_lo + k], zc[k]);
    for (int k = threadIdx.x; k < nkeys; k += FIN_T) {
        const int b = (int)key0 + k;
        const int n_b = cnt[k];
        const int start = cur[k] - n_b;
        if (n_b > SMALL_MAX) {
            list_big_bucket(big_list, big_n, n_buckets, b, n_b);
            continue;  // k_sort_listed sorts it, places it and writes bucket_z
        }
        uint64_t first = ~0ull;
        if (n_b > 0) {
            // sorted slots become table points right away
            const float4 *pc = bucket_pcam(so, b);
            if (n_b == 1) {
                first = skey[start];
                put_slot(so, pc, start, first);
            } else if (n_b <= 4) {
                first = sort_bucket_to_slots<4>(skey, start, n_b, so, pc);
            } else if (n_b <= 8) {
                first = sort_bucket_to_slots<8>(skey, start, n_b, so, pc);
            } else {
                first = sort_bucket_to_slots<16>(skey, start, n_b, so, pc);
            }
        }
        bucket_z[b] = n_b > 0 ? __uint_as_float((uint32_t)(first >> 32)) : __builtin_inff();
    }
}

constexpr int BIG_T = 256;
constexpr int BIG_LDS = 4096;

// Bitonic sort of cnt keys with all comparators placing the minimum at the
// lower index ("flip" form): virtual +inf keys beyond cnt never move, so the
// length need not be a power of two.
template <typename Load, typename Store>
__device__ void block_flip_bitonic(int cnt, Load ld, Store st)
{
    int P = 1;
    while (P < cnt) P <<= 1;
    for (int s = 2; s <= P; s <<= 1) {
        for (int j = s >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P / 2; i += blockDim.x) {
                // comparator i of this stage joins positions lo < hi
                int lo, hi;
                if (j == (s >> 1)) {
                    const int blk = i / j, off = i % j;
                    lo = blk * s + off;
                    hi = blk * s + s - 1 - off;
                } else {
                    const int blk = i / j, off = i % j;
                    lo = blk * 2 * j + off;
                    hi = lo + j;
                }
                if (hi < cnt) {
                    const uint64_t a = ld(lo), b = ld(hi);
                    if (b < a) {
                        st(lo, b);
                        st(hi, a);
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Buckets of 17..128 points: one wave each, a register bitonic sort across
// the wave (one or two keys per lane), no LDS and no workgroup barrier.
// (workgroup `blk` of `nblk` taking this role)
__device__ __forceinline__ void sort_mid(const int32_t *__restrict__ offsets,
                                         uint64_t *__restrict__ skey,
                                         const int32_t *__restrict__ big_list,
                                         const int32_t *__restrict__ big_n,
                                         float *__restrict__ bucket_z, const SlotOut &so, int blk,
                                         int nblk)
{
    const int nbig = big_n[0];
    const int l = lane_id();
    const int waves = blockDim.x / WAVE;
    for (int it = blk * waves + (threadIdx.x >> 6); it < nbig; it += nblk * waves) {
        const int b = big_list[it];
        const int start = offsets[b];
        const int cnt = offsets[b + 1] - start;
        uint64_t x = l < cnt ? skey[start + l] : ~0ull;
        if (cnt <= WAVE) {
            x = wave_sort_fast(x);
        } else {
            // 128 keys: an ascending and a descending run, the lane-wise
            // half-cleaner, then both halves sorted
            uint64_t y = WAVE + l < cnt ? skey[start + WAVE + l] : ~0ull;
            x = wave_sort_fast(x);
            y = wave_sort_desc(y);
            const uint64_t lo = umin64(x, y), hi = umax64(x, y);
            x = wave_merge_low_fast(lo, ~0ull);
            y = wave_merge_low_fast(hi, ~0ull);
            if (WAVE + l < cnt) {
                if (so.pts) put_slot(so, bucket_pcam(so, b), start + WAVE + l, y);
                else skey[start + WAVE + l] = y;
            }
        }
        if (l < cnt) {
            if (so.pts) put_slot(so, bucket_pcam(so, b), start + l, x);
            else skey[start + l] = x;
        }
        if (l == 0) bucket_z[b] = __uint_as_float((uint32_t)(x >> 32));
    }
}

// Buckets of more than 128 points: one workgroup each, bitonic in LDS (in
// global memory beyond BIG_LDS entries).
__device__ __forceinline__ void sort_big(const int32_t *__restrict__ offsets,
                                         uint64_t *__restrict__ skey,
                                         const int32_t *__restrict__ big_list,
                                         const int32_t *__restrict__ big_n,
                                         float *__restrict__ bucket_z, int64_t cap, const SlotOut &so,
                                         uint64_t *sh, int blk, int nblk)
{
    const int nbig = big_n[1];
    for (int it = blk; it < nbig; it += nblk) {
        const int b = big_list[cap - 1 - it];
        const int start = offsets[b];
        const int cnt = offsets[b + 1] - start;
        uint64_t *g = skey + start;
        if (cnt <= BIG_LDS) {
            for (int i = threadIdx.x; i < cnt; i += blockDim.x) sh[i] = g[i];
            __syncthreads();
            block_flip_bitonic(cnt, [&](int i) { return sh[i]; }, [&](int i, uint64_t v) { sh[i] = v; });
            for (int i = threadIdx.x; i < cnt; i += blockDim.x) g[i] = sh[i];
        } else {
            block_flip_bitonic(cnt, [&](int i) { return g[i]; },
                               [&](int i, uint64_t v) { g[i] = v; });
        }
        __syncthreads();
        if (so.pts) {
            const float4 *pc = bucket_pcam(so, b);
            for (int i = threadIdx.x; i < cnt; i += blockDim.x) put_slot(so, pc, start + i, g[i]);
        }
        if (threadIdx.x == 0) bucket_z[b] = __uint_as_float((uint32_t)(g[0] >> 32));
        __syncthreads();
    }
}

// The listed buckets in one launch: the first MID_BLOCKS workgroups sort those
// of 17..128 points (a wave each), the other BIG_BLOCKS the larger ones.
constexpr int MID_BLOCKS = 1024;
constexpr int BIG_BLOCKS = 256;
static_assert(BIG_T == 256, "both roles run 256-thread workgroups");

__global__ void __launch_bounds__(256) k_sort_listed(const int32_t *__restrict__ offsets,
                                                     uint64_t *__restrict__ skey,
                                                     const int32_t *__restrict__ big_list,
                                                     const int32_t *__restrict__ big_n,
                                                     float *__restrict__ bucket_z, int64_t cap,
                                                     SlotOut so)
{
    __shared__ uint64_t sh[BIG_LDS];
    if (blockIdx.x < MID_BLOCKS)
        sort_mid(offsets, skey, big_list, big_n, bucket_z, so, blockIdx.x, MID_BLOCKS);
    else
        sort_big(offsets, skey, big_list, big_n, bucket_z, cap, so, sh, blockIdx.x - MID_BLOCKS,
                 BIG_BLOCKS);
}

// Minimum depth of each CELL x CELL block of buckets, from the buckets'
// first (nearest) points.  One wave per cell, grid (cells / 4, views).
__global__ void __launch_bounds__(256) k_cell_zmin(const float *__restrict__ bucket_z,
                                                   const ViewK *__restrict__ views, int layout,
                                                   uint32_t *__restrict__ cell_zmin)
{
    const ViewK &V = views[blockIdx.y];
    const int cell = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int ncy = (V.Hg + CELL - 1) / CELL;
    if (cell >= V.ncx * ncy) return;
    const int l = threadIdx.x & 63;
    const int bx = (cell % V.ncx) * CELL + (l & (CELL - 1));
    const int by = (cell / V.ncx) * CELL + (l >> CELL_SHIFT);
    float z = __builtin_inff();
    if (bx < V.Wg && by < V.Hg) z = bucket_z[bucket_of(V, layout, bx, by)];
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) z = __builtin_fminf(z, __shfl_xor(z, o, WAVE));
    if (l == 0) cell_zmin[V.cell_base + cell] = __float_as_uint(z);
}

// first slot of every view (views are contiguous in the bucket space)
__global__ void k_view_slots(const int32_t *__restrict__ offsets, ViewK *views, int n_views)
{
    const int i = threadIdx.x;
    if (i < n_views) views[i].slot_base = offsets[views[i].bucket_base];
}

__global__ void __launch_bounds__(256) k_materialize(const uint64_t *__restrict__ skey,
                                                     const int32_t *__restrict__ n_in_ptr,
                                                     const float4 *__restrict__ pcam, int64_t n,
                                                     const ViewK *__restrict__ views, int n_views,
                                                     float4 *__restrict__ pts,
                                                     int32_t *__restrict__ perm)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= *n_in_ptr) return;
    int vi = 0;
    while (vi + 1 < n_views && views[vi + 1].slot_base <= s) ++vi;
    const int32_t idx = (int32_t)(uint32_t)skey[s];
    pts[s] = pcam[(int64_t)vi * n + idx];
    perm[s] = idx;
}

}  // namespace hp

namespace hp {

static void finish_build(const float *xyz, int64_t n, const ViewSet &vs, const TableWs &tw,
                         bool materialize, hipStream_t s);

hipError_t launch_build(const float *xyz, int64_t n, const ViewSet &vs, int64_t n_buckets,
                        int64_t n_cells, const TableWs &tw, hipStream_t s)
{
    const int V = vs.n;
    const int64_t nv = n * V;
    const int64_t nsb = (n_buckets + SB - 1) / SB;
    // the projection passes count a view's points per superbucket in LDS, so
    // each view may span at most SB_MAX superbuckets (the table as a whole
    // may span more)
    int64_t view_sb_max = 0;
    for (int i = 0; i < V; ++i) {
        const ViewK &vk = vs.v[i];
        const int64_t lo = vk.bucket_base >> SB_SHIFT;
        const int64_t hi = ((int64_t)vk.bucket_base + (int64_t)vk.Wg * vk.Hg - 1) >> SB_SHIFT;
        view_sb_max = max(view_sb_max, hi - lo + 1);
    }
    if (view_sb_max <= SB_MAX && nsb <= INT32_MAX / SB) {
        // two-level build: superbucket totals, records by superbucket, then
        // each superbucket's buckets in LDS
        // totals, cursors, big_n[2]; the depth cells, which the superbuckets'
        // workgroups lower
        k_build_begin<<<64, 256, 0, s>>>(vs, tw.views, tw.sb_count, tw.sb_words, tw.cell_zmin, n_cells);
        if (nv > 0) {
            const dim3 grid((unsigned)((n + SB_T * SB_PER - 1) / (SB_T * SB_PER)), V);
            k_project_sb<<<grid, SB_T, 0, s>>>(xyz, n, tw.views, vs.layout, tw.kz, tw.pcam,
                                               tw.sb_count);
            if (nsb <= SCAN_SB) {
                k_scatter_sb<true><<<grid, SB_T, 0, s>>>(tw.kz, n, tw.views, tw.sb_off, tw.sb_cursor,
                                                         reinterpret_cast<int4 *>(tw.pts), tw.sb_count,
                                                         (int)nsb, tw.offsets + n_buckets);
            } else {
                k_sb_scan<<<1, 1024, 0, s>>>(tw.sb_count, (int)nsb, tw.sb_off, tw.offsets + n_buckets);
                k_scatter_sb<false><<<grid, SB_T, 0, s>>>(tw.kz, n, tw.views, tw.sb_off, tw.sb_cursor,
                                                          reinterpret_cast<int4 *>(tw.pts), nullptr,
                                                          (int)nsb, nullptr);
            }
        } else {
            k_sb_scan<<<1, 1024, 0, s>>>(tw.sb_count, (int)nsb, tw.sb_off, tw.offsets + n_buckets);
        }
        // (the records sit in pts: a superbucket's workgroup overwrites only
        // its own range, after reading all of it)
        const SlotOut so{tw.pcam, n, tw.views, V, tw.pts, tw.perm};
        k_finalize_sb<<<(unsigned)nsb, FIN_T, 0, s>>>(reinterpret_cast<const int4 *>(tw.pts), tw.sb_off,
                                                     n_buckets, tw.offsets, tw.skey, tw.big_list,
                                                     tw.big_n, tw.bucket_z, so, vs.layout, tw.cell_zmin);
        k_sort_listed<<<MID_BLOCKS + BIG_BLOCKS, 256, 0, s>>>(tw.offsets, tw.skey, tw.big_list, tw.big_n,
                                                            tw.bucket_z, n_buckets, so);
        return hipGetLastError();
    }
    // one level (a view beyond SB_MAX superbuckets): a counter per bucket
    k_build_begin<<<1024, 256, 0, s>>>(vs, tw.views, tw.count, n_buckets, nullptr, 0);
    k_fill_i32<<<1, 64, 0, s>>>(tw.big_n, 0, 2);
    if (n > 0)
        k_project<<<dim3((unsigned)((n + 256 * PROJ_PER - 1) / (256 * PROJ_PER)), V), 256, 0, s>>>(
            xyz, n, tw.views, vs.layout, tw.kz, tw.pcam, tw.count, tw.perm);
    const int64_t nblk = (n_buckets + SCAN_TILE - 1) / SCAN_TILE;
    k_scan_reduce<<<(unsigned)nblk, SCAN_T, 0, s>>>(tw.count, n_buckets, tw.block_sums);
    k_scan_blocks<<<1, SCAN_T, 0, s>>>(tw.block_sums, nblk);
    k_scan_apply<<<(unsigned)nblk, SCAN_T, 0, s>>>(tw.count, n_buckets, tw.block_sums, tw.offsets);
    if (nv > 0) k_scatter<<<(unsigned)((nv + 255) / 256), 256, 0, s>>>(tw.kz, tw.perm, nv, n, tw.offsets, tw.skey);
    k_sort_small<<<(unsigned)((n_buckets + 255) / 256), 256, 0, s>>>(tw.offsets, n_buckets, tw.skey, tw.big_list, tw.big_n, tw.bucket_z);
    const SlotOut none{nullptr, 0, nullptr, 0, nullptr, nullptr};
    k_sort_listed<<<MID_BLOCKS + BIG_BLOCKS, 256, 0, s>>>(tw.offsets, tw.skey, tw.big_list, tw.big_n,
                                                        tw.bucket_z, n_buckets, none);
    finish_build(xyz, n, vs, tw, true, s);
    return hipGetLastError();
}

// depth cells; with `materialize`, the views' first slots and the table
// points per slot (the two-level build places them while sorting)
static void finish_build(const float *xyz, int64_t n, const ViewSet &vs, const TableWs &tw,
                         bool materialize, hipStream_t s)
{
    const int V = vs.n;
    const int64_t nv = n * V;
    int max_cells = 0;
    for (int i = 0; i < V; ++i) {
        const ViewK &vk = vs.v[i];
        max_cells = max(max_cells, vk.ncx * ((vk.Hg + CELL - 1) / CELL));
    }
    k_cell_zmin<<<dim3((unsigned)((max_cells + 3) / 4), V), 256, 0, s>>>(tw.bucket_z, tw.views, vs.layout, tw.cell_zmin);
    if (!materialize) return;
    k_view_slots<<<1, HP_MAX_VIEWS, 0, s>>>(tw.offsets, tw.views, V);
    if (nv > 0)
        k_materialize<<<(unsigned)((nv + 255) / 256), 256, 0, s>>>(tw.skey, tw.offsets + tw.n_buckets, tw.pcam, n, tw.views, V, tw.pts, tw.perm);
}

}  // namespace hp
