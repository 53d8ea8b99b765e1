// Layout of the table workspace (device memory owned by the caller).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hp_device.hpp"

namespace hp {

// Superbuckets of the two-level build: SB = 2^SB_SHIFT consecutive bucket
// keys; tables whose views each span at most SB_MAX of them (2^23 buckets)
// take that path.
constexpr int SB_SHIFT = 10;
constexpr int SB_MAX = 8192;

struct TableWs {
    ViewK *views;          // [HP_MAX_VIEWS]  per-view constants
    int32_t *count;        // [n_buckets]     per-bucket counters
    int32_t *offsets;      // [n_buckets + 1] bucket offsets (the table)
    int32_t *block_sums;   // [scan blocks]
    int2 *kz;              // [n_views * n]   (bucket, z bits) per point and view
    uint64_t *skey;        // [n_views * n]   (z bits, index) per slot
    float4 *pts;           // [n_views * n]   camera-space point per slot
    int32_t *perm;         // [n_views * n]   point index per slot
    float4 *pcam;          // [n_views * n]   camera-space point (x, y, z, index bits) per point and view
    int32_t *big_list;     // [n_buckets]     buckets too large for one lane
    int32_t *sb_count;     // [n_sb]          points per superbucket, then
    int32_t *sb_cursor;    // [n_sb]          records placed per superbucket, then
    int32_t *big_n;        // [2]             entries of big_list (one region, zeroed at once)
    int64_t sb_words;      //                 2 n_sb + 2
    int32_t *sb_off;       // [n_sb + 1]      first record of each superbucket
    int64_t n_buckets;
    float *bucket_z;       // [n_buckets]     depth of the first point (+inf if empty)
    uint32_t *cell_zmin;   // [n_cells]       min depth bits per cell (+inf if empty)
    size_t bytes;
};

inline TableWs table_ws_layout(void *base, int64_t n, int n_views, int64_t n_buckets,
                               int64_t n_cells)
{
    TableWs w;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? (void *)((char *)base + off) : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    const int64_t nv = n * n_views;
    const int64_t nvs = nv > 0 ? nv : 1;
    const int64_t scan_blocks = (n_buckets + 4095) / 4096 + 1;
    w.views = (ViewK *)take(sizeof(ViewK) * HP_MAX_VIEWS);
    w.count = (int32_t *)take(sizeof(int32_t) * n_buckets);
    w.offsets = (int32_t *)take(sizeof(int32_t) * (n_buckets + 1));
    w.block_sums = (int32_t *)take(sizeof(int32_t) * scan_blocks);
    w.kz = (int2 *)take(sizeof(int2) * nvs);
    w.skey = (uint64_t *)take(sizeof(uint64_t) * nvs);
    w.pts = (float4 *)take(sizeof(float4) * nvs);
    w.perm = (int32_t *)take(sizeof(int32_t) * nvs);
    w.pcam = (float4 *)take(sizeof(float4) * nvs);
    w.big_list = (int32_t *)take(sizeof(int32_t) * n_buckets);
    const int64_t n_sb = (n_buckets + (1 << SB_SHIFT) - 1) >> SB_SHIFT;
    w.sb_count = (int32_t *)take(sizeof(int32_t) * (2 * n_sb + 64));
    w.sb_cursor = base ? w.sb_count + n_sb : nullptr;
    w.big_n = base ? w.sb_count + 2 * n_sb : nullptr;
    w.sb_words = 2 * n_sb + 2;
    w.sb_off = (int32_t *)take(sizeof(int32_t) * (n_sb + 1));
    w.n_buckets = n_buckets;
    w.bucket_z = (float *)take(sizeof(float) * n_buckets);
    w.cell_zmin = (uint32_t *)take(sizeof(uint32_t) * (n_cells > 0 ? n_cells : 1));
    w.bytes = off;
    return w;
}

}  // namespace hp
