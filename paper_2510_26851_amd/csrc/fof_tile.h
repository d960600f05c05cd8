// Tiles of the coarse grid shared by the LDS-tiled kernels (hard linking and the
// candidate edges of stochastic linking): a block owns kTileX x kTileY x kTileZ coarse cells
// and stages them with a one-cell halo.  With cells z fastest every (x, y) row of the halo
// is one contiguous run of particles in cell order.
#pragma once

#include "fof_internal.h"

namespace fof {
namespace {

constexpr int kHX = kTileX + 2, kHY = kTileY + 2, kHZ = kTileZ + 2;
constexpr int kRowsH = kHX * kHY;
constexpr int kHalo = kRowsH * kHZ;
constexpr int kTileBlock = 256;
constexpr int kPerT = (kHalo + kTileBlock - 1) / kTileBlock;  // halo cells per thread
constexpr int kTileCap = 1024;                                  // staged particles per tile
constexpr int kStagePerT = kTileCap / kTileBlock;
constexpr int kOwnRows = kTileX * kTileY;
static_assert(kTileCap % kTileBlock == 0, "staging assumes whole rounds");
static_assert(kRowsH <= kWave && kHZ <= kTileBlock, "row scans use one wave");

constexpr int top_pow2(int n) { return n < 2 ? 1 : 2 * top_pow2(n / 2); }

// Box owning tile t: the last box whose first tile is <= t.  Boxes without tiles share
// their tile_base with the next box, which comes later, so they are never chosen.
__device__ __forceinline__ int find_box_tile(const BoxDesc *d, int nbox, int64_t t)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile_base <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The last index h in [0, N) with off[h] <= s, for non-decreasing off with off[0] <= s.
// Fixed trip count, so a thread's independent searches interleave.
template <int N>
__device__ __forceinline__ int last_le(const int *off, int s)
{
    constexpr int kTop = top_pow2(N - 1);  // evaluated at compile time
    int pos = 0;
#pragma unroll
    for (int step = kTop; step > 0; step >>= 1)
        if (pos + step < N && off[pos + step] <= s)
            pos += step;
    return pos;
}

struct TileGeom {
    int x0, y0, z0;     // first own cell
    int hxe, hye, hze;  // last halo index in use per axis (own cells stop at the box edge)
};

__device__ __forceinline__ TileGeom tile_geom(const BoxDesc &B, int64_t tile)
{
    // a box has fewer tiles than cells (< 2^31), so 32-bit division suffices
    int tl = (int)(tile - B.tile_base);
    const int tz = tl % B.ntile[2];
    tl /= B.ntile[2];
    const int ty = tl % B.ntile[1];
    const int tx = tl / B.ntile[1];
    TileGeom g;
    g.x0 = tx * kTileX;
    g.y0 = ty * kTileY;
    g.z0 = tz * kTileZ;
    g.hxe = min(kTileX, B.nc[0] - g.x0) + 1;
    g.hye = min(kTileY, B.nc[1] - g.y0) + 1;
    g.hze = min(kTileZ, B.nc[2] - g.z0) + 1;
    return g;
}

// Halo table of a tile: the staged count of every halo cell and its global start, or for a
// cell with a clique table -1 - its dense id (halo coordinates lie in [-1, nc], so one wrap
// suffices), then the running offsets.  Ends with a block barrier; returns the staged total.
__device__ int build_halo(const Work &w, const BoxDesc &B, const TileGeom &g, bool box_dense,
                          int *hoff, int *gst, int *scr)
{
    static_assert(kHZ % kPerT == 0, "a thread's halo cells share one row");
    const int t = threadIdx.x, lane = lane_id(), wid = t / kWave;
    int cnt_local[kPerT];
    int sum = 0;
    const int h0 = t * kPerT;
    const int hz0 = h0 % kHZ, row = h0 / kHZ, hy = row % kHY, hx = row / kHY;
    const bool row_in = h0 < kHalo && hx <= g.hxe && hy <= g.hye;
    // the row's (x, y) column, once per thread
    const int64_t col = row_in ? coarse_cell(B, wrap_cell(g.x0 - 1 + hx, B.nc[0]),
                                             wrap_cell(g.y0 - 1 + hy, B.nc[1]), 0)
                               : 0;
#pragma unroll
    for (int k = 0; k < kPerT; ++k) {
        const int h = h0 + k, hz = hz0 + k;
        int cnt = 0;
        if (h < kHalo) {
            int tag = -1, s = 0;
            if (row_in && hz <= g.hze) {
                const int64_t c = col + wrap_cell(g.z0 - 1 + hz, B.nc[2]);
                s = w.cell_start[c];
                cnt = w.cell_start[c + 1] - s;
                if (box_dense && cnt > w.dense_threshold && w.cell_count[c] >= 0) {
                    tag = w.cell_count[c];
                    cnt = 0;
                }
            }
            gst[h] = tag >= 0 ? -1 - tag : s;
        }
        cnt_local[k] = cnt;
        sum += cnt;
    }
    // exclusive scan of staged counts; each thread owns kPerT consecutive halo cells
    const int x = wave_incl_sum(sum);
    if (lane == kWave - 1)
        scr[wid] = x;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int k = 0; k < kTileBlock / kWave; ++k) {
        if (k < wid)
            pre += scr[k];
        tot += scr[k];
    }
    int run = pre + x - sum;
#pragma unroll
    for (int k = 0; k < kPerT; ++k) {
        const int h = t * kPerT + k;
        if (h < kHalo)
            hoff[h] = run;
        run += cnt_local[k];
    }
    if (t == 0)
        hoff[kHalo] = tot;
    __syncthreads();
    return tot;
}

}  // namespace
}  // namespace fof
