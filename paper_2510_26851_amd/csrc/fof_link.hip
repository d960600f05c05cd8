// Friends-of-Friends linking (paper Sec. 2 steps (iii)-(v), Alg. 2): candidate search over
// the 27-cell stencil of the coarse grid, the exact minimum-image predicate, and connected
// components by a lock-free union-find instead of a fixed number of label sweeps.
//
// One thread per particle in cell-sorted order.  Each thread tests every candidate in the
// neighbour cells that its own position can reach (a neighbour cell is skipped when the
// particle is farther than `reach` from the shared face), so every pair is tested from
// both ends.  That lets a particle that finds no friend at all write its final label
// (itself) at once; only particles with at least one friend are marked in the flag bitmap
// and resolved by the compress pass.  Each friend pair is hooked once, by its lower
// sorted index.
//
// Cells with clique tables (fof_dense.hip) are linked by the dense kernels; their
// particles skip the search here and are only marked.  A particle of an ordinary cell
// reaches a dense neighbour through its units: only the fine cells within reach are
// visited, and one friend in a unit (a clique) joins the particle to all of it.
#include "fof_internal.h"

namespace fof {

namespace {

// Offsets to visit along one axis, deduplicated when the grid has fewer than 3 cells.
struct AxisSpan {
    int lo, hi;  // visit o in [lo, hi] (o = -1, 0, +1), skipping none in between
};

__device__ __forceinline__ AxisSpan axis_span(float x, int ix, float side, int nc, float reach)
{
    if (nc == 1)
        return {0, 0};
    float g_lo = x - (float)ix * side;          // distance to the lower face
    float g_hi = (float)(ix + 1) * side - x;    // distance to the upper face
    bool need_lo = g_lo < reach;
    bool need_hi = g_hi < reach;
    if (nc == 2)  // the single other cell is both the lower and the upper neighbour
        return {0, (need_lo || need_hi) ? 1 : 0};
    return {need_lo ? -1 : 0, need_hi ? 1 : 0};
}

__device__ __forceinline__ int wrap_cell(int c, int nc)
{
    return c < 0 ? c + nc : (c >= nc ? c - nc : c);
}

// Fine-key range of a neighbour dense cell that a particle at fine coordinate f (relative
// to that cell's origin, in the particle's periodic frame) can reach.
__device__ __forceinline__ void key_range(float f, float rf, int m, int &lo, int &hi)
{
    lo = (int)floorf(f - rf);
    hi = (int)floorf(f + rf);
    lo = lo < 0 ? 0 : lo;
    hi = hi > m - 1 ? m - 1 : hi;
}

// Links particle i (position p) to the units of dense cell c2 at offset (ox, oy, oz) from
// its own cell (ix, iy, iz).  Returns true if any friend was found.
__device__ bool link_dense_neighbour(const Work &w, const BoxDesc &B, uint32_t i, float4 p,
                                     int ix, int iy, int iz, int ox, int oy, int oz, int32_t s2,
                                     int32_t n2, int32_t d2)
{
    const int m = B.m;
    const int W = w.table_words;
    const int32_t *T = w.table + (int64_t)d2 * w.table_stride;
    const int u = T[2], ncomp = T[1];
    int x0, x1, y0, y1, z0, z1;
    FOF_STAT(w.ctr, ST_DN_CALLS, 1);
    key_range(p.x * B.inv_fine[0] - (float)((ix + ox) * m), B.reach * B.inv_fine[0], m, x0, x1);
    key_range(p.y * B.inv_fine[1] - (float)((iy + oy) * m), B.reach * B.inv_fine[1], m, y0, y1);
    key_range(p.z * B.inv_fine[2] - (float)((iz + oz) * m), B.reach * B.inv_fine[2], m, z0, z1);
    bool any = false;
    uint64_t seen = 0;  // components (numbers < 64) already joined
    for (int bz = z0; bz <= z1; ++bz)
        for (int by = y0; by <= y1; ++by)
            for (int bx = x0; bx <= x1; ++bx) {
                const int kb = (bz * m + by) * m + bx;
                const uint32_t word = (uint32_t)T[kTableHeader + (kb >> 5)];
                if (!((word >> (kb & 31)) & 1u))
                    continue;
                const int rb = T[kTableHeader + W + (kb >> 5)] +
                               __popc(word & ((1u << (kb & 31)) - 1u));
                const int comp = w.cnt[s2 + rb];
                if (comp < 64 && ((seen >> comp) & 1ull))
                    continue;
                const int32_t b0 = w.rank[s2 + rb];
                const int32_t b1 = rb + 1 < u ? w.rank[s2 + rb + 1] : s2 + n2;
                FOF_STAT(w.ctr, ST_DN_UNITS, 1);
                FOF_STAT(w.ctr, ST_DN_MEMBER_TESTS, b1 - b0);
                for (int32_t j = b0; j < b1; ++j) {
                    const float4 q = w.sorted[j];
                    if (linked(B, p.x, p.y, p.z, q.x, q.y, q.z)) {
                        uf_union(w.parent, i, (uint32_t)j);
                        any = true;
                        if (comp < 64)
                            seen |= 1ull << comp;
                        break;
                    }
                }
                if (any && ncomp == 1)
                    return true;
            }
    return any;
}

// Whether particle p (sorted index i) sits in a cell linked by the dense kernels.
__device__ __forceinline__ bool in_dense_cell(const Work &w, const BoxDesc &B, int ix, int iy,
                                              int iz)
{
    if (!(w.dense_cap > 0 && w.dense_threshold >= 0 && B.dense_ok))
        return false;
    const int64_t c0 = coarse_cell(B, ix, iy, iz);
    return w.cell_start[c0 + 1] - w.cell_start[c0] > w.dense_threshold && w.cell_count[c0] >= 0;
}

// Candidate search of one particle straight from global memory.  Returns true if it has a
// friend (its hooks are done).
__device__ bool link_particle_global(const Work &w, const BoxDesc &B, int64_t i, float4 p,
                                     int ix, int iy, int iz)
{
    const bool box_dense = w.dense_cap > 0 && w.dense_threshold >= 0 && B.dense_ok;
    bool has_friend = false;
    const AxisSpan sx = axis_span(p.x, ix, B.side[0], B.nc[0], B.reach);
    const AxisSpan sy = axis_span(p.y, iy, B.side[1], B.nc[1], B.reach);
    const AxisSpan sz = axis_span(p.z, iz, B.side[2], B.nc[2], B.reach);
    for (int ox = sx.lo; ox <= sx.hi; ++ox) {
        const int cx = wrap_cell(ix + ox, B.nc[0]);
        for (int oy = sy.lo; oy <= sy.hi; ++oy) {
            const int cy = wrap_cell(iy + oy, B.nc[1]);
            for (int oz = sz.lo; oz <= sz.hi; ++oz) {
                const int cz = wrap_cell(iz + oz, B.nc[2]);
                const int64_t c = coarse_cell(B, cx, cy, cz);
                const int32_t s = w.cell_start[c], e = w.cell_start[c + 1];
                if (box_dense && e - s > w.dense_threshold) {
                    const int32_t d2 = w.cell_count[c];
                    if (d2 >= 0) {
                        has_friend |= link_dense_neighbour(w, B, (uint32_t)i, p, ix, iy, iz, ox,
                                                           oy, oz, s, e - s, d2);
                        continue;
                    }
                }
                FOF_STAT(w.ctr, ST_PAIRS_GLOBAL, e - s);
                for (int32_t j = s; j < e; ++j) {
                    if (j == i)
                        continue;
                    const float4 q = w.sorted[j];
                    if (linked(B, p.x, p.y, p.z, q.x, q.y, q.z)) {
                        has_friend = true;
                        // each pair is hooked from the end with the smaller original index,
                        // the rule every link path shares (the other end may be staged)
                        if (__float_as_int(p.w) < __float_as_int(q.w))
                            uf_union(w.parent, (uint32_t)i, (uint32_t)j);
                    }
                }
            }
        }
    }
    return has_friend;
}

__device__ __forceinline__ void finish_particle(const Work &w, int32_t *root, int64_t i,
                                                int32_t orig, bool has_friend)
{
    if (has_friend)
        atomicOr((unsigned long long *)(w.flags + (i >> 6)), 1ull << (i & 63));
    else
        root[orig] = orig;
}

// Per-particle kernel for boxes the tiled kernel does not take (fewer than 3 cells on an
// axis).  Dense-cell particles were marked by the dense kernels.
__global__ void k_link(Work w, int32_t *__restrict__ root)
{
    const int64_t i = gtid_xcd();
    if (i >= w.n)
        return;
    const BoxDesc &B = w.desc[find_box(w.desc, w.nbox, i)];
    if (B.tiled)
        return;
    const float4 p = w.sorted[i];
    const int ix = fine_index(p.x, B.inv_fine[0], B.nf[0]) / B.m;
    const int iy = fine_index(p.y, B.inv_fine[1], B.nf[1]) / B.m;
    const int iz = fine_index(p.z, B.inv_fine[2], B.nf[2]) / B.m;
    if (in_dense_cell(w, B, ix, iy, iz))
        return;
    finish_particle(w, root, i, __float_as_int(p.w), link_particle_global(w, B, i, p, ix, iy, iz));
}

// ---------------------------------------------------------------------------------------
// LDS-tiled linking.  A block owns kTileX x kTileY x kTileZ coarse cells and stages them
// with a one-cell halo in LDS.  With cells z fastest, a particle's candidates in one
// neighbour row (up to three consecutive cells) form one contiguous LDS range.  Staging is
// flat: staged slot s belongs to the halo cell whose offset range holds s, found by a
// fixed-length binary search, so each thread issues its few global loads back to back.
// Cells with clique tables are not staged: particles reach them through their unit
// tables.  A tile whose staged particles do not fit searches from global memory.
// ---------------------------------------------------------------------------------------
constexpr int kHX = kTileX + 2, kHY = kTileY + 2, kHZ = kTileZ + 2;
constexpr int kRowsH = kHX * kHY;
constexpr int kHalo = kRowsH * kHZ;
constexpr int kTileBlock = 256;
constexpr int kPerT = (kHalo + kTileBlock - 1) / kTileBlock;  // halo cells per thread
constexpr int kTileCap = 1024;                                  // staged particles per tile
constexpr int kStagePerT = kTileCap / kTileBlock;
constexpr int kOwnRows = kTileX * kTileY;
static_assert(kTileCap % kTileBlock == 0, "staging assumes whole rounds");

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

__device__ __forceinline__ int mod_cell(int c, int nc)
{
    int r = c % nc;
    return r < 0 ? r + nc : r;
}

// Halo cell holding staged slot s: the last h with hoff[h] <= s (hoff non-decreasing,
// hoff[0] = 0 <= s < hoff[kHalo]).  Fixed trip count, so independent searches interleave.
__device__ __forceinline__ int halo_cell_of(const int *hoff, int s)
{
    int pos = 0;
#pragma unroll
    for (int step = 512; step > 0; step >>= 1)
        if (pos + step < kHalo && hoff[pos + step] <= s)
            pos += step;
    return pos;
}
static_assert(kHalo <= 1024, "halo_cell_of searches at most 1024 cells");

__global__ __launch_bounds__(kTileBlock) void k_link_tiled(Work w, int32_t *__restrict__ root)
{
    __shared__ float4 part[kTileCap];
    __shared__ int hoff[kHalo + 1];  // staged offset of each halo cell
    __shared__ int gst[kHalo];       // global (sorted) start of each halo cell
    __shared__ int htag[kHalo];      // dense id (>= 0) or -1
    __shared__ int ownoff[kOwnRows + 1];
    __shared__ int scr[kTileBlock / kWave];

    const int64_t tile = xcd_block();
    if (tile >= w.ntiles)
        return;
    const BoxDesc &B = w.desc[find_box_tile(w.desc, w.nbox, tile)];
    int64_t tl = tile - B.tile_base;
    const int tz = (int)(tl % B.ntile[2]);
    tl /= B.ntile[2];
    const int ty = (int)(tl % B.ntile[1]);
    const int tx = (int)(tl / B.ntile[1]);
    const int x0 = tx * kTileX, y0 = ty * kTileY, z0 = tz * kTileZ;
    // last halo index (inclusive) in use per axis: own cells stop at the box edge
    const int hxe = min(kTileX, B.nc[0] - x0) + 1;
    const int hye = min(kTileY, B.nc[1] - y0) + 1;
    const int hze = min(kTileZ, B.nc[2] - z0) + 1;
    const bool box_dense = w.dense_cap > 0 && w.dense_threshold >= 0 && B.dense_ok;
    const int t = threadIdx.x;

    int cnt_local[kPerT];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kPerT; ++k) {
        const int h = t * kPerT + k;
        int cnt = 0;
        if (h < kHalo) {
            const int hz = h % kHZ, row = h / kHZ, hy = row % kHY, hx = row / kHY;
            int tag = -1, s = 0;
            if (hx <= hxe && hy <= hye && hz <= hze) {
                const int64_t c = coarse_cell(B, mod_cell(x0 - 1 + hx, B.nc[0]),
                                              mod_cell(y0 - 1 + hy, B.nc[1]),
                                              mod_cell(z0 - 1 + hz, B.nc[2]));
                s = w.cell_start[c];
                cnt = w.cell_start[c + 1] - s;
                if (box_dense && cnt > w.dense_threshold && w.cell_count[c] >= 0) {
                    tag = w.cell_count[c];
                    cnt = 0;
                }
            }
            gst[h] = s;
            htag[h] = tag;
        }
        cnt_local[k] = cnt;
        sum += cnt;
    }
    {  // exclusive scan of staged counts; each thread owns kPerT consecutive halo cells
        const int lane = lane_id(), wid = t / kWave;
        int x = sum;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            int y = __shfl_up(x, o, kWave);
            if (lane >= o)
                x += y;
        }
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
    }
    __syncthreads();
    if (t <= kOwnRows) {  // own particles before each own row
        int acc = 0;
        for (int r = 0; r < t; ++r) {
            const int hx = 1 + r / kTileY, hy = 1 + r % kTileY;
            const int rb = (hx * kHY + hy) * kHZ;
            if (hx <= hxe - 1 && hy <= hye - 1)
                acc += hoff[rb + hze] - hoff[rb + 1];
        }
        ownoff[t] = acc;
    }
    const int total = hoff[kHalo];
    const bool staged = total <= kTileCap;
    if (t == 0) {
        FOF_STAT(w.ctr, ST_TILES, 1);
        if (!staged)
            FOF_STAT(w.ctr, ST_TILES_OVERFLOW, 1);
    }
    if (staged) {
        int src[kStagePerT];
#pragma unroll
        for (int k = 0; k < kStagePerT; ++k) {
            const int sl = t + k * kTileBlock;
            src[k] = -1;
            if (sl < total) {
                const int h = halo_cell_of(hoff, sl);
                src[k] = gst[h] + (sl - hoff[h]);
            }
        }
        float4 v[kStagePerT];
#pragma unroll
        for (int k = 0; k < kStagePerT; ++k)
            if (src[k] >= 0)
                v[k] = w.sorted[src[k]];
#pragma unroll
        for (int k = 0; k < kStagePerT; ++k)
            if (src[k] >= 0)
                part[t + k * kTileBlock] = v[k];
    }
    __syncthreads();

    const int nown = ownoff[kOwnRows];
    if (t == 0)
        FOF_STAT(w.ctr, staged ? ST_OWN_STAGED : ST_OWN_GLOBAL, nown);
    for (int k = t; k < nown; k += kTileBlock) {
        int r = 0;
        while (ownoff[r + 1] <= k)
            ++r;
        const int rhx = 1 + r / kTileY, rhy = 1 + r % kTileY;
        const int slot = hoff[(rhx * kHY + rhy) * kHZ + 1] + (k - ownoff[r]);
        const int hs = halo_cell_of(hoff, slot);
        const int64_t i = gst[hs] + (slot - hoff[hs]);
        const float4 p = staged ? part[slot] : w.sorted[i];
        const int32_t oi = __float_as_int(p.w);
        const int ix = fine_index(p.x, B.inv_fine[0], B.nf[0]) / B.m;
        const int iy = fine_index(p.y, B.inv_fine[1], B.nf[1]) / B.m;
        const int iz = fine_index(p.z, B.inv_fine[2], B.nf[2]) / B.m;
        if (!staged) {
            finish_particle(w, root, i, oi, link_particle_global(w, B, i, p, ix, iy, iz));
            continue;
        }
        const int hx = ix - x0 + 1, hy = iy - y0 + 1, hz = iz - z0 + 1;
        bool has_friend = false;
        const AxisSpan sx = axis_span(p.x, ix, B.side[0], B.nc[0], B.reach);
        const AxisSpan sy = axis_span(p.y, iy, B.side[1], B.nc[1], B.reach);
        const AxisSpan sz = axis_span(p.z, iz, B.side[2], B.nc[2], B.reach);
        for (int ox = sx.lo; ox <= sx.hi; ++ox)
            for (int oy = sy.lo; oy <= sy.hi; ++oy) {
                const int rb = ((hx + ox) * kHY + hy + oy) * kHZ;
                const int a = hoff[rb + hz + sz.lo], e = hoff[rb + hz + sz.hi + 1];
                FOF_STAT(w.ctr, ST_PAIRS_TILED, e - a);
                for (int j = a; j < e; ++j) {
                    if (j == slot)
                        continue;
                    const float4 q4 = part[j];
                    if (linked(B, p.x, p.y, p.z, q4.x, q4.y, q4.z)) {
                        has_friend = true;
                        if (oi < __float_as_int(q4.w)) {  // each pair hooked from one end
                            const int hj = halo_cell_of(hoff, j);
                            uf_union(w.parent, (uint32_t)i, (uint32_t)(gst[hj] + (j - hoff[hj])));
                        }
                    }
                }
                if (box_dense)
                    for (int oz = sz.lo; oz <= sz.hi; ++oz) {
                        const int tag = htag[rb + hz + oz];
                        if (tag < 0)
                            continue;
                        const int64_t c2 = coarse_cell(B, wrap_cell(ix + ox, B.nc[0]),
                                                       wrap_cell(iy + oy, B.nc[1]),
                                                       wrap_cell(iz + oz, B.nc[2]));
                        const int32_t s2 = gst[rb + hz + oz];
                        has_friend |= link_dense_neighbour(w, B, (uint32_t)i, p, ix, iy, iz, ox, oy,
                                                           oz, s2, w.cell_start[c2 + 1] - s2, tag);
                    }
            }
        finish_particle(w, root, i, oi, has_friend);
    }
}

// Particles with a friend: follow the union-find to the root and write the root's key
// (its original index, the smallest in the component) as the label.  Also leaves every
// flagged entry pointing straight at its root for the group passes.  The lookup must not
// halve paths: a halving write by one thread could replace the root another thread has
// just stored in its own entry with a stale grandparent.
__global__ void k_compress(const float4 *__restrict__ sorted, int64_t n,
                           uint64_t *__restrict__ parent, const uint64_t *__restrict__ flags,
                           int32_t *__restrict__ root)
{
    const int64_t i = gtid_xcd();
    if (i >= n)
        return;
    if (!((flags[i >> 6] >> (i & 63)) & 1ull))
        return;
    const uint64_t r = uf_find_ro(parent, (uint32_t)i);
    st_relaxed(parent + i, r);
    root[__float_as_int(sorted[i].w)] = (int32_t)uf_key(r);
}

}  // namespace

hipError_t launch_link(const Work &w, int32_t *root, hipStream_t s)
{
    if (w.n <= 0)
        return hipSuccess;
    hipError_t e = launch_fill_u64(w.flags, (w.n + 63) / 64, 0ull, s);
    if (e != hipSuccess)
        return e;
    e = launch_dense(w, s);
    if (e != hipSuccess)
        return e;
    const unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
    if (w.ntiles > 0)
        hipLaunchKernelGGL(k_link_tiled, dim3((unsigned)w.ntiles), dim3(kTileBlock), 0, s, w,
                           root);
    hipLaunchKernelGGL(k_link, dim3(nb), dim3(w.block), 0, s, w, root);
    hipLaunchKernelGGL(k_compress, dim3(nb), dim3(w.block), 0, s, w.sorted, w.n, w.parent,
                       w.flags, root);
    return hipGetLastError();
}

}  // namespace fof
