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

__global__ void k_link(Work w, int32_t *__restrict__ root)
{
    const int64_t i = gtid();
    const bool dense_on = w.dense_cap > 0 && w.dense_threshold >= 0;
    bool has_friend = false;
    if (i < w.n) {
        const BoxDesc &B = w.desc[find_box(w.desc, w.nbox, i)];
        const float4 p = w.sorted[i];
        const int ix = fine_index(p.x, B.inv_fine[0], B.nf[0]) / B.m;
        const int iy = fine_index(p.y, B.inv_fine[1], B.nf[1]) / B.m;
        const int iz = fine_index(p.z, B.inv_fine[2], B.nf[2]) / B.m;
        const bool box_dense = dense_on && B.dense_ok;
        bool own_dense = false;
        if (box_dense) {
            const int64_t c0 = coarse_cell(B, ix, iy, iz);
            own_dense = w.cell_start[c0 + 1] - w.cell_start[c0] > w.dense_threshold &&
                        w.cell_count[c0] >= 0;
        }
        if (own_dense) {
            has_friend = true;  // linked by the dense kernels, resolved by compress
        } else {
            const AxisSpan sx = axis_span(p.x, ix, B.side[0], B.nc[0], B.reach);
            const AxisSpan sy = axis_span(p.y, iy, B.side[1], B.nc[1], B.reach);
            const AxisSpan sz = axis_span(p.z, iz, B.side[2], B.nc[2], B.reach);
            for (int oz = sz.lo; oz <= sz.hi; ++oz) {
                const int cz = wrap_cell(iz + oz, B.nc[2]);
                for (int oy = sy.lo; oy <= sy.hi; ++oy) {
                    const int cy = wrap_cell(iy + oy, B.nc[1]);
                    for (int ox = sx.lo; ox <= sx.hi; ++ox) {
                        const int cx = wrap_cell(ix + ox, B.nc[0]);
                        const int64_t c = coarse_cell(B, cx, cy, cz);
                        const int32_t s = w.cell_start[c], e = w.cell_start[c + 1];
                        if (box_dense && e - s > w.dense_threshold) {
                            const int32_t d2 = w.cell_count[c];
                            if (d2 >= 0) {
                                has_friend |= link_dense_neighbour(w, B, (uint32_t)i, p, ix, iy,
                                                                   iz, ox, oy, oz, s, e - s, d2);
                                continue;
                            }
                        }
                        for (int32_t j = s; j < e; ++j) {
                            if (j == i)
                                continue;
                            const float4 q = w.sorted[j];
                            if (linked(B, p.x, p.y, p.z, q.x, q.y, q.z)) {
                                has_friend = true;
                                if (i < j)
                                    uf_union(w.parent, (uint32_t)i, (uint32_t)j);
                            }
                        }
                    }
                }
            }
        }
        if (!has_friend)
            root[__float_as_int(p.w)] = __float_as_int(p.w);
    }
    const uint64_t m = ballot(has_friend);
    if (lane_id() == 0 && i < w.n)
        w.flags[i >> 6] = m;
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
    const int64_t i = gtid();
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
    hipError_t e = launch_dense(w, s);
    if (e != hipSuccess)
        return e;
    const unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
    hipLaunchKernelGGL(k_link, dim3(nb), dim3(w.block), 0, s, w, root);
    hipLaunchKernelGGL(k_compress, dim3(nb), dim3(w.block), 0, s, w.sorted, w.n, w.parent,
                       w.flags, root);
    return hipGetLastError();
}

}  // namespace fof
