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

__global__ void k_link(const float4 *__restrict__ sorted, int64_t n,
                       const BoxDesc *__restrict__ desc, int nbox,
                       const int32_t *__restrict__ cell_start, uint64_t *__restrict__ parent,
                       uint64_t *__restrict__ flags, int32_t *__restrict__ root)
{
    const int64_t i = gtid();
    bool has_friend = false;
    if (i < n) {
        const BoxDesc &B = desc[find_box(desc, nbox, i)];
        const float4 p = sorted[i];
        const int ix = fine_index(p.x, B.inv_fine[0], B.nf[0]) / B.m;
        const int iy = fine_index(p.y, B.inv_fine[1], B.nf[1]) / B.m;
        const int iz = fine_index(p.z, B.inv_fine[2], B.nf[2]) / B.m;
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
                    const int32_t s = cell_start[c], e = cell_start[c + 1];
                    for (int32_t j = s; j < e; ++j) {
                        if (j == i)
                            continue;
                        const float4 q = sorted[j];
                        if (linked(B, p.x, p.y, p.z, q.x, q.y, q.z)) {
                            has_friend = true;
                            if (i < j)
                                uf_union(parent, (uint32_t)i, (uint32_t)j);
                        }
                    }
                }
            }
        }
        if (!has_friend)
            root[__float_as_int(p.w)] = __float_as_int(p.w);
    }
    const uint64_t m = ballot(has_friend);
    if (lane_id() == 0 && i < n)
        flags[i >> 6] = m;
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
    const unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
    hipLaunchKernelGGL(k_link, dim3(nb), dim3(w.block), 0, s, w.sorted, w.n, w.desc, w.nbox,
                       w.cell_start, w.parent, w.flags, root);
    hipLaunchKernelGGL(k_compress, dim3(nb), dim3(w.block), 0, s, w.sorted, w.n, w.parent,
                       w.flags, root);
    return hipGetLastError();
}

}  // namespace fof
