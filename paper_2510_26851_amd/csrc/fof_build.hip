// Cell binning as a counting sort (paper Alg. 2: cell indexing with x fastest, then the
// particles sorted by cell).  Three steps:
//   count    validate the coordinate, compute the coarse cell, take a rank inside the cell
//            with one atomic increment of the cell counter;
//   scan     exclusive scan of the counters gives cell_start;
//   scatter  sorted[cell_start[c] + rank] = (x, y, z, original index), and the union-find
//            entry of that sorted slot is initialised to itself.
// Within a cell the order is whatever the atomics produced; no result depends on it.
#include "fof_internal.h"

namespace fof {

namespace {

struct CellOf {
    int64_t cell;
    bool ok;
};

// Coarse cell of a particle.  Invalid coordinates (NaN, negative, >= L) are replaced by 0 in
// place, so every later kernel sees in-range positions; the status word reports them.
__device__ __forceinline__ CellOf cell_of(const BoxDesc &B, float &x, float &y, float &z)
{
    // Valid coordinates are finite and 0 <= x < L, compared in double (NaN fails).
    bool ok = ((double)x >= 0.0) & ((double)x < B.L[0]) & ((double)y >= 0.0) &
              ((double)y < B.L[1]) & ((double)z >= 0.0) & ((double)z < B.L[2]);
    if (!ok) {  // keep the index in range; the status word reports the bad input
        x = (x >= 0.0f && x < (float)B.L[0]) ? x : 0.0f;
        y = (y >= 0.0f && y < (float)B.L[1]) ? y : 0.0f;
        z = (z >= 0.0f && z < (float)B.L[2]) ? z : 0.0f;
    }
    int ix = fine_index(x, B.inv_fine[0], B.nf[0]) / B.m;
    int iy = fine_index(y, B.inv_fine[1], B.nf[1]) / B.m;
    int iz = fine_index(z, B.inv_fine[2], B.nf[2]) / B.m;
    return {coarse_cell(B, ix, iy, iz), ok};
}

__global__ void k_count(const float *__restrict__ pos, int64_t n, const BoxDesc *__restrict__ desc,
                        int nbox, int32_t *__restrict__ cell_count, int32_t *__restrict__ rank,
                        Counters *__restrict__ ctr)
{
    int64_t i = gtid();
    if (i >= n)
        return;
    const BoxDesc &B = desc[find_box(desc, nbox, i)];
    float x = pos[3 * i + 0], y = pos[3 * i + 1], z = pos[3 * i + 2];
    CellOf c = cell_of(B, x, y, z);
    if (!c.ok)
        atomicOr(&ctr->status, (int32_t)FOF_STATUS_RANGE);
    rank[i] = atomicAdd(cell_count + c.cell, 1);
}

__global__ void k_scatter(const float *__restrict__ pos, int64_t n,
                          const BoxDesc *__restrict__ desc, int nbox,
                          const int32_t *__restrict__ cell_start, const int32_t *__restrict__ rank,
                          float4 *__restrict__ sorted, uint64_t *__restrict__ parent)
{
    int64_t i = gtid();
    if (i >= n)
        return;
    const BoxDesc &B = desc[find_box(desc, nbox, i)];
    float x = pos[3 * i + 0], y = pos[3 * i + 1], z = pos[3 * i + 2];
    CellOf c = cell_of(B, x, y, z);
    int32_t dst = cell_start[c.cell] + rank[i];
    sorted[dst] = make_float4(x, y, z, __int_as_float((int32_t)i));
    parent[dst] = ((uint64_t)(uint32_t)i << 32) | (uint32_t)dst;
}

__global__ void k_clear_counters(Counters *ctr)
{
    if (threadIdx.x < sizeof(Counters) / sizeof(int32_t))
        ((int32_t *)ctr)[threadIdx.x] = 0;
}

}  // namespace

hipError_t launch_build(const Work &w, const float *pos, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(64), 0, s, w.ctr);
    hipError_t e = launch_fill_i32(w.cell_count, w.ncell, 0, s);
    if (e != hipSuccess)
        return e;
    if (w.n > 0) {
        unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
        hipLaunchKernelGGL(k_count, dim3(nb), dim3(w.block), 0, s, pos, w.n, w.desc, w.nbox,
                           w.cell_count, w.rank, w.ctr);
    }
    e = launch_scan_i32(w.cell_count, w.cell_start, w.ncell, w.scan, s);
    if (e != hipSuccess)
        return e;
    if (w.n > 0) {
        unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
        hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(w.block), 0, s, pos, w.n, w.desc, w.nbox,
                           w.cell_start, w.rank, w.sorted, w.parent);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        return launch_dense_build(w, s);
    }
    return hipGetLastError();
}

}  // namespace fof
