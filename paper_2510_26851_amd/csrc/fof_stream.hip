// Streaming (bounded-workspace) labelling of one box in z-slabs (paper Sec. 2.3: the box is
// cut into slabs, each slab is linked together with a ghost layer of its neighbours'
// particles, and the components that share a particle are fused into global groups).
//
// Slab k owns the particles with k L/S <= z < (k + 1) L/S (S slabs, z in double).  Its
// ghosts are the particles of the two neighbouring slabs (periodically) closer than g to
// the shared face, g >= b.  A friend pair has |dz| < b, so either both ends are owned by
// one slab or one end is a ghost of the other's slab: every friend pair is linked in some
// slab.  Each slab is an ordinary periodic box of the full lengths holding only those
// particles (the predicate sees the original coordinates, so every link it finds is a true
// link), planned on the same cell grid as the whole box.  Its labels (smallest slab index
// of the component) are fused into the global labels: for every slab particle, its original
// index and the original index of its slab label are merged in one union-find over the
// output array, whose roots only move to smaller indices, so the final root of a particle is
// the smallest original index of its global component.
//
//   k_slab_count        members of every slab (own + ghost), one atomic per block and slab
//   k_slab_chunk_count  members of slab k per chunk of the input
//   scan                chunk offsets
//   k_slab_gather       members of slab k, in ascending original index: positions and the
//                       map slab index -> original index
//   (fof_build_grid + fof_link on the slab)
//   k_slab_fuse         union of (original index, original index of the slab label)
//   k_fuse_final        root[i] = final root
#include "fof_internal.h"

namespace fof {

namespace {

constexpr int kSlabBlock = 256;
constexpr int kSlabChunk = 4096;  // particles per gather block
constexpr int kSlabPer = kSlabChunk / kSlabBlock;
constexpr int kMaxSlabs = 4096;

// Slab membership of a particle at height z (in double): its own slab, and whether it is a
// ghost of the slab above (own + 1 mod S) or of the slab below (own - 1 mod S).
struct SlabOf {
    int own;
    bool up, down;
};

__device__ __forceinline__ SlabOf slab_of(const SlabGeom &G, float zf)
{
    const double z = (double)zf;
    int k = (int)floor(z * (double)G.nslab / G.Lz);
    k = k < 0 ? 0 : (k >= G.nslab ? G.nslab - 1 : k);
    const double lo = (double)k * G.width, hi = (double)(k + 1) * G.width;
    SlabOf s;
    s.own = k;
    s.up = G.nslab > 1 && hi - z < G.ghost;
    s.down = G.nslab > 1 && z - lo < G.ghost;
    return s;
}

__device__ __forceinline__ bool in_slab(const SlabGeom &G, float z, int k)
{
    const SlabOf s = slab_of(G, z);
    const int S = G.nslab;
    return s.own == k || (s.up && (s.own + 1) % S == k) || (s.down && (s.own - 1 + S) % S == k);
}

__global__ __launch_bounds__(kSlabBlock) void k_slab_count(const float *__restrict__ pos,
                                                           int64_t n, SlabGeom G,
                                                           int64_t *__restrict__ counts)
{
    __shared__ int32_t lc[kMaxSlabs];
    for (int k = threadIdx.x; k < G.nslab; k += kSlabBlock)
        lc[k] = 0;
    __syncthreads();
    const int S = G.nslab;
    for (int64_t i = (int64_t)blockIdx.x * kSlabBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kSlabBlock) {
        const SlabOf s = slab_of(G, pos[3 * i + 2]);
        atomicAdd(lc + s.own, 1);
        if (s.up)
            atomicAdd(lc + (s.own + 1) % S, 1);
        if (s.down)
            atomicAdd(lc + (s.own - 1 + S) % S, 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < S; k += kSlabBlock)
        if (lc[k])
            atomicAdd((unsigned long long *)(counts + k), (unsigned long long)lc[k]);
}

// Block-wide exclusive scan of one int per thread.
__device__ int32_t slab_block_scan(int32_t v, int32_t *total)
{
    __shared__ int32_t wsum[kSlabBlock / kWave];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t y = __shfl_up(x, o, kWave);
        if (lane >= o)
            x += y;
    }
    if (lane == kWave - 1)
        wsum[wid] = x;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int k = 0; k < kSlabBlock / kWave; ++k) {
        if (k < wid)
            pre += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

// Members of slab k in each chunk of kSlabChunk input particles; thread t owns the chunk's
// particles t * kSlabPer .. (t + 1) * kSlabPer - 1, so the gather keeps input order.
__global__ __launch_bounds__(kSlabBlock) void k_slab_chunk_count(const float *__restrict__ pos,
                                                                 int64_t n, SlabGeom G, int k,
                                                                 int32_t *__restrict__ ccount)
{
    const int64_t base = (int64_t)blockIdx.x * kSlabChunk + (int64_t)threadIdx.x * kSlabPer;
    int32_t c = 0;
#pragma unroll
    for (int q = 0; q < kSlabPer; ++q) {
        const int64_t i = base + q;
        if (i < n && in_slab(G, pos[3 * i + 2], k))
            ++c;
    }
    int32_t tot;
    slab_block_scan(c, &tot);
    if (threadIdx.x == 0)
        ccount[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kSlabBlock) void k_slab_gather(const float *__restrict__ pos,
                                                            int64_t n, SlabGeom G, int k,
                                                            const int32_t *__restrict__ coff,
                                                            int64_t cap, float *__restrict__ spos,
                                                            int32_t *__restrict__ map,
                                                            int32_t *__restrict__ status)
{
    const int64_t base = (int64_t)blockIdx.x * kSlabChunk + (int64_t)threadIdx.x * kSlabPer;
    uint32_t mine = 0;
    int32_t c = 0;
#pragma unroll
    for (int q = 0; q < kSlabPer; ++q) {
        const int64_t i = base + q;
        if (i < n && in_slab(G, pos[3 * i + 2], k)) {
            mine |= 1u << q;
            ++c;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && (int64_t)coff[gridDim.x] != cap)
        atomicOr(status, (int32_t)FOF_STATUS_SLAB_CAP);  // counts[k] was not this slab's size
    int32_t tot;
    int64_t s = (int64_t)coff[blockIdx.x] + slab_block_scan(c, &tot);
#pragma unroll
    for (int q = 0; q < kSlabPer; ++q) {
        if (!((mine >> q) & 1u))
            continue;
        const int64_t i = base + q;
        if (s < cap) {
            spos[3 * s + 0] = pos[3 * i + 0];
            spos[3 * s + 1] = pos[3 * i + 1];
            spos[3 * s + 2] = pos[3 * i + 2];
            map[s] = (int32_t)i;
        } else {
            atomicOr(status, (int32_t)FOF_STATUS_SLAB_CAP);
        }
        ++s;
    }
}

// Union-find over the int32 output array: parent[x] <= x, roots only move to smaller
// indices (compare-and-swap of a root), halving writes only non-root entries.
__device__ __forceinline__ int32_t find32(int32_t *P, int32_t x)
{
    for (;;) {
        const int32_t p = __hip_atomic_load(P + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p == x)
            return x;
        const int32_t g = __hip_atomic_load(P + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (g == p)
            return p;
        __hip_atomic_store(P + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = g;
    }
}

__device__ __forceinline__ void union32(int32_t *P, int32_t a, int32_t b)
{
    for (;;) {
        a = find32(P, a);
        b = find32(P, b);
        if (a == b)
            return;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(P + b, b, a) == b)
            return;
    }
}

// The slab's labels into the global forest.  map entries past the slab's true member count
// hold -1 (filled before the gather) and are skipped.
__global__ void k_slab_fuse(const int32_t *__restrict__ map, const int32_t *__restrict__ sroot,
                            int64_t m, int32_t *__restrict__ root)
{
    for (int64_t s = gtid(); s < m; s += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = sroot[s];
        if (r == (int32_t)s || r < 0 || r >= m)
            continue;
        const int32_t a = map[s], b = map[r];
        if (a >= 0 && b >= 0)
            union32(root, a, b);
    }
}

__global__ void k_fuse_init(int32_t *__restrict__ root, int64_t n)
{
    for (int64_t i = gtid(); i < n; i += (int64_t)gridDim.x * blockDim.x)
        root[i] = (int32_t)i;
}

// After every union: each entry points at its root (a reader that meets an entry already
// rewritten sees the root, still an ancestor).
__global__ void k_fuse_final(int32_t *__restrict__ root, int64_t n)
{
    for (int64_t i = gtid(); i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t x = (int32_t)i;
        int32_t p = __hip_atomic_load(root + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (p != x) {
            x = p;
            p = __hip_atomic_load(root + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __hip_atomic_store(root + i, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_zero_i64(int64_t *__restrict__ p, int64_t n)
{
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        p[i] = 0;
}

// The slab run's status bits into the stream's own status word.
__global__ void k_or_status(const Counters *__restrict__ from, int32_t *__restrict__ to)
{
    if (threadIdx.x == 0 && from->status)
        atomicOr(to, from->status);
}

unsigned grid_for(int64_t n, int per_block)
{
    int64_t b = (n + per_block - 1) / per_block;
    b = b < 1 ? 1 : (b > 65536 ? 65536 : b);
    return (unsigned)b;
}

}  // namespace

int64_t slab_chunks(int64_t n) { return (n + kSlabChunk - 1) / kSlabChunk; }
int slab_max() { return kMaxSlabs; }

hipError_t launch_slab_count(const float *pos, int64_t n, const SlabGeom &G, int64_t *counts,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(256), 0, s, counts, (int64_t)G.nslab);
    if (n > 0)
        hipLaunchKernelGGL(k_slab_count, dim3(grid_for(n, kSlabBlock * 16)), dim3(kSlabBlock), 0,
                           s, pos, n, G, counts);
    return hipGetLastError();
}

hipError_t launch_slab_gather(const float *pos, int64_t n, const SlabGeom &G, int k,
                              int32_t *ccount, int32_t *coff, int32_t *scan_scratch, int64_t cap,
                              float *spos, int32_t *map, int32_t *status, hipStream_t s)
{
    const int64_t nch = slab_chunks(n);
    hipError_t e = launch_fill_i32(map, cap, -1, s);
    if (e != hipSuccess || n <= 0)
        return e;
    hipLaunchKernelGGL(k_slab_chunk_count, dim3((unsigned)nch), dim3(kSlabBlock), 0, s, pos, n, G,
                       k, ccount);
    if ((e = launch_scan_i32(ccount, coff, nch, scan_scratch, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_slab_gather, dim3((unsigned)nch), dim3(kSlabBlock), 0, s, pos, n, G, k,
                       coff, cap, spos, map, status);
    return hipGetLastError();
}

hipError_t launch_fuse_init(int32_t *root, int64_t n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_fuse_init, dim3(grid_for(n, 1024)), dim3(256), 0, s, root, n);
    return hipGetLastError();
}

hipError_t launch_slab_fuse(const int32_t *map, const int32_t *sroot, int64_t m, int32_t *root,
                            hipStream_t s)
{
    if (m > 0)
        hipLaunchKernelGGL(k_slab_fuse, dim3(grid_for(m, 1024)), dim3(256), 0, s, map, sroot, m,
                           root);
    return hipGetLastError();
}

hipError_t launch_or_status(const Counters *from, int32_t *to, hipStream_t s)
{
    hipLaunchKernelGGL(k_or_status, dim3(1), dim3(64), 0, s, from, to);
    return hipGetLastError();
}

hipError_t launch_fuse_final(int32_t *root, int64_t n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_fuse_final, dim3(grid_for(n, 1024)), dim3(256), 0, s, root, n);
    return hipGetLastError();
}

}  // namespace fof
