// Cell binning as a counting sort (paper Alg. 2: cell indexing, then the particles sorted
// by cell).
//
// Bucketed form (every grid of up to kBinMaxBuckets << kBinMaxShift cells).  Cells are
// grouped into buckets of 2^shift consecutive ids; G blocks each own one contiguous chunk of
// the input.  No global atomics:
//   k_bin_count  per block, an LDS histogram of its particles over buckets (also validates
//                the coordinates), written out as column g of a [bucket][block] table;
//   scan         exclusive scan of the table: where each block's share of each bucket goes;
//   k_bin_place  per block, LDS cursors from the scanned table; every particle goes, as
//                (x, y, z, input index), to its bucket's slot of the staging array;
//   k_bin_sort   one block per bucket: reads its particles (coalesced, into registers),
//                counts them per cell in LDS, scans (cell_start of the bucket's cells), then
//                writes sorted[dst] and the union-find entry of dst, all inside the bucket's
//                own stretch of the output.
// Particles stored in lattice order land in few buckets per block, so the staging writes and
// the final scatter stay local, whatever the displacement of each particle from its cell.
//
// Grids with more cells than 16384 sorting buckets hold (a 1024^3 box) take one more pass:
// the placed buckets are larger, and k_bin_split cuts each into its sorting buckets.
//
// Per-particle form (still larger grids, or few particles on a huge grid): one atomic
// increment per particle gives its rank in the cell, a scan gives cell_start, and a
// scatter writes the sorted copy.
//
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
    // Valid coordinates are 0 <= x < L (NaN fails).  For a float x, x < L holds exactly when
    // x < Lup, the smallest float >= L, so the test needs no double arithmetic.
    const bool okx = (x >= 0.0f) & (x < B.Lup[0]);
    const bool oky = (y >= 0.0f) & (y < B.Lup[1]);
    const bool okz = (z >= 0.0f) & (z < B.Lup[2]);
    x = okx ? x : 0.0f;
    y = oky ? y : 0.0f;
    z = okz ? z : 0.0f;
    int ix = coarse_index(x, B, 0);
    int iy = coarse_index(y, B, 1);
    int iz = coarse_index(z, B, 2);
    return {coarse_cell(B, ix, iy, iz), okx && oky && okz};
}

// Calls f with the descriptor of particle i's box.  When every active lane of the wave lies
// in the box of the wave's first active lane (the usual case), that descriptor is found and
// read with scalar loads; otherwise each lane searches for its own.
template <class F>
__device__ __forceinline__ void with_box(const BoxDesc *__restrict__ desc, int nbox, int64_t i,
                                         F &&f)
{
    const int64_t i0 =
        (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(i >> 32)) << 32) |
                  (uint32_t)__builtin_amdgcn_readfirstlane((int)i));
    const BoxDesc &B0 = desc[find_box(desc, nbox, i0)];
    if (ballot(i < B0.off || i >= B0.off + B0.n) == 0)
        f(B0);
    else
        f(desc[find_box(desc, nbox, i)]);
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

constexpr int kBinBlock = 1024;  // k_bin_count / k_bin_place
constexpr int kSortBlock = 1024;  // k_bin_sort
constexpr int kSortPer = 16;     // particles per k_bin_sort thread held in registers

constexpr int kBinUnroll = 4;  // particles per thread whose loads are issued together

// Positions of particles r + threadIdx.x + u * kBinBlock (u < kBinUnroll) below i1, loaded
// before any is used, so that each thread keeps several loads in flight.
struct BinBatch {
    float x[kBinUnroll], y[kBinUnroll], z[kBinUnroll];
};

__device__ __forceinline__ BinBatch load_batch(const float *__restrict__ pos, int64_t r,
                                               int64_t i1)
{
    BinBatch q;
#pragma unroll
    for (int u = 0; u < kBinUnroll; ++u) {
        const int64_t i = r + threadIdx.x + (int64_t)u * kBinBlock;
        if (i < i1) {
            q.x[u] = pos[3 * i + 0];
            q.y[u] = pos[3 * i + 1];
            q.z[u] = pos[3 * i + 2];
        }
    }
    return q;
}

// Adds one to LDS counter k for every active lane and returns each lane's value before its
// own increment.  Particles stored in lattice order put a whole wave in one bucket: then a
// single atomic serves the wave (the lanes of one address would otherwise serialise);
// otherwise every lane does its own.
__device__ __forceinline__ int32_t wave_lds_inc(int32_t *cnt, int k)
{
    const uint64_t act = __ballot(true);
    const int k0 = __builtin_amdgcn_readfirstlane(k);
    if (__ballot(k == k0) == act) {
        const int lane = lane_id();
        const int first = __ffsll((unsigned long long)act) - 1;
        int32_t base = 0;
        if (lane == first)
            base = atomicAdd(cnt + k0, __popcll(act));
        base = __shfl(base, first, kWave);
        return base + __popcll(act & ((1ull << lane) - 1ull));
    }
    return atomicAdd(cnt + k, 1);
}

__global__ __launch_bounds__(kBinBlock) void k_bin_count(const float *__restrict__ pos,
                                                         const BoxDesc *__restrict__ desc,
                                                         int nbox, int64_t n, BinShape bs,
                                                         int32_t *__restrict__ hist,
                                                         Counters *__restrict__ ctr)
{
    extern __shared__ int32_t lh[];  // bs.nbk counters
    for (int64_t k = threadIdx.x; k < bs.nbk; k += kBinBlock)
        lh[k] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * bs.chunk;
    const int64_t i1 = i0 + bs.chunk < n ? i0 + bs.chunk : n;
    bool bad = false;
    for (int64_t r = i0; r < i1; r += (int64_t)kBinBlock * kBinUnroll) {
        BinBatch q = load_batch(pos, r, i1);
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u) {
            const int64_t i = r + threadIdx.x + (int64_t)u * kBinBlock;
            if (i < i1)
                with_box(desc, nbox, i, [&](const BoxDesc &B) {
                    const CellOf c = cell_of(B, q.x[u], q.y[u], q.z[u]);
                    bad |= !c.ok;
                    wave_lds_inc(lh, (int)(c.cell >> bs.shift));
                });
        }
    }
    if (bad)
        atomicOr(&ctr->status, (int32_t)FOF_STATUS_RANGE);
    __syncthreads();
    for (int64_t k = threadIdx.x; k < bs.nbk; k += kBinBlock)
        hist[k * bs.G + blockIdx.x] = lh[k];
}

__global__ __launch_bounds__(kBinBlock) void k_bin_place(const float *__restrict__ pos,
                                                         const BoxDesc *__restrict__ desc,
                                                         int nbox, int64_t n, BinShape bs,
                                                         const int32_t *__restrict__ off,
                                                         float4 *__restrict__ stage)
{
    extern __shared__ int32_t cur[];  // bs.nbk cursors
    for (int64_t k = threadIdx.x; k < bs.nbk; k += kBinBlock)
        cur[k] = off[k * bs.G + blockIdx.x];
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * bs.chunk;
    const int64_t i1 = i0 + bs.chunk < n ? i0 + bs.chunk : n;
    for (int64_t r = i0; r < i1; r += (int64_t)kBinBlock * kBinUnroll) {
        BinBatch q = load_batch(pos, r, i1);
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u) {
            const int64_t i = r + threadIdx.x + (int64_t)u * kBinBlock;
            if (i < i1)
                with_box(desc, nbox, i, [&](const BoxDesc &B) {
                    const CellOf c = cell_of(B, q.x[u], q.y[u], q.z[u]);
                    stage[wave_lds_inc(cur, (int)(c.cell >> bs.shift))] =
                        make_float4(q.x[u], q.y[u], q.z[u], __int_as_float((int32_t)i));
                });
        }
    }
}

// Exclusive scan of one int per thread over a kSortBlock-thread block.
__device__ __forceinline__ int32_t sort_block_scan(int32_t v, int32_t *wsum)
{
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
    int32_t pre = 0;
    for (int k = 0; k < wid; ++k)
        pre += wsum[k];
    __syncthreads();
    return pre + x - v;
}

// Exclusive scan of one int per thread over a kSortBlock-thread block, with the total.
__device__ __forceinline__ int32_t sort_block_scan_total(int32_t v, int32_t *wsum, int32_t *total)
{
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int32_t x = wave_incl_sum(v);
    if (lane == kWave - 1)
        wsum[wid] = x;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int k = 0; k < kSortBlock / kWave; ++k) {
        pre += k < wid ? wsum[k] : 0;
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

// Where the sorting blocks put the dense-cell index (cells over the threshold, in boxes that
// allow clique tables): thr < 0 or cap == 0 means none.
struct DenseOut {
    int32_t thr, cap;
    int32_t *cell_count, *dense_list, *big_list;
    Counters *ctr;
};

// Cell of a staged particle relative to the bucket's first cell (coordinates were already
// made valid by the placing pass, so this is the cell that pass used).
__device__ __forceinline__ int staged_cell(const BoxDesc *__restrict__ desc, int nbox,
                                           float4 p, int64_t c0)
{
    int lc = 0;
    with_box(desc, nbox, __float_as_int(p.w), [&](const BoxDesc &B) {
        lc = (int)(cell_of(B, p.x, p.y, p.z).cell - c0);
    });
    return lc;
}

// LDS slot of a sorting bucket's cell counter: one pad word after every 32, so the scan's
// threads, each owning a run of consecutive cells, hit distinct banks.
__device__ __forceinline__ int lpad(int j) { return j + (j >> 5); }

// Dense cells among a thread's cells [j0, j1) of the bucket: ids from one atomic per block,
// in cell order inside it, and places in the big list for cells over kSmallCell.  A cell past
// the table capacity, or in a box without clique tables, gets -1 in cell_count.
__device__ void number_dense_cells(const DenseOut &dn, const BoxDesc *__restrict__ desc,
                                   int nbox, int64_t c0, const int32_t *lc, int j0, int j1,
                                   int32_t *wsum, int32_t *sbase)
{
    uint32_t dmask = 0;
    int a = 0;
    for (int j = j0; j < j1; ++j)
        if (lc[lpad(j)] > dn.thr) {
            if (desc[find_box_cell(desc, nbox, c0 + j)].dense_ok) {
                dmask |= 1u << (j - j0);
                ++a;
            } else {
                dn.cell_count[c0 + j] = -1;
            }
        }
    int32_t tot;
    int32_t d = sort_block_scan_total(a, wsum, &tot);
    if (threadIdx.x == 0)
        *sbase = tot ? atomicAdd(&dn.ctr->n_dense, tot) : 0;
    __syncthreads();
    d += *sbase;
    uint32_t bmask = 0;
    int nbig = 0;
    bool over = false;
    const int dfirst = d;
    for (uint32_t m = dmask; m; m &= m - 1u) {
        const int j = j0 + __ffs(m) - 1;
        if (d < dn.cap) {
            dn.cell_count[c0 + j] = d;
            dn.dense_list[d] = (int32_t)(c0 + j);
            if (lc[lpad(j)] > kSmallCell) {
                bmask |= 1u << (j - j0);
                ++nbig;
            }
        } else {
            dn.cell_count[c0 + j] = -1;
            over = true;
        }
        ++d;
    }
    if (over)
        atomicOr(&dn.ctr->status, (int32_t)FOF_STATUS_DENSE_CAP);
    __syncthreads();  // every thread has read sbase
    int32_t bg = sort_block_scan_total(nbig, wsum, &tot);
    if (threadIdx.x == 0)
        *sbase = tot ? atomicAdd(&dn.ctr->n_big, tot) : 0;
    __syncthreads();
    bg += *sbase;
    d = dfirst;
    for (uint32_t m = dmask; m; m &= m - 1u, ++d)
        if ((bmask >> (__ffs(m) - 1)) & 1u)
            dn.big_list[bg++] = d;
    __syncthreads();  // sbase is free again
}

// Sorting bucket b's particles are stage[bounds[b * stride], bounds[(b + 1) * stride]).
__global__ __launch_bounds__(kSortBlock) void k_bin_sort(const BoxDesc *__restrict__ desc,
                                                         int nbox, int64_t ncell, BinShape bs,
                                                         const int32_t *__restrict__ bounds,
                                                         int64_t stride,
                                                         const float4 *__restrict__ stage,
                                                         int32_t *__restrict__ cell_start,
                                                         float4 *__restrict__ sorted,
                                                         uint64_t *__restrict__ parent,
                                                         DenseOut dn)
{
    extern __shared__ int32_t lc[];  // per-cell counters, then cursors, at lpad(cell)
    __shared__ int32_t wsum[kSortBlock / kWave];
    __shared__ int32_t sbase;
    constexpr int64_t kCap = (int64_t)kSortBlock * kSortPer;
    const int64_t b = blockIdx.x;
    const int64_t c0 = b << bs.sshift;
    const int nc = (int)((c0 + (1ll << bs.sshift) < ncell ? (1ll << bs.sshift) : ncell - c0));
    const int64_t base = bounds[b * stride], end = bounds[(b + 1) * stride];
    for (int k = threadIdx.x; k < nc; k += kSortBlock)
        lc[lpad(k)] = 0;
    __syncthreads();
    // Items k0 + threadIdx.x + r * kSortBlock (r < kSortPer) of a chunk live in registers; a
    // bucket of at most kCap particles is read once, larger ones chunk by chunk, twice.
    float4 it[kSortPer];
    int cl[kSortPer];
    for (int64_t k0 = base; k0 < end; k0 += kCap) {
#pragma unroll
        for (int r = 0; r < kSortPer; ++r) {
            const int64_t k = k0 + threadIdx.x + (int64_t)r * kSortBlock;
            if (k < end)
                it[r] = stage[k];
        }
#pragma unroll
        for (int r = 0; r < kSortPer; ++r) {
            const int64_t k = k0 + threadIdx.x + (int64_t)r * kSortBlock;
            if (k < end) {
                cl[r] = staged_cell(desc, nbox, it[r], c0);
                atomicAdd(lc + lpad(cl[r]), 1);
            }
        }
    }
    __syncthreads();
    // thread t owns cells [t * per, (t + 1) * per) of the bucket (per <= 8)
    const int per = (nc + kSortBlock - 1) / kSortBlock;
    const int j0 = threadIdx.x * per;
    const int j1 = j0 + per < nc ? j0 + per : nc;
    if (dn.thr >= 0 && dn.cap > 0)  // uniform
        number_dense_cells(dn, desc, nbox, c0, lc, j0, j1, wsum, &sbase);
    // exclusive scan of the counts
    int32_t sum = 0;
    for (int j = j0; j < j1; ++j)
        sum += lc[lpad(j)];
    int32_t run = (int32_t)base + sort_block_scan(sum, wsum);
    for (int j = j0; j < j1; ++j) {
        const int32_t v = lc[lpad(j)];
        lc[lpad(j)] = run;
        run += v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nc; j += kSortBlock)
        cell_start[c0 + j] = lc[lpad(j)];
    if (c0 + nc == ncell && threadIdx.x == 0)
        cell_start[ncell] = (int32_t)end;
    __syncthreads();
    const bool one_chunk = end - base <= kCap;
    for (int64_t k0 = base; k0 < end; k0 += kCap) {
        if (!one_chunk) {
#pragma unroll
            for (int r = 0; r < kSortPer; ++r) {
                const int64_t k = k0 + threadIdx.x + (int64_t)r * kSortBlock;
                if (k < end) {
                    it[r] = stage[k];
                    cl[r] = staged_cell(desc, nbox, it[r], c0);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < kSortPer; ++r) {
            const int64_t k = k0 + threadIdx.x + (int64_t)r * kSortBlock;
            if (k < end) {
                const int32_t dst = atomicAdd(lc + lpad(cl[r]), 1);
                const uint32_t i = (uint32_t)__float_as_int(it[r].w);
                sorted[dst] = it[r];
                parent[dst] = ((uint64_t)i << 32) | (uint32_t)dst;
            }
        }
    }
}

// Two-level binning: placed bucket b (stage[off[b * G], off[(b + 1) * G])) is split into
// its 2^(shift - sshift) sorting buckets, counted in LDS, then copied into `out` by sorting
// bucket; the sorting buckets' bounds go to sub_off[b * nsplit + j] (and the total to
// sub_off[nbk * nsplit]).
constexpr int kSplitBlock = 1024;
constexpr int kSplitBatch = 4;

__global__ __launch_bounds__(kSplitBlock) void k_bin_split(const BoxDesc *__restrict__ desc,
                                                           int nbox, BinShape bs,
                                                           const int32_t *__restrict__ off,
                                                           const float4 *__restrict__ in,
                                                           float4 *__restrict__ out,
                                                           int32_t *__restrict__ sub_off)
{
    __shared__ int32_t cnt[1 << kBinMaxSplit];
    const int64_t b = blockIdx.x;
    const int nsplit = 1 << (bs.shift - bs.sshift);
    const int64_t base = off[b * bs.G], end = off[(b + 1) * bs.G];
    const int64_t c0 = b << bs.shift;
    if (threadIdx.x < nsplit)
        cnt[threadIdx.x] = 0;
    __syncthreads();
    // kSplitBatch loads in flight per thread in both sweeps
    for (int64_t k0 = base; k0 < end; k0 += (int64_t)kSplitBatch * kSplitBlock) {
        float4 p[kSplitBatch];
#pragma unroll
        for (int r = 0; r < kSplitBatch; ++r) {
            const int64_t k = k0 + threadIdx.x + (int64_t)r * kSplitBlock;
            if (k < end)
                p[r] = in[k];
        }
#pragma unroll
        for (int r = 0; r < kSplitBatch; ++r)
            if (k0 + threadIdx.x + (int64_t)r * kSplitBlock < end)
                wave_lds_inc(cnt, staged_cell(desc, nbox, p[r], c0) >> bs.sshift);
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // counts -> starts (at most 64 of them)
        int32_t run = (int32_t)base;
        for (int j = 0; j < nsplit; ++j) {
            const int32_t v = cnt[j];
            cnt[j] = run;
            sub_off[b * nsplit + j] = run;
            run += v;
        }
        if (b == bs.nbk - 1)
            sub_off[bs.nbk * nsplit] = run;
    }
    __syncthreads();
    for (int64_t k0 = base; k0 < end; k0 += (int64_t)kSplitBatch * kSplitBlock) {
        float4 p[kSplitBatch];
#pragma unroll
        for (int r = 0; r < kSplitBatch; ++r) {
            const int64_t k = k0 + threadIdx.x + (int64_t)r * kSplitBlock;
            if (k < end)
                p[r] = in[k];
        }
#pragma unroll
        for (int r = 0; r < kSplitBatch; ++r)
            if (k0 + threadIdx.x + (int64_t)r * kSplitBlock < end)
                out[wave_lds_inc(cnt, staged_cell(desc, nbox, p[r], c0) >> bs.sshift)] = p[r];
    }
}

__global__ void k_clear_counters(Counters *ctr)
{
    if (threadIdx.x < sizeof(Counters) / sizeof(int32_t))
        ((int32_t *)ctr)[threadIdx.x] = 0;
}

}  // namespace

// Dynamic LDS of k_bin_sort: one counter per cell of a sorting bucket, padded (lpad).
static size_t sort_lds(const BinShape &bs)
{
    const size_t nc = (size_t)1 << bs.sshift;
    return sizeof(int32_t) * (nc + nc / 32);
}

static DenseOut dense_out(const Work &w)
{
    DenseOut dn;
    dn.thr = w.dense_threshold;
    dn.cap = w.dense_cap;
    dn.cell_count = w.cell_count;
    dn.dense_list = w.dense_list;
    dn.big_list = w.big_list;
    dn.ctr = w.ctr;
    return dn;
}

hipError_t launch_build(const Work &w, const float *pos, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(64), 0, s, w.ctr);
    hipError_t e;
    if (w.n <= 0)  // every cell empty
        return launch_fill_i32(w.cell_start, w.ncell + 1, 0, s);
    const BinShape bs = bin_shape(w.n, w.ncell);
    if (bs.ok) {
        int32_t *hist = w.bin_hist, *off = w.bin_hist + bs.nbk * bs.G;
        const size_t lds_b = sizeof(int32_t) * (size_t)bs.nbk;
        hipLaunchKernelGGL(k_bin_count, dim3(bs.G), dim3(kBinBlock), lds_b, s, pos, w.desc,
                           w.nbox, w.n, bs, hist, w.ctr);
        e = launch_scan_i32(hist, off, bs.nbk * bs.G, w.scan, s);
        if (e != hipSuccess)
            return e;
        if (bs.shift == bs.sshift) {
            hipLaunchKernelGGL(k_bin_place, dim3(bs.G), dim3(kBinBlock), lds_b, s, pos, w.desc,
                               w.nbox, w.n, bs, off, w.temp);
            hipLaunchKernelGGL(k_bin_sort, dim3((unsigned)bs.nsb), dim3(kSortBlock), sort_lds(bs),
                               s, w.desc, w.nbox, w.ncell, bs, off, (int64_t)bs.G, w.temp,
                               w.cell_start, w.sorted, w.parent, dense_out(w));
        } else {  // placed buckets staged in `sorted`, split into `temp`, sorted into `sorted`
            int32_t *sub_off = hist;  // the counts are spent once scanned into off
            hipLaunchKernelGGL(k_bin_place, dim3(bs.G), dim3(kBinBlock), lds_b, s, pos, w.desc,
                               w.nbox, w.n, bs, off, w.sorted);
            hipLaunchKernelGGL(k_bin_split, dim3((unsigned)bs.nbk), dim3(kSplitBlock), 0, s,
                               w.desc, w.nbox, bs, off, w.sorted, w.temp, sub_off);
            hipLaunchKernelGGL(k_bin_sort, dim3((unsigned)bs.nsb), dim3(kSortBlock), sort_lds(bs),
                               s, w.desc, w.nbox, w.ncell, bs, sub_off, (int64_t)1, w.temp,
                               w.cell_start, w.sorted, w.parent, dense_out(w));
        }
    } else {
        e = launch_fill_i32(w.cell_count, w.ncell, 0, s);
        if (e != hipSuccess)
            return e;
        const unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
        hipLaunchKernelGGL(k_count, dim3(nb), dim3(w.block), 0, s, pos, w.n, w.desc, w.nbox,
                           w.cell_count, w.rank, w.ctr);
        e = launch_scan_i32(w.cell_count, w.cell_start, w.ncell, w.scan, s);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(w.block), 0, s, pos, w.n, w.desc, w.nbox,
                           w.cell_start, w.rank, w.sorted, w.parent);
    }
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_dense_build(w, s, bs.ok);
}

}  // namespace fof
