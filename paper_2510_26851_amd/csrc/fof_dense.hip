// Clique-cell path for dense cells.
//
// Inside a coarse cell that holds many particles, pair testing is quadratic.  The cell is
// cut into m^3 fine cells whose side is small enough (<= 0.999 b / sqrt(3), allowing for the
// float32 index error) that any two particles of one fine cell are friends: every
// non-empty fine cell is a clique ("unit"), the idea of cell-based FoF with cells of side
// b/sqrt(3) that the paper's linked-cell section cites as its inspiration.  Units then only
// need one friend pair to be joined, so tests stop at the first hit.
//
// Build stage (index construction):
//   k_classify_* cells with more than `dense_threshold` particles get a dense id (in cell
//                order, by a count / scan / assign over chunks of cells) and a table
//   k_dense_sort sort each dense cell by fine key (in LDS when it fits, else through a
//                staging buffer) and write the key bitmask, its popcount prefix and the
//                start of every unit
// Link stage:
//   k_dense_cc   union-find over the units of one cell in LDS (first hit joins two units),
//                then every member's entry points at the component member with the
//                smallest original index; units record their component number
//   k_dense_cross units of neighbouring dense cells, each cell pair handled once (by the
//                lower cell index), stopping as soon as two single-component cells meet
//   k_dense_sparse (after the sparse link kernels) the particles of ordinary cells around
//                a dense cell: each one within reach is tested against the units its
//                position can reach, one friend per component, straight from LDS
#include "fof_internal.h"

namespace fof {

namespace {

constexpr int kDenseBlock = 256;
constexpr int kBigBlock = 512;    // block of a big cell's components pass: 8 waves
constexpr int kLdsCap = 2048;     // particles a dense cell may hold to be sorted in LDS
constexpr int kHookBuf = 64;      // LDS buffer of a worker's deferred sparse-dense hooks
constexpr int kPairCell = 64;     // dense cells up to this size are joined by all their pairs

struct CellXYZ {
    int x, y, z;
};

__device__ __forceinline__ CellXYZ cell_xyz(const BoxDesc &B, int64_t c)
{
    int64_t l = c - B.cell_base;  // z fastest, see coarse_cell
    CellXYZ r;
    r.z = (int)(l % B.nc[2]);
    l /= B.nc[2];
    r.y = (int)(l % B.nc[1]);
    r.x = (int)(l / B.nc[1]);
    return r;
}

// Fine key of a particle inside its coarse cell (cx, cy, cz).
__device__ __forceinline__ int fine_key(const BoxDesc &B, const CellXYZ &cc, float4 p)
{
    const int m = B.m;
    int fx = fine_index(p.x, B.inv_fine[0], B.nf[0]) - cc.x * m;
    int fy = fine_index(p.y, B.inv_fine[1], B.nf[1]) - cc.y * m;
    int fz = fine_index(p.z, B.inv_fine[2], B.nf[2]) - cc.z * m;
    return (fz * m + fy) * m + fx;
}

// LDS union-find over fine keys: hook the larger root under the smaller.
__device__ __forceinline__ int lfind(int *uf, int x)
{
    for (;;) {
        const int p = __hip_atomic_load(uf + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p == x)
            return x;
        const int g = __hip_atomic_load(uf + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (g != p)  // halving: only non-root entries are rewritten, never a root
            __hip_atomic_store(uf + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = g;
    }
}

__device__ __forceinline__ void lunion(int *uf, int a, int b)
{
    for (;;) {
        a = lfind(uf, a);
        b = lfind(uf, b);
        if (a == b)
            return;
        if (a < b) {
            int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(uf + a, a, b) == a)
            return;
    }
}

// Capacity of the sparse-dense pass's deferred hooks (at most the 2n int2 pairs the staging
// buffer holds, and the plan's hook capacity).
__device__ __forceinline__ int64_t dense_edge_cap(const Work &w)
{
    return w.dense_edge_cap < INT32_MAX ? w.dense_edge_cap : INT32_MAX;
}

// One hook straight to the deferred list (when a worker's LDS buffer is full).
__device__ __forceinline__ void defer_dense_hook(const Work &w, int2 h)
{
    const int32_t slot = atomicAdd(&w.ctr->n_dense_edges, 1);
    if ((int64_t)slot < dense_edge_cap(w))
        reinterpret_cast<int2 *>(w.temp)[slot] = h;
    else
        w.ctr->dense_edge_over = 1;
}

// Block-wide exclusive scan of one int per thread (kDenseBlock threads).
__device__ int block_scan(int v, int *total, int *scratch /* kDenseBlock / kWave ints */)
{
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(x, o, kWave);
        if (lane >= o)
            x += y;
    }
    if (lane == kWave - 1)
        scratch[wid] = x;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int k = 0; k < kDenseBlock / kWave; ++k) {
        int s = scratch[k];
        if (k < wid)
            pre += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

__device__ __forceinline__ int dense_count(const Counters *ctr, int cap)
{
    int nd = __hip_atomic_load(&ctr->n_dense, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return nd < cap ? nd : cap;
}

// Cells holding more than dense_threshold particles (in boxes that allow clique tables)
// get a dense id; those over kSmallCell also a place in the big list.  Ids follow cell
// order and are assigned without atomics in two passes over chunks of kClassChunk cells:
// k_classify_count counts per chunk, a scan gives each chunk its first ids, and
// k_classify_assign ranks the cells inside the chunk.  A cell whose id would pass the
// table capacity gets none (-1) and raises FOF_STATUS_DENSE_CAP.
constexpr int kClassChunk = 4096;
constexpr int kClassBlock = 256;
constexpr int kClassPer = kClassChunk / kClassBlock;

// 0: ordinary cell, 1: dense, 2: dense and big; -1: above the threshold, no table allowed.
__device__ __forceinline__ int cell_class(const Work &w, int64_t c)
{
    const int32_t cnt = w.cell_start[c + 1] - w.cell_start[c];
    if (cnt <= w.dense_threshold)
        return 0;
    if (!w.desc[find_box_cell(w.desc, w.nbox, c)].dense_ok)
        return -1;
    return cnt > kSmallCell ? 2 : 1;
}

// Block-wide exclusive scan of two small counts per thread (kClassBlock threads).
__device__ __forceinline__ int2 block_scan2(int a, int b, int2 *total, int2 *scr)
{
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int xa = a, xb = b;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int ya = __shfl_up(xa, o, kWave), yb = __shfl_up(xb, o, kWave);
        if (lane >= o) {
            xa += ya;
            xb += yb;
        }
    }
    if (lane == kWave - 1)
        scr[wid] = make_int2(xa, xb);
    __syncthreads();
    int2 pre = make_int2(0, 0), tot = make_int2(0, 0);
    for (int k = 0; k < kClassBlock / kWave; ++k) {
        if (k < wid) {
            pre.x += scr[k].x;
            pre.y += scr[k].y;
        }
        tot.x += scr[k].x;
        tot.y += scr[k].y;
    }
    __syncthreads();  // scr is reused by the next call
    *total = tot;
    return make_int2(pre.x + xa - a, pre.y + xb - b);
}

__global__ __launch_bounds__(kClassBlock) void k_classify_count(Work w, int64_t nchunk,
                                                                 int32_t *__restrict__ nd,
                                                                 int32_t *__restrict__ nbig)
{
    __shared__ int2 scr[kClassBlock / kWave];
    for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        int a = 0, b = 0;
        for (int k = 0; k < kClassPer; ++k) {
            const int64_t c = ch * kClassChunk + k * kClassBlock + threadIdx.x;
            if (c < w.ncell) {
                const int cl = cell_class(w, c);
                a += cl > 0;
                b += cl == 2;
            }
        }
        int2 tot;
        block_scan2(a, b, &tot, scr);
        if (threadIdx.x == 0) {
            nd[ch] = tot.x;
            nbig[ch] = tot.y;
        }
    }
}

__global__ void k_classify_totals(Counters *ctr, int64_t nchunk, const int32_t *nd_pre,
                                  const int32_t *nbig_pre)
{
    if (threadIdx.x == 0) {
        ctr->n_dense = nd_pre[nchunk];
        ctr->n_big = nbig_pre[nchunk];
    }
}

// Thread t of chunk ch owns cells ch * kClassChunk + t * kClassPer + [0, kClassPer): one
// scan per chunk numbers the dense cells in cell order.
__global__ __launch_bounds__(kClassBlock) void k_classify_assign(Work w, int64_t nchunk,
                                                                  const int32_t *__restrict__ nd_pre,
                                                                  const int32_t *__restrict__ nbig_pre)
{
    __shared__ int2 scr[kClassBlock / kWave];
    for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        const int64_t c0 = ch * kClassChunk + (int64_t)threadIdx.x * kClassPer;
        int a = 0, b = 0;
        bool any = false;
        for (int k = 0; k < kClassPer; ++k) {
            const int cl = c0 + k < w.ncell ? cell_class(w, c0 + k) : 0;
            a += cl > 0;
            b += cl == 2;
            any |= cl != 0;
        }
        int2 tot;
        const int2 r = block_scan2(a, b, &tot, scr);
        if (!any)
            continue;
        int next_d = nd_pre[ch] + r.x, next_b = nbig_pre[ch] + r.y;
        for (int k = 0; k < kClassPer; ++k) {
            const int64_t c = c0 + k;
            const int cl = c < w.ncell ? cell_class(w, c) : 0;
            if (cl == 0)
                continue;
            int32_t d = -1;
            if (cl > 0) {
                d = next_d++;
                const int bg = cl == 2 ? next_b++ : -1;
                if (d < w.dense_cap) {
                    w.dense_list[d] = (int32_t)c;
                    if (cl == 2)
                        w.big_list[bg] = d;
                } else {
                    atomicOr(&w.ctr->status, (int32_t)FOF_STATUS_DENSE_CAP);
                    if (cl == 2)  // big ids past this one have no table either
                        atomicMin(&w.ctr->n_big, bg);
                    d = -1;
                }
            }
            w.cell_count[c] = d;
        }
    }
}

// ---------------------------------------------------------------------------------------
// Sort one dense cell by fine key and write its tables.
// ---------------------------------------------------------------------------------------
// LDS of one cell's sort: per-key counts and offsets, the key bitmask and its popcount
// prefix.
struct SortLds {
    int kcnt[kMaxFineKeys];
    int koff[kMaxFineKeys + 1];
    uint32_t kbits[kMaxTableWords];
    int kpre[kMaxTableWords];
};

// One cell of at most kSmallCell particles, by the calling wave (every particle in
// registers, kSmallCell / kWave per lane; wave barriers only).
__device__ void sort_small_cell(const Work &w, int d, SortLds &S)
{
    constexpr int kPer = kSmallCell / kWave;
    constexpr int kKeysPerLane = (kMaxFineKeys + kWave - 1) / kWave;
    const int lane = lane_id();
    const int64_t c = w.dense_list[d];
    const int32_t s = w.cell_start[c];
    const int32_t n = w.cell_start[c + 1] - s;
    const BoxDesc &B = uniform_box(w.desc, find_box(w.desc, w.nbox, s));
    const CellXYZ cc = cell_xyz(B, c);
    const int K = B.m * B.m * B.m;
    const int W = w.table_words;
    int32_t *T = w.table + (int64_t)d * w.table_stride;

    for (int k = lane; k < K; k += kWave)
        S.kcnt[k] = 0;
    for (int k = lane; k < kMaxTableWords; k += kWave)
        S.kbits[k] = 0u;
    wave_sync();
    // keys and per-key ranks
    float4 preg[kPer];
    int kreg[kPer], rreg[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int t = lane + j * kWave;
        if (t < n) {
            preg[j] = w.sorted[s + t];
            kreg[j] = fine_key(B, cc, preg[j]);
            rreg[j] = atomicAdd(S.kcnt + kreg[j], 1);
        }
    }
    wave_sync();
    // exclusive scan over keys: lane l owns keys [l * per, (l + 1) * per)
    const int per = (K + kWave - 1) / kWave;
    const int k0 = lane * per;
    int sum = 0;
    for (int q = 0; q < per && q < kKeysPerLane; ++q)
        sum += k0 + q < K ? S.kcnt[k0 + q] : 0;
    int run = wave_incl_sum(sum) - sum;
    for (int q = 0; q < per && q < kKeysPerLane; ++q) {
        const int k = k0 + q;
        if (k < K) {
            const int v = S.kcnt[k];
            S.koff[k] = run;
            if (v > 0)
                atomicOr(S.kbits + (k >> 5), 1u << (k & 31));
            run += v;
        }
    }
    if (lane == 0)
        S.koff[K] = n;
    wave_sync();
    // popcount prefix of the bitmask words (W <= kWave)
    const int pc = lane < W ? __popc(S.kbits[lane]) : 0;
    const int pre = wave_incl_sum(pc) - pc;
    if (lane < W)
        S.kpre[lane] = pre;
    wave_sync();
    // place the particles in key order (all of them are in registers)
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int t = lane + j * kWave;
        if (t < n)
            w.sorted[s + S.koff[kreg[j]] + rreg[j]] = preg[j];
    }
    // tables: header, bitmask, popcount prefix, unit starts (absolute sorted index)
    if (lane == 0) {
        T[0] = (int32_t)c;
        T[1] = 0;
        T[2] = S.kpre[W - 1] + __popc(S.kbits[W - 1]);
        T[3] = 0;
    }
    for (int q = lane; q < W; q += kWave) {
        T[kTableHeader + q] = (int32_t)S.kbits[q];
        T[kTableHeader + W + q] = S.kpre[q];
    }
    for (int k = lane; k < K; k += kWave) {
        if ((S.kbits[k >> 5] >> (k & 31)) & 1u) {
            const int r = S.kpre[k >> 5] + __popc(S.kbits[k >> 5] & ((1u << (k & 31)) - 1u));
            w.rank[s + r] = s + S.koff[k];
        }
    }
    wave_sync();  // the LDS of this cell is read before the next cell overwrites it
}

// One cell of more than kSmallCell particles, by the whole block (those of at most kLdsCap
// held in registers, larger ones sorted through the staging buffer).
__device__ void sort_big_cell(const Work &w, int d, SortLds &S, int *scr)
{
    int *kcnt = S.kcnt, *koff = S.koff, *kpre = S.kpre;
    uint32_t *kbits = S.kbits;
    constexpr int kPer = kLdsCap / kDenseBlock;
    const int64_t c = w.dense_list[d];
    const int32_t s = w.cell_start[c];
    const int32_t n = w.cell_start[c + 1] - s;
    const BoxDesc &B = uniform_box(w.desc, find_box(w.desc, w.nbox, s));
    const CellXYZ cc = cell_xyz(B, c);
    const int K = B.m * B.m * B.m;
    const int W = w.table_words;
    int32_t *T = w.table + (int64_t)d * w.table_stride;
    const bool lds = n <= kLdsCap;

    for (int k = threadIdx.x; k < K; k += kDenseBlock)
        kcnt[k] = 0;
    for (int k = threadIdx.x; k < kMaxTableWords; k += kDenseBlock)
        kbits[k] = 0u;
    __syncthreads();

    // keys and per-key ranks
    float4 preg[kPer];
    int kreg[kPer], rreg[kPer];
    if (lds) {
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int t = threadIdx.x + j * kDenseBlock;
            if (t < n) {
                preg[j] = w.sorted[s + t];
                kreg[j] = fine_key(B, cc, preg[j]);
                rreg[j] = atomicAdd(kcnt + kreg[j], 1);
            }
        }
    } else {
        for (int t = threadIdx.x; t < n; t += kDenseBlock)
            atomicAdd(kcnt + fine_key(B, cc, w.sorted[s + t]), 1);
    }
    __syncthreads();

    // exclusive scan over keys (each thread owns 4 consecutive keys: K <= 1024)
    int loc[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = threadIdx.x * 4 + q;
        loc[q] = k < K ? kcnt[k] : 0;
        sum += loc[q];
    }
    int tot;
    int run = block_scan(sum, &tot, scr);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = threadIdx.x * 4 + q;
        if (k < K) {
            koff[k] = run;
            if (loc[q] > 0)
                atomicOr(kbits + (k >> 5), 1u << (k & 31));
        }
        run += loc[q];
    }
    if (threadIdx.x == 0)
        koff[K] = n;
    __syncthreads();
    if ((int)threadIdx.x < W) {
        int pre = 0;
        for (int q = 0; q < (int)threadIdx.x; ++q)
            pre += __popc(kbits[q]);
        kpre[threadIdx.x] = pre;
    }
    __syncthreads();

    // place the particles in key order
    if (lds) {
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int t = threadIdx.x + j * kDenseBlock;
            if (t < n)
                w.sorted[s + koff[kreg[j]] + rreg[j]] = preg[j];
        }
    } else {
        for (int k = threadIdx.x; k < K; k += kDenseBlock)
            kcnt[k] = 0;  // reused as per-key cursors
        __syncthreads();
        for (int t = threadIdx.x; t < n; t += kDenseBlock) {
            const float4 p = w.sorted[s + t];
            const int k = fine_key(B, cc, p);
            w.temp[s + koff[k] + atomicAdd(kcnt + k, 1)] = p;
        }
        __threadfence();
        __syncthreads();
        for (int t = threadIdx.x; t < n; t += kDenseBlock)
            w.sorted[s + t] = w.temp[s + t];
    }

    // tables: header, bitmask, popcount prefix, unit starts (absolute sorted index)
    if (threadIdx.x == 0) {
        T[0] = (int32_t)c;
        T[1] = 0;
        T[2] = kpre[W - 1] + __popc(kbits[W - 1]);
        T[3] = 0;
    }
    for (int q = threadIdx.x; q < W; q += kDenseBlock) {
        T[kTableHeader + q] = (int32_t)kbits[q];
        T[kTableHeader + W + q] = kpre[q];
    }
    for (int k = threadIdx.x; k < K; k += kDenseBlock) {
        if ((kbits[k >> 5] >> (k & 31)) & 1u) {
            const int r = kpre[k >> 5] + __popc(kbits[k >> 5] & ((1u << (k & 31)) - 1u));
            w.rank[s + r] = s + koff[k];
        }
    }
    __syncthreads();
}

// Dense-cell sort: the big cells first, one block each (few, long), then the cells of at
// most kSmallCell particles one wave each (many, short: they even out the blocks' ends).
__global__ __launch_bounds__(kDenseBlock) void k_dense_sort(Work w)
{
    __shared__ SortLds lds[kDenseBlock / kWave];
    __shared__ int scr[kDenseBlock / kWave];
    const int nb = __hip_atomic_load(&w.ctr->n_big, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int kb = blockIdx.x; kb < nb; kb += gridDim.x)
        sort_big_cell(w, w.big_list[kb], lds[0], scr);
    __syncthreads();
    const int nd = dense_count(w.ctr, w.dense_cap);
    const int nw = gridDim.x * (kDenseBlock / kWave);
    SortLds &S = lds[threadIdx.x / kWave];
    for (int d = blockIdx.x * (kDenseBlock / kWave) + (int)threadIdx.x / kWave; d < nd; d += nw) {
        const int64_t c = w.dense_list[d];
        if (w.cell_start[c + 1] - w.cell_start[c] <= kSmallCell)  // wave-uniform
            sort_small_cell(w, d, S);
    }
}

// ---------------------------------------------------------------------------------------
// Link stage.  Cells of up to kSmallCell particles are handled by one wave each (four per
// block, each with its own LDS slice); larger cells by a whole block.  The code is shared
// through the group type G.
// ---------------------------------------------------------------------------------------

template <int G>
struct Grp;

template <>
struct Grp<kWave> {
    static constexpr int per_block = kDenseBlock / kWave;
    static __device__ int tid() { return lane_id(); }
    static __device__ int slot() { return threadIdx.x / kWave; }
    static __device__ void sync()
    {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
};

template <>
struct Grp<kDenseBlock> {
    static constexpr int per_block = 1;
    static __device__ int tid() { return threadIdx.x; }
    static __device__ int slot() { return 0; }
    static __device__ void sync() { __syncthreads(); }
};

template <>
struct Grp<kBigBlock> {
    static constexpr int per_block = 1;
    static __device__ int tid() { return threadIdx.x; }
    static __device__ int slot() { return 0; }
    static __device__ void sync() { __syncthreads(); }
};

template <int UMAX, int CAP>
struct CellLds {
    float4 part[CAP];               // the cell's particles, when it has at most CAP
    int uf[UMAX];                   // union-find over unit ranks
    unsigned long long umin[UMAX];  // (original index << 32 | sorted index) minimum
    int ustart[UMAX + 1];           // absolute sorted index of each unit's first member
    int umark[UMAX];                // unit counts per root, then the units outside the giant
    short uxyz[UMAX];               // fine coordinates: x | y << 4 | z << 8
    short ucomp[UMAX];              // component number of each unit
    uint32_t bits[kMaxTableWords];  // key bitmask of the cell (or of a neighbour, in cross)
    int pre[kMaxTableWords];
    uint32_t pairbits[32];
    int ncomp, nnb, done, giant, nmark;
    int2 hk[kHookBuf];              // deferred sparse-dense hooks of the cell, then flushed
    int nhk, hkbase;
    int nb[26];                     // neighbour dense ids (cross), or sparse cell starts
    short nbo[26];                  // their offsets: (ox+1) | (oy+1) << 2 | (oz+1) << 4
    int nbp[27];                    // sparse neighbours: running particle count
#ifdef FOF_TIMING
    long long phase[8], tlast;      // diagnostic builds: clock ticks per phase of a pass
#endif
};

#ifdef FOF_TIMING
#define FOF_PHASE(L, lead, k)                                                                 \
    do {                                                                                      \
        if (lead) {                                                                           \
            const long long now_ = clock64();                                                 \
            (L).phase[k] += now_ - (L).tlast;                                                 \
            (L).tlast = now_;                                                                 \
        }                                                                                     \
    } while (0)
#define FOF_PHASE_START(L, lead)                                                              \
    do {                                                                                      \
        if (lead) {                                                                           \
            for (int k_ = 0; k_ < 8; ++k_)                                                    \
                (L).phase[k_] = 0;                                                            \
            (L).tlast = clock64();                                                            \
        }                                                                                     \
    } while (0)
#define FOF_PHASE_FLUSH(L, lead, ctr, base)                                                   \
    do {                                                                                      \
        if (lead)                                                                             \
            for (int k_ = 0; k_ < 8; ++k_)                                                    \
                atomicAdd(&(ctr)->stats[(base) + k_], (unsigned long long)(L).phase[k_]);     \
    } while (0)
#else
#define FOF_PHASE(L, lead, k) ((void)0)
#define FOF_PHASE_START(L, lead) ((void)0)
#define FOF_PHASE_FLUSH(L, lead, ctr, base) ((void)0)
#endif

__device__ __forceinline__ int rank_in(const uint32_t *bits, const int *pre, int k)
{
    return pre[k >> 5] + __popc(bits[k >> 5] & ((1u << (k & 31)) - 1u));
}

// Box of global fine cell (gx, gy, gz) (any periodic image), widened by the slack.
struct FineBox {
    float lo[3], hi[3];
};

__device__ __forceinline__ FineBox fine_box(const BoxDesc &B, int gx, int gy, int gz)
{
    FineBox f;
    const int g[3] = {gx, gy, gz};
    for (int a = 0; a < 3; ++a) {
        f.lo[a] = (float)g[a] * B.fine[a] - B.slack;
        f.hi[a] = (float)(g[a] + 1) * B.fine[a] + B.slack;
    }
    return f;
}

// True when every point of the unit lies at least b from p, so the pair tests of p against
// the unit can be skipped.  The box is widened by the slack (>= 5 L 2^-23: float error of
// its bounds, the members' index error and the rounding of the differences), so the
// computed gaps never exceed the true ones; the float sum of three squares is within
// 2e-7 relative, covered by the factor 1 + 1e-6 on b^2.
__device__ __forceinline__ bool far_from(const BoxDesc &B, const FineBox &f, float4 p)
{
    const float c[3] = {p.x, p.y, p.z};
    float s = 0.0f;
    for (int a = 0; a < 3; ++a) {
        const float g = fmaxf(0.0f, fmaxf(f.lo[a] - c[a], c[a] - f.hi[a]));
        s += g * g;
    }
    return s >= (float)B.b2 * 1.000001f;
}

// Index of the first member of memB[b0, b1) that is a friend of p, or -1.  Members are
// read four at a time so that their loads (LDS or global) overlap.
__device__ __forceinline__ int first_friend(const Pred &P, float4 p, const float4 *memB, int b0,
                                            int b1)
{
    int j = b0;
    for (; j + 4 <= b1; j += 4) {
        const float4 q0 = memB[j], q1 = memB[j + 1], q2 = memB[j + 2], q3 = memB[j + 3];
        const bool h0 = linked(P, p.x, p.y, p.z, q0.x, q0.y, q0.z);
        const bool h1 = linked(P, p.x, p.y, p.z, q1.x, q1.y, q1.z);
        const bool h2 = linked(P, p.x, p.y, p.z, q2.x, q2.y, q2.z);
        const bool h3 = linked(P, p.x, p.y, p.z, q3.x, q3.y, q3.z);
        if (h0 | h1 | h2 | h3)
            return h0 ? j : (h1 ? j + 1 : (h2 ? j + 2 : j + 3));
    }
    for (; j < b1; ++j) {
        const float4 q = memB[j];
        if (linked(P, p.x, p.y, p.z, q.x, q.y, q.z))
            return j;
    }
    return -1;
}

// Is some member of unit A (memA[a0, a1)) a friend of some member of unit B (memB[b0, b1))?
// Members of A far from B's fine box are skipped.
__device__ __forceinline__ bool units_meet(const BoxDesc &B, const Pred &P, const float4 *memA,
                                           int a0, int a1, const float4 *memB, int b0, int b1,
                                           const FineBox &fb)
{
    for (int i = a0; i < a1; ++i) {
        const float4 p = memA[i];
        if (far_from(B, fb, p))
            continue;
        if (first_friend(P, p, memB, b0, b1) >= 0)
            return true;
    }
    return false;
}

// Own units of dense cell d: keys, coordinates, member ranges; bitmask into L.bits.
template <int G, bool kLds, int UMAX, int CAP>
__device__ void load_units(const Work &w, const int32_t *T, int32_t s, int32_t n, int m, int u,
                           CellLds<UMAX, CAP> &L)
{
    const int W = w.table_words;
    const int t = Grp<G>::tid();
    for (int q = t; q < W; q += G) {
        L.bits[q] = (uint32_t)T[kTableHeader + q];
        L.pre[q] = T[kTableHeader + W + q];
    }
    for (int r = t; r < u; r += G)
        L.ustart[r] = w.rank[s + r];
    if (t == 0)
        L.ustart[u] = s + n;
    if (kLds)
        for (int k = t; k < n; k += G)
            L.part[k] = w.sorted[s + k];
    Grp<G>::sync();
    for (int q = t; q < W; q += G) {
        uint32_t bits = L.bits[q];
        int r = L.pre[q];
        while (bits) {
            const int k = q * 32 + __ffs(bits) - 1;
            bits &= bits - 1u;
            L.uxyz[r] = (short)((k % m) | (((k / m) % m) << 4) | ((k / (m * m)) << 8));
            ++r;
        }
    }
    Grp<G>::sync();
}

// Occupancy bits of fine keys [key0, key0 + nb) (nb <= 31) of a key bitmask in LDS
// holding W words: bit i of the result is key key0 + i.
__device__ __forceinline__ uint32_t row_bits(const uint32_t *bits, int W, int key0, int nb)
{
    const int w0 = key0 >> 5, sh = key0 & 31;
    uint64_t v = bits[w0];
    if (sh + nb > 32 && w0 + 1 < W)
        v |= (uint64_t)bits[w0 + 1] << 32;
    return (uint32_t)(v >> sh) & ((1u << nb) - 1u);
}

// Largest S with S fs^2 < b^2 (slightly below, so that pruning by it stays conservative):
// fine cells whose squared gap, in whole fine cells per axis, exceeds S hold no friend.
__device__ __forceinline__ int gap_budget(const BoxDesc &B)
{
    const double fs2 = (double)B.fine_side * (double)B.fine_side * (1.0 - 1e-12);
    int K = (int)(B.b2 / fs2);
    while (K > 0 && (double)K * fs2 >= B.b2)
        --K;
    while ((double)(K + 1) * fs2 < B.b2)
        ++K;
    return K;
}

// Joins units of the staged cell with their neighbour units.  pass 0: every unit, the
// forward half of the nearest shell (offsets in [-1, 1]^3).  pass 1: the units listed in
// umark[0, nmark) (those outside the largest component), every offset in [-R, R]^3 outside
// the nearest shell, in both directions (a pair with an unlisted end is then still examined
// from the other).  pass 2: every unit, the forward half of the offsets in [-R, R]^3
// outside the nearest shell (cheaper than pass 1 when the largest component holds fewer
// than about half the units: each pair once instead of twice from every listed unit).
// The work items are (unit, fine row of offsets) pairs spread over all threads; the
// occupied neighbours of one row are read as a bit field of the key bitmask, so empty fine
// cells cost nothing.  A pair already in one component is skipped, otherwise its first
// friend pair joins it.
template <int G, int UMAX, int CAP>
__device__ void join_units(const Work &w, const BoxDesc &B, const Pred &P, const CellXYZ &cc,
                           int m, int R, int u, int32_t s, const float4 *mem,
                           CellLds<UMAX, CAP> &L, int pass)
{
    const int W = w.table_words;
    const int reach = pass == 0 ? 1 : R;
    const int span = 2 * reach + 1;
    // (dz, dy) rows per unit; pass 2: dz = 0 with dy in [0, R], then dz in [1, R]
    const int rows = pass == 0 ? 5 : (pass == 1 ? span * span : R + 1 + R * span);
    const int nitems = (pass == 1 ? L.nmark : u) * rows;
    for (int item = Grp<G>::tid(); item < nitems; item += G) {
        const int r = pass == 1 ? L.umark[item / rows] : item / rows;
        const int q = item % rows;
        int dz, dy;
        if (pass == 0) {  // forward rows: (0, 0) with dx > 0, (0, 1), (1, -1), (1, 0), (1, 1)
            dz = q < 2 ? 0 : 1;
            dy = q < 2 ? q : q - 3;
        } else if (pass == 1) {
            dz = q / span - reach;
            dy = q % span - reach;
        } else {
            dz = q <= R ? 0 : 1 + (q - R - 1) / span;
            dy = q <= R ? q : (q - R - 1) % span - R;
        }
        const int xyz = L.uxyz[r];
        const int ax = xyz & 15, ay = (xyz >> 4) & 15, az = xyz >> 8;
        const int bz = az + dz, by = ay + dy;
        if (bz < 0 || bz >= m || by < 0 || by >= m)
            continue;
        int lo = -reach, hi = reach;  // dx range of this row
        if ((pass == 0 || pass == 2) && q == 0)
            lo = 1;
        const bool skip_core = pass != 0 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
        lo = max(lo, -ax);
        hi = min(hi, m - 1 - ax);
        if (lo > hi)
            continue;
        const int key0 = (bz * m + by) * m + ax + lo, nb = hi - lo + 1;
        uint32_t row = row_bits(L.bits, W, key0, nb);
        if (skip_core)  // positions of dx = -1, 0, 1 relative to lo
            for (int dx = -1; dx <= 1; ++dx)
                if (dx >= lo && dx <= hi)
                    row &= ~(1u << (dx - lo));
        while (row) {
            const int bpos = __ffs(row) - 1;
            row &= row - 1u;
            const int bx = ax + lo + bpos;
            const int kb = key0 + bpos;
            const int rb = rank_in(L.bits, L.pre, kb);
            if (lfind(L.uf, r) == lfind(L.uf, rb)) {
                FOF_STAT(w.ctr, ST_CC_SKIPS, 1);
                continue;
            }
            const FineBox fb = fine_box(B, cc.x * m + bx, cc.y * m + by, cc.z * m + bz);
            FOF_STAT(w.ctr, ST_CC_UNIT_PAIRS, 1);
            if (units_meet(B, P, mem, L.ustart[r] - s, L.ustart[r + 1] - s, mem,
                           L.ustart[rb] - s, L.ustart[rb + 1] - s, fb))
                lunion(L.uf, r, rb);
        }
    }
}

// Components of a cell of at most kPairCell particles (most of whose clique cells hold one
// member, so units save nothing): every pair of its particles is tested, pair p of the
// strict upper triangle on lane p mod 64, into an LDS union-find over the particles.  Then,
// as for units: every member points at its component's smallest original index, every unit
// records its component number (a unit is a clique, so all its members share one).
__device__ __forceinline__ int tri_row_start(int i, int n) { return i * (2 * n - i - 1) / 2; }

template <int G, int UMAX, int CAP>
__device__ void cc_cell_pairs(const Work &w, const Pred &P, int32_t s, int n, int u,
                              const float4 *mem, int32_t *T, CellLds<UMAX, CAP> &L)
{
    const int t = Grp<G>::tid();
    for (int k = t; k < n; k += G) {
        L.uf[k] = k;
        L.umin[k] = ~0ull;
    }
    Grp<G>::sync();
    const int np = n * (n - 1) / 2;
    for (int p = t; p < np; p += G) {
        // row i of pair p: the largest i with tri_row_start(i) <= p (float estimate, then
        // exact integer correction)
        const float q = (float)(2 * n - 1);
        int i = (int)((q - sqrtf(q * q - 8.0f * (float)p)) * 0.5f);
        i = max(0, min(i, n - 2));
        while (i > 0 && tri_row_start(i, n) > p)
            --i;
        while (i < n - 2 && tri_row_start(i + 1, n) <= p)
            ++i;
        const int j = p - tri_row_start(i, n) + i + 1;
        const float4 a = mem[i], b = mem[j];
        if (linked(P, a.x, a.y, a.z, b.x, b.y, b.z))
            lunion(L.uf, i, j);
    }
    Grp<G>::sync();
    for (int k = t; k < n; k += G) {
        const int r = lfind(L.uf, k);
        const unsigned long long v =
            ((unsigned long long)(uint32_t)__float_as_int(mem[k].w) << 32) | (uint32_t)(s + k);
        atomicMin(L.umin + r, v);
        if (r == k)
            L.umark[k] = atomicAdd(&L.ncomp, 1);
    }
    Grp<G>::sync();
    for (int k = t; k < n; k += G)
        w.parent[s + k] = L.umin[lfind(L.uf, k)];
    for (int r = t; r < u; r += G)
        w.cnt[s + r] = L.umark[lfind(L.uf, L.ustart[r] - s)];
    // mark every particle of the cell for the compress pass
    for (int64_t q = (s >> 6) + t; q <= ((int64_t)s + n - 1) >> 6; q += G) {
        const int64_t lo = q << 6, hi = lo + 64;
        const int64_t a = lo > s ? lo : s, b = hi < s + n ? hi : s + n;
        const uint64_t mask = (b - a == 64) ? ~0ull : (((1ull << (b - a)) - 1ull) << (a - lo));
        atomicOr((unsigned long long *)(w.flags + q), (unsigned long long)mask);
    }
    if (t == 0)
        T[1] = L.ncomp;
    Grp<G>::sync();
}

// kLds: the cell's particles are staged in LDS (it holds at most CAP), else read from HBM;
// fixed per instantiation, so every member access compiles to one kind of load.
template <int G, bool kLds, int UMAX, int CAP>
__device__ void cc_cell(const Work &w, int d, CellLds<UMAX, CAP> &L)
{
    const int t = Grp<G>::tid();
    const int64_t c = w.dense_list[d];
    const int32_t s = w.cell_start[c];
    const int32_t n = w.cell_start[c + 1] - s;
    const BoxDesc &B = uniform_box(w.desc, find_box(w.desc, w.nbox, s));
    const CellXYZ cc = cell_xyz(B, c);
    const Pred P = pred_of(B);
    const int m = B.m, R = B.R;
    int32_t *T = w.table + (int64_t)d * w.table_stride;
    const int u = T[2];
    const float4 *mem = kLds ? L.part : w.sorted + s;  // indexed by (sorted index - s)

    if (t == 0)
        L.ncomp = 0;
    load_units<G, kLds>(w, T, s, n, m, u, L);
    FOF_PHASE(L, t == 0, 0);
    if (G == kWave && n <= kPairCell) {  // uniform
        cc_cell_pairs<G>(w, P, s, n, u, mem, T, L);
        return;
    }

    // unit minima, one thread per member (a unit of a clump core can hold thousands); a
    // member's unit is the rank of its fine key, the key the cell was sorted by
    for (int r = t; r < u; r += G) {
        L.umin[r] = ~0ull;
        L.uf[r] = r;
    }
    Grp<G>::sync();
    for (int k = t; k < n; k += G) {
        const float4 p = mem[k];
        const unsigned long long v =
            ((unsigned long long)(uint32_t)__float_as_int(p.w) << 32) | (uint32_t)(s + k);
        atomicMin(L.umin + rank_in(L.bits, L.pre, fine_key(B, cc, p)), v);
    }
    Grp<G>::sync();
    FOF_PHASE(L, t == 0, 1);

    // join units of this cell: first friend pair wins.  The nearest shell goes first; when
    // it already leaves one component (the usual case inside a clump) the rest is skipped.
    join_units<G>(w, B, P, cc, m, R, u, s, mem, L, 0);
    Grp<G>::sync();
    FOF_PHASE(L, t == 0, 2);
    // components after the nearest shell: a far pair of two different components has at
    // least one end outside the largest one, so only those units search the far offsets
    if (t == 0) {
        L.ncomp = 0;
        L.giant = 0;
    }
    for (int r = t; r < u; r += G)
        L.umark[r] = 0;
    Grp<G>::sync();
    for (int r = t; r < u; r += G) {
        const int root = lfind(L.uf, r);
        atomicAdd(&L.umark[root], 1);
        if (root == r)
            atomicAdd(&L.ncomp, 1);
    }
    Grp<G>::sync();
    for (int r = t; r < u; r += G)
        if (L.umark[r])
            atomicMax(&L.giant, (L.umark[r] << 16) | r);  // unit count < 2^15, r < 2^16
    Grp<G>::sync();
    const bool far = L.ncomp > 1;  // uniform: every thread reads the same count
    FOF_PHASE(L, t == 0, 3);
    if (far && t == 0)
        FOF_STAT(w.ctr, ST_CC_FAR_CELLS, 1);
    if (far) {
        const int giant = L.giant & 0xFFFF, gsize = L.giant >> 16;
        const int span = 2 * R + 1;
        if (span * span * (u - gsize) <= (R + 1 + R * span) * u) {
            if (t == 0)
                L.nmark = 0;
            Grp<G>::sync();
            for (int r = t; r < u; r += G)  // umark becomes the list of units outside the giant
                if (lfind(L.uf, r) != giant)
                    L.umark[atomicAdd(&L.nmark, 1)] = r;
            Grp<G>::sync();
            join_units<G>(w, B, P, cc, m, R, u, s, mem, L, 1);
        } else {
            join_units<G>(w, B, P, cc, m, R, u, s, mem, L, 2);
        }
    }
    Grp<G>::sync();
    FOF_PHASE(L, t == 0, 4);
    if (t == 0)
        L.ncomp = 0;
    Grp<G>::sync();

    // flatten: component minimum and component numbers
    for (int r = t; r < u; r += G) {
        const int root = lfind(L.uf, r);
        if (root != r)
            atomicMin(L.umin + root, L.umin[r]);
        else
            L.ucomp[r] = (short)atomicAdd(&L.ncomp, 1);
    }
    Grp<G>::sync();
    FOF_PHASE(L, t == 0, 5);

    // every member points at its component's smallest original index; every unit records
    // its component number.  Cells of one wave hold few members per unit: one lane per
    // unit; in a block's cell a unit can hold thousands: one thread per member.
    if (G == kWave) {
        for (int r = t; r < u; r += G) {
            const int root = lfind(L.uf, r);
            const unsigned long long lead = L.umin[root];
            for (int i = L.ustart[r]; i < L.ustart[r + 1]; ++i)
                w.parent[i] = lead;
            w.cnt[s + r] = L.ucomp[root];
        }
    } else {
        for (int r = t; r < u; r += G)
            w.cnt[s + r] = L.ucomp[lfind(L.uf, r)];
        for (int k = t; k < n; k += G) {
            const int r = rank_in(L.bits, L.pre, fine_key(B, cc, mem[k]));
            w.parent[s + k] = L.umin[lfind(L.uf, r)];
        }
    }
    // mark every particle of the cell for the compress pass
    for (int64_t q = (s >> 6) + t; q <= ((int64_t)s + n - 1) >> 6; q += G) {
        const int64_t lo = q << 6, hi = lo + 64;
        const int64_t a = lo > s ? lo : s, b = hi < s + n ? hi : s + n;
        const uint64_t mask = (b - a == 64) ? ~0ull : (((1ull << (b - a)) - 1ull) << (a - lo));
        atomicOr((unsigned long long *)(w.flags + q), (unsigned long long)mask);
    }
    if (t == 0)
        T[1] = L.ncomp;
    Grp<G>::sync();
    FOF_PHASE(L, t == 0, 6);
}

// kLds: the cell's particles are staged in LDS (it holds at most CAP), else read from HBM;
// fixed per instantiation, so every member access compiles to one kind of load.
template <int G, bool kLds, int UMAX, int CAP>
__device__ void cross_cell(const Work &w, int d, CellLds<UMAX, CAP> &L)
{
    const int t = Grp<G>::tid();
    const int64_t c = w.dense_list[d];
    const int32_t s = w.cell_start[c];
    const int32_t n = w.cell_start[c + 1] - s;
    const BoxDesc &B = uniform_box(w.desc, find_box(w.desc, w.nbox, s));
    const CellXYZ cc = cell_xyz(B, c);
    const Pred P = pred_of(B);
    const int m = B.m, R = B.R;
    const int W = w.table_words;
    const int32_t *T = w.table + (int64_t)d * w.table_stride;
    const int u = T[2], ncomp = T[1];
    const int K = gap_budget(B);

    // neighbour dense cells with a higher index: this cell handles those pairs
    if (t == 0)
        L.nnb = 0;
    Grp<G>::sync();
    if (t < 27 && t != 13) {
        const int ox = t % 3 - 1, oy = (t / 3) % 3 - 1, oz = t / 9 - 1;
        int nx = cc.x + ox, ny = cc.y + oy, nz = cc.z + oz;
        nx += nx < 0 ? B.nc[0] : (nx >= B.nc[0] ? -B.nc[0] : 0);
        ny += ny < 0 ? B.nc[1] : (ny >= B.nc[1] ? -B.nc[1] : 0);
        nz += nz < 0 ? B.nc[2] : (nz >= B.nc[2] ? -B.nc[2] : 0);
        const int64_t c2 = coarse_cell(B, nx, ny, nz);
        if (c2 > c && w.cell_start[c2 + 1] - w.cell_start[c2] > w.dense_threshold) {
            const int32_t d2 = w.cell_count[c2];
            if (d2 >= 0) {
                const int k = atomicAdd(&L.nnb, 1);
                L.nb[k] = d2;
                L.nbo[k] = (short)((ox + 1) | ((oy + 1) << 2) | ((oz + 1) << 4));
            }
        }
    }
    Grp<G>::sync();
    const int nnb = L.nnb;
    FOF_PHASE(L, t == 0, 0);
    if (nnb == 0) {  // uniform: every thread read the same count
        Grp<G>::sync();
        return;
    }
    const float4 *mem = kLds ? L.part : w.sorted + s;
    for (int r = t; r < u; r += G) {
        L.ustart[r] = w.rank[s + r];
        L.ucomp[r] = (short)w.cnt[s + r];
    }
    if (t == 0)
        L.ustart[u] = s + n;
    if (kLds)
        for (int k = t; k < n; k += G)
            L.part[k] = w.sorted[s + k];
    for (int q = t; q < W; q += G) {
        uint32_t bits = (uint32_t)T[kTableHeader + q];
        int r = T[kTableHeader + W + q];
        while (bits) {
            const int k = q * 32 + __ffs(bits) - 1;
            bits &= bits - 1u;
            L.uxyz[r] = (short)((k % m) | (((k / m) % m) << 4) | ((k / (m * m)) << 8));
            ++r;
        }
    }
    Grp<G>::sync();
    FOF_PHASE(L, t == 0, 1);

    for (int k = 0; k < nnb; ++k) {
        const int d2 = L.nb[k];
        const int o = L.nbo[k];
        const int ox = (o & 3) - 1, oy = ((o >> 2) & 3) - 1, oz = (o >> 4) - 1;
        const int32_t *T2 = w.table + (int64_t)d2 * w.table_stride;
        const int64_t c2 = T2[0];
        const int32_t s2 = w.cell_start[c2];
        const int32_t n2 = w.cell_start[c2 + 1] - s2;
        const int u2 = T2[2], ncomp2 = T2[1];
        const bool dedupe = ncomp * ncomp2 <= 1024;
        const bool single = ncomp == 1 && ncomp2 == 1;
        if (t == 0)
            FOF_STAT(w.ctr, ST_CROSS_CELLPAIRS, 1);
        for (int q = t; q < W; q += G) {
            L.bits[q] = (uint32_t)T2[kTableHeader + q];
            L.pre[q] = T2[kTableHeader + W + q];
        }
        for (int q = t; q < 32; q += G)
            L.pairbits[q] = 0u;
        if (t == 0)
            L.done = 0;
        // the neighbour's unit components and member starts, in LDS when they fit; a pair of
        // single-component cells stops at its first friend pair, so it reads the few member
        // starts it needs from global memory instead
        const bool staged2 = u2 < UMAX && !single;
        int *ncomp_of = L.umark;
        int *nstart = reinterpret_cast<int *>(L.umin);  // 2 * UMAX ints
        if (staged2) {
            for (int q = t; q < u2; q += G) {
                ncomp_of[q] = w.cnt[s2 + q];
                nstart[q] = w.rank[s2 + q];
            }
            if (t == 0)
                nstart[u2] = s2 + n2;
        }
        // units of this cell within R fine cells of the shared face, edge or corner: only
        // they can reach the neighbour's units
        if (t == 0)
            L.nmark = 0;
        Grp<G>::sync();
        for (int r = t; r < u; r += G) {
            const int xyz = L.uxyz[r];
            const int ax = xyz & 15, ay = (xyz >> 4) & 15, az = xyz >> 8;
            const bool near = (ox == 0 || (ox > 0 ? ax >= m - R : ax < R)) &&
                              (oy == 0 || (oy > 0 ? ay >= m - R : ay < R)) &&
                              (oz == 0 || (oz > 0 ? az >= m - R : az < R));
            if (near)
                L.uf[atomicAdd(&L.nmark, 1)] = r;
        }
        Grp<G>::sync();
        FOF_PHASE(L, t == 0, 2);
        // items: (candidate unit, (dz, dy) row of the neighbour) spread over every thread
        const int span = 2 * R + 1;
        const int nitems = L.nmark * span * span;
        for (int item = t; item < nitems; item += G) {
            if (__hip_atomic_load(&L.done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                break;
            const int r = L.uf[item / (span * span)];
            const int dz = (item % (span * span)) / span - R, dy = item % span - R;
            const int xyz = L.uxyz[r];
            // unit r in the frame of the neighbour cell
            const int rx = (xyz & 15) - ox * m, ry = ((xyz >> 4) & 15) - oy * m,
                      rz = (xyz >> 8) - oz * m;
            const int bz = rz + dz, by = ry + dy;
            if (bz < 0 || bz >= m || by < 0 || by >= m)
                continue;
            const int kz = max(0, abs(dz) - 1), ky = max(0, abs(dy) - 1);
            const int rem = K - kz * kz - ky * ky;
            if (rem < 0)
                continue;  // this row lies b or more from unit r
            const int sp = min(R, (int)sqrtf((float)rem) + 1);
            const int lo = max(-sp, -rx), hi = min(sp, m - 1 - rx);
            if (lo > hi)
                continue;
            const int key0 = (bz * m + by) * m + rx + lo;
            uint32_t row = row_bits(L.bits, W, key0, hi - lo + 1);
            while (row) {
                const int bpos = __ffs(row) - 1;
                row &= row - 1u;
                const int bx = rx + lo + bpos;
                const int rb = rank_in(L.bits, L.pre, key0 + bpos);
                const int cb = single ? 0 : (staged2 ? ncomp_of[rb] : w.cnt[s2 + rb]);
                const int bit = L.ucomp[r] * ncomp2 + cb;
                if (dedupe && ((L.pairbits[bit >> 5] >> (bit & 31)) & 1u))
                    continue;
                const int32_t b0 = staged2 ? nstart[rb] : w.rank[s2 + rb];
                const int32_t b1 = staged2 ? nstart[rb + 1]
                                           : (rb + 1 < u2 ? w.rank[s2 + rb + 1] : s2 + n2);
                // unit B's box in the own cell's periodic frame
                const FineBox fb = fine_box(B, (cc.x + ox) * m + bx, (cc.y + oy) * m + by,
                                            (cc.z + oz) * m + bz);
                FOF_STAT(w.ctr, ST_CROSS_UNIT_PAIRS, 1);
                int hit_i = -1, hit_j = -1;
                for (int i = L.ustart[r]; i < L.ustart[r + 1] && hit_i < 0; ++i) {
                    const float4 p = mem[i - s];
                    if (far_from(B, fb, p))
                        continue;
                    const int j = first_friend(P, p, w.sorted, b0, b1);
                    if (j >= 0) {
                        hit_i = i;
                        hit_j = j;
                    }
                }
                if (hit_i >= 0) {
                    uf_union(w.parent, (uint32_t)hit_i, (uint32_t)hit_j);
                    if (dedupe)
                        atomicOr(L.pairbits + (bit >> 5), 1u << (bit & 31));
                    if (single) {
                        __hip_atomic_store(&L.done, 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                        break;
                    }
                }
            }
        }
        Grp<G>::sync();
        FOF_PHASE(L, t == 0, 3);
    }
}

// Ordinary (sparse) particles around dense cell d, after the components.  A particle q of a
// neighbouring cell
// without a clique table is tested only if this cell lies within reach of q's position
// (the face test of the sparse search, from q's side), then only against the fine cells
// within reach of q, one friend per component of this cell.  q is then marked in the flag
// bitmap, so the compress pass gives it its component's label.
// kLds: the cell's particles are staged in LDS (it holds at most CAP), else read from HBM;
// fixed per instantiation, so every member access compiles to one kind of load.
// kDefer: hooks are appended to the deferred list (pairs in Work::temp, which the link stage
// does not otherwise use) for k_dense_edges, so the pass can run beside the tiled kernel,
// whose plain stores to ordinary particles' parents would overwrite a direct hook.
template <int G, bool kLds, bool kDefer, int UMAX, int CAP>
__device__ void sparse_cell(const Work &w, int d, CellLds<UMAX, CAP> &L)
{
    const int t = Grp<G>::tid();
    const int64_t c = w.dense_list[d];
    const int32_t s = w.cell_start[c];
    const int32_t n = w.cell_start[c + 1] - s;
    const BoxDesc &B = uniform_box(w.desc, find_box(w.desc, w.nbox, s));
    const CellXYZ cc = cell_xyz(B, c);
    const Pred P = pred_of(B);
    const int m = B.m;
    const int W = w.table_words;
    const int32_t *T = w.table + (int64_t)d * w.table_stride;
    const int u = T[2], ncomp = T[1];

    if (t == 0)
        L.nnb = 0;
    Grp<G>::sync();
    if (t < 27 && t != 13) {  // dense_ok boxes have nc >= 3: the 26 neighbours are distinct
        const int ox = t % 3 - 1, oy = (t / 3) % 3 - 1, oz = t / 9 - 1;
        const int64_t c2 = coarse_cell(B, wrap_cell(cc.x + ox, B.nc[0]),
                                       wrap_cell(cc.y + oy, B.nc[1]), wrap_cell(cc.z + oz, B.nc[2]));
        const int32_t s2 = w.cell_start[c2], n2 = w.cell_start[c2 + 1] - s2;
        if (n2 > 0 && !(n2 > w.dense_threshold && w.cell_count[c2] >= 0)) {
            const int k = atomicAdd(&L.nnb, 1);
            L.nb[k] = s2;
            L.nbp[k] = n2;
            L.nbo[k] = (short)((ox + 1) | ((oy + 1) << 2) | ((oz + 1) << 4));
        }
    }
    Grp<G>::sync();
    const int nnb = L.nnb;
    FOF_PHASE(L, t == 0, 0);
    if (nnb == 0) {  // uniform: every thread read the same count
        Grp<G>::sync();
        return;
    }
    if (t == 0) {  // counts -> running offsets (at most 26 entries)
        int acc = 0;
        for (int k = 0; k < nnb; ++k) {
            const int c2 = L.nbp[k];
            L.nbp[k] = acc;
            acc += c2;
        }
        L.nbp[nnb] = acc;
    }
    for (int q = t; q < W; q += G) {
        L.bits[q] = (uint32_t)T[kTableHeader + q];
        L.pre[q] = T[kTableHeader + W + q];
    }
    for (int r = t; r < u; r += G) {
        L.ustart[r] = w.rank[s + r];
        L.ucomp[r] = (short)w.cnt[s + r];
    }
    if (t == 0)
        L.ustart[u] = s + n;
    if (kLds)
        for (int k = t; k < n; k += G)
            L.part[k] = w.sorted[s + k];
    Grp<G>::sync();
    const float4 *mem = kLds ? L.part : w.sorted + s;
    const int total = L.nbp[nnb];
    FOF_PHASE(L, t == 0, 1);
    for (int e = t; e < total; e += G) {
        int k = 0;
        while (L.nbp[k + 1] <= e)
            ++k;
        const int o = L.nbo[k];
        const int ox = (o & 3) - 1, oy = ((o >> 2) & 3) - 1, oz = (o >> 4) - 1;
        const int32_t j = L.nb[k] + (e - L.nbp[k]);
        const float4 q = w.sorted[j];
        // q's cell, and this cell's coordinate in q's periodic frame (q's cell minus o)
        const int qx = wrap_cell(cc.x + ox, B.nc[0]), qy = wrap_cell(cc.y + oy, B.nc[1]),
                  qz = wrap_cell(cc.z + oz, B.nc[2]);
        const AxisSpan sx = axis_span(q.x, qx, B.side[0], B.nc[0], B.reach);
        const AxisSpan sy = axis_span(q.y, qy, B.side[1], B.nc[1], B.reach);
        const AxisSpan sz = axis_span(q.z, qz, B.side[2], B.nc[2], B.reach);
        if (-ox < sx.lo || -ox > sx.hi || -oy < sy.lo || -oy > sy.hi || -oz < sz.lo || -oz > sz.hi)
            continue;
        int x0, x1, y0, y1, z0, z1;
        key_range(q.x * B.inv_fine[0] - (float)((qx - ox) * m), B.reach * B.inv_fine[0], m, x0, x1);
        key_range(q.y * B.inv_fine[1] - (float)((qy - oy) * m), B.reach * B.inv_fine[1], m, y0, y1);
        key_range(q.z * B.inv_fine[2] - (float)((qz - oz) * m), B.reach * B.inv_fine[2], m, z0, z1);
        FOF_STAT(w.ctr, ST_DN_CALLS, 1);
        bool any = false;
        uint64_t seen = 0;  // components (numbers < 64) already joined
        for (int bz = z0; bz <= z1; ++bz)
            for (int by = y0; by <= y1 && x0 <= x1; ++by) {
                const int key0 = (bz * m + by) * m + x0;
                uint32_t row = row_bits(L.bits, W, key0, x1 - x0 + 1);
                while (row) {
                    const int bpos = __ffs(row) - 1;
                    row &= row - 1u;
                    const int rb = rank_in(L.bits, L.pre, key0 + bpos);
                    const int comp = L.ucomp[rb];
                    if (comp < 64 && ((seen >> comp) & 1ull))
                        continue;
                    FOF_STAT(w.ctr, ST_DN_UNITS, 1);
                    const int hit =
                        first_friend(P, q, mem, L.ustart[rb] - s, L.ustart[rb + 1] - s);
                    if (hit >= 0) {
                        if (kDefer) {
                            const int k = atomicAdd(&L.nhk, 1);
                            if (k < kHookBuf)
                                L.hk[k] = make_int2(j, s + hit);
                            else
                                defer_dense_hook(w, make_int2(j, s + hit));
                        } else {
                            uf_union(w.parent, (uint32_t)j, (uint32_t)(s + hit));
                        }
                        any = true;
                        if (comp < 64)
                            seen |= 1ull << comp;
                    }
                    if (any && ncomp == 1)
                        goto done;
                }
            }
    done:
        if (any)
            atomicOr((unsigned long long *)(w.flags + (j >> 6)), 1ull << (j & 63));
    }
    Grp<G>::sync();
    if (kDefer) {  // the cell's buffered hooks go to the list with one global atomic
        const int nh = min(L.nhk, kHookBuf);
        if (t == 0 && nh > 0)
            L.hkbase = atomicAdd(&w.ctr->n_dense_edges, nh);
        Grp<G>::sync();
        for (int k = t; k < nh; k += G) {
            if ((int64_t)(L.hkbase + k) < dense_edge_cap(w))
                reinterpret_cast<int2 *>(w.temp)[L.hkbase + k] = L.hk[k];
            else
                w.ctr->dense_edge_over = 1;
        }
        if (t == 0)
            L.nhk = 0;
        Grp<G>::sync();
    }
    FOF_PHASE(L, t == 0, 2);
}

// Work distribution of a dense pass.  Items (dense ids) are dealt to kCursorGroups groups,
// item d to group d % G; worker k (a wave or a block, of `nworkers`) serves group
// k % G, first taking item g + G * (k / G) and then further items of its group from the
// group's cursor.  Item costs differ widely, so the cursors balance the load; the groups
// keep each cursor's atomics few and on its own line.  The cursor is read before it is
// incremented, so that workers with nothing left do not queue on the atomic.
struct Deal {
    int32_t *cursor;
    int g, per_group;  // this worker's group, workers per group
};

__device__ __forceinline__ Deal deal(int32_t *cursors, int pass, int worker, int nworkers)
{
    const int G = kCursorGroups;
    const int g = worker % G;
    Deal dl;
    dl.cursor = cursors + (pass * G + g) * kCursorStride;
    dl.g = g;
    dl.per_group = (nworkers - g + G - 1) / G;  // workers k < nworkers with k % G == g
    return dl;
}

__device__ __forceinline__ int deal_first(const Deal &dl, int worker)
{
    return dl.g + kCursorGroups * (worker / kCursorGroups);
}

__device__ __forceinline__ int deal_next(const Deal &dl, int n)
{
    const int G = kCursorGroups;
    const int k0 = __hip_atomic_load(dl.cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (dl.g + G * (dl.per_group + k0) >= n)
        return n;
    return dl.g + G * (dl.per_group + atomicAdd(dl.cursor, 1));
}

// Small cells: one wave per cell, iterating over every dense id and skipping big cells.
// kMode: 0 components inside the cell, 1 dense neighbours, 2 ordinary neighbours (hooks
// deferred), 3 ordinary neighbours with direct hooks, run only when the deferred list
// overflowed.
template <int kMode>
__global__ __launch_bounds__(kDenseBlock) void k_dense_small(Work w)
{
    if (kMode == 3 && !w.ctr->dense_edge_over)  // uniform: every thread reads the same word
        return;
    __shared__ CellLds<kSmallCell, kSmallCell> lds[Grp<kWave>::per_block];
    CellLds<kSmallCell, kSmallCell> &L = lds[Grp<kWave>::slot()];
    if (lane_id() == 0)
        L.nhk = 0;
    Grp<kWave>::sync();
    const int nd = dense_count(w.ctr, w.dense_cap);
    const int nworkers = gridDim.x * Grp<kWave>::per_block;
    const int worker = blockIdx.x * Grp<kWave>::per_block + Grp<kWave>::slot();
    const Deal dl = deal(w.cursors, 2 * kMode, worker, nworkers);
    FOF_PHASE_START(L, lane_id() == 0);
    int d = deal_first(dl, worker);
    while (d < nd) {
        const int64_t c = w.dense_list[d];
        if (w.cell_start[c + 1] - w.cell_start[c] <= kSmallCell) {
            if (kMode == 1)
                cross_cell<kWave, true>(w, d, L);
            else if (kMode >= 2)
                sparse_cell<kWave, true, kMode == 2>(w, d, L);
            else
                cc_cell<kWave, true>(w, d, L);
        }
        int nx = 0;
        if (lane_id() == 0)
            nx = deal_next(dl, nd);
        d = __shfl(nx, 0, kWave);
        FOF_PHASE(L, lane_id() == 0, 7);
    }
    FOF_PHASE(L, lane_id() == 0, 7);
    FOF_PHASE_FLUSH(L, lane_id() == 0 && kMode == 0, w.ctr, 0);
#if defined(FOF_TIMING) && !defined(FOF_TIMING_BIG)
    if (lane_id() == 0 && (kMode == 1 || kMode == 2))
        for (int k = 0; k < 4; ++k)
            atomicAdd(&w.ctr->stats[16 + 4 * (kMode - 1) + k], (unsigned long long)L.phase[k]);
#endif
}

// Big cells: one block per cell, over the list of big dense ids (BLOCK threads: 512 for the
// components pass, whose loops over units and members gain from twice the waves per CU;
// the pair passes run slower that way beside the tiled kernel, so they keep 256).
template <int kMode, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_dense_big(Work w)
{
    if (kMode == 3 && !w.ctr->dense_edge_over)
        return;
    __shared__ CellLds<kMaxFineKeys, kLdsCap> L;
    __shared__ int next;
    if (threadIdx.x == 0)
        L.nhk = 0;
    __syncthreads();
    const int nb = __hip_atomic_load(&w.ctr->n_big, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const Deal dl = deal(w.cursors, 2 * kMode + 1, blockIdx.x, gridDim.x);
    FOF_PHASE_START(L, threadIdx.x == 0);
    for (int k = deal_first(dl, blockIdx.x); k < nb;) {
        const int d = w.big_list[k];
        const int64_t c = w.dense_list[d];
        if (w.cell_start[c + 1] - w.cell_start[c] <= kLdsCap) {
            if (kMode == 1)
                cross_cell<BLOCK, true>(w, d, L);
            else if (kMode >= 2)
                sparse_cell<BLOCK, true, kMode == 2>(w, d, L);
            else
                cc_cell<BLOCK, true>(w, d, L);
        } else {
            if (kMode == 1)
                cross_cell<BLOCK, false>(w, d, L);
            else if (kMode >= 2)
                sparse_cell<BLOCK, false, kMode == 2>(w, d, L);
            else
                cc_cell<BLOCK, false>(w, d, L);
        }
        if (threadIdx.x == 0)
            next = deal_next(dl, nb);
        __syncthreads();
        k = next;
        __syncthreads();  // every thread has read `next` before it is overwritten
        FOF_PHASE(L, threadIdx.x == 0, 7);
    }
    FOF_PHASE(L, threadIdx.x == 0, 7);
    FOF_PHASE_FLUSH(L, threadIdx.x == 0 && kMode == 0, w.ctr, 8);
#if defined(FOF_TIMING) && defined(FOF_TIMING_BIG)  // diagnostic: big cells' pair passes
    if (threadIdx.x == 0 && (kMode == 1 || kMode == 2))
        for (int k = 0; k < 4; ++k)
            atomicAdd(&w.ctr->stats[16 + 4 * (kMode - 1) + k], (unsigned long long)L.phase[k]);
#endif

}

// The sparse-dense pass's deferred hooks, once the tiled kernel's plain stores are done.
__global__ void k_dense_edges(Work w)
{
    const int64_t cap = dense_edge_cap(w);
    const int64_t m = min((int64_t)w.ctr->n_dense_edges, cap);
    const int2 *e = reinterpret_cast<const int2 *>(w.temp);
    for (int64_t k = gtid(); k < m; k += (int64_t)gridDim.x * blockDim.x)
        uf_union(w.parent, (uint32_t)e[k].x, (uint32_t)e[k].y);
}

// Blocks of a dense pass: enough to fill the chip, at most one per possible item, and at
// least one worker per cursor group (every group's items need a worker).
unsigned persistent_blocks(int cap)
{
    int b = cap < 4096 ? cap : 4096;
    return (unsigned)(b > kCursorGroups ? b : kCursorGroups);
}

void launch_dense_sorts(const Work &w, hipStream_t s)
{
    hipLaunchKernelGGL(k_dense_sort, dim3(persistent_blocks(w.dense_cap)), dim3(kDenseBlock), 0, s,
                       w);
}

}  // namespace

hipError_t launch_dense_build(const Work &w, hipStream_t s, bool classified)
{
    if (w.dense_cap <= 0 || w.dense_threshold < 0)
        return hipSuccess;
    if (classified) {  // the bucketed sort numbered the dense cells already
        launch_dense_sorts(w, s);
        return hipGetLastError();
    }
    const int64_t nchunk = (w.ncell + kClassChunk - 1) / kClassChunk;
    int32_t *nd = w.classify, *nd_pre = nd + (nchunk + 1);
    int32_t *nbig = nd_pre + (nchunk + 1), *nbig_pre = nbig + (nchunk + 1);
    const unsigned cb = (unsigned)(nchunk < 65536 ? (nchunk > 0 ? nchunk : 1) : 65536);
    hipLaunchKernelGGL(k_classify_count, dim3(cb), dim3(kClassBlock), 0, s, w, nchunk, nd, nbig);
    hipError_t e = launch_scan_i32(nd, nd_pre, nchunk, w.scan, s);
    if (e != hipSuccess)
        return e;
    e = launch_scan_i32(nbig, nbig_pre, nchunk, w.scan, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_classify_totals, dim3(1), dim3(64), 0, s, w.ctr, nchunk, nd_pre,
                       nbig_pre);
    hipLaunchKernelGGL(k_classify_assign, dim3(cb), dim3(kClassBlock), 0, s, w, nchunk, nd_pre,
                       nbig_pre);
    launch_dense_sorts(w, s);
    return hipGetLastError();
}

// Components, the ordinary neighbours of dense cells (hooks deferred), then pairs of dense
// cells; `hooks_listed` (optional) is recorded once the deferred hooks are all listed.
hipError_t launch_dense(const Work &w, hipStream_t s, hipEvent_t hooks_listed)
{
    if (w.dense_cap <= 0 || w.dense_threshold < 0)
        return hipSuccess;
    hipError_t e = launch_fill_i32(w.cursors, kCursorInts, 0, s);
    if (e == hipSuccess)
        e = launch_fill_i32(&w.ctr->n_dense_edges, 2, 0, s);  // n_dense_edges, dense_edge_over
    if (e != hipSuccess)
        return e;
    const unsigned pb = persistent_blocks(w.dense_cap);
    // in each pass the big cells first: their few long blocks then overlap the small cells'
    // many short ones of the next pass instead of ending the chain (about 0.07 ms at 512^3)
    hipLaunchKernelGGL((k_dense_big<0, kBigBlock>), dim3(pb), dim3(kBigBlock), 0, s, w);
    hipLaunchKernelGGL(k_dense_small<0>, dim3(pb), dim3(kDenseBlock), 0, s, w);
    hipLaunchKernelGGL((k_dense_big<2, kDenseBlock>), dim3(pb), dim3(kDenseBlock), 0, s, w);
    hipLaunchKernelGGL(k_dense_small<2>, dim3(pb), dim3(kDenseBlock), 0, s, w);
    if (hooks_listed && (e = hipEventRecord(hooks_listed, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_dense_big<1, kDenseBlock>), dim3(pb), dim3(kDenseBlock), 0, s, w);
    hipLaunchKernelGGL(k_dense_small<1>, dim3(pb), dim3(kDenseBlock), 0, s, w);
    return hipGetLastError();
}

// After every plain store of the tiled kernel: the deferred sparse-dense hooks, then (only
// if their list overflowed) the sparse-dense pass again with direct hooks.
hipError_t launch_dense_hooks(const Work &w, hipStream_t s)
{
    if (w.dense_cap <= 0 || w.dense_threshold < 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_dense_edges, dim3(1024), dim3(256), 0, s, w);
    const unsigned pb = persistent_blocks(w.dense_cap);
    hipLaunchKernelGGL(k_dense_small<3>, dim3(pb), dim3(kDenseBlock), 0, s, w);
    hipLaunchKernelGGL((k_dense_big<3, kDenseBlock>), dim3(pb), dim3(kDenseBlock), 0, s, w);
    return hipGetLastError();
}

}  // namespace fof
